"""Python front end of the FP64 CPU oracle (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this module.  It wraps ``liboracle.so`` (built from
``rt_oracle.c`` with gcc, ``-ffp-contract=off``) and applies it slab by slab
to a multi-slab problem: the slabs are independent, so the operator is block
diagonal and every solver runs per slab.

It takes plain arrays (a ``Problem`` from the input generators, or any object
with the same fields); it imports nothing from the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# A test may point the wrapper at another build of the same source (the
# mutation test plants mistakes in a temporary copy and loads that build).
_LIB_OVERRIDE = os.environ.get("RT_ORACLE_LIB")
_lock = threading.Lock()
_lib = None

STATUS = {0: "converged", 1: "maxit", 2: "breakdown", -1: "nomem"}


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C99, FP64, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
                               "-fPIC", "-shared", "-Wall", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Slab(C.Structure):
    _fields_ = [
        ("ns", C.c_int), ("tau", C.POINTER(C.c_double)),
        ("nmu", C.c_int), ("mu", C.POINTER(C.c_double)), ("wmu", C.POINTER(C.c_double)),
        ("nnu", C.c_int), ("wnu", C.POINTER(C.c_double)), ("phi", C.POINTER(C.c_double)),
        ("opac", C.POINTER(C.c_double)),
        ("eps", C.c_double), ("W2", C.c_double), ("Ibot", C.c_double),
        ("B", C.POINTER(C.c_double)),
        ("fs", C.c_int), ("normalize", C.c_int),
    ]


class _Prec(C.Structure):
    _fields_ = [("kind", C.c_int), ("dinv", C.POINTER(C.c_double)),
                ("A", C.POINTER(C.c_double)), ("omega", C.c_double)]


PRECONDITIONERS = {"none": 0, "jacobi": 1, "sor": 2, "ssor": 3}


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if _LIB_OVERRIDE:
                L = C.CDLL(_LIB_OVERRIDE)
            else:
                if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                    build(force=True)
                L = C.CDLL(_LIB)
            P = C.POINTER(_Slab)
            D = C.POINTER(C.c_double)
            I = C.POINTER(C.c_int)
            L.orc_t20.argtypes = [C.c_double, D, D]
            L.orc_delo_linear.argtypes = [C.c_double, D, D, D]
            L.orc_trapezoid.argtypes = [C.c_double, D, D]
            L.orc_implicit_euler.argtypes = [C.c_double, D, D]
            L.orc_delo_parabolic.argtypes = [C.c_double, C.c_double, D, D, D, D]
            L.orc_exp_moments.argtypes = [C.c_double, D]
            L.orc_ray.argtypes = [C.c_int, D, C.c_double, C.c_int, C.c_int, D, C.c_double, D]
            L.orc_weights.argtypes = [P, D]
            L.orc_apply.argtypes = [P, D, D]
            L.orc_rhs.argtypes = [P, D]
            L.orc_diag.argtypes = [P, C.c_int, I, D]
            L.orc_assemble.argtypes = [P, D]
            L.orc_apply_I.argtypes = [P, D, D]
            L.orc_rhs_I.argtypes = [P, D]
            L.orc_sigma_from_I.argtypes = [P, D, D]
            Q = C.POINTER(_Prec)
            L.orc_gmres.argtypes = [P, D, D, Q, C.c_int, C.c_double, C.c_int, I, I, D, D, C.c_int,
                                    C.c_int]
            L.orc_bicgstab.argtypes = [P, D, D, Q, C.c_double, C.c_int, I, I, D]
            L.orc_richardson.argtypes = [P, D, D, Q, C.c_double, C.c_int, I, I, D]
            L.orc_cgs.argtypes = [P, D, D, Q, C.c_double, C.c_int, I, I, D]
            for f in ("orc_apply", "orc_rhs", "orc_diag", "orc_assemble", "orc_gmres",
                      "orc_apply_I", "orc_rhs_I", "orc_sigma_from_I",
                      "orc_bicgstab", "orc_richardson", "orc_cgs"):
                getattr(L, f).restype = C.c_int
            _lib = L
        return _lib


class _SlabView:
    """Keeps the numpy buffers of one slab alive while C holds pointers."""

    def __init__(self, prob, i):
        off = prob.offsets
        s = slice(int(off[i]), int(off[i + 1]))
        self.tau = np.ascontiguousarray(prob.tau[s], dtype=np.float64)
        self.B = np.ascontiguousarray(prob.B[s], dtype=np.float64)
        self.mu = np.ascontiguousarray(prob.mu, dtype=np.float64)
        self.wmu = np.ascontiguousarray(prob.w_mu, dtype=np.float64)
        self.wnu = np.ascontiguousarray(prob.w_nu, dtype=np.float64)
        self.phi = np.ascontiguousarray(prob.phi[i], dtype=np.float64)
        self.opac = np.ascontiguousarray(prob.opac[i], dtype=np.float64)
        self.ns = int(prob.ns[i])
        self.c = _Slab(self.ns, _dp(self.tau), self.mu.shape[0], _dp(self.mu), _dp(self.wmu),
                       self.wnu.shape[0], _dp(self.wnu), _dp(self.phi), _dp(self.opac),
                       float(prob.eps[i]), float(prob.W2[i]), float(prob.I_bot[i]), _dp(self.B),
                       int(prob.formal_solver), int(bool(prob.normalize_profile)))

    @property
    def ref(self):
        return C.byref(self.c)


def _slices(prob):
    off = 2 * prob.offsets
    return [slice(int(off[i]), int(off[i + 1])) for i in range(prob.n_atm)]


# ----------------------------------------------------------------------------
# scalar building blocks (exposed for the pins)
# ----------------------------------------------------------------------------

def t20(mu):
    a, b = C.c_double(), C.c_double()
    lib().orc_t20(float(mu), C.byref(a), C.byref(b))
    return a.value, b.value


def delo_linear(d):
    E, pu, pk = C.c_double(), C.c_double(), C.c_double()
    lib().orc_delo_linear(float(d), C.byref(E), C.byref(pu), C.byref(pk))
    return E.value, pu.value, pk.value


def trapezoid(d):
    a, b = C.c_double(), C.c_double()
    lib().orc_trapezoid(float(d), C.byref(a), C.byref(b))
    return a.value, b.value


def implicit_euler(d):
    a, b = C.c_double(), C.c_double()
    lib().orc_implicit_euler(float(d), C.byref(a), C.byref(b))
    return a.value, b.value


def delo_parabolic(d, dd):
    """(E, c_u, c_k, c_d) of a DELO-parabolic step with upwind optical step d
    and downwind step dd."""
    E, pu, pk, pd = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    lib().orc_delo_parabolic(float(d), float(dd), C.byref(E), C.byref(pu), C.byref(pk),
                             C.byref(pd))
    return E.value, pu.value, pk.value, pd.value


def exp_moments(d):
    """int_0^d t^n exp(-t) dt for n = 0, 1, 2."""
    w = np.zeros(3)
    lib().orc_exp_moments(float(d), _dp(w))
    return w


def ray(tau, kappa, upward, S, I_entry=0.0, fs=0):
    tau = np.ascontiguousarray(tau, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    I = np.zeros_like(tau)
    lib().orc_ray(tau.shape[0], _dp(tau), float(kappa), int(bool(upward)), int(fs), _dp(S),
                  float(I_entry), _dp(I))
    return I


def weights(prob, i=0):
    v = _SlabView(prob, i)
    q = np.zeros(prob.n_mu * prob.n_nu)
    lib().orc_weights(v.ref, _dp(q))
    return q.reshape(prob.n_mu, prob.n_nu)


# ----------------------------------------------------------------------------
# operator, right-hand side, diagonal
# ----------------------------------------------------------------------------

def apply(prob, sigma_in):
    """sigma_out = A sigma_in = sigma_in - J Lambda T sigma_in over all slabs."""
    x = np.ascontiguousarray(sigma_in, dtype=np.float64)
    y = np.empty_like(x)
    for i, s in enumerate(_slices(prob)):
        v = _SlabView(prob, i)
        xs = np.ascontiguousarray(x[s])
        ys = np.empty_like(xs)
        if lib().orc_apply(v.ref, _dp(xs), _dp(ys)) != 0:
            raise MemoryError("oracle apply")
        y[s] = ys
    return y


def apply_slab(prob, i, sigma_slab):
    v = _SlabView(prob, i)
    xs = np.ascontiguousarray(sigma_slab, dtype=np.float64)
    ys = np.empty_like(xs)
    if lib().orc_apply(v.ref, _dp(xs), _dp(ys)) != 0:
        raise MemoryError("oracle apply")
    return ys


def rhs(prob):
    out = np.empty(prob.n_unknowns)
    for i, s in enumerate(_slices(prob)):
        v = _SlabView(prob, i)
        bs = np.empty(s.stop - s.start)
        lib().orc_rhs(v.ref, _dp(bs))
        out[s] = bs
    return out


def diag(prob, indices=None):
    """Diagonal of A from unit vectors; ``indices`` are global (all slabs)."""
    n = prob.n_unknowns
    idx = np.arange(n) if indices is None else np.asarray(indices, dtype=np.int64)
    out = np.empty(idx.shape[0])
    sl = _slices(prob)
    starts = np.array([s.start for s in sl])
    for i, s in enumerate(sl):
        sel = np.nonzero((idx >= s.start) & (idx < s.stop))[0]
        if sel.size == 0:
            continue
        v = _SlabView(prob, i)
        loc = np.ascontiguousarray(idx[sel] - starts[i], dtype=np.int32)
        d = np.empty(sel.size)
        lib().orc_diag(v.ref, loc.shape[0], loc.ctypes.data_as(C.POINTER(C.c_int)), _dp(d))
        out[sel] = d
    return out


def assemble(prob, i=0):
    """Dense A of slab i, column by column (Sect. 3.3)."""
    v = _SlabView(prob, i)
    n = 2 * int(prob.ns[i])
    A = np.empty((n, n))
    lib().orc_assemble(v.ref, _dp(A))
    return A


# ----------------------------------------------------------------------------
# the field as unknown (eq. crd_linear_system2), one slab at a time; field
# index ((st * nmu + m) * nnu + p) * ns + k, st = 0 for I, 1 for Q
# ----------------------------------------------------------------------------

def field_size(prob, i=0):
    return 2 * int(prob.ns[i]) * len(prob.mu) * len(prob.w_nu)


def apply_I(prob, field, i=0):
    """(Id - Lambda T J) I for slab i."""
    v = _SlabView(prob, i)
    f = np.ascontiguousarray(field, dtype=np.float64)
    out = np.empty_like(f)
    lib().orc_apply_I(v.ref, _dp(f), _dp(out))
    return out


def rhs_I(prob, i=0):
    """Lambda T c + t for slab i."""
    v = _SlabView(prob, i)
    out = np.empty(field_size(prob, i))
    lib().orc_rhs_I(v.ref, _dp(out))
    return out


def sigma_from_I(prob, field, i=0):
    """sigma = J I + c for slab i."""
    v = _SlabView(prob, i)
    f = np.ascontiguousarray(field, dtype=np.float64)
    out = np.empty(2 * int(prob.ns[i]))
    lib().orc_sigma_from_I(v.ref, _dp(f), _dp(out))
    return out


# ----------------------------------------------------------------------------
# solvers (per slab)
# ----------------------------------------------------------------------------

def _solve(kind, prob, b, x0, prec, tol, maxit, restart=30, hist_len=0, left=False):
    """prec: None, or ("jacobi", dinv over all slabs), or ("sor" | "ssor", omega)."""
    n = prob.n_unknowns
    b = np.ascontiguousarray(b if b is not None else rhs(prob), dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    info = []
    hists = []
    for i, s in enumerate(_slices(prob)):
        v = _SlabView(prob, i)
        bs = np.ascontiguousarray(b[s])
        xs = np.ascontiguousarray(x[s])
        it, mv, rr = C.c_int(), C.c_int(), C.c_double()
        keep = None
        if prec is None:
            dptr = None
        elif prec[0] == "jacobi":
            keep = np.ascontiguousarray(prec[1][s], dtype=np.float64)
            dptr = C.byref(_Prec(1, _dp(keep), None, 1.0))
        else:
            keep = np.empty((bs.size, bs.size))
            lib().orc_assemble(v.ref, _dp(keep))
            dptr = C.byref(_Prec(PRECONDITIONERS[prec[0]], None, _dp(keep), float(prec[1])))
        if kind == "gmres":
            h = np.zeros(max(hist_len, 1))
            st = lib().orc_gmres(v.ref, _dp(bs), _dp(xs), dptr, int(restart), float(tol),
                                 int(maxit), C.byref(it), C.byref(mv), C.byref(rr), _dp(h),
                                 int(hist_len), int(bool(left)))
            hists.append(h[:min(hist_len, it.value + 1)] if hist_len else None)
        elif kind == "bicgstab":
            st = lib().orc_bicgstab(v.ref, _dp(bs), _dp(xs), dptr, float(tol), int(maxit),
                                    C.byref(it), C.byref(mv), C.byref(rr))
        elif kind == "richardson":
            st = lib().orc_richardson(v.ref, _dp(bs), _dp(xs), dptr, float(tol), int(maxit),
                                      C.byref(it), C.byref(mv), C.byref(rr))
        elif kind == "cgs":
            st = lib().orc_cgs(v.ref, _dp(bs), _dp(xs), dptr, float(tol), int(maxit),
                               C.byref(it), C.byref(mv), C.byref(rr))
        else:
            raise ValueError(kind)
        x[s] = xs
        info.append(dict(status=STATUS.get(st, st), iterations=it.value, matvecs=mv.value,
                         relres=rr.value))
    _ = n
    if hist_len:
        return x, info, hists
    return x, info


def jacobi_inverse(prob):
    return 1.0 / diag(prob)


def _prec(prob, precond, dinv, omega):
    """Preconditioner spec (Sect. 2.3): True or "jacobi" (P = D), False or
    "none", "sor" or "ssor" (relaxation omega, from the assembled A)."""
    if precond is True:
        precond = "jacobi"
    if precond is False or precond is None or precond == "none":
        return None
    if precond == "jacobi":
        return ("jacobi", jacobi_inverse(prob) if dinv is None else dinv)
    if precond in ("sor", "ssor"):
        if not 0.0 < omega < 2.0:
            raise ValueError("omega must lie in (0, 2)")
        return (precond, float(omega))
    raise ValueError(f"unknown preconditioner {precond!r}")


def gmres(prob, b=None, x0=None, precond=True, tol=1e-10, maxit=10000, restart=30,
          dinv=None, hist_len=0, left=False, omega=1.0):
    """GMRES(restart) of Sect. 2.1, right-preconditioned by default (minimizes
    and tests the true residual).  left=True preconditions from the left and
    minimizes and tests the preconditioned residual ||P^-1 (b - A x)||."""
    if x0 is None:
        x0 = _x0(prob)
    return _solve("gmres", prob, b, x0, _prec(prob, precond, dinv, omega), tol, maxit, restart,
                  hist_len, left)


def bicgstab(prob, b=None, x0=None, precond=True, tol=1e-10, maxit=10000, dinv=None,
             omega=1.0):
    if x0 is None:
        x0 = _x0(prob)
    return _solve("bicgstab", prob, b, x0, _prec(prob, precond, dinv, omega), tol, maxit)


def cgs(prob, b=None, x0=None, precond=True, tol=1e-10, maxit=10000, dinv=None, omega=1.0):
    if x0 is None:
        x0 = _x0(prob)
    return _solve("cgs", prob, b, x0, _prec(prob, precond, dinv, omega), tol, maxit)


def richardson(prob, b=None, x0=None, precond=True, tol=1e-10, maxit=100000, dinv=None,
               omega=1.0):
    if x0 is None:
        x0 = _x0(prob)
    return _solve("richardson", prob, b, x0, _prec(prob, precond, dinv, omega), tol, maxit)


def _x0(prob):
    x0 = np.zeros(prob.n_unknowns)
    x0[0::2] = 1.0
    return x0
