"""ctypes binding of librt.so (include/rt.h, include/rt_ext.h).

Argument marshalling only: every step of the operator and of the solvers runs
in the gfx950 kernels of the library.  Vectors are torch CUDA (HIP) float64
tensors; streams are torch streams (default: torch's current stream).  There is
no CPU fallback: if the library is missing or no gfx950 device is present the
calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librt.so")

RT_OK, RT_EINVAL, RT_ENOMEM, RT_EDEVICE, RT_ENOCONV, RT_EBREAKDOWN = 0, -1, -2, -3, 1, 2
RT_FS_DELO_LINEAR, RT_FS_TRAPEZOIDAL, RT_FS_IMPLICIT_EULER, RT_FS_DELO_PARABOLIC = 0, 1, 2, 3
RT_PREC_FP64, RT_PREC_MIXED = 0, 1
RT_PC_JACOBI, RT_PC_SOR, RT_PC_SSOR = 0, 1, 2
RT_COEF_AUTO, RT_COEF_PAIRS, RT_COEF_STREAM_W, RT_COEF_RECOMPUTE, RT_COEF_RECOMPUTE_FP32 = \
    0, 1, 2, 3, 4
RT_MAX_NS = 2048
RT_MAX_RESTART = 128
STATUS_NAMES = {RT_OK: "converged", RT_ENOCONV: "maxit", RT_EBREAKDOWN: "breakdown"}

# every function the headers declare
EXPORTS = ["rt_default_options", "rt_setup", "rt_destroy", "rt_num_unknowns", "rt_apply_op",
           "rt_precond_jacobi", "rt_get_rhs", "rt_get_jacobi_diag", "rt_solve_gmres",
           "rt_solve_bicgstab", "rt_solve_richardson", "rt_solve_cgs", "rt_last_error",
           "rt_apply_op_fp32", "rt_apply_op_noalloc",
           "rt_plan_info", "rt_sweep_config", "rt_sweep_coef_mode", "rt_validate",
           "rt_tuned_plan_status", "rt_sweep_source_hash", "rt_plan_key", "rt_get_options", "rt_assembled_size", "rt_assemble",
           "rt_precond_apply", "rt_solve_lu", "rt_field_size", "rt_apply_op_field",
           "rt_get_rhs_field", "rt_sigma_from_field", "rt_solve_field_gmres",
           "rt_set_redistribution", "rt_prd_size", "rt_apply_op_prd", "rt_apply_op_prd_bf16x3", "rt_get_rhs_prd",
           "rt_get_jacobi_diag_prd", "rt_solve_prd_gmres"]


class RTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"rt error {code}: {msg}")
        self.code = code


class rt_problem(C.Structure):
    _fields_ = [
        ("n_atm", C.c_int), ("ns", C.POINTER(C.c_int)), ("tau", C.POINTER(C.c_double)),
        ("n_mu", C.c_int), ("mu", C.POINTER(C.c_double)), ("w_mu", C.POINTER(C.c_double)),
        ("n_nu", C.c_int), ("w_nu", C.POINTER(C.c_double)), ("phi", C.POINTER(C.c_double)),
        ("opac", C.POINTER(C.c_double)), ("eps", C.POINTER(C.c_double)),
        ("W2", C.POINTER(C.c_double)), ("B", C.POINTER(C.c_double)),
        ("I_bot", C.POINTER(C.c_double)), ("formal_solver", C.c_int),
        ("normalize_profile", C.c_int), ("R", C.POINTER(C.c_double)),
    ]


class rt_options(C.Structure):
    _fields_ = [
        ("precision", C.c_int), ("restart", C.c_int), ("maxit", C.c_int), ("rtol", C.c_double),
        ("inner_rtol", C.c_double), ("inner_maxit", C.c_int), ("max_outer", C.c_int),
        ("chunk", C.c_int), ("wave_batches", C.c_int), ("prefetch", C.c_int),
        ("check_every", C.c_int), ("sweep_waves", C.c_int), ("graphs", C.c_int),
        ("precond", C.c_int), ("omega", C.c_double), ("coef_mode", C.c_int),
        ("autotune", C.c_int), ("plan_file", C.c_char_p),
    ]


class rt_solve_info(C.Structure):
    _fields_ = [("status", C.c_int), ("iterations", C.c_int), ("matvecs", C.c_int),
                ("outer_steps", C.c_int), ("relres", C.c_double)]


_lib = None


def lib():
    """Load librt.so; raise if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build() or "
                              "python paper_2110_11873_amd/csrc/build.py")
        L = C.CDLL(LIB_PATH)
        vp, dp = C.c_void_p, C.POINTER(C.c_double)
        L.rt_default_options.argtypes = [C.POINTER(rt_options)]
        L.rt_default_options.restype = None
        L.rt_setup.argtypes = [C.POINTER(vp), C.POINTER(rt_problem), C.POINTER(rt_options)]
        L.rt_destroy.argtypes = [vp]
        L.rt_destroy.restype = None
        L.rt_num_unknowns.argtypes = [vp]
        for f in ("rt_apply_op", "rt_apply_op_fp32", "rt_apply_op_noalloc", "rt_precond_jacobi",
                  "rt_precond_apply"):
            getattr(L, f).argtypes = [vp, vp, vp, vp]
        for f in ("rt_get_rhs", "rt_get_jacobi_diag"):
            getattr(L, f).argtypes = [vp, vp, vp]
        for f in ("rt_solve_gmres", "rt_solve_bicgstab", "rt_solve_richardson", "rt_solve_cgs",
                  "rt_solve_lu", "rt_solve_field_gmres", "rt_solve_prd_gmres"):
            getattr(L, f).argtypes = [vp, vp, vp, C.POINTER(rt_solve_info), vp]
        L.rt_last_error.argtypes = []
        L.rt_last_error.restype = C.c_char_p
        L.rt_plan_info.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                   C.POINTER(C.c_longlong), C.POINTER(C.c_longlong)]
        L.rt_sweep_config.argtypes = [vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.rt_sweep_coef_mode.argtypes = [vp, C.c_int, C.POINTER(C.c_int)]
        L.rt_tuned_plan_status.argtypes = [vp]
        L.rt_get_options.argtypes = [vp, C.POINTER(rt_options)]
        L.rt_sweep_source_hash.argtypes = []
        L.rt_sweep_source_hash.restype = C.c_char_p
        L.rt_plan_key.argtypes = [C.POINTER(rt_problem), C.c_int, C.c_char_p, C.c_char_p, C.c_int]
        L.rt_validate.argtypes = [C.POINTER(rt_problem), C.POINTER(rt_options)]
        L.rt_assembled_size.argtypes = [vp, C.POINTER(C.c_longlong)]
        L.rt_field_size.argtypes = [vp, C.POINTER(C.c_longlong)]
        L.rt_set_redistribution.argtypes = [vp, C.POINTER(C.c_double)]
        L.rt_prd_size.argtypes = [vp, C.POINTER(C.c_longlong)]
        L.rt_apply_op_prd.argtypes = [vp, vp, vp, vp]
        L.rt_apply_op_prd_bf16x3.argtypes = [vp, vp, vp, vp]
        L.rt_get_rhs_prd.argtypes = [vp, vp, vp]
        L.rt_get_jacobi_diag_prd.argtypes = [vp, vp, vp]
        L.rt_apply_op_field.argtypes = [vp, vp, vp, vp]
        L.rt_get_rhs_field.argtypes = [vp, vp, vp]
        L.rt_sigma_from_field.argtypes = [vp, vp, vp, vp]
        L.rt_assemble.argtypes = [vp, vp, vp]
        _ = dp
        _lib = L
    return _lib


def last_error() -> str:
    return lib().rt_last_error().decode()


def _check(rc):
    if rc < 0:
        raise RTError(rc, last_error())
    return rc


def default_options(**kw) -> rt_options:
    o = rt_options()
    lib().rt_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        if k == "plan_file" and isinstance(v, str):
            v = v.encode()
        setattr(o, k, v)
    return o


def sweep_source_hash() -> str:
    """Hash of the sweep sources the loaded library was built from."""
    return lib().rt_sweep_source_hash().decode()


def plan_key(prob, mixed: bool, arch: Optional[str] = None) -> str:
    """The key under which the launch plan of `prob` is stored (rt_plan_key)."""
    pb = _ProblemBuffers(prob)
    buf = C.create_string_buffer(256)
    _check(lib().rt_plan_key(C.byref(pb.c), RT_PREC_MIXED if mixed else RT_PREC_FP64,
                             arch.encode() if arch else None, buf, 256))
    return buf.value.decode()


class _ProblemBuffers:
    """Holds contiguous host copies while rt_setup reads them."""

    def __init__(self, prob, R=None):
        f = lambda a: np.ascontiguousarray(a, dtype=np.float64)  # noqa: E731
        self.ns = np.ascontiguousarray(prob.ns, dtype=np.int32)
        self.tau, self.mu, self.w_mu = f(prob.tau), f(prob.mu), f(prob.w_mu)
        self.w_nu, self.phi, self.opac = f(prob.w_nu), f(prob.phi), f(prob.opac)
        self.eps, self.W2, self.B, self.I_bot = f(prob.eps), f(prob.W2), f(prob.B), f(prob.I_bot)
        d = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
        self.c = rt_problem(
            int(self.ns.shape[0]), self.ns.ctypes.data_as(C.POINTER(C.c_int)), d(self.tau),
            int(self.mu.shape[0]), d(self.mu), d(self.w_mu), int(self.w_nu.shape[0]), d(self.w_nu),
            d(self.phi), d(self.opac), d(self.eps), d(self.W2), d(self.B), d(self.I_bot),
            int(prob.formal_solver), int(bool(prob.normalize_profile)))
        # optional redistribution matrices, R[s][p][q] (one (n_nu, n_nu) matrix
        # serves a single slab)
        self.R = None if R is None else f(R)
        if self.R is not None:
            self.c.R = d(self.R)


def validate(prob, options: Optional[rt_options] = None) -> int:
    """rt_validate: host-side checks only (no device needed)."""
    pb = _ProblemBuffers(prob)
    return lib().rt_validate(C.byref(pb.c), C.byref(options) if options is not None else None)


@dataclass
class SolveInfo:
    status: str
    iterations: int
    matvecs: int
    outer_steps: int
    relres: float


def _ptr(t) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 \
            or not t.is_contiguous():
        raise TypeError("vectors must be contiguous float64 tensors on the GPU")
    return t.data_ptr()


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Handle:
    """An rt_handle: a problem set up on the current GPU."""

    def __init__(self, prob, options: Optional[rt_options] = None, R=None, **kw):
        self.options = options if options is not None else default_options(**kw)
        pb = _ProblemBuffers(prob, R)
        h = C.c_void_p()
        _check(lib().rt_setup(C.byref(h), C.byref(pb.c), C.byref(self.options)))
        self._h = h
        self.n = lib().rt_num_unknowns(h)
        self.n_atm = int(pb.ns.shape[0])
        self.ns = [int(n) for n in pb.ns]

    def close(self):
        if getattr(self, "_h", None):
            lib().rt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _new(self):
        import torch
        return torch.empty(self.n, dtype=torch.float64, device="cuda")

    # -- operator and preconditioner ------------------------------------------
    def apply_op(self, sigma_in, sigma_out=None, stream=None):
        out = self._new() if sigma_out is None else sigma_out
        _check(lib().rt_apply_op(self._h, C.c_void_p(_ptr(sigma_in)), C.c_void_p(_ptr(out)),
                                 _stream(stream)))
        return out

    def apply_op_fp32(self, sigma_in, sigma_out=None, stream=None):
        out = self._new() if sigma_out is None else sigma_out
        _check(lib().rt_apply_op_fp32(self._h, C.c_void_p(_ptr(sigma_in)), C.c_void_p(_ptr(out)),
                                      _stream(stream)))
        return out

    def apply_op_noalloc(self, sigma_in, sigma_out=None, stream=None):
        """rt_apply_op_noalloc: the FP64 operator with its partial sums in the
        library's fixed device array (no allocation in the call)."""
        out = self._new() if sigma_out is None else sigma_out
        _check(lib().rt_apply_op_noalloc(self._h, C.c_void_p(_ptr(sigma_in)),
                                         C.c_void_p(_ptr(out)), _stream(stream)))
        return out

    def precond_jacobi(self, v, z=None, stream=None):
        out = self._new() if z is None else z
        _check(lib().rt_precond_jacobi(self._h, C.c_void_p(_ptr(v)), C.c_void_p(_ptr(out)),
                                       _stream(stream)))
        return out

    def precond_apply(self, v, z=None, stream=None):
        """z = P^-1 v with the handle's preconditioner (options.precond)."""
        out = self._new() if z is None else z
        _check(lib().rt_precond_apply(self._h, C.c_void_p(_ptr(v)), C.c_void_p(_ptr(out)),
                                      _stream(stream)))
        return out

    def get_rhs(self, stream=None):
        b = self._new()
        _check(lib().rt_get_rhs(self._h, C.c_void_p(_ptr(b)), _stream(stream)))
        return b

    def get_jacobi_diag(self, stream=None):
        d = self._new()
        _check(lib().rt_get_jacobi_diag(self._h, C.c_void_p(_ptr(d)), _stream(stream)))
        return d

    def plan_info(self):
        L, nb = C.c_int(), C.c_int()
        npairs, nint = C.c_longlong(), C.c_longlong()
        _check(lib().rt_plan_info(self._h, C.byref(L), C.byref(nb), C.byref(npairs),
                                  C.byref(nint)))
        return dict(chunk=L.value, blocks=nb.value, pairs=npairs.value, intervals=nint.value)

    def sweep_config(self, fp32=False):
        """Waves per sweep workgroup, prefetch (0/1) and the coefficient mode
        (0 pairs streamed, 1 w streamed, 2 computed in the sweep)."""
        w, pf, cm = C.c_int(), C.c_int(), C.c_int()
        _check(lib().rt_sweep_config(self._h, 1 if fp32 else 0, C.byref(w), C.byref(pf)))
        _check(lib().rt_sweep_coef_mode(self._h, 1 if fp32 else 0, C.byref(cm)))
        return dict(waves=w.value, prefetch=pf.value, coef_mode=cm.value)

    def effective_options(self) -> rt_options:
        """The options the handle runs with (a stored plan applied)."""
        o = rt_options()
        _check(lib().rt_get_options(self._h, C.byref(o)))
        return o

    def tuned_plan_status(self):
        """'none', 'current' (a stored plan measured with the sweep sources
        this library was built from was applied) or 'stale' (one measured with other
        sources)."""
        return {0: "none", 1: "current", 2: "stale"}[lib().rt_tuned_plan_status(self._h)]

    def sweep_kernel_name(self, fp32=False):
        """The sweep kernel rt_apply_op(_fp32) launches, as profilers name it."""
        c = self.sweep_config(fp32)
        return "rt::sweep::sweep_kernel<%s, %d, %d, %d, %d>" % (
            "float" if fp32 else "double", self.plan_info()["chunk"], c["waves"], c["prefetch"],
            c["coef_mode"])

    # -- frequency redistribution -------------------------------------------------
    def set_redistribution(self, R):
        """R: (n_atm, n_nu, n_nu) or (n_nu, n_nu) host array, R[s][p][q]."""
        R = np.ascontiguousarray(R, dtype=np.float64)
        _check(lib().rt_set_redistribution(self._h, R.ctypes.data_as(C.POINTER(C.c_double))))

    def prd_size(self):
        n = C.c_longlong()
        _check(lib().rt_prd_size(self._h, C.byref(n)))
        return n.value

    def _new_prd(self):
        import torch
        return torch.empty(self.prd_size(), dtype=torch.float64, device="cuda")

    def apply_op_prd(self, sigma_in, sigma_out=None, stream=None):
        out = self._new_prd() if sigma_out is None else sigma_out
        _check(lib().rt_apply_op_prd(self._h, C.c_void_p(_ptr(sigma_in)), C.c_void_p(_ptr(out)),
                                     _stream(stream)))
        return out

    def apply_op_prd_bf16x3(self, sigma_in, sigma_out=None, stream=None):
        out = self._new_prd() if sigma_out is None else sigma_out
        _check(lib().rt_apply_op_prd_bf16x3(self._h, C.c_void_p(_ptr(sigma_in)),
                                            C.c_void_p(_ptr(out)), _stream(stream)))
        return out

    def get_rhs_prd(self, stream=None):
        b = self._new_prd()
        _check(lib().rt_get_rhs_prd(self._h, C.c_void_p(_ptr(b)), _stream(stream)))
        return b

    def get_jacobi_diag_prd(self, stream=None):
        d = self._new_prd()
        _check(lib().rt_get_jacobi_diag_prd(self._h, C.c_void_p(_ptr(d)), _stream(stream)))
        return d

    def solve_prd_gmres(self, x, b=None, stream=None):
        return self._solve("rt_solve_prd_gmres", b, x, stream)

    # -- the field as unknown ------------------------------------------------------
    def field_size(self):
        n = C.c_longlong()
        _check(lib().rt_field_size(self._h, C.byref(n)))
        return n.value

    def _new_field(self):
        import torch
        return torch.empty(self.field_size(), dtype=torch.float64, device="cuda")

    def apply_op_field(self, I_in, I_out=None, stream=None):
        """(Id - Lambda T J) I (rt_apply_op_field)."""
        out = self._new_field() if I_out is None else I_out
        _check(lib().rt_apply_op_field(self._h, C.c_void_p(_ptr(I_in)), C.c_void_p(_ptr(out)),
                                       _stream(stream)))
        return out

    def get_rhs_field(self, stream=None):
        """Lambda T c + t (rt_get_rhs_field)."""
        b = self._new_field()
        _check(lib().rt_get_rhs_field(self._h, C.c_void_p(_ptr(b)), _stream(stream)))
        return b

    def solve_field_gmres(self, I, b_field=None, stream=None):
        """Unpreconditioned GMRES on the field system (I: initial guess in,
        solution out)."""
        return self._solve("rt_solve_field_gmres", b_field, I, stream)

    def sigma_from_field(self, I, stream=None):
        """sigma = J I + c (rt_sigma_from_field)."""
        out = self._new()
        _check(lib().rt_sigma_from_field(self._h, C.c_void_p(_ptr(I)), C.c_void_p(_ptr(out)),
                                         _stream(stream)))
        return out

    # -- dense route -------------------------------------------------------------
    def assembled_size(self):
        n = C.c_longlong()
        _check(lib().rt_assembled_size(self._h, C.byref(n)))
        return n.value

    def assemble(self, out=None, stream=None):
        """rt_assemble into a flat float64 tensor (allocated if out is None)."""
        import torch
        A = out if out is not None else torch.empty(self.assembled_size(), dtype=torch.float64,
                                                    device="cuda")
        _check(lib().rt_assemble(self._h, C.c_void_p(_ptr(A)), _stream(stream)))
        return A

    def dense_blocks(self, A):
        """Views of the slabs' (2 ns) x (2 ns) blocks of a flat assembled A."""
        out, off = [], 0
        for n in self.ns:
            out.append(A[off:off + 4 * n * n].view(2 * n, 2 * n))
            off += 4 * n * n
        return out

    # -- solvers ---------------------------------------------------------------
    def _solve(self, fn, b, x, stream):
        info = (rt_solve_info * self.n_atm)()
        bp = C.c_void_p(_ptr(b)) if b is not None else None
        rc = getattr(lib(), fn)(self._h, bp, C.c_void_p(_ptr(x)), info, _stream(stream))
        _check(rc)
        return rc, [SolveInfo(STATUS_NAMES.get(i.status, str(i.status)), i.iterations, i.matvecs,
                              i.outer_steps, i.relres) for i in info]

    def solve_gmres(self, x, b=None, stream=None):
        return self._solve("rt_solve_gmres", b, x, stream)

    def solve_bicgstab(self, x, b=None, stream=None):
        return self._solve("rt_solve_bicgstab", b, x, stream)

    def solve_richardson(self, x, b=None, stream=None):
        return self._solve("rt_solve_richardson", b, x, stream)

    def solve_cgs(self, x, b=None, stream=None):
        return self._solve("rt_solve_cgs", b, x, stream)

    def solve_lu(self, x, b=None, stream=None):
        """Direct solve with the LU factors of the assembled A (x is output only)."""
        return self._solve("rt_solve_lu", b, x, stream)


def setup(prob, options: Optional[rt_options] = None, autotune: bool = False, **kw) -> Handle:
    """Set up `prob` on the current GPU.  autotune=True sets options.autotune:
    the library applies the launch plan stored for this problem shape and
    precision (paper_2110_11873_amd.autotune writes it) where the caller did
    not set the field."""
    if autotune and options is None:
        kw = {"autotune": 1, **kw}
    return Handle(prob, options, **kw)
