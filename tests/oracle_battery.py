"""A fast battery of the oracle's pins, runnable against any build of it.

``python tests/oracle_battery.py`` runs every check and exits 0 only if all
pass.  The mutation test runs it with ``RT_ORACLE_LIB`` pointing at a build of
the oracle with a planted mistake and expects a non-zero exit.  Each check
compares the oracle against something independent of it (see the pin tests).
"""
import math
import os
import sys

import numpy as np
from scipy import integrate

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import dense as D  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_2110_11873_amd import workloads as W  # noqa: E402


def chk_moments():
    mu, w = W.gauss_legendre(8)
    t = np.array([O.t20(m) for m in mu])
    h = 0.5 * w
    return (abs((h * t[:, 0]).sum()) < 1e-14 and abs((h * t[:, 0] ** 2).sum() - 0.1) < 1e-14
            and abs((h * (t[:, 0] ** 2 + t[:, 1] ** 2)).sum() - 0.7) < 1e-14
            and abs((h * t[:, 1]).sum() + math.sqrt(2) / 2) < 1e-14)


def chk_delo():
    for d in [1e-6, 0.05, 0.3, 5.0]:
        E, pu, pk = O.delo_linear(d)
        ru = d * integrate.quad(lambda u: u * math.exp(-d * u), 0, 1, epsabs=0, epsrel=1e-13)[0]
        rk = d * integrate.quad(lambda u: (1 - u) * math.exp(-d * u), 0, 1, epsabs=0,
                                epsrel=1e-13)[0]
        if not (abs(E - math.exp(-d)) < 1e-16 and abs(pu - ru) < 1e-13 * ru
                and abs(pk - rk) < 1e-13 * rk):
            return False
    return True


def chk_trapezoid():
    errs = []
    for n in [41, 81, 161]:
        tau = np.linspace(0.0, 4.0, n)
        I = O.ray(tau, 1.0, False, 2.0 + 3.0 * tau, I_entry=5.0, fs=1)
        ex = (2.0 + 3.0 * tau - 3.0) + 6.0 * np.exp(-tau)
        errs.append(np.abs(I - ex).max())
    a, b = O.trapezoid(0.7)
    return abs(a + 2 * b - 1) < 1e-15 and 3.8 < errs[0] / errs[1] < 4.2 and \
        3.8 < errs[1] / errs[2] < 4.2


def chk_implicit_euler():
    errs = []
    for n in [41, 81, 161]:
        tau = np.linspace(0.0, 4.0, n)
        I = O.ray(tau, 1.0, False, 2.0 + 3.0 * tau, I_entry=5.0, fs=2)
        ex = (2.0 + 3.0 * tau - 3.0) + 6.0 * np.exp(-tau)
        errs.append(np.abs(I - ex).max())
    a, b = O.implicit_euler(0.7)
    up = O.ray(np.linspace(0.0, 4.0, 41), 1.0, True, np.full(41, 0.8), I_entry=0.8, fs=2)
    return (abs(a + b - 1) < 1e-15 and 1.85 < errs[0] / errs[1] < 2.15
            and 1.85 < errs[1] / errs[2] < 2.15 and np.abs(up - 0.8).max() < 1e-14)


def chk_linear_source():
    tau = np.logspace(-3, 2, 60)
    a, b, kap = 0.3, 0.7, 0.37
    m = 1 / kap
    S = a + b * tau
    up = O.ray(tau, kap, True, S, I_entry=1.3)
    ex_up = (a + b * tau + b * m) - (a + b * tau[-1] + b * m - 1.3) * np.exp(-(tau[-1] - tau) / m)
    dn = O.ray(tau, kap, False, S, I_entry=0.2)
    ex_dn = (a + b * tau - b * m) - (a + b * tau[0] - b * m - 0.2) * np.exp(-(tau - tau[0]) / m)
    return (np.abs(up - ex_up).max() < 1e-12 * np.abs(ex_up).max()
            and np.abs(dn - ex_dn).max() < 1e-12 * np.abs(ex_dn).max())


def chk_dense():
    for fs in ("delo_linear", "trapezoidal", "implicit_euler"):
        p = W.config1_subgrid(fs)
        d = D.Dense(p)
        v = W.random_vector(p.n_unknowns, 0)
        if not (np.abs(O.apply(p, v) - d.A @ v).max() < 1e-13
                and np.abs(O.rhs(p) - d.b).max() < 1e-14
                and np.abs(O.diag(p) - np.diag(d.A)).max() < 1e-14):
            return False
        sub = [3, 7, 11]
        if np.abs(O.diag(p, sub) - np.diag(d.A)[sub]).max() > 1e-14:
            return False
    return True


def chk_solvers_vs_lu():
    p = W.config1_subgrid()
    ref = D.Dense(p).solve()
    for s in (O.gmres, O.bicgstab, O.richardson, O.cgs):
        x, info = s(p, tol=1e-13, maxit=5000)
        if info[0]["status"] != "converged" or np.abs(x - ref).max() > 1e-10 * np.abs(ref).max():
            return False
    for kw in (dict(restart=4), dict(restart=4, left=True)):
        x, info = O.gmres(p, tol=1e-13, maxit=5000, **kw)
        if info[0]["status"] != "converged" or np.abs(x - ref).max() > 1e-10 * np.abs(ref).max():
            return False
    return True


def chk_paper_counts():
    p = W.paper_replica(20, scale="integrated", normalize=False)
    _, g = O.gmres(p, precond=False, restart=0, tol=1e-6, maxit=1000)
    _, r = O.richardson(p, precond=True, tol=1e-6, maxit=10000)
    p40 = W.paper_replica(40, scale="integrated", normalize=False)
    _, g40 = O.gmres(p40, precond=False, restart=0, tol=1e-6, maxit=1000)
    p80 = W.paper_replica(80, scale="integrated", normalize=False)
    _, bi = O.bicgstab(p80, precond=True, tol=1e-6, maxit=1000)
    _, cg = O.cgs(p80, precond=True, tol=1e-6, maxit=1000)
    _, gl = O.gmres(p80, precond=True, restart=0, tol=1e-6, maxit=1000, left=True)
    _, gl40 = O.gmres(p40, precond=True, restart=0, tol=1e-6, maxit=1000, left=True)
    return (g[0]["iterations"] == 28 and r[0]["iterations"] + 1 == 67
            and g40[0]["iterations"] == 48 and 18 <= bi[0]["iterations"] <= 19
            and cg[0]["iterations"] == 26 and gl[0]["iterations"] == 29
            and gl40[0]["iterations"] == 18)


def chk_sor_ssor_counts():
    """Tables tab:sor and tab:ssor at N_s = 40 (Richardson with omega = 1.5
    counted as the paper's loop index; GMRES left-preconditioned)."""
    p40 = W.paper_replica(40, scale="integrated", normalize=False)
    out = []
    for pc, rich, gm, cg in (("sor", 26, 17, 12), ("ssor", 20, 9, 7)):
        _, r = O.richardson(p40, precond=pc, omega=1.5, tol=1e-6, maxit=10000)
        _, g = O.gmres(p40, precond=pc, restart=0, tol=1e-6, maxit=1000, left=True)
        _, c = O.cgs(p40, precond=pc, tol=1e-6, maxit=1000)
        out += [r[0]["iterations"] + 1 == rich, g[0]["iterations"] == gm,
                c[0]["iterations"] == cg]
    return all(out)


def chk_delo_parabolic():
    """DELO-parabolic: coefficients against their defining integrals, a
    quadratic source integrated exactly, and the operator equal to the dense
    route on the tiny grid."""
    for d, dd in ((0.02, 0.05), (0.6, 0.4), (3.0, 9.0)):
        E, pu, pk, pd = O.delo_parabolic(d, dd)
        fs = (lambda t: t * (t + dd) / (d * (d + dd)), lambda t: (d - t) * (t + dd) / (d * dd),
              lambda t: t * (t - d) / (dd * (d + dd)))
        for got, f in zip((pu, pk, pd), fs):
            ref = integrate.quad(lambda t: f(t) * np.exp(-t), 0.0, d, epsabs=0.0, epsrel=1e-13)[0]
            if abs(got - ref) > 1e-12 * (1.0 - E):
                return False
    tau = np.logspace(-3, 1.5, 40)
    s = tau - tau[0]
    S = 0.3 + 0.7 * s + 0.05 * s * s
    exact = S - (0.7 + 0.1 * s) + 0.1 - (0.3 - 0.7 + 0.1) * np.exp(-s)
    I = O.ray(tau, 1.0, False, S, fs=3)
    if np.abs(I[:-1] - exact[:-1]).max() > 1e-11:
        return False
    s_up = tau[-1] - tau
    S = 0.3 + 0.7 * s_up + 0.05 * s_up * s_up
    exact = S - (0.7 + 0.1 * s_up) + 0.1 - (0.3 - 0.7 + 0.1) * np.exp(-s_up)
    I = O.ray(tau, 1.0, True, S, fs=3)
    if np.abs(I[1:] - exact[1:]).max() > 1e-11:
        return False
    p = W.config1_subgrid("delo_parabolic")
    return np.abs(O.assemble(p) - D.Dense(p).A).max() <= 1e-13


def chk_field_formulation():
    """Field-unknown operator, right-hand side and sigma recovery (eq.
    crd_linear_system2) against the dense route."""
    p = W.config1_subgrid()
    d = D.Dense(p)
    K = np.eye(d.Lam.shape[0]) - d.Lam @ d.T @ d.J
    f = np.random.default_rng(0).uniform(-1, 1, K.shape[0])
    return (np.abs(O.apply_I(p, f) - K @ f).max() <= 1e-13
            and np.abs(O.rhs_I(p) - (d.Lam @ d.T @ d.c + d.t)).max() <= 1e-14
            and np.abs(O.sigma_from_I(p, f) - (d.J @ f + d.c)).max() <= 1e-13)


def chk_special_cases():
    p = W.config1_subgrid().with_(eps=np.array([1.0]))
    if np.abs(O.assemble(p) - np.eye(p.n_unknowns)).max() != 0.0:
        return False
    p = W.config1_subgrid().with_(W2=np.array([0.0]))
    x, _ = O.gmres(p, tol=1e-12)
    return np.abs(x[1::2]).max() == 0.0


CHECKS = [chk_moments, chk_delo, chk_trapezoid, chk_implicit_euler, chk_linear_source, chk_dense,
          chk_solvers_vs_lu, chk_paper_counts, chk_sor_ssor_counts, chk_delo_parabolic,
          chk_field_formulation, chk_special_cases]


def run():
    failed = []
    for c in CHECKS:
        try:
            ok = bool(c())
        except Exception as e:  # a crash or NaN path counts as a failed pin
            print(f"{c.__name__}: exception {e!r}")
            ok = False
        if not ok:
            failed.append(c.__name__)
    return failed


if __name__ == "__main__":
    f = run()
    print("FAILED: " + ",".join(f) if f else "ALL PASS")
    sys.exit(1 if f else 0)
