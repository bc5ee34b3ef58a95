"""Pins of the FP64 CPU oracle against facts fixed by the paper and by mathematics.

None of these checks re-types an oracle formula: each compares the oracle to
something independent of it -- numbers printed in the paper, closed forms,
definite integrals evaluated by adaptive quadrature, analytic solutions of the
transfer equation, a separately assembled dense operator solved by LAPACK, or
structural properties the paper states.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import dense as D
from oracle import oracle as O
from paper_2110_11873_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_iteration_counts.json")


# --------------------------------------------------------------------------
# Quadrature and polarization tensor (eqs. sourceI/sourceQ, J00/J02)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n_mu", [4, 8, 20, 32])
def test_t20_angular_moments(n_mu):
    """Angular moments of T^2_{0,1}, T^2_{0,2} over (1/2) int_{-1}^{1} dmu are
    exact for Gauss-Legendre with >= 3 nodes: <1> = 1, <T1> = 0, <T2> = -sqrt2/2,
    <T1^2> = 1/10, <T1^2 + T2^2> = 7/10 (moments <mu^2> = 1/3, <mu^4> = 1/5)."""
    mu, w = W.gauss_legendre(n_mu)
    t = np.array([O.t20(m) for m in mu])
    h = 0.5 * w
    assert abs(h.sum() - 1.0) < 1e-14
    assert abs((h * t[:, 0]).sum()) < 1e-14
    assert abs((h * t[:, 1]).sum() + math.sqrt(2.0) / 2.0) < 1e-14
    assert abs((h * t[:, 0] ** 2).sum() - 0.1) < 1e-14
    assert abs((h * (t[:, 0] ** 2 + t[:, 1] ** 2)).sum() - 0.7) < 1e-14
    # Q's factor vanishes for grazing-free vertical rays and T1 at mu^2 = 1/3
    assert abs(O.t20(1.0)[1]) < 1e-15
    assert abs(O.t20(1.0 / math.sqrt(3.0))[0]) < 1e-15


def test_weights_normalized_sum_to_one():
    p = W.config1()
    q = O.weights(p)
    assert q.shape == (p.n_mu, p.n_nu)
    assert abs(q.sum() - 1.0) < 1e-14
    # unnormalized: the spectral integral of the truncated Voigt profile is < 1
    q2 = O.weights(p.with_(normalize_profile=False))
    assert 0.99 < q2.sum() < 1.0


# --------------------------------------------------------------------------
# Formal-solver step coefficients (Sect. 4.1)
# --------------------------------------------------------------------------

DELTAS = [1e-10, 1e-7, 1e-4, 1e-2, 0.05, 0.0999999, 0.1, 0.1000001, 0.3, 1.0, 3.0, 10.0,
          50.0, 300.0]


@pytest.mark.parametrize("d", DELTAS)
def test_delo_linear_coefficients_are_the_defining_integrals(d):
    """psi_u = int_0^d (s/d) e^{-s} ds, psi_k = int_0^d ((d-s)/d) e^{-s} ds,
    E = e^{-d}: the exact integrals of a linearly interpolated source
    function along the ray, evaluated here by adaptive Gauss-Kronrod."""
    E, pu, pk = O.delo_linear(d)
    # substitute s = d u so the integrand lives on [0, 1]
    ref_u = d * integrate.quad(lambda u: u * math.exp(-d * u), 0.0, 1.0, epsabs=0,
                               epsrel=1e-13, limit=200)[0]
    ref_k = d * integrate.quad(lambda u: (1.0 - u) * math.exp(-d * u), 0.0, 1.0, epsabs=0,
                               epsrel=1e-13, limit=200)[0]
    assert abs(E - math.exp(-d)) <= 1e-16 * max(1.0, math.exp(-d))
    assert abs(pu - ref_u) <= 1e-13 * abs(ref_u)
    assert abs(pk - ref_k) <= 1e-13 * abs(ref_k)


def test_delo_linear_limits_and_branch_continuity():
    # large d: E -> 0, psi_u -> 1/d, psi_k -> 1 - 1/d
    for d in [800.0, 1e4, 1e9]:
        E, pu, pk = O.delo_linear(d)
        assert E == 0.0
        assert abs(pu - 1.0 / d) <= 1e-15 / d
        assert abs(pk - (1.0 - 1.0 / d)) <= 1e-15
    # small d: psi_u ~ d/2 - d^2/3 + d^3/8, psi_k ~ d/2 - d^2/6 + d^3/24
    d = 1e-5
    E, pu, pk = O.delo_linear(d)
    assert abs(pu - (d / 2 - d * d / 3 + d ** 3 / 8)) < 1e-15 * d
    assert abs(pk - (d / 2 - d * d / 6 + d ** 3 / 24)) < 1e-15 * d
    # the two branches meet at the switch
    a = O.delo_linear(np.nextafter(0.1, 0.0))
    b = O.delo_linear(0.1)
    assert abs(a[1] - b[1]) < 1e-15 and abs(a[2] - b[2]) < 1e-15
    # consistency: a constant source is reproduced exactly, E + psi_u + psi_k = 1
    for d in DELTAS:
        E, pu, pk = O.delo_linear(d)
        assert abs(E + pu + pk - 1.0) < 4e-16


def test_trapezoid_is_second_order_and_preserves_constants():
    """Crank-Nicolson on dI/dt = S - I: constants preserved (a + 2b = 1) and
    global error O(h^2) against the exact solution for S = 2 + 3 t."""
    for d in [1e-8, 0.3, 2.0, 1e3, 1e8]:
        a, b = O.trapezoid(d)
        assert abs(a + 2 * b - 1.0) < 1e-15
        assert abs(a) <= 1.0
    errs = []
    for n in [41, 81, 161, 321]:
        tau = np.linspace(0.0, 4.0, n)
        S = 2.0 + 3.0 * tau
        I = O.ray(tau, 1.0, False, S, I_entry=5.0, fs=1)
        exact = (2.0 + 3.0 * tau - 3.0) + (5.0 - (2.0 - 3.0)) * np.exp(-tau)
        errs.append(np.abs(I - exact).max())
    rates = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(3.8 < r < 4.2 for r in rates), rates


def test_implicit_euler_is_first_order_and_L_stable():
    """Implicit Euler (Sect. 4.1) on dI/dt = S - I: constants preserved
    (a + b = 1), the step damps every mode (0 < a < 1, a -> 0 as d grows: L-
    stable, unlike the trapezoid), and the global error against the exact
    solution for S = 2 + 3 t is O(h): it halves when the step halves."""
    for d in [1e-8, 0.3, 2.0, 1e3, 1e8]:
        a, b = O.implicit_euler(d)
        assert abs(a + b - 1.0) < 1e-15
        assert 0.0 < a < 1.0 and b > 0.0
    assert O.implicit_euler(1e8)[0] < 1e-7
    errs = []
    for n in [41, 81, 161, 321]:
        tau = np.linspace(0.0, 4.0, n)
        S = 2.0 + 3.0 * tau
        I = O.ray(tau, 1.0, False, S, I_entry=5.0, fs=2)
        exact = (2.0 + 3.0 * tau - 3.0) + (5.0 - (2.0 - 3.0)) * np.exp(-tau)
        errs.append(np.abs(I - exact).max())
    rates = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(1.85 < r < 2.15 for r in rates), rates


@pytest.mark.parametrize("d", [1e-7, 1e-3, 0.05, 0.7, 0.999, 1.0, 1.3, 5.0, 60.0])
@pytest.mark.parametrize("ratio", [0.2, 1.0, 7.0])
def test_delo_parabolic_coefficients_are_the_defining_integrals(d, ratio):
    """DELO-parabolic (Sect. 4.1): c_u, c_k, c_d are the integrals of
    exp(-t) against the quadratic Lagrange basis through t = d (upwind),
    0 (current) and -dd (downwind), on [0, d]; they sum to 1 - E."""
    dd = ratio * d
    E, pu, pk, pd = O.delo_parabolic(d, dd)
    basis = {
        "u": lambda t: t * (t + dd) / (d * (d + dd)),
        "k": lambda t: (d - t) * (t + dd) / (d * dd),
        "d": lambda t: t * (t - d) / (dd * (d + dd)),
    }
    ref = {key: integrate.quad(lambda t, f=f: f(t) * math.exp(-t), 0.0, d, epsabs=0.0,
                               epsrel=1e-13, limit=200)[0] for key, f in basis.items()}
    scale = max(1.0 - math.exp(-d), 1e-300)
    for key, got in (("u", pu), ("k", pk), ("d", pd)):
        assert abs(got - ref[key]) <= 1e-12 * scale + 1e-300, (key, got, ref[key])
    assert abs(pu + pk + pd - (-math.expm1(-d))) <= 1e-14 * scale
    assert E == math.exp(-d)


@pytest.mark.parametrize("kappa", [0.37, 1.0, 6.0])
def test_delo_parabolic_exact_for_quadratic_source(kappa):
    """With S quadratic in the ray's optical path s, I(s) = P(s) - P(0) e^{-s}
    + I0 e^{-s} with P = S - S' + S'' solves dI/ds = S - I exactly; the
    parabola through three nodes is S itself, so every point but the ray's
    last (where the step is DELO-linear) is exact."""
    tau = np.logspace(-3, 1.5, 40)
    a, b, c = 0.3, 0.7, 0.05
    for upward in (False, True):
        s = kappa * (tau[-1] - tau) if upward else kappa * (tau - tau[0])
        S = a + b * s + c * s * s
        P = S - (b + 2 * c * s) + 2 * c
        I0 = 0.4
        exact = P - (a - b + 2 * c) * np.exp(-s) + I0 * np.exp(-s)
        I = O.ray(tau, kappa, upward, S, I_entry=I0, fs=3)
        # the upward ray ends at index 0, the downward one at the last index
        inner = slice(1, len(tau)) if upward else slice(0, -1)
        assert np.abs(I[inner] - exact[inner]).max() <= 1e-11 * np.abs(exact).max(), upward
        last = 0 if upward else -1
        assert abs(I[last] - exact[last]) <= 1e-2 * abs(exact[last])


def test_delo_parabolic_is_third_order():
    """Global error O(h^3) on a smooth source: it drops about eightfold when
    the step halves (DELO-linear: fourfold)."""
    errs = []
    for n in [21, 41, 81, 161]:
        tau = np.linspace(0.0, 4.0, n)
        S = np.sin(tau)
        I = O.ray(tau, 1.0, False, S, I_entry=0.0, fs=3)
        exact = 0.5 * (np.sin(tau) - np.cos(tau)) + 0.5 * np.exp(-tau)
        errs.append(np.abs(I - exact).max())
    rates = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(6.5 < r < 9.5 for r in rates), rates


# --------------------------------------------------------------------------
# Formal solution along a ray (eqs. RTE_delo1/2, boundary conditions Sect. 3.1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kappa", [0.37, 1.0, 6.0])
def test_delo_linear_exact_for_linear_source(kappa):
    """DELO-linear integrates a linear source exactly.  With S = a + b tau and
    m = 1/kappa (= |mu|/r_p): upward from tau_max with I(tau_max) = Ib,
       I = (a + b tau + b m) - (a + b tau_max + b m - Ib) e^{-(tau_max - tau)/m};
    downward from tau_1 with I(tau_1) = It,
       I = (a + b tau - b m) - (a + b tau_1 - b m - It) e^{-(tau - tau_1)/m}."""
    tau = np.logspace(-3, 2, 60)
    a, b, m = 0.3, 0.7, 1.0 / kappa
    S = a + b * tau
    Ib, It = 1.3, 0.2
    up = O.ray(tau, kappa, True, S, I_entry=Ib)
    ex_up = (a + b * tau + b * m) - (a + b * tau[-1] + b * m - Ib) * np.exp(-(tau[-1] - tau) / m)
    dn = O.ray(tau, kappa, False, S, I_entry=It)
    ex_dn = (a + b * tau - b * m) - (a + b * tau[0] - b * m - It) * np.exp(-(tau - tau[0]) / m)
    assert np.abs(up - ex_up).max() <= 1e-12 * np.abs(ex_up).max()
    assert np.abs(dn - ex_dn).max() <= 1e-12 * np.abs(ex_dn).max()


@pytest.mark.parametrize("fs", [0, 1, 2, 3])
def test_constant_source_with_matching_inflow_is_stationary(fs):
    tau = np.logspace(-4, 8, 50)
    S = np.full(50, 0.8)
    I = O.ray(tau, 2.5, True, S, I_entry=0.8, fs=fs)
    assert np.abs(I - 0.8).max() < 1e-14


@pytest.mark.parametrize("fs", [0, 1, 2, 3])
def test_point_source_has_exact_upwind_zeros(fs):
    """A point-like source at z_j leaves the intensity zero on the upwind side
    of the ray and decaying on the downwind side (Sect. 4.4 run-time remarks;
    stated in z, here in tau: mu<0 rays are zero above the source, mu>0 rays
    zero below it).  DELO-parabolic's parabola reaches one point further
    upwind: the point just before the source sees it through c_d."""
    tau = np.logspace(-2, 3, 30)
    j = 13
    S = np.zeros(30)
    S[j] = 1.0
    dn = O.ray(tau, 1.0, False, S, fs=fs)
    up = O.ray(tau, 1.0, True, S, fs=fs)
    reach = 1 if fs == 3 else 0
    assert np.all(dn[:j - reach] == 0.0) and dn[j] > 0
    assert np.all(up[j + 1 + reach:] == 0.0) and up[j] > 0
    if fs == 3:
        assert dn[j - 1] != 0.0 and up[j + 1] != 0.0
    if fs in (0, 2):   # DELO, implicit Euler: nonnegative, decaying past the source's interval
        assert np.all(np.diff(dn[j + 1:]) <= 0) and np.all(dn[j:] >= 0)
        assert np.all(np.diff(up[:j]) >= 0) and np.all(up[:j + 1] >= 0)


# --------------------------------------------------------------------------
# The operator against an independently assembled dense route (Sect. 3.2-3.3)
# --------------------------------------------------------------------------

@pytest.fixture(scope="module", params=[0, 1, 2, 3], ids=["delo", "trap", "euler", "parab"])
def sub(request):
    p = W.config1_subgrid(["delo_linear", "trapezoidal", "implicit_euler",
                           "delo_parabolic"][request.param])
    return p, D.Dense(p)


def test_matvec_columns_equal_dense_operator(sub):
    p, d = sub
    A = O.assemble(p)
    assert np.abs(A - d.A).max() <= 1e-13
    for seed in range(3):
        v = W.random_vector(p.n_unknowns, seed)
        assert np.abs(O.apply(p, v) - d.A @ v).max() <= 1e-13 * np.abs(v).max()


def test_rhs_and_diag_equal_dense(sub):
    p, d = sub
    assert np.abs(O.rhs(p) - d.b).max() <= 1e-14
    assert np.abs(O.diag(p) - np.diag(d.A)).max() <= 1e-14


def test_I_formulation_gives_same_sigma(sub):
    p, d = sub
    s1 = d.solve()
    s2, _ = d.solve_I_formulation()
    assert np.abs(s1 - s2).max() <= 1e-12 * np.abs(s1).max()


def test_field_formulation_equals_dense(sub):
    """The field-unknown operator, right-hand side and sigma = J I + c of eq.
    crd_linear_system2 against the dense route's explicit matrices; and the
    field I = Lambda T sigma* + t of the sigma solution solves it."""
    p, d = sub
    K = np.eye(d.Lam.shape[0]) - d.Lam @ d.T @ d.J
    for seed in range(2):
        f = np.random.default_rng(seed).uniform(-1, 1, K.shape[0])
        assert np.abs(O.apply_I(p, f) - K @ f).max() <= 1e-13 * np.abs(f).max()
        assert np.abs(O.sigma_from_I(p, f) - (d.J @ f + d.c)).max() <= 1e-13
    bI = O.rhs_I(p)
    assert np.abs(bI - (d.Lam @ d.T @ d.c + d.t)).max() <= 1e-14
    sig = d.solve()
    Istar = d.Lam @ d.T @ sig + d.t
    assert np.abs(O.apply_I(p, Istar) - bI).max() <= 1e-11 * np.abs(bI).max()
    assert np.abs(O.sigma_from_I(p, Istar) - sig).max() <= 1e-11 * np.abs(sig).max()


def test_solvers_agree_with_LU(sub):
    p, d = sub
    ref = d.solve()
    for solve in (O.gmres, O.bicgstab, O.cgs):
        x, info = solve(p, tol=1e-13)
        assert info[0]["status"] == "converged", (solve, info)
        assert np.abs(x - ref).max() <= 1e-11 * np.abs(ref).max(), solve
    # Jacobi-Richardson converges iff the spectral radius of Id - D^-1 A is < 1:
    # true for DELO-linear and implicit Euler (nonnegative steps), false for
    # the trapezoidal solver, whose step amplification tends to -1 on
    # optically thick intervals.
    rho = np.abs(np.linalg.eigvals(np.eye(d.A.shape[0]) - d.A / np.diag(d.A)[:, None])).max()
    x, info = O.richardson(p, tol=1e-13, maxit=20000)
    if rho < 1.0:
        assert info[0]["status"] == "converged"
        assert np.abs(x - ref).max() <= 1e-11 * np.abs(ref).max()
    else:
        assert info[0]["status"] in ("breakdown", "maxit")
    assert (rho < 1.0) == (p.formal_solver != 1)


def test_unrestarted_gmres_terminates_within_N_steps(sub):
    """Krylov methods terminate in at most N steps in exact arithmetic (Sect. 2)."""
    p, d = sub
    N = p.n_unknowns
    x, info = O.gmres(p, precond=False, restart=0, tol=1e-13, maxit=N)
    assert info[0]["status"] == "converged" and info[0]["iterations"] <= N


def test_A_is_positive_definite_nonsymmetric(sub):
    """A is nonsymmetric and positive definite for the paper's formal solvers
    (Sect. 3.2).  The trapezoidal solver is not among them and loses the
    property (its steps are not L-stable); its eigenvalues stay in the right
    half-plane, which is all GMRES(m) needs here."""
    p, d = sub
    A = d.A
    assert np.abs(A - A.T).max() > 1e-3
    if p.formal_solver in (0, 2):
        assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0
    assert np.linalg.eigvals(A).real.min() > 0


def test_paper_sized_A_positive_definite():
    p = W.paper_replica(20, scale="integrated", normalize=False)
    A = O.assemble(p)
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0


def test_unpolarized_block_is_an_M_matrix():
    """W2 = 0 with DELO-linear: the sigma00 block of xi J Lambda T is entrywise
    nonnegative with row sums <= xi, so Id - xi J Lambda T is an M-matrix and
    Jacobi-Richardson converges."""
    p = W.config1().with_(W2=np.array([0.0]))
    A = O.assemble(p)
    A00 = A[0::2, 0::2]
    K = np.eye(A00.shape[0]) - A00
    xi = 1.0 - p.eps[0]
    assert K.min() >= 0.0
    assert K.sum(axis=1).max() <= xi * (1 + 1e-14)
    # sigma20 rows are exactly the identity
    assert np.abs(A[1::2] - np.eye(p.n_unknowns)[1::2]).max() == 0.0


def test_solvers_agree_with_LU_on_tiny_config():
    p = W.config1()
    ref = np.linalg.solve(O.assemble(p), O.rhs(p))
    x, info = O.gmres(p, tol=1e-12, restart=30)
    assert info[0]["status"] == "converged"
    assert np.abs(x - ref).max() <= 1e-9 * np.abs(ref).max()
    x, info = O.bicgstab(p, tol=1e-12)
    assert info[0]["status"] == "converged"
    assert np.abs(x - ref).max() <= 1e-9 * np.abs(ref).max()


# --------------------------------------------------------------------------
# Special cases and physics limits
# --------------------------------------------------------------------------

def test_eps_one_gives_identity_and_planck():
    p = W.config1_subgrid().with_(eps=np.array([1.0]))
    assert np.abs(O.assemble(p) - np.eye(p.n_unknowns)).max() == 0.0
    x, info = O.gmres(p, tol=1e-14)
    assert np.abs(x[0::2] - p.B).max() < 1e-15 and np.abs(x[1::2]).max() == 0.0
    assert info[0]["iterations"] <= 1


def test_zero_polarizability_gives_zero_sigma20():
    p = W.config1().with_(W2=np.array([0.0]))
    b = O.rhs(p)
    assert np.abs(b[1::2]).max() == 0.0
    x, _ = O.gmres(p, tol=1e-12)
    assert np.abs(x[1::2]).max() == 0.0


def test_sqrt_eps_surface_law_and_deep_thermalization():
    """Semi-infinite isothermal slab, CRD, conservative scattering: the exact
    surface source function is sqrt(eps) B and deep layers thermalize to B.
    The discrete value must approach sqrt(eps) under refinement."""
    eps = 1e-2
    ratios = []
    for ns, nmu, nnu, X in [(60, 4, 21, 8), (120, 8, 41, 10), (240, 16, 101, 16)]:
        p = W.make_slabs([ns], [(1e-6, 1e10)], nmu, nnu, X, [1e-3], [eps], [0.0], normalize=True)
        x, info = O.gmres(p, precond=False, restart=0, tol=1e-12, maxit=2 * ns)
        assert info[0]["status"] == "converged"
        ratios.append(x[0] / math.sqrt(eps))
        assert abs(x[-2] - 1.0) < 1e-10        # thermalized at depth
        assert np.abs(x[1::2]).max() == 0.0
    assert ratios[0] < ratios[1] < ratios[2] <= 1.0 + 1e-3, ratios
    assert abs(ratios[-1] - 1.0) < 0.02, ratios


def test_solver_status_paths():
    p = W.config1_subgrid()
    x, info = O.gmres(p, tol=1e-14, maxit=1)
    assert info[0]["status"] == "maxit" and info[0]["iterations"] == 1
    z = np.zeros(p.n_unknowns)
    x, info = O.gmres(p, b=z)
    assert np.all(x == 0) and info[0]["status"] == "converged"
    x, info = O.bicgstab(p, b=z)
    assert np.all(x == 0)
    ref = D.Dense(p).solve()
    x, info = O.gmres(p, x0=ref, tol=1e-10)
    assert info[0]["iterations"] == 0


# --------------------------------------------------------------------------
# The paper's printed iteration counts (weak pins of the whole operator)
# --------------------------------------------------------------------------

with open(GOLDEN) as f:
    _G = json.load(f)


def _replica(ns, nmunu=20):
    # frequency-integrated optical depth (r_p = phi_p), profile not renormalized
    return W.paper_replica(ns, n_mu=nmunu, n_nu=nmunu, scale="integrated", normalize=False)


@pytest.mark.parametrize("ns,expected", list(zip(_G["no_preconditioner_gmres"]["ns"],
                                                _G["no_preconditioner_gmres"]["iterations"])))
def test_paper_unpreconditioned_gmres_counts(ns, expected):
    p = _replica(ns)
    _, info = O.gmres(p, precond=False, restart=0, tol=1e-6, maxit=1000)
    assert info[0]["iterations"] == expected


@pytest.mark.parametrize("ns,expected", list(zip(_G["jacobi_gmres"]["ns"],
                                                _G["jacobi_gmres"]["iterations"])))
def test_paper_jacobi_gmres_counts(ns, expected):
    """Jacobi-GMRES without restarts (Table tab:jacobi): the printed counts
    exactly, with left preconditioning and the preconditioned-residual test."""
    p = _replica(ns)
    _, info = O.gmres(p, precond=True, restart=0, tol=1e-6, maxit=1000, left=True)
    assert info[0]["status"] == "converged"
    assert info[0]["iterations"] == expected


def test_left_and_right_gmres_solve_the_same_system():
    """Both preconditioning sides converge to the LU solution (Sect. 2.1)."""
    p = _replica(20)
    ref = D.Dense(p).solve()
    for left in (False, True):
        x, info = O.gmres(p, tol=1e-13, restart=0, maxit=200, left=left)
        assert info[0]["status"] == "converged"
        assert np.max(np.abs(x - ref)) < 1e-9 * np.max(np.abs(ref))


@pytest.mark.parametrize("ns,expected", list(zip(_G["jacobi_richardson"]["ns"],
                                                _G["jacobi_richardson"]["iterations"])))
def test_paper_jacobi_richardson_counts(ns, expected):
    p = _replica(ns)
    _, info = O.richardson(p, precond=True, tol=1e-6, maxit=100000)
    assert info[0]["iterations"] + 1 == expected


@pytest.mark.parametrize("n,expected", list(zip(
    _G["gmres_vs_angular_spectral_resolution"]["n_mu_eq_n_nu"],
    _G["gmres_vs_angular_spectral_resolution"]["iterations"])))
def test_paper_gmres_counts_vs_resolution(n, expected):
    p = _replica(40, n)
    _, info = O.gmres(p, precond=False, restart=0, tol=1e-6, maxit=1000)
    assert info[0]["iterations"] == expected


@pytest.mark.parametrize("ns,expected", list(zip(_G["jacobi_bicgstab"]["ns"],
                                                _G["jacobi_bicgstab"]["iterations"])))
def test_paper_jacobi_bicgstab_counts(ns, expected):
    p = _replica(ns)
    _, info = O.bicgstab(p, precond=True, tol=1e-6, maxit=1000)
    assert expected <= info[0]["iterations"] <= expected + 1


@pytest.mark.parametrize("ns,expected", list(zip(_G["jacobi_cgs"]["ns"],
                                                _G["jacobi_cgs"]["iterations"])))
def test_paper_jacobi_cgs_counts(ns, expected):
    """Jacobi-CGS (Sect. 2.2, Table tab:jacobi): the printed counts exactly."""
    p = _replica(ns)
    _, info = O.cgs(p, precond=True, tol=1e-6, maxit=1000)
    assert info[0]["status"] == "converged"
    assert info[0]["iterations"] == expected


def test_paper_unpreconditioned_cgs_count_small_grid():
    """Table tab:no_prec, CGS at N_s = 20 (the larger grids' entries depend on
    rounding and are not pinned)."""
    g = _G["no_preconditioner_cgs_ns20"]
    _, info = O.cgs(_replica(g["ns"]), precond=False, tol=1e-6, maxit=1000)
    assert info[0]["iterations"] == g["iterations"]


# SOR and SSOR (Sect. 2.3, 4.2; Tables tab:sor and tab:ssor): relaxation 1.5 for
# Richardson, none for the Krylov methods.
_SOR_CASES = [(pc, method, ns, exp) for pc in ("sor", "ssor")
              for method in ("richardson", "gmres", "bicgstab", "cgs")
              for ns, exp in zip(_G[pc]["ns"], _G[pc][method])]


@pytest.mark.parametrize("pc,method,ns,expected", _SOR_CASES)
def test_paper_sor_ssor_counts(pc, method, ns, expected):
    p = _replica(ns)
    if method == "richardson":
        _, info = O.richardson(p, precond=pc, omega=1.5, tol=1e-6, maxit=10000)
        assert info[0]["iterations"] + 1 == expected
        return
    if method == "gmres":
        _, info = O.gmres(p, precond=pc, restart=0, tol=1e-6, maxit=1000, left=True)
    else:
        _, info = getattr(O, method)(p, precond=pc, tol=1e-6, maxit=1000)
    assert info[0]["status"] == "converged"
    if method == "bicgstab":
        assert expected <= info[0]["iterations"] <= expected + 1
    else:
        assert info[0]["iterations"] == expected


@pytest.mark.parametrize("pc", ["sor", "ssor"])
@pytest.mark.parametrize("omega", [0.7, 1.0, 1.5])
def test_sor_ssor_preconditioner_is_the_textbook_matrix(pc, omega):
    """P^-1 v from the oracle equals a dense solve with P built from the
    triangles of the assembled A (Sect. 2.3), on the tiny grid."""
    p = W.config1_subgrid()
    A = O.assemble(p)
    n = A.shape[0]
    D = np.diag(np.diag(A))
    L, U = np.tril(A, -1), np.triu(A, 1)
    if pc == "sor":
        P = D / omega + U
    else:
        P = omega / (2.0 - omega) * (D / omega + U) @ np.linalg.inv(D) @ (D / omega + L)
    # one Richardson update from x = 0 is exactly P^-1 b
    b = np.random.default_rng(5).uniform(-1, 1, n)
    x, info = O.richardson(p, b=b, x0=np.zeros(n), precond=pc, omega=omega, tol=1e-300, maxit=1)
    assert np.allclose(x, np.linalg.solve(P, b), rtol=1e-12, atol=1e-12 * np.abs(x).max())


def test_sor_with_omega_one_is_gauss_seidel_on_the_upper_triangle():
    """omega = 1: SOR is Gauss-Seidel (Sect. 2.3), here sweeping from the last
    unknown up; SSOR is symmetric Gauss-Seidel, that sweep followed by D and a
    forward sweep.  Written as explicit loops over the assembled A."""
    p = W.config1_subgrid()
    A = O.assemble(p)
    n = A.shape[0]
    b = np.random.default_rng(6).uniform(-1, 1, n)
    x, _ = O.richardson(p, b=b, x0=np.zeros(n), precond="sor", omega=1.0, tol=1e-300, maxit=1)
    ref = np.zeros(n)
    for i in range(n - 1, -1, -1):     # Gauss-Seidel, last unknown first
        ref[i] = (b[i] - A[i, i + 1:] @ ref[i + 1:]) / A[i, i]
    assert np.allclose(x, ref, rtol=1e-13, atol=1e-14)
    y, _ = O.richardson(p, b=b, x0=np.zeros(n), precond="ssor", omega=1.0, tol=1e-300, maxit=1)
    z = np.diag(A) * ref
    fw = np.zeros(n)
    for i in range(n):                 # then forward, first unknown first
        fw[i] = (z[i] - A[i, :i] @ fw[:i]) / A[i, i]
    assert np.allclose(y, fw, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("pc", ["sor", "ssor"])
def test_sor_ssor_solvers_agree_with_LU(pc):
    p = W.config1_subgrid()
    ref = D.Dense(p).solve()
    for solve in (O.gmres, O.bicgstab, O.cgs):
        x, info = solve(p, precond=pc, tol=1e-13, maxit=2000)
        assert info[0]["status"] == "converged"
        assert np.max(np.abs(x - ref)) < 1e-10 * np.max(np.abs(ref))


# --------------------------------------------------------------------------
# Frequency redistribution (the benchmark's fifth configuration)
# --------------------------------------------------------------------------

from oracle import redistrib as RDO  # noqa: E402


def test_redistribution_columns_are_normalized():
    p, R = W.config5(ns=8, n_mu=4, n_nu=31)
    assert np.abs((p.w_nu[:, None] * R).sum(0) - p.phi[0]).max() <= 1e-15


@pytest.mark.parametrize("fs", ["delo_linear", "delo_parabolic"])
def test_redistribution_gamma0_is_complete_redistribution(fs):
    """gamma = 0: R proportional to phi phi', and a frequency-independent
    sigma gives the CRD operator (and right-hand side) at every frequency."""
    p = W.config1_subgrid(fs)
    R0 = W.redistribution_matrix(p.x, p.w_nu, p.phi[0], 0.0)
    ns, nnu = int(p.ns[0]), len(p.w_nu)
    s = W.random_vector(2 * ns, 3)
    sig = np.repeat(s.reshape(ns, 1, 2), nnu, axis=1).ravel()
    y = RDO.apply(p, R0, sig).reshape(ns, nnu, 2)
    assert np.abs(y - O.apply(p, s).reshape(ns, 2)[:, None, :]).max() <= 1e-13
    b = RDO.rhs(p, R0).reshape(ns, nnu, 2)
    assert np.abs(b - O.rhs(p).reshape(ns, 2)[:, None, :]).max() <= 1e-13


@pytest.mark.parametrize("gamma", [0.0, 0.5, 1.0])
def test_redistribution_operator_equals_dense_route(gamma):
    p = W.config1_subgrid()
    R = W.redistribution_matrix(p.x, p.w_nu, p.phi[0], gamma)
    A = D.redistribution_matrix_A(p, R)
    for seed in range(2):
        v = np.random.default_rng(seed).uniform(-1, 1, A.shape[0])
        assert np.abs(RDO.apply(p, R, v) - A @ v).max() <= 1e-13 * np.abs(v).max()


# Photon conservation of the redistribution.  R's columns are normalized so
# that sum_p w_p R(p, q) = phi_q (the discrete int R(x, x') dx = phi(x')), so
# for ANY monochromatic J the contraction Jt(k, p) = sum_q R(p, q) w_q J(k, q)
# satisfies sum_p w_p Jt(k, p) = sum_q w_q phi_q J(k, q).  A transposed R, or
# a dropped w_q, breaks it as soon as R is not symmetric (gamma > 0: the
# Gaussian part phi(x') g(x - x') is not), which the gamma = 0 reduction to
# complete redistribution cannot see (phi phi' is symmetric).

def _conservation_error(contract, p, R, seed=0):
    ns, nnu = 6, len(p.w_nu)
    J = np.random.default_rng(seed).uniform(0.1, 1.0, (ns, nnu))
    Jt = contract(J)
    lhs = Jt @ p.w_nu
    rhs = J @ (p.w_nu * p.phi[0])
    return np.abs(lhs - rhs).max() / np.abs(rhs).max()


@pytest.mark.parametrize("gamma", [0.5, 1.0])
def test_redistribution_contraction_conserves_photons(gamma):
    p, R = W.config5(gamma=gamma, ns=8, n_mu=4, n_nu=31)
    assert np.abs(R - R.T).max() > 1e-3 * np.abs(R).max()  # the pin can see a transpose
    err = _conservation_error(lambda J: RDO._contract(p, 0, R, J), p, R)
    assert err <= 1e-13, err
    # a point mass at frequency q0 comes back as column q0 of R, times w_q0
    q0 = 7
    J = np.zeros((1, len(p.w_nu)))
    J[0, q0] = 1.0
    assert np.abs(RDO._contract(p, 0, R, J)[0] - R[:, q0] * p.w_nu[q0]).max() <= 1e-15


@pytest.mark.parametrize("gamma", [0.5, 1.0])
def test_redistribution_dense_route_conserves_photons(gamma):
    """The same law through the explicit A of the dense route: for any sigma,
    sum_p w_p phi_p ((Id - A) sigma)^K(k, p) = xi W_K sum_q w_q phi_q J^K_q(k),
    with J^K_q the monochromatic angle quadrature of the formal solution
    (computed by the redistribution oracle's own ray sweeps)."""
    p = W.config1_subgrid()
    R = W.redistribution_matrix(p.x, p.w_nu, p.phi[0], gamma)
    A = D.redistribution_matrix_A(p, R)
    ns, nnu = int(p.ns[0]), len(p.w_nu)
    sig = np.random.default_rng(2).uniform(-1, 1, A.shape[0])
    lhs = ((sig - A @ sig).reshape(ns, nnu, 2) * (p.w_nu * p.phi[0])[None, :, None]).sum(1)
    s3 = sig.reshape(ns, nnu, 2)
    J0, J2 = RDO._mono_J(p, 0, s3[:, :, 0], s3[:, :, 1], False)
    xi, W2 = 1.0 - float(p.eps[0]), float(p.W2[0])
    wphi = p.w_nu * p.phi[0]
    rhs = np.stack([xi * (J0 @ wphi), xi * W2 * (J2 @ wphi)], axis=1)
    assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(rhs).max()


def _mutated_module(path, name, old, new):
    import types
    src = open(path).read()
    assert old in src, (name, old)
    mod = types.ModuleType("oracle._mut_" + name)
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new, 1), path + ":" + name, "exec"), mod.__dict__)
    return mod


_RDO_SRC = os.path.join(os.path.dirname(RDO.__file__), "redistrib.py")
_DENSE_SRC = os.path.join(os.path.dirname(D.__file__), "dense.py")
_CONTRACT = "return J @ (R * np.asarray(prob.w_nu)[None, :]).T"
_DENSE_C0 = "Cm[sidx(k, p, 0), sidx(k, q, 0)] = xi * R[p, q] * wnu[q] / phi[p]"


@pytest.mark.parametrize("name,old,new", [
    ("transposed_R", _CONTRACT, "return J @ (R.T * np.asarray(prob.w_nu)[None, :]).T"),
    ("dropped_w", _CONTRACT, "return J @ R.T"),
])
def test_redistribution_pin_rejects_planted_contraction_mistakes(name, old, new):
    p, R = W.config5(gamma=0.5, ns=8, n_mu=4, n_nu=31)
    mut = _mutated_module(_RDO_SRC, name, old, new)
    assert _conservation_error(lambda J: mut._contract(p, 0, R, J), p, R) > 1e-6, name


@pytest.mark.parametrize("name,new", [
    ("dense_transposed_R", "Cm[sidx(k, p, 0), sidx(k, q, 0)] = xi * R[q, p] * wnu[q] / phi[p]"),
    ("dense_dropped_w", "Cm[sidx(k, p, 0), sidx(k, q, 0)] = xi * R[p, q] / phi[p]"),
])
def test_redistribution_dense_pin_rejects_planted_mistakes(name, new):
    p = W.config1_subgrid()
    R = W.redistribution_matrix(p.x, p.w_nu, p.phi[0], 0.5)
    mut = _mutated_module(_DENSE_SRC, name, _DENSE_C0, new)
    A = mut.redistribution_matrix_A(p, R)
    ns, nnu = int(p.ns[0]), len(p.w_nu)
    sig = np.random.default_rng(2).uniform(-1, 1, A.shape[0])
    lhs = ((sig - A @ sig).reshape(ns, nnu, 2)[:, :, 0] * (p.w_nu * p.phi[0])[None, :]).sum(1)
    s3 = sig.reshape(ns, nnu, 2)
    J0, _ = RDO._mono_J(p, 0, s3[:, :, 0], s3[:, :, 1], False)
    rhs = (1.0 - float(p.eps[0])) * (J0 @ (p.w_nu * p.phi[0]))
    assert np.abs(lhs - rhs).max() > 1e-6 * np.abs(rhs).max(), name
