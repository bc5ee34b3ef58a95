"""GPU parity of the frequency-redistribution variant (the benchmark's fifth
configuration): operator, right-hand side, Jacobi diagonal and GMRES against
the redistribution oracle and its dense route, and the complete-redistribution
limit (gamma = 0) against the CRD operator.  Tolerance: normwise 1e-12 in
FP64 (the contraction runs on the FP64 matrix cores)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dense as D  # noqa: E402
from oracle import oracle as O  # noqa: E402
from oracle import redistrib as RDO  # noqa: E402
from paper_2110_11873_amd import binding as B  # noqa: E402
from paper_2110_11873_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def normwise(ref, y, v):
    return np.abs(y - ref).max() / (np.abs(v).max() + np.abs(v - ref).max())


@pytest.mark.parametrize("gamma", [0.0, 0.5])
@pytest.mark.parametrize("fs", ["delo_linear", "trapezoidal", "implicit_euler", "delo_parabolic"])
def test_prd_subgrid_against_oracle_and_dense(gamma, fs):
    p = W.config1_subgrid(fs)
    R = W.redistribution_matrix(p.x, p.w_nu, p.phi[0], gamma)
    A = D.redistribution_matrix_A(p, R)
    v = np.random.default_rng(1).uniform(-1, 1, A.shape[0])
    with B.setup(p) as h:
        h.set_redistribution(R)
        y = host(h.apply_op_prd(dev(v)))
        b = host(h.get_rhs_prd())
        d = host(h.get_jacobi_diag_prd())
    assert normwise(RDO.apply(p, R, v), y, v) <= 1e-12
    assert normwise(A @ v, y, v) <= 1e-12
    rb = RDO.rhs(p, R)
    assert np.abs(b - rb).max() <= 1e-12 * np.abs(rb).max()
    assert np.abs(d - np.diag(A)).max() <= 1e-12


def test_prd_gamma0_is_the_crd_operator():
    """R proportional to phi phi': a frequency-independent sigma gives the CRD
    operator at every frequency (GPU against GPU, and against the oracle)."""
    p = W.config1()
    R0 = W.redistribution_matrix(p.x, p.w_nu, p.phi[0], 0.0)
    ns, nnu = int(p.ns[0]), len(p.w_nu)
    s = W.random_vector(2 * ns, 4)
    sig = np.repeat(s.reshape(ns, 1, 2), nnu, axis=1).ravel()
    with B.setup(p) as h:
        h.set_redistribution(R0)
        y = host(h.apply_op_prd(dev(sig))).reshape(ns, nnu, 2)
        yc = host(h.apply_op(dev(s))).reshape(ns, 2)
    assert np.abs(y - yc[:, None, :]).max() <= 1e-12 * (np.abs(s).max() + 1.0)
    assert np.abs(y - O.apply(p, s).reshape(ns, 2)[:, None, :]).max() <= 1e-12 * (np.abs(s).max() + 1.0)


def test_prd_reduced_config5_solve():
    p, R = W.config5(ns=64, n_mu=16, n_nu=64)
    v = np.random.default_rng(2).uniform(-1, 1, 2 * 64 * 64)
    with B.setup(p, rtol=1e-9, restart=30, maxit=3000) as h:
        h.set_redistribution(R)
        y = host(h.apply_op_prd(dev(v)))
        x = dev(np.zeros(h.prd_size()))
        rc, info = h.solve_prd_gmres(x)
        xs = host(x)
    assert normwise(RDO.apply(p, R, v), y, v) <= 1e-12
    assert rc == 0 and info[0].status == "converged"
    b = RDO.rhs(p, R)
    rel = np.linalg.norm(b - RDO.apply(p, R, xs)) / np.linalg.norm(b)
    assert rel < 1e-9, rel


def test_prd_config5_full_operator():
    """256 depths x 32 mu x 256 nu, gamma = 0.5: the operator against the
    oracle, and the solve to 1e-9 checked by the oracle's residual."""
    p, R = W.config5()
    v = np.random.default_rng(3).uniform(-1, 1, 2 * 256 * 256)
    with B.setup(p, rtol=1e-9, restart=30, maxit=5000) as h:
        h.set_redistribution(R)
        y = host(h.apply_op_prd(dev(v)))
        x = dev(np.zeros(h.prd_size()))
        rc, info = h.solve_prd_gmres(x)
        xs = host(x)
    assert normwise(RDO.apply(p, R, v), y, v) <= 1e-12
    assert rc == 0
    b = RDO.rhs(p, R)
    rel = np.linalg.norm(b - RDO.apply(p, R, xs)) / np.linalg.norm(b)
    assert rel < 1e-9, rel


def _batch_case(ns_list, n_mu, n_nu, fs, gamma, seed):
    ranges = [(1e-3, 1e5), (1e-4, 1e8), (1e-2, 1e4)]
    n = len(ns_list)
    p = W.make_slabs(ns_list, [ranges[i % 3] for i in range(n)], n_mu, n_nu, 6.0,
                     [1e-3 * (i + 1) for i in range(n)], [1e-2 / (i + 1) for i in range(n)],
                     [0.5 - 0.1 * i for i in range(n)], formal_solver=fs)
    R = np.stack([W.redistribution_matrix(p.x, p.w_nu, p.phi[i], gamma) for i in range(n)])
    v = np.random.default_rng(seed).uniform(-1, 1, 2 * n_nu * int(np.sum(ns_list)))
    return p, R, v


def _check_batch(p, R, v):
    nnu = len(p.w_nu)
    with B.setup(p) as h:
        h.set_redistribution(R)
        y = host(h.apply_op_prd(dev(v)))
        b = host(h.get_rhs_prd())
    off = 0
    for i, ns in enumerate(int(n) for n in p.ns):
        seg = slice(2 * nnu * off, 2 * nnu * (off + ns))
        assert normwise(RDO.apply(p, R[i], v[seg], i=i), y[seg], v[seg]) <= 1e-12, i
        rb = RDO.rhs(p, R[i], i=i)
        assert np.abs(b[seg] - rb).max() <= 1e-12 * np.abs(rb).max(), i
        off += ns


@pytest.mark.parametrize("fs", ["delo_linear", "delo_parabolic"])
def test_prd_uneven_batch(fs):
    """Three slabs of 7, 23 and 40 depths with their own R, profiles and
    parameters: per-slab depth chunks (some empty) and slab offsets."""
    _check_batch(*_batch_case([7, 23, 40], 8, 12, fs, 0.5, 5))


@pytest.mark.parametrize("fs", ["delo_linear", "trapezoidal", "implicit_euler", "delo_parabolic"])
def test_prd_ragged_depth_chunks(fs):
    """16 |mu| and slabs of 250, 77 and 130 depths: 32 depth chunks per ray of
    8, 3 and 5 points, ragged last chunks and empty ones, for every formal
    solver."""
    _check_batch(*_batch_case([250, 77, 130], 32, 10, fs, 0.5, 9))


def test_prd_R_given_at_setup_equals_set_redistribution():
    """rt_problem.R hands the matrices to rt_setup: the operator, right-hand
    side and solve are those of a handle given R afterwards, bit for bit."""
    p, R, v = _batch_case([23, 40], 8, 12, "delo_linear", 0.5, 10)
    with B.setup(p) as h:
        h.set_redistribution(R)
        y0 = host(h.apply_op_prd(dev(v)))
        b0 = host(h.get_rhs_prd())
    with B.setup(p, R=R) as h:
        y1 = host(h.apply_op_prd(dev(v)))
        b1 = host(h.get_rhs_prd())
    assert np.array_equal(y0, y1) and np.array_equal(b0, b1)


@pytest.mark.parametrize("fs", ["delo_linear", "delo_parabolic"])
def test_prd_one_direction_pair_two_frequencies(fs):
    """One pair of directions (one lane per depth chunk, up to 300 chunks of
    one point) and two frequencies, slabs of 2, 3, 40 and 300 depths."""
    _check_batch(*_batch_case([2, 3, 40, 300], 2, 2, fs, 0.5, 11))


def test_prd_long_rays_global_stage():
    """700 depths x 16 |mu|: the per-frequency quadrature stage exceeds the
    LDS budget and lives in global memory; a 300-depth slab beside it."""
    _check_batch(*_batch_case([700, 300], 32, 6, "delo_linear", 0.5, 6))


def test_prd_tiny_slabs():
    """2-, 3- and 5-depth slabs: chunks of one point and empty chunks."""
    _check_batch(*_batch_case([2, 3, 5], 4, 3, "delo_linear", 0.3, 7))


# BF16x3 contraction: each operand split into bf16 hi + lo carries about 16
# significant bits (relative error <= 2^-17 each, from FP32), the dropped
# lo.lo term is below 2^-16 of a product, and 256 FP32 additions add at most
# 256 * 2^-24 relative to the sum of |products| (R w >= 0 and the largest J
# terms dominate): together below 2e-5 of |xi J~ / phi|, so normwise (as in
# the FP64 tests) below 2e-5.
BF16X3_TOL = 2e-5


@pytest.mark.parametrize("fs", ["delo_linear", "delo_parabolic"])
def test_prd_bf16x3_operator_against_oracle(fs):
    p, R, v = _batch_case([7, 23, 40], 8, 12, fs, 0.5, 8)
    nnu = len(p.w_nu)
    with B.setup(p) as h:
        h.set_redistribution(R)
        y = host(h.apply_op_prd_bf16x3(dev(v)))
        y64 = host(h.apply_op_prd(dev(v)))
    off = 0
    for i, ns in enumerate(int(n) for n in p.ns):
        seg = slice(2 * nnu * off, 2 * nnu * (off + ns))
        ref = RDO.apply(p, R[i], v[seg], i=i)
        assert normwise(ref, y[seg], v[seg]) <= BF16X3_TOL, i
        off += ns
    # it is the BF16 path: not bit-equal to the FP64 contraction
    assert np.abs(y - y64).max() > 0.0


def test_prd_bf16x3_config5_operator():
    p, R = W.config5()
    v = np.random.default_rng(9).uniform(-1, 1, 2 * 256 * 256)
    with B.setup(p) as h:
        h.set_redistribution(R)
        y = host(h.apply_op_prd_bf16x3(dev(v)))
    assert normwise(RDO.apply(p, R, v), y, v) <= BF16X3_TOL


@pytest.mark.parametrize("shape", [(64, 16, 64), (256, 32, 256)])
def test_prd_mixed_refinement_solve(shape):
    """MIXED: FP64 refinement around BF16x3 inner solves reaches 1e-9 by the
    oracle's FP64 residual."""
    ns, n_mu, n_nu = shape
    p, R = W.config5(ns=ns, n_mu=n_mu, n_nu=n_nu)
    with B.setup(p, rtol=1e-9, restart=30, maxit=5000, precision=B.RT_PREC_MIXED) as h:
        h.set_redistribution(R)
        x = dev(np.zeros(h.prd_size()))
        rc, info = h.solve_prd_gmres(x)
        xs = host(x)
    assert rc == 0 and info[0].status == "converged", info
    assert info[0].outer_steps >= 2
    b = RDO.rhs(p, R)
    rel = np.linalg.norm(b - RDO.apply(p, R, xs)) / np.linalg.norm(b)
    assert rel < 1e-9, rel


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_prd_batch_solve_per_slab(precision):
    """Three uneven slabs with their own R: each slab's solve (FP64 GMRES, or
    the refinement around BF16x3 inner solves) reaches 1e-9 by the oracle's
    residual of that slab."""
    p, R, _ = _batch_case([7, 23, 40], 8, 12, "delo_linear", 0.5, 10)
    nnu = len(p.w_nu)
    prec = B.RT_PREC_MIXED if precision == "mixed" else B.RT_PREC_FP64
    with B.setup(p, rtol=1e-9, restart=30, maxit=5000, precision=prec) as h:
        h.set_redistribution(R)
        x = dev(np.zeros(h.prd_size()))
        rc, info = h.solve_prd_gmres(x)
        xs = host(x)
    assert rc == 0 and all(i.status == "converged" for i in info), info
    off = 0
    for i, ns in enumerate(int(n) for n in p.ns):
        seg = slice(2 * nnu * off, 2 * nnu * (off + ns))
        b = RDO.rhs(p, R[i], i=i)
        rel = np.linalg.norm(b - RDO.apply(p, R[i], xs[seg], i=i)) / np.linalg.norm(b)
        assert rel < 1e-9, (i, rel)
        off += ns


def test_prd_requires_R():
    p = W.config1_subgrid()
    with B.setup(p) as h:
        with pytest.raises(B.RTError):
            h.get_rhs_prd()
        with pytest.raises(B.RTError):
            h.set_redistribution(np.full((5, 5), np.nan))


def _random_case(seed):
    """A random redistribution problem (inputs only): 1 to 3 slabs of 2 to
    700 points, 2 to 16 angles, 2 to 33 frequencies, any formal solver, a
    redistribution parameter per slab."""
    rng = np.random.default_rng(110873 + seed)
    n = int(rng.integers(1, 4))
    ns = [int(v) for v in rng.choice([2, 3, 9, 40, 77, 130, 256, 700], n)]
    n_mu = int(rng.choice([2, 4, 8, 16]))
    n_nu = int(rng.choice([2, 3, 9, 17, 33]))
    fs = ["delo_linear", "trapezoidal", "implicit_euler", "delo_parabolic"][seed % 4]
    ranges = [(10.0 ** rng.uniform(-4, -2), 10.0 ** rng.uniform(2, 6)) for _ in ns]
    p = W.make_slabs(ns, ranges, n_mu, n_nu, float(rng.uniform(3.0, 7.0)),
                     list(10.0 ** rng.uniform(-4, -2, n)), list(10.0 ** rng.uniform(-3, -1, n)),
                     list(rng.uniform(0.0, 1.0, n)), formal_solver=fs)
    R = np.stack([W.redistribution_matrix(p.x, p.w_nu, p.phi[i], float(rng.uniform(0.0, 1.0)))
                  for i in range(n)])
    v = rng.uniform(-1, 1, 2 * n_nu * int(np.sum(ns)))
    return p, R, v


@pytest.mark.parametrize("seed", range(16))
def test_prd_random_shapes(seed):
    """Seeded random shapes (all within the cached sweep's chunk length;
    longer chunks: test_prd_long_rays_global_stage): FP64 operator and
    right-hand side per slab
    against the redistribution oracle, the BF16x3 operator within its 2e-5
    bound, and Jacobi-GMRES by the oracle's residual."""
    p, R, v = _random_case(seed)
    print(f"case {seed}: ns={list(p.ns)} n_mu={p.n_mu} n_nu={p.n_nu} fs={p.formal_solver}",
          flush=True)
    nnu = len(p.w_nu)
    with B.setup(p, rtol=1e-9, restart=30, maxit=20000) as h:
        h.set_redistribution(R)
        y = host(h.apply_op_prd(dev(v)))
        y3 = host(h.apply_op_prd_bf16x3(dev(v)))
        b = host(h.get_rhs_prd())
        x = torch.zeros(h.prd_size(), dtype=torch.float64, device="cuda")
        rc, info = h.solve_prd_gmres(x)
        xs = host(x)
    assert rc == 0 and all(i.status == "converged" for i in info), info
    off = 0
    for i, ns in enumerate(int(n) for n in p.ns):
        seg = slice(2 * nnu * off, 2 * nnu * (off + ns))
        ref = RDO.apply(p, R[i], v[seg], i=i)
        assert normwise(ref, y[seg], v[seg]) <= 1e-12, i
        assert normwise(ref, y3[seg], v[seg]) <= 2e-5, i
        rb = RDO.rhs(p, R[i], i=i)
        assert np.abs(b[seg] - rb).max() <= 1e-12 * np.abs(rb).max(), i
        rel = np.linalg.norm(rb - RDO.apply(p, R[i], xs[seg], i=i)) / np.linalg.norm(rb)
        assert rel < 1e-9, (i, rel)
        off += ns
