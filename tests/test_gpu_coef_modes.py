"""GPU parity of the sweep's coefficient modes against the FP64 CPU oracle.

The sweep takes each ray-interval's step coefficients (E, w) from one of
three places (options.coef_mode): both streamed from tiles built at setup,
w streamed with E = 1 - w d derived from the optical step d = kappa dtau, or
both computed in the sweep from d.  Every mode must give the operator of
Algorithm 1 (Sect. 3.3) for every two-point formal solver of Sect. 4.1:

  * FP64 operator: normwise error <= 1e-12 against the oracle (the bound of
    the other parity tests), and <= 1e-13 between modes;
  * FP32 operator (the inner solves of the mixed-precision refinement):
    normwise error below 1e-5, and above 1e-12 (it does run in FP32);
  * identity steps (padding frequencies, intervals past a slab's bottom, the
    zero-length last step of a short chunk) exercised by ragged depth grids
    and odd frequency counts for every chunk length;
  * solves in both precisions reach the oracle's own residual.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dense as D  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_2110_11873_amd import binding as B  # noqa: E402
from paper_2110_11873_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

MODES = {"pairs": B.RT_COEF_PAIRS, "stream_w": B.RT_COEF_STREAM_W,
         "recompute": B.RT_COEF_RECOMPUTE, "recompute_fp32": B.RT_COEF_RECOMPUTE_FP32}
FS = ["delo_linear", "trapezoidal", "implicit_euler"]
# resolved kernel modes (0 pairs, 1 w streamed, 2 recomputed) of (FP64, FP32)
RESOLVED = {"pairs": (0, 0), "stream_w": (1, 1), "recompute": (2, 2), "recompute_fp32": (1, 2)}


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def normwise(ref, v, y):
    return np.abs(y - ref).max() / (np.abs(v).max() + np.abs(v - ref).max())


def check_both(p, h, seed, tol64=1e-12, tol32=1e-5):
    v = W.random_vector(p.n_unknowns, seed)
    ref = O.apply(p, v)
    y64 = host(h.apply_op(dev(v)))
    y32 = host(h.apply_op_fp32(dev(v)))
    e64, e32 = normwise(ref, v, y64), normwise(ref, v, y32)
    assert e64 <= tol64, ("fp64", e64)
    assert 1e-12 < e32 < tol32, ("fp32", e32)
    return e64, e32


@pytest.mark.parametrize("mode", list(MODES))
def test_mode_resolution(mode):
    p = W.config1()
    with B.setup(p, coef_mode=MODES[mode]) as h:
        got = (h.sweep_config(False)["coef_mode"], h.sweep_config(True)["coef_mode"])
    assert got == RESOLVED[mode]


@pytest.mark.parametrize("fs", FS)
@pytest.mark.parametrize("mode", list(MODES))
def test_mode_unit_columns_subgrid(mode, fs):
    """Columns of A from unit vectors against the dense route (eqs.
    matricial_form_1 / crd_linear_system, assembled independently)."""
    p = W.config1_subgrid(fs)
    A = D.Dense(p).A
    with B.setup(p, coef_mode=MODES[mode]) as h:
        for j in range(p.n_unknowns):
            e = np.zeros(p.n_unknowns)
            e[j] = 1.0
            col = host(h.apply_op(dev(e)))
            assert np.abs(col - A[:, j]).max() <= 1e-13, (mode, fs, j)


@pytest.mark.parametrize("fs", FS)
@pytest.mark.parametrize("mode", list(MODES))
def test_mode_config1_config2(mode, fs):
    for p in (W.config1(fs), W.config2(fs)):
        with B.setup(p, coef_mode=MODES[mode]) as h:
            check_both(p, h, seed=21)


@pytest.mark.parametrize("mode", ["stream_w", "recompute"])
@pytest.mark.parametrize("chunk", [4, 8, 16, 32])
@pytest.mark.parametrize("ns", [2, 3, 10, 33, 41, 97])
def test_mode_forced_chunks_and_ragged_tails(mode, chunk, ns):
    """Identity steps in the derived modes: a single interval (2), chunks made
    of padding only (10 with chunk 4), exact fits (33), and 7 frequencies
    (padding rays in every wave-batch)."""
    if (ns - 1) > 64 * chunk:
        pytest.skip("chunk too short for this grid")
    p = W.make_slabs([ns], [(1e-3, 1e5)], 6, 7, 6.0, [1e-3], [1e-3], [0.6])
    with B.setup(p, chunk=chunk, coef_mode=MODES[mode]) as h:
        assert h.plan_info()["chunk"] == chunk
        check_both(p, h, seed=3)


@pytest.mark.parametrize("mode", ["stream_w", "recompute"])
@pytest.mark.parametrize("chunk", [4, 8])
@pytest.mark.parametrize("waves", [4, 8])
def test_mode_kernel_variants(mode, chunk, waves):
    """Every chunk count (8..64) and several chunk lengths in one launch,
    with wave-batch counts that leave some waves idle."""
    ns = [2, 20, 33, 64, 65, 130, 200, 257]
    ns = [n for n in ns if n - 1 <= 64 * chunk]
    p = W.make_slabs(ns, [(1e-3, 1e5)] * len(ns), 6, 21, 6.0, [1e-3] * len(ns),
                     [1e-3] * len(ns), [0.6] * len(ns))
    with B.setup(p, chunk=chunk, sweep_waves=waves, wave_batches=3,
                 coef_mode=MODES[mode]) as h:
        check_both(p, h, seed=11)


@pytest.mark.parametrize("mode", list(MODES))
def test_mode_rhs_and_diag(mode):
    """The right-hand side runs the FP64 sweep with the bottom inflow, which
    crosses the identity steps past a slab's bottom."""
    for p in (W.config1(), W.make_slabs([10, 41], [(1e-3, 1e5)] * 2, 6, 7, 6.0, [1e-3] * 2,
                                        [1e-3, 1e-2], [0.6, 0.2])):
        with B.setup(p, chunk=4, coef_mode=MODES[mode]) as h:
            b = host(h.get_rhs())
            d = host(h.get_jacobi_diag())
        ref = O.rhs(p)
        assert np.abs(b - ref).max() <= 1e-13 * np.abs(ref).max(), mode
        assert np.abs(d - O.diag(p)).max() <= 1e-13, mode


@pytest.mark.parametrize("mode", list(MODES))
def test_mode_full_batch_sampled_slabs(mode):
    """The 512-slab batch (Ns 64..512, 16 mu x 101 nu, DELO-linear) in the
    bench's launch plan, sampled slabs against the oracle slab by slab."""
    p = W.config4(n_slabs=512)
    v = W.random_vector(p.n_unknowns, 5)
    with B.setup(p, coef_mode=MODES[mode]) as h:
        y64 = host(h.apply_op(dev(v)))
        y32 = host(h.apply_op_fp32(dev(v)))
    sl = O._slices(p)
    for i in [0, 7, 123, 300, 511]:
        ref = O.apply_slab(p, i, v[sl[i]])
        assert normwise(ref, v[sl[i]], y64[sl[i]]) <= 1e-12, (mode, i)
        assert normwise(ref, v[sl[i]], y32[sl[i]]) < 1e-5, (mode, i)


@pytest.mark.parametrize("mode", ["stream_w", "recompute"])
def test_mode_config3_full(mode):
    """One 1024-point slab, 32 mu x 201 nu (chunks of 16, 64 per ray)."""
    p = W.config3()
    with B.setup(p, coef_mode=MODES[mode]) as h:
        check_both(p, h, seed=6)


def test_modes_agree_with_each_other():
    """FP64 operator of every mode within 1e-13 (normwise) of the pairs mode
    on the paper-shaped slab, for every formal solver."""
    for fs in FS:
        p = W.config2(fs)
        v = W.random_vector(p.n_unknowns, 31)
        out = {}
        for mode, cm in MODES.items():
            with B.setup(p, coef_mode=cm) as h:
                out[mode] = host(h.apply_op(dev(v)))
        for mode in MODES:
            err = np.abs(out[mode] - out["pairs"]).max() / (np.abs(v).max() + np.abs(out["pairs"]).max())
            assert err <= 1e-13, (fs, mode, err)


def _c4_subset(step):
    p = W.config4(n_slabs=512)
    sel = list(range(0, 512, step))
    sub = W.make_slabs([int(p.ns[i]) for i in sel],
                       [(p.tau[p.offsets[i]], p.tau[p.offsets[i + 1] - 1]) for i in sel],
                       p.n_mu, p.n_nu, 10.0, [0.0] * len(sel), list(p.eps[sel]), list(p.W2[sel]))
    return sub.with_(phi=p.phi[sel].copy(), opac=p.opac[sel].copy())


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("mixed", [False, True])
def test_mode_batched_solve(mode, mixed):
    """14 slabs of the 512-slab batch solved by Jacobi-GMRES(30) to 1e-9 in
    FP64 and in mixed precision, checked by the oracle's own residual."""
    sub = _c4_subset(37)
    prec = B.RT_PREC_MIXED if mixed else B.RT_PREC_FP64
    with B.setup(sub, rtol=1e-9, maxit=20000, precision=prec, coef_mode=MODES[mode]) as h:
        x = dev(W.initial_guess(sub))
        rc, info = h.solve_gmres(x)
        xs = host(x)
    assert all(i.status == "converged" for i in info), info
    b = O.rhs(sub)
    for i, s in enumerate(O._slices(sub)):
        r = b[s] - O.apply_slab(sub, i, xs[s])
        assert np.linalg.norm(r) / np.linalg.norm(b[s]) < 1e-9, (mode, mixed, i)
