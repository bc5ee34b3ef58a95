"""GPU parity of the field-unknown formulation (eq. crd_linear_system2):
(Id - Lambda T J) I, Lambda T c + t and sigma = J I + c against the oracle
(which orders a slab's field depth-fastest; the library orders it
ray-fastest, so the tests permute), and the consistency of the two
formulations.  Tolerance: normwise 1e-12 in FP64, as for the operator.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dense as D  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_2110_11873_amd import binding as B  # noqa: E402
from paper_2110_11873_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def to_gpu_order(p, f_oracle, i):
    """Oracle slab field [st][m][p][k] -> library slab field [st][k][m][p]."""
    ns, nmu, nnu = int(p.ns[i]), len(p.mu), len(p.w_nu)
    return f_oracle.reshape(2, nmu, nnu, ns).transpose(0, 3, 1, 2).ravel()


def to_oracle_order(p, f_gpu, i):
    ns, nmu, nnu = int(p.ns[i]), len(p.mu), len(p.w_nu)
    return f_gpu.reshape(2, ns, nmu, nnu).transpose(0, 2, 3, 1).ravel()


def slab_fields(p, f):
    out, off = [], 0
    for i in range(p.n_atm):
        n = O.field_size(p, i)
        out.append(f[off:off + n])
        off += n
    return out


@pytest.mark.parametrize("fs", ["delo_linear", "trapezoidal", "implicit_euler", "delo_parabolic"])
@pytest.mark.parametrize("maker", [W.config1_subgrid, W.config1])
def test_field_operator_rhs_and_sigma(fs, maker):
    p = maker(fs)
    rng = np.random.default_rng(7)
    with B.setup(p) as h:
        n = h.field_size()
        f = rng.uniform(-1, 1, n)
        y = host(h.apply_op_field(dev(f)))
        bI = host(h.get_rhs_field())
        sg = host(h.sigma_from_field(dev(f)))
    fo = to_oracle_order(p, f, 0)
    ref = O.apply_I(p, fo)
    scale = np.abs(f).max() + np.abs(fo - ref).max()
    assert np.abs(to_oracle_order(p, y, 0) - ref).max() / scale <= 1e-12
    rb = O.rhs_I(p)
    assert np.abs(to_oracle_order(p, bI, 0) - rb).max() <= 1e-12 * np.abs(rb).max()
    rs = O.sigma_from_I(p, fo)
    assert np.abs(sg - rs).max() <= 1e-12 * np.abs(rs).max()


def test_field_of_the_sigma_solution_solves_the_field_system():
    """I* = Lambda T sigma* + t satisfies (Id - Lambda T J) I* = Lambda T c + t
    and gives back sigma* = J I* + c (the two formulations agree)."""
    p = W.config1_subgrid()
    d = D.Dense(p)
    sig = d.solve()
    Istar = to_gpu_order(p, d.Lam @ d.T @ sig + d.t, 0)
    with B.setup(p) as h:
        y = host(h.apply_op_field(dev(Istar)))
        bI = host(h.get_rhs_field())
        s2 = host(h.sigma_from_field(dev(Istar)))
    assert np.abs(y - bI).max() <= 1e-11 * np.abs(bI).max()
    assert np.abs(s2 - sig).max() <= 1e-11 * np.abs(sig).max()


def test_field_batch():
    p = W.config4(6)
    rng = np.random.default_rng(8)
    with B.setup(p) as h:
        f = rng.uniform(-1, 1, h.field_size())
        y = host(h.apply_op_field(dev(f)))
    for i, (fi, yi) in enumerate(zip(slab_fields(p, f), slab_fields(p, y))):
        if i not in (0, 5):
            continue
        fo = to_oracle_order(p, fi, i)
        ref = O.apply_I(p.slab(i), fo)
        scale = np.abs(fi).max() + np.abs(fo - ref).max()
        assert np.abs(to_oracle_order(p, yi, i) - ref).max() / scale <= 1e-12, i


# ------------------------------------------------------------- field GMRES

@pytest.mark.parametrize("fs", ["delo_linear", "trapezoidal", "implicit_euler", "delo_parabolic"])
def test_field_gmres_matches_dense_field_solution(fs):
    p = W.config1_subgrid(fs)
    sig_ref, I_ref = D.Dense(p).solve_I_formulation()
    with B.setup(p, rtol=1e-13, restart=40, maxit=2000) as h:
        I = dev(np.zeros(h.field_size()))
        rc, info = h.solve_field_gmres(I)
        sig = host(h.sigma_from_field(I))
    assert rc == 0 and info[0].status == "converged" and info[0].relres < 1e-13
    Ig = to_oracle_order(p, host(I), 0)
    assert np.abs(Ig - I_ref).max() <= 1e-10 * np.abs(I_ref).max()
    assert np.abs(sig - sig_ref).max() <= 1e-10 * np.abs(sig_ref).max()


def test_field_gmres_config1_oracle_residual():
    p = W.config1()
    with B.setup(p, rtol=1e-10, restart=30, maxit=5000) as h:
        I = dev(np.zeros(h.field_size()))
        rc, info = h.solve_field_gmres(I)
        b = host(h.get_rhs_field())
    assert rc == 0
    Io, bo = to_oracle_order(p, host(I), 0), to_oracle_order(p, b, 0)
    r = O.rhs_I(p) - O.apply_I(p, Io)
    assert np.abs(bo - O.rhs_I(p)).max() <= 1e-12 * np.abs(bo).max()
    assert np.linalg.norm(r) / np.linalg.norm(O.rhs_I(p)) < 1e-10
    assert abs(info[0].relres - np.linalg.norm(r) / np.linalg.norm(O.rhs_I(p))) < 1e-11


def test_field_gmres_batch_per_slab():
    """Uneven slabs converge independently; the maxit limit is honoured."""
    p = W.config4(3)
    with B.setup(p, rtol=1e-10, restart=30, maxit=5000) as h:
        I = dev(np.zeros(h.field_size()))
        rc, info = h.solve_field_gmres(I)
        If = host(I)
    with B.setup(p, rtol=1e-14, restart=10, maxit=7) as h:
        I2 = dev(np.zeros(h.field_size()))
        rc2, info2 = h.solve_field_gmres(I2)
    assert rc == 0 and all(i.status == "converged" for i in info)
    for i, fi in enumerate(slab_fields(p, If)):
        ps = p.slab(i)
        fo = to_oracle_order(p, fi, i)
        r = O.rhs_I(ps) - O.apply_I(ps, fo)
        assert np.linalg.norm(r) / np.linalg.norm(O.rhs_I(ps)) < 1e-10, i
    assert rc2 == B.RT_ENOCONV and all(i.iterations == 7 for i in info2)


def _random_case(seed):
    """A random field-unknown problem (inputs only): 1 to 3 slabs of 2 to 130
    points, 2 to 8 angles, 2 to 13 frequencies, any formal solver."""
    rng = np.random.default_rng(3211 + seed)
    n = int(rng.integers(1, 4))
    ns = [int(v) for v in rng.choice([2, 3, 9, 40, 77, 130], n)]
    fs = ["delo_linear", "trapezoidal", "implicit_euler", "delo_parabolic"][seed % 4]
    ranges = [(10.0 ** rng.uniform(-3, -1), 10.0 ** rng.uniform(1, 4)) for _ in ns]
    return W.make_slabs(ns, ranges, int(rng.choice([2, 4, 8])), int(rng.choice([2, 3, 9, 13])),
                        float(rng.uniform(3.0, 7.0)), list(10.0 ** rng.uniform(-4, -2, n)),
                        list(10.0 ** rng.uniform(-2, -1, n)), list(rng.uniform(0.0, 1.0, n)),
                        formal_solver=fs)


@pytest.mark.parametrize("seed", range(12))
def test_field_random_shapes(seed):
    """Seeded random shapes: per slab the field operator, its right-hand
    side and sigma = J I + c against the oracle, and field GMRES by the
    oracle's own residual."""
    p = _random_case(seed)
    print(f"case {seed}: ns={list(p.ns)} n_mu={p.n_mu} n_nu={p.n_nu} fs={p.formal_solver}",
          flush=True)
    rng = np.random.default_rng(seed)
    with B.setup(p, rtol=1e-10, restart=30, maxit=20000) as h:
        f = rng.uniform(-1, 1, h.field_size())
        y = host(h.apply_op_field(dev(f)))
        bI = host(h.get_rhs_field())
        sg = host(h.sigma_from_field(dev(f)))
        I = dev(np.zeros(h.field_size()))
        rc, info = h.solve_field_gmres(I)
        If = host(I)
    assert rc == 0 and all(i.status == "converged" for i in info), info
    sl = O._slices(p)
    for i, (fi, yi, bi, xi) in enumerate(zip(slab_fields(p, f), slab_fields(p, y),
                                             slab_fields(p, bI), slab_fields(p, If))):
        ps = p.slab(i)
        fo = to_oracle_order(p, fi, i)
        ref = O.apply_I(ps, fo)
        scale = np.abs(fi).max() + np.abs(fo - ref).max()
        assert np.abs(to_oracle_order(p, yi, i) - ref).max() / scale <= 1e-12, i
        rb = O.rhs_I(ps)
        assert np.abs(to_oracle_order(p, bi, i) - rb).max() <= 1e-12 * np.abs(rb).max(), i
        rs = O.sigma_from_I(ps, fo)
        assert np.abs(sg[sl[i]] - rs).max() <= 1e-12 * np.abs(rs).max(), i
        r = rb - O.apply_I(ps, to_oracle_order(p, xi, i))
        assert np.linalg.norm(r) / np.linalg.norm(rb) < 1e-10, i
