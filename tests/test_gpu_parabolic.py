"""GPU parity of the DELO-parabolic formal solver (Sect. 4.1), which runs the
ray-per-lane FP64 sweep, against the FP64 CPU oracle and its dense route.

Tolerances as for the other formal solvers: operator, right-hand side and
diagonal normwise 1e-12 (unit columns 1e-13 absolute); solves by the oracle's
own residual below the requested rtol.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dense as D  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_2110_11873_amd import binding as B  # noqa: E402
from paper_2110_11873_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

FS = "delo_parabolic"


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def normwise(p, v, y):
    ref = O.apply(p, v)
    return np.abs(y - ref).max() / (np.abs(v).max() + np.abs(v - ref).max())


def oracle_relres(p, x, b=None):
    b = O.rhs(p) if b is None else b
    out = []
    for i, s in enumerate(O._slices(p)):
        r = b[s] - O.apply_slab(p, i, x[s])
        out.append(np.linalg.norm(r) / np.linalg.norm(b[s]))
    return np.array(out)


def test_unit_columns_equal_dense_route():
    p = W.config1_subgrid(FS)
    A = D.Dense(p).A
    with B.setup(p) as h:
        for j in range(p.n_unknowns):
            e = np.zeros(p.n_unknowns)
            e[j] = 1.0
            assert np.abs(host(h.apply_op(dev(e))) - A[:, j]).max() <= 1e-13, j


@pytest.mark.parametrize("maker", [lambda: W.config1(FS), lambda: W.config2(FS)])
def test_operator_rhs_diag(maker):
    p = maker()
    with B.setup(p) as h:
        for sd in (0, 1):
            v = W.random_vector(p.n_unknowns, sd)
            assert normwise(p, v, host(h.apply_op(dev(v)))) <= 1e-12
            # the FP32 entry point runs the same FP64 sweep for this solver
            assert normwise(p, v, host(h.apply_op_fp32(dev(v)))) <= 1e-12
        b = host(h.get_rhs())
        d = host(h.get_jacobi_diag())
    assert np.abs(b - O.rhs(p)).max() <= 1e-12 * np.abs(O.rhs(p)).max()
    # the oracle's diagonal is (A e_i)_i, one application per entry: sampled
    idx = sorted({0, 1, 2, 3, p.n_unknowns // 2, p.n_unknowns - 2, p.n_unknowns - 1})
    assert np.abs(d[idx] - O.diag(p, idx)).max() <= 1e-12


def test_batched_operator():
    """8 uneven slabs: few rays, so each ray is cut into depth chunks."""
    p = W.config4(8).with_(formal_solver=W.FS_DELO_PARABOLIC)
    v = W.random_vector(p.n_unknowns, 2)
    with B.setup(p) as h:
        y = host(h.apply_op(dev(v)))
    assert normwise(p, v, y) <= 1e-12


def test_many_slab_operator_unchunked():
    """160 small slabs x 13 groups of 64 rays: enough wavefronts that each ray
    is one lane from top to bottom (the path of the 512-slab batch)."""
    rng = np.random.default_rng(12)
    n = 160
    ns = [int(v) for v in rng.integers(2, 12, n)]
    p = W.make_slabs(ns, [(1e-4, float(10 ** rng.uniform(4, 8))) for _ in range(n)], 16, 101, 10.0,
                     list(10 ** rng.uniform(-4, -2, n)), list(10 ** rng.uniform(-6, -2, n)),
                     list(rng.uniform(0, 0.7, n)), formal_solver=FS)
    v = W.random_vector(p.n_unknowns, 3)
    with B.setup(p) as h:
        y = host(h.apply_op(dev(v)))
        b = host(h.get_rhs())
    assert normwise(p, v, y) <= 1e-12
    rb = O.rhs(p)
    assert np.abs(b - rb).max() <= 1e-12 * np.abs(rb).max()


@pytest.mark.parametrize("kind,maker", [("gmres", W.config2), ("bicgstab", W.config2),
                                        ("cgs", W.config1)])
def test_solvers(kind, maker):
    """(CGS breaks down on the 200-point slab with either DELO solver, in the
    oracle too; it is checked on the 40-point one.)"""
    p = maker(FS)
    with B.setup(p) as h:
        x = dev(np.zeros(p.n_unknowns))
        rc, info = getattr(h, "solve_" + kind)(x)
    assert rc == 0 and info[0].status == "converged"
    assert oracle_relres(p, host(x)).max() < 1e-10


def test_mixed_precision_gmres():
    p = W.config2(FS)
    with B.setup(p, precision=B.RT_PREC_MIXED) as h:
        x = dev(np.zeros(p.n_unknowns))
        rc, info = h.solve_gmres(x)
    assert rc == 0
    assert oracle_relres(p, host(x)).max() < 1e-10


def test_dense_routes_reject_the_three_point_stencil():
    p = W.config1(FS)
    with B.setup(p) as h:
        with pytest.raises(B.RTError):
            h.assemble()
        x = dev(np.zeros(p.n_unknowns))
        with pytest.raises(B.RTError):
            h.solve_lu(x)
    with B.setup(p, precond=B.RT_PC_SSOR) as h:
        with pytest.raises(B.RTError):
            h.solve_gmres(dev(np.zeros(p.n_unknowns)))
