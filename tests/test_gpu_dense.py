"""GPU parity of the dense route: the assembled A (rt_assemble) against the
oracle's column-by-column assembly and its independent dense route.

Tolerance: every entry of A is a sum of nonnegative-weighted intensities
bounded by one, so entries are compared absolutely at 1e-13 (FP64, the sum over
up to 3216 rays in a different order from the oracle's).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dense as D  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_2110_11873_amd import binding as B  # noqa: E402
from paper_2110_11873_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

ENTRY_TOL = 1e-13


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def assembled_blocks(p, **kw):
    with B.setup(p, **kw) as h:
        A = h.assemble()
        return [host(b) for b in h.dense_blocks(A)]


@pytest.mark.parametrize("fs", ["delo_linear", "trapezoidal", "implicit_euler"])
def test_assemble_subgrid_equals_dense_route(fs):
    p = W.config1_subgrid(fs)
    (Ag,) = assembled_blocks(p)
    assert np.abs(Ag - D.Dense(p).A).max() <= ENTRY_TOL


@pytest.mark.parametrize("fs", ["delo_linear", "trapezoidal", "implicit_euler"])
def test_assemble_config1_equals_oracle(fs):
    p = W.config1(fs)
    (Ag,) = assembled_blocks(p)
    assert np.abs(Ag - O.assemble(p)).max() <= ENTRY_TOL


@pytest.mark.parametrize("ns", [20, 65, 140])
def test_assemble_paper_replica(ns):
    """One ray slice, 64-column blocks with a ragged last block."""
    p = W.paper_replica(ns, scale="integrated", normalize=False)
    (Ag,) = assembled_blocks(p)
    assert np.abs(Ag - O.assemble(p)).max() <= ENTRY_TOL


def test_assemble_several_ray_slices():
    """101 frequencies x 10 |mu|: the rays do not fit one workgroup, so the
    slices' moments are combined by a second pass."""
    p = W.paper_replica(70, n_mu=20, n_nu=101, scale="integrated", normalize=False)
    (Ag,) = assembled_blocks(p)
    assert np.abs(Ag - O.assemble(p)).max() <= ENTRY_TOL


def test_assemble_config2_columns():
    """Sampled columns of the 200-point slab against the oracle's matvec of
    unit vectors (three ray slices)."""
    p = W.config2()
    (Ag,) = assembled_blocks(p)
    n = p.n_unknowns
    for j in (0, 1, 63, 64, 127, 128, 200, 398, 399):
        e = np.zeros(n)
        e[j] = 1.0
        assert np.abs(Ag[:, j] - O.apply(p, e)).max() <= ENTRY_TOL, j


def test_assemble_batch_matches_operator_and_oracle():
    """Uneven batch: every slab's block times a random vector equals
    rt_apply_op, and sampled slabs equal the oracle's assembly."""
    p = W.config4(24)
    v = W.random_vector(p.n_unknowns, 3)
    with B.setup(p) as h:
        A = h.assemble()
        y_op = host(h.apply_op(dev(v)))
        blocks = [host(b) for b in h.dense_blocks(A)]
        A2 = host(h.assemble())
    assert np.array_equal(host(A), A2), "assembly is not deterministic"
    off = 0
    for i, Ab in enumerate(blocks):
        n = Ab.shape[0]
        y = Ab @ v[off:off + n]
        scale = np.abs(v[off:off + n]).max() + np.abs(v[off:off + n] - y_op[off:off + n]).max()
        assert np.abs(y - y_op[off:off + n]).max() / scale <= 1e-12, i
        off += n
    for i in (0, 7, 23):
        assert np.abs(blocks[i] - O.assemble(p.slab(i))).max() <= ENTRY_TOL, i


def test_assemble_full_batch_operator_property():
    """The 512-slab batch at full size: A x equals rt_apply_op(x) slab by slab
    (a property that holds at any size), plus two sampled slabs against the
    oracle's assembly."""
    p = W.config4(512)
    v = W.random_vector(p.n_unknowns, 4)
    with B.setup(p) as h:
        A = h.assemble()
        vd = dev(v)
        y_op = h.apply_op(vd)
        torch.cuda.synchronize()
        blocks = h.dense_blocks(A)
        off = 0
        worst = 0.0
        for Ab in blocks:
            n = Ab.shape[0]
            y = Ab @ vd[off:off + n]
            scale = vd[off:off + n].abs().max() + (vd[off:off + n] - y_op[off:off + n]).abs().max()
            worst = max(worst, float(((y - y_op[off:off + n]).abs().max() / scale).item()))
            off += n
        sample = {i: host(blocks[i]) for i in (5, 300)}
    assert worst <= 1e-12, worst
    for i, Ab in sample.items():
        assert np.abs(Ab - O.assemble(p.slab(i))).max() <= ENTRY_TOL, i
