"""rt_apply_op_noalloc (the operator for callers that cannot allocate) against
rt_apply_op through the C ABI: the same result bit for bit on two calls in a
row, the second on a smaller problem, with the library's one fixed array
reused; and a clean error for a handle whose sweep needs more partial sums
than the array holds."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2110_11873_amd import binding as B  # noqa: E402
from paper_2110_11873_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def _pair(p, seed, **kw):
    v = torch.from_numpy(W.random_vector(p.n_unknowns, seed)).cuda()
    with B.setup(p, **kw) as h:
        ref = h.apply_op(v).cpu().numpy()
        out = torch.full_like(v, np.nan)
        h.apply_op_noalloc(v, out)
        got = out.cpu().numpy()
        # in place, as rt_apply_op allows
        w = v.clone()
        h.apply_op_noalloc(w, w)
        inplace = w.cpu().numpy()
    return v.cpu().numpy(), ref, got, inplace


def test_noalloc_matches_apply_op_on_two_calls_second_smaller():
    big = W.config4(n_slabs=512)         # about 2.4 million partial sums
    small = W.config1()                  # 80 unknowns
    for p, seed in ((big, 1), (small, 2)):
        v, ref, got, inplace = _pair(p, seed)
        assert np.array_equal(got, ref), p.name
        assert np.array_equal(inplace, ref), p.name
    # and against the oracle on the small one (the second call)
    ref_o = O.apply(small, v)
    assert np.abs(got - ref_o).max() / (np.abs(v).max() + np.abs(v - ref_o).max()) <= 1e-12


@pytest.mark.parametrize("mode", [B.RT_COEF_PAIRS, B.RT_COEF_RECOMPUTE])
def test_noalloc_other_coefficient_modes(mode):
    p = W.config2()
    v, ref, got, _ = _pair(p, 3, coef_mode=mode)
    assert np.array_equal(got, ref)


def test_noalloc_rejects_sweeps_beyond_its_array():
    # one wave-batch per wave: hundreds of workgroups per slab, tens of
    # millions of partial sums
    p = W.config4(n_slabs=512)
    with B.setup(p, wave_batches=1) as h:
        v = torch.zeros(h.n, dtype=torch.float64, device="cuda")
        with pytest.raises(B.RTError) as e:
            h.apply_op_noalloc(v, torch.empty_like(v))
        assert e.value.code == B.RT_EINVAL
        assert "partial sums" in str(e.value)
