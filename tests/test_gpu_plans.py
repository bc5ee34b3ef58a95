"""Stored launch plans applied by the library itself (options.autotune, the
plan file read by rt_setup), so a C caller gets the autotuner's plan."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2110_11873_amd import binding as B  # noqa: E402
from paper_2110_11873_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def _write(path, entries):
    with open(path, "w") as fh:
        fh.write("# test plans\n")
        for e in entries:
            fh.write(" ".join(str(x) for x in e) + "\n")


def _check_operator(p, h):
    v = W.random_vector(p.n_unknowns, 2)
    y = h.apply_op(torch.from_numpy(v).cuda()).cpu().numpy()
    ref = O.apply(p, v)
    assert np.abs(y - ref).max() / (np.abs(v).max() + np.abs(v - ref).max()) <= 1e-12


def test_stored_plan_applied_and_reported(tmp_path):
    p = W.config1()
    key = B.plan_key(p, True)
    path = str(tmp_path / "plans.txt")
    src = B.sweep_source_hash()
    _write(path, [(B.plan_key(p, False), 8, 4, 1, 0, 2, src),
                  (key, 4, 8, 2, 3, 1, src)])
    with B.setup(p, precision=B.RT_PREC_MIXED, autotune=True, plan_file=path) as h:
        assert h.tuned_plan_status() == "current"
        o = h.effective_options()
        assert (o.chunk, o.sweep_waves, o.prefetch, o.wave_batches, o.coef_mode) == (4, 8, 2, 3, 1)
        assert h.plan_info()["chunk"] == 4
        assert h.sweep_config(True) == dict(waves=8, prefetch=1, coef_mode=0)
        _check_operator(p, h)
    # the caller's own settings win over the stored plan's
    with B.setup(p, precision=B.RT_PREC_MIXED, autotune=True, plan_file=path, chunk=8,
                 coef_mode=B.RT_COEF_RECOMPUTE) as h:
        o = h.effective_options()
        assert (o.chunk, o.sweep_waves, o.coef_mode) == (8, 8, B.RT_COEF_RECOMPUTE)
        _check_operator(p, h)
    # the FP64 key
    with B.setup(p, autotune=True, plan_file=path) as h:
        assert h.tuned_plan_status() == "current"
        assert h.sweep_config(False)["coef_mode"] == 1
    # no autotune: the file is not read
    with B.setup(p, precision=B.RT_PREC_MIXED, plan_file=path) as h:
        assert h.tuned_plan_status() == "none"
        assert h.effective_options().chunk == 0


def test_stale_missing_and_unusable_plans(tmp_path):
    p = W.config1()
    path = str(tmp_path / "plans.txt")
    _write(path, [(B.plan_key(p, True), 4, 4, 1, 0, 2, "0123456789abcdef")])
    with B.setup(p, precision=B.RT_PREC_MIXED, autotune=True, plan_file=path) as h:
        assert h.tuned_plan_status() == "stale"
        assert h.effective_options().chunk == 4
    with B.setup(W.config2(), autotune=True, plan_file=path) as h:
        assert h.tuned_plan_status() == "none"
    with B.setup(p, autotune=True, plan_file=str(tmp_path / "absent.txt")) as h:
        assert h.tuned_plan_status() == "none"
    # a plan whose chunk is too short for the slab (64 * 4 < 1023) is not applied
    q = W.config3()
    _write(path, [(B.plan_key(q, False), 4, 4, 1, 0, 2, B.sweep_source_hash())])
    with B.setup(q, autotune=True, plan_file=path) as h:
        assert h.tuned_plan_status() == "none"
        assert h.plan_info()["chunk"] == 16


def test_shipped_plans_are_current_for_the_benchmark_batch():
    """The plan index next to the library holds plans for the 512-slab batch
    measured with the sweep sources the library was built from."""
    p = W.config4(512)
    for prec in (B.RT_PREC_MIXED, B.RT_PREC_FP64):
        with B.setup(p, precision=prec, autotune=True) as h:
            assert h.tuned_plan_status() == "current", prec
