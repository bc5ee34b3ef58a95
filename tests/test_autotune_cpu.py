"""Host logic of the launch-plan autotuner and of the library's stored-plan
lookup: shape keys, candidate plans, the JSON cache and the plan index the
library reads (no GPU needed)."""
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2110_11873_amd import autotune as AT  # noqa: E402
from paper_2110_11873_amd import binding as B  # noqa: E402
from paper_2110_11873_amd import workloads as W  # noqa: E402


def test_candidates_respect_chunk_limits_and_cover_every_coefficient_mode():
    p = W.config4(512)
    cs = AT.candidates(p, mixed=True)
    assert {c["chunk"] for c in cs} == {8, 16, 32}  # 64 * 4 < 511
    assert {c["coef_mode"] for c in cs} == {AT.COEF_PAIRS, AT.COEF_STREAM_W, AT.COEF_RECOMPUTE,
                                            AT.COEF_RECOMPUTE_FP32}
    assert AT.COEF_RECOMPUTE_FP32 not in {c["coef_mode"] for c in AT.candidates(p, mixed=False)}
    for c in cs:
        if c["chunk"] > 8:
            assert c["sweep_waves"] == 4 and c["prefetch"] == 1
        if c["coef_mode"] != AT.COEF_PAIRS:
            assert c["prefetch"] == 1  # prefetch is compiled for the streamed pairs only
    small = W.config1_subgrid()
    assert {c["chunk"] for c in AT.candidates(small)} == {4, 8, 16}
    for c in cs:  # every candidate passes the library's validation
        assert B.validate(p, B.default_options(**c)) == 0, (c, B.last_error())


def test_plan_key_separates_shapes_precisions_and_architectures():
    a, b = W.config4(512), W.config2()
    ka, kb = AT.shape_key(a, True, "gfx950"), AT.shape_key(b, True, "gfx950")
    assert ka != kb
    assert ka != AT.shape_key(a, False, "gfx950")
    assert ka != AT.shape_key(a, True, "gfx942")
    assert ka == AT.shape_key(W.config4(512), True, "gfx950")  # seeded: same shape
    assert " " not in ka and ka.startswith("gfx950|mixed|0|16|101|512|512|")
    # the depth counts enter through their hash: same size, other depths
    c = a.slab(0)
    d = W.make_slabs([int(c.ns[0]) + 1], [(1e-4, 1e6)], 16, 101, 10.0, [1e-3], [1e-4], [0.5])
    assert AT.shape_key(c, True, "gfx950").split("|")[-1] != AT.shape_key(d, True, "gfx950").split("|")[-1]


def test_store_lookup_roundtrip_and_index(tmp_path):
    path = str(tmp_path / "plans.json")
    p = W.config2()
    opts = dict(chunk=8, sweep_waves=4, prefetch=2, wave_batches=0, coef_mode=AT.COEF_PAIRS)
    assert AT.lookup(p, False, arch="gfx950", path=path) is None
    AT.store(p, False, opts, [dict(options=opts, cost=1.0)], arch="gfx950", path=path)
    assert AT.lookup(p, False, arch="gfx950", path=path) == opts
    assert AT.lookup(p, True, arch="gfx950", path=path) is None
    assert AT.lookup(W.config1(), False, arch="gfx950", path=path) is None
    ent = AT.entry(p, False, arch="gfx950", path=path)
    assert ent["source_hash"] == B.sweep_source_hash()
    lines = [ln.split() for ln in open(AT.index_path(path)) if not ln.startswith("#")]
    assert lines == [[AT.shape_key(p, False, "gfx950"), "8", "4", "2", "0", "1",
                      B.sweep_source_hash()]]


def test_library_embeds_the_sweep_source_hash():
    from paper_2110_11873_amd.csrc import build
    assert B.sweep_source_hash() == build.sweep_source_hash()


def test_shipped_cache_entries_are_valid_plans():
    """Every stored plan is one the library accepts for its shape, the index
    the library reads matches the JSON cache, and every entry records the
    sweep sources it was measured with."""
    if not os.path.exists(AT.DEFAULT_CACHE):
        pytest.skip("no shipped cache")
    with open(AT.DEFAULT_CACHE) as fh:
        cache = json.load(fh)
    idx = {ln.split()[0]: ln.split()[1:] for ln in open(AT.index_path(AT.DEFAULT_CACHE))
           if ln.strip() and not ln.startswith("#")}
    assert set(idx) == set(cache)
    for key, ent in cache.items():
        o = ent["options"]
        assert set(o) == set(AT.TUNED_FIELDS), key
        assert o["chunk"] in (4, 8, 16, 32) and o["sweep_waves"] in (4, 8)
        assert o["prefetch"] in (1, 2) and 0 <= o["wave_batches"] <= 64
        assert 1 <= o["coef_mode"] <= 4
        assert not (o["sweep_waves"] == 8 and o["chunk"] > 8)
        assert idx[key] == [str(o[f]) for f in AT.TUNED_FIELDS] + [ent["source_hash"]]
