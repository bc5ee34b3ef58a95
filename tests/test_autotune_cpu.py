"""Host logic of the launch-plan autotuner: shape keys, candidate plans and
the JSON cache (no GPU needed)."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2110_11873_amd import autotune as AT  # noqa: E402
from paper_2110_11873_amd import workloads as W  # noqa: E402


def test_candidates_respect_chunk_limits():
    p = W.config4(512)
    cs = AT.candidates(p)
    assert {c["chunk"] for c in cs} == {8, 16, 32}  # 64 * 4 < 511
    for c in cs:
        if c["chunk"] > 8:
            assert c["sweep_waves"] == 4 and c["prefetch"] == 1
    small = W.config1_subgrid()
    assert {c["chunk"] for c in AT.candidates(small)} == {4, 8, 16}


def test_shape_key_separates_shapes_and_precisions():
    a, b = W.config4(512), W.config2()
    ka, kb = AT.shape_key(a, True, "gfx950"), AT.shape_key(b, True, "gfx950")
    assert ka != kb
    assert ka != AT.shape_key(a, False, "gfx950")
    assert ka != AT.shape_key(a, True, "gfx942")
    assert ka == AT.shape_key(W.config4(512), True, "gfx950")  # seeded: same shape


def test_store_and_lookup_roundtrip(tmp_path):
    path = str(tmp_path / "plans.json")
    p = W.config2()
    opts = dict(chunk=8, sweep_waves=4, prefetch=2, wave_batches=0)
    assert AT.lookup(p, False, arch="gfx950", path=path) is None
    AT.store(p, False, opts, [dict(options=opts, cost=1.0)], arch="gfx950", path=path)
    assert AT.lookup(p, False, arch="gfx950", path=path) == opts
    assert AT.lookup(p, True, arch="gfx950", path=path) is None
    assert AT.lookup(W.config1(), False, arch="gfx950", path=path) is None


def test_shipped_cache_entries_are_valid_plans():
    """Every stored plan is one the library accepts for its shape."""
    import json
    if not os.path.exists(AT.DEFAULT_CACHE):
        pytest.skip("no shipped cache")
    with open(AT.DEFAULT_CACHE) as fh:
        cache = json.load(fh)
    for key, ent in cache.items():
        o = ent["options"]
        assert set(o) == set(AT.TUNED_FIELDS), key
        assert o["chunk"] in (4, 8, 16, 32) and o["sweep_waves"] in (4, 8)
        assert o["prefetch"] in (1, 2) and 0 <= o["wave_batches"] <= 64
        assert not (o["sweep_waves"] == 8 and o["chunk"] > 8)
