"""Host logic of the benchmark's measurements (no GPU needed): the
algorithmic bytes of an operator application, the roofline fractions, and
the counter summaries (HBM traffic from FETCH_SIZE / WRITE_SIZE scaled by a
copy of known size; VALU issue from SQ_INSTS_VALU) with their source-hash
gating."""
import csv
import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2110_11873_amd import workloads as W  # noqa: E402


def test_op_bytes_of_the_batch_match_a_count_from_the_grids():
    """The bytes the bench divides by: per ray-interval the streamed
    coefficients, per ray the weight (and kappa), per depth point dtau, per
    unknown sigma in and out; ray-intervals counted from the depth grids."""
    p = W.config4(512)
    ns = np.asarray(p.ns, dtype=np.int64)
    rays_per_slab = (p.n_mu // 2) * p.n_nu
    intervals = int(np.sum(ns - 1)) * rays_per_slab
    assert intervals == 120_746_712
    assert p.n_unknowns == 2 * int(np.sum(ns)) == 299_902
    plan = {"intervals": intervals}
    n_rays = p.n_atm * rays_per_slab
    sig = 16 * p.n_unknowns
    assert bench.op_bytes(p, plan, 0, 4) == 8 * intervals + 8 * n_rays + sig
    assert bench.op_bytes(p, plan, 0, 8) == 16 * intervals + 8 * n_rays + sig
    w32 = 4 * intervals + 16 * n_rays + 8 * int(np.sum(ns)) + sig
    assert bench.op_bytes(p, plan, 1, 4) == w32 == 495_604_024
    assert bench.op_bytes(p, plan, 2, 8) == 24 * n_rays + 8 * int(np.sum(ns)) + sig


def test_roofline_fractions():
    r = bench.roofline_hbm(4e9, 1000.0, "k", None)  # 4 GB in 1 ms
    assert r["bound"] == "hbm" and r["achieved"] == pytest.approx(4000.0)
    assert r["frac"] == pytest.approx(0.5)
    a = bench.roofline_alu(7.86e9, 1000.0, "k", None)  # 7.86 GFLOP in 1 ms
    assert a["bound"] == "alu" and a["frac"] == pytest.approx(0.1)


def _write_counters(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (k, c, v) in enumerate(rows):
            w.writerow([i, k, c, v])


def _log(path, n):
    with open(path, "w") as fh:
        fh.write("noise line\n")
        fh.write(json.dumps({"op": "x", "applications": n}) + "\n")


def test_traffic_and_valu_summaries_roundtrip(tmp_path, monkeypatch):
    root = tmp_path / "pmc"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    monkeypatch.setattr(bench, "VALU_FILE", str(tmp_path / "valu.json"))
    monkeypatch.setattr(bench, "sweep_source_hash", lambda: "h1")
    kib = bench.COPY_BYTES // 1024
    # the copy reads half its size on FETCH_SIZE and all of it on WRITE_SIZE
    _write_counters(str(root / "copy_fetch" / "a" / "run_counter_collection.csv"),
                    [("__amd_rocclr_copyBuffer", "FETCH_SIZE", kib / 2)] * 3)
    _write_counters(str(root / "copy_write" / "a" / "run_counter_collection.csv"),
                    [("__amd_rocclr_copyBuffer", "WRITE_SIZE", kib)] * 3)
    for kind, kname in (("fp32", "void rt::sweep::sweep_kernel<float, 8, 4, 0, 1>(rt::SweepArgs)"),
                        ("fp64", "void rt::sweep::sweep_kernel<double, 8, 4, 0, 1>(rt::SweepArgs)")):
        # one set-up dispatch of each kernel before the two timed ones (excluded)
        fe = [(kname, "FETCH_SIZE", 999.0), ("rt::finalize_kernel(rt::SweepArgs)", "FETCH_SIZE", 999.0)]
        wr = [(kname, "WRITE_SIZE", 999.0), ("rt::finalize_kernel(rt::SweepArgs)", "WRITE_SIZE", 999.0)]
        sq = [(kname, "SQ_INSTS_VALU", 1.0), (kname, "SQ_WAVES", 1.0)]
        for _ in range(2):
            fe += [(kname, "FETCH_SIZE", 100.0), ("rt::finalize_kernel(rt::SweepArgs)", "FETCH_SIZE", 10.0)]
            wr += [(kname, "WRITE_SIZE", 20.0), ("rt::finalize_kernel(rt::SweepArgs)", "WRITE_SIZE", 2.0)]
            sq += [(kname, "SQ_INSTS_VALU", 6.0e7), (kname, "SQ_WAVES", 16384.0)]
        _write_counters(str(root / (kind + "_fetch") / "a" / "run_counter_collection.csv"), fe)
        _write_counters(str(root / (kind + "_write") / "a" / "run_counter_collection.csv"), wr)
        _write_counters(str(root / (kind + "_sq") / "a" / "run_counter_collection.csv"), sq)
        for sub in ("_fetch", "_write", "_sq"):
            _log(str(root / (kind + sub + ".log")), 2)
    bench.summarize_pmc(str(root))
    t = json.load(open(tmp_path / "traffic.json"))
    assert t["fetch_factor"] == pytest.approx(2.0) and t["write_factor"] == pytest.approx(1.0)
    want = 1024 * ((100.0 * 2 + 20.0) + (10.0 * 2 + 2.0))
    assert bench.measured_traffic("fp32") == pytest.approx(want)
    assert bench.measured_traffic("fp64") == pytest.approx(want)
    bench.summarize_valu(str(root))
    assert bench.measured_valu("fp32") == pytest.approx(6.0e7)
    # 6e7 wave instructions x 4 cycles over 1024 SIMDs at 2.4 GHz in 125 us
    assert bench.valu_issue_frac("fp32", 125.0) == pytest.approx(6.0e7 * 4 / (1024 * 2.4e9 * 125e-6))
    # other sweep sources: the summaries no longer apply
    monkeypatch.setattr(bench, "sweep_source_hash", lambda: "h2")
    assert bench.measured_traffic("fp32") is None
    assert bench.measured_valu("fp64") is None and bench.valu_issue_frac("fp64", 1.0) is None
