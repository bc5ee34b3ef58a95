"""Benchmark of the matrix-free (Id - J Lambda T) operator and its Jacobi-Krylov solves.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

A step is one Jacobi-preconditioned GMRES(30) solve, in FP64, of the
paper-shaped slab (Ns = 200 log-spaced in tau in [1e-4, 1e8], 20 Gauss-Legendre
directions, 101 frequencies on x in [-10, 10], Voigt a = 1e-3, eps = 1e-4,
W2 = 0.5, DELO-linear) to ||b - A x|| / ||b|| < 1e-10 from x0 = [1, 0, ...],
with the inputs already resident on the GPU.  `value` is solves per second.

Also reported on the same line: the operator alone (matvecs/s, with the
achieved bandwidth of the sweep kernel against the HBM peak, timed with HIP
events on the stream the kernel runs on), the same solve in mixed precision,
BiCGSTAB and Jacobi-Richardson, a batched 512-slab workload, and the FP64 CPU
oracle timed on this host.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "(Id−TΛ) matvecs/s, HBM GB/s frac; GMRES solves/s to 1e-9, FP64 vs mixed"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes_fp64(plan, n_unknowns):
    # one (c_u, c_k) FP64 pair per ray-interval, sigma in and sigma out
    return 16.0 * plan["intervals"] + 16.0 * n_unknowns


def time_matvecs(torch, h, v, out, n):
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(10):
        h.apply_op(v, out)
    e0.record(s)
    for _ in range(n):
        h.apply_op(v, out)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / n  # ms per launch


def time_solves(torch, h, x0, kind, steps, warmup):
    x = x0.clone()
    fn = getattr(h, "solve_" + kind)
    info = None
    for _ in range(warmup):
        x.copy_(x0)
        _, info = fn(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        x.copy_(x0)
        _, info = fn(x)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, info, x


def cpu_baseline(p):
    """The FP64 oracle on this host: one Jacobi-GMRES(30) solve of the same
    slab (its Jacobi diagonal computed beforehand, untimed, as the GPU's is
    at setup)."""
    from oracle import oracle as O
    dinv = 1.0 / O.diag(p)
    b = O.rhs(p)
    t0 = time.perf_counter()
    x, info = O.gmres(p, b=b, dinv=dinv, tol=1e-10, restart=30)
    dt = time.perf_counter() - t0
    return dict(value=1.0 / dt, unit="solves/s", cores=1, kind="oracle",
                sample=f"one full Jacobi-GMRES(30) FP64 solve of the same slab to 1e-10 "
                       f"({info[0]['iterations']} iterations, {info[0]['matvecs']} matvecs, "
                       f"{dt:.2f} s single-threaded); Jacobi diagonal precomputed untimed")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--matvecs", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the slabs are independent and a single slab's "
              "solve is latency-bound, so this build measures one GPU's throughput "
              "(see the sharding notes in the design document).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2110_11873_amd import binding as B
    from paper_2110_11873_amd import workloads as W

    torch.cuda.set_device(0)
    p = W.config2("delo_linear")
    x0 = torch.from_numpy(W.initial_guess(p)).cuda()
    out = {}
    with B.setup(p, rtol=1e-10, restart=30) as h:
        plan = h.plan_info()
        dt, info, _ = time_solves(torch, h, x0, "gmres", args.steps, args.warmup)
        ms_step = 1e3 * dt / args.steps
        value = args.steps / dt
        v = torch.from_numpy(W.random_vector(p.n_unknowns, 0)).cuda()
        y = torch.empty_like(v)
        mv_ms = time_matvecs(torch, h, v, y, args.matvecs)
        bytes_mv = algorithmic_bytes_fp64(plan, p.n_unknowns)
        achieved = bytes_mv / (mv_ms * 1e-3) / 1e9
        out["gmres_iterations"] = info[0].iterations
        out["gmres_matvecs"] = info[0].matvecs
        out["gmres_relres"] = info[0].relres
        out["matvecs_per_s"] = 1e3 / mv_ms
        out["matvec_us"] = mv_ms * 1e3
        out["sweep_plan"] = plan
        if not args.no_extras:
            dtb, infob, _ = time_solves(torch, h, x0, "bicgstab", max(3, args.steps // 4), 1)
            out["bicgstab_solves_per_s"] = max(3, args.steps // 4) / dtb
            out["bicgstab_iterations"] = infob[0].iterations
    if not args.no_extras:
        with B.setup(p, rtol=1e-10, restart=30, precision=B.RT_PREC_MIXED) as hm:
            dtm, infom, _ = time_solves(torch, hm, x0, "gmres", max(3, args.steps // 2), 1)
            out["mixed_solves_per_s"] = max(3, args.steps // 2) / dtm
            out["mixed_outer_steps"] = infom[0].outer_steps
            out["mixed_relres"] = infom[0].relres
            v32 = torch.empty_like(v)
            s = torch.cuda.current_stream()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            for _ in range(10):
                hm.apply_op_fp32(v, v32)
            e0.record(s)
            for _ in range(args.matvecs):
                hm.apply_op_fp32(v, v32)
            e1.record(s)
            e1.synchronize()
            out["matvec_fp32_us"] = e0.elapsed_time(e1) / args.matvecs * 1e3

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "single slab Ns=200, 20 mu, 101 nu, DELO-linear, "
                               "Jacobi-GMRES(30) FP64 to 1e-10",
                   "ns": 200, "n_mu": 20, "n_nu": 101, "tau": [1e-4, 1e8], "eps": 1e-4,
                   "W2": 0.5, "a": 1e-3, "restart": 30, "rtol": 1e-10},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "sweep_kernel<double,L,4>",
                     "bytes_per_launch": bytes_mv, "launch_us": mv_ms * 1e3},
    }
    line.update(out)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(p)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
