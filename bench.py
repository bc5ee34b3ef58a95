"""Benchmark of the matrix-free (Id - J Lambda T) operator and its Jacobi-Krylov solves.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
    python bench.py --op-only fp32|fp64|prd|prd_bf16|lu [--matvecs N] [--coef-mode M]  # one leg alone
    python bench.py --copy-calib                        # 512 MiB device copy x3
    python bench.py --summarize-pmc DIR                 # counters -> profiles/
    python bench.py --summarize-valu DIR                # VALU counters -> profiles/

Workload: a batch of 512 independent isothermal slabs of uneven depth
(Ns ~ U{64..512}, tau in [1e-4, tau_max], tau_max ~ logU[1e4, 1e8], 16
Gauss-Legendre directions, 101 frequencies on x in [-10, 10], Voigt profiles
with a ~ logU[1e-4, 1e-2], eps ~ logU[1e-6, 1e-2], W2 ~ U[0, 0.7], DELO-linear),
seeded.  A step is one Jacobi-preconditioned GMRES(30) solve of every slab to
||b - A x|| / ||b|| < 1e-9, in mixed precision (FP32 sweeps inside inner
GMRES solves, FP64 residuals and refinement), starting from x0 = [1, 0, ...]
with the inputs resident on the GPU.  `value` counts solved slabs per second.

Also on the same JSON line: the same solve in plain FP64; the operator alone
(FP64 and FP32 applications per second and their achieved bandwidth against
the HBM peak, timed with HIP events on the stream the kernels run on), in the
tuned launch plan and in each coefficient mode of the sweep; the single
1024-point slab (32 mu, 201 nu) solved in mixed precision to 1e-10; errors
against the FP64 oracle (the FP32 operator's, the refined solutions' residual
by the oracle's own operator, and their forward error against LU solutions of
the oracle's assembled A, with its condition number); the single
paper-shaped slab (Ns = 200, 20 mu, 101 nu) solved by Jacobi-GMRES, BiCGSTAB
and Richardson in FP64; and the FP64 CPU oracle timed on this host, on one
core and on several.
"""
import argparse
import csv
import glob
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "(Id−TΛ) matvecs/s, HBM GB/s frac; GMRES solves/s to 1e-9, FP64 vs mixed"
HBM_PEAK_GBS = 8000.0
RT_MAX_RESTART_USED = 128  # no restart on the paper's grids (their counts stay below)
RTOL = 1e-9
COPY_BYTES = 512 * 1024 * 1024
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_c4.json")
VALU_FILE = os.path.join(ROOT, "profiles", "sweep_valu_c4.json")
SIMDS, CLOCK_HZ, VALU_CYCLES = 1024, 2.4e9, 4  # 256 CUs x 4 SIMDs; a wave64 VALU op: 4 cycles
CPU_SHARE = 16  # host cores of one GPU's share on the benchmark machines


def sweep_source_hash():
    """Hash of the sweep sources the library was built from (built in)."""
    from paper_2110_11873_amd import binding as B
    return B.sweep_source_hash()


def measured_traffic(kind):
    """HBM bytes per operator application (sweep + finalize) from the committed
    counter summary, or None if there is none or the kernels changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != sweep_source_hash() or kind not in t:
        return None
    return t[kind]["hbm_bytes_per_launch"]


def measured_valu(kind):
    """VALU instructions (per wavefront, summed over the dispatch) of one
    sweep launch from the committed counter summary, or None if there is none
    or the kernels changed since."""
    try:
        with open(VALU_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != sweep_source_hash() or kind not in t:
        return None
    return t[kind]["valu_insts_per_launch"]


def valu_issue_frac(kind, us):
    """Share of the operator's time that its sweep's VALU instructions keep
    the 1024 SIMDs issuing (4 cycles per wave64 instruction at 2.4 GHz)."""
    n = measured_valu(kind)
    return None if n is None else n * VALU_CYCLES / (SIMDS * CLOCK_HZ * us * 1e-6)


def op_only(kind, n, coef_mode=0):
    """The operator leg alone (for counter passes): n applications, in the
    tuned launch plan of the mixed solve (FP32) or of the FP64 solve (FP64),
    or with its coefficient mode replaced; or the frequency-redistribution
    operator (256 depths, 32 mu, 256 nu, gamma = 0.5) with its contraction on
    the FP64 (prd) or the BF16 (prd_bf16) matrix cores; or (lu) n direct
    solves of the 512-slab batch, each on a fresh handle, so that each
    assembles and factors the batch once."""
    import torch
    from paper_2110_11873_amd import binding as B
    from paper_2110_11873_amd import workloads as W
    torch.cuda.set_device(0)
    if kind == "lu":
        p = W.config4(512)
        for _ in range(n):
            with B.setup(p, precision=B.RT_PREC_MIXED) as h:
                x = torch.zeros(p.n_unknowns, dtype=torch.float64, device="cuda")
                rc, info = h.solve_lu(x)
                torch.cuda.synchronize()
        print(json.dumps(dict(op=kind, factorizations=n, relres_max=max(i.relres for i in info))),
              flush=True)
        return
    if kind.startswith("prd"):
        p5, R5 = W.config5()
        with B.setup(p5) as h:
            h.set_redistribution(R5)
            v = torch.from_numpy(np.random.default_rng(0).uniform(-1, 1, h.prd_size())).cuda()
            y = torch.empty_like(v)
            f = h.apply_op_prd_bf16x3 if kind == "prd_bf16" else h.apply_op_prd
            for _ in range(n):
                f(v, y)
            torch.cuda.synchronize()
            print(json.dumps(dict(op=kind, applications=n)), flush=True)
        return
    p = W.config4(512)
    # the handle (and launch plan) the bench times the operator on
    kw = dict(coef_mode=coef_mode) if coef_mode else {}
    prec = B.RT_PREC_MIXED if kind == "fp32" else B.RT_PREC_FP64
    with B.setup(p, precision=prec, autotune=True, **kw) as h:
        v = torch.from_numpy(W.random_vector(p.n_unknowns, 0)).cuda()
        y = torch.empty_like(v)
        f = h.apply_op_fp32 if kind == "fp32" else h.apply_op
        for _ in range(n):
            f(v, y)
        torch.cuda.synchronize()
        print(json.dumps(dict(op=kind, applications=n, plan=h.plan_info(),
                              kernel=h.sweep_kernel_name(kind == "fp32"))), flush=True)


def copy_calib():
    """A plain device-to-device copy of known size, three times."""
    import torch
    x = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps(dict(copy_bytes=COPY_BYTES, copies=3)), flush=True)


def _counters(path):
    """{kernel name: {counter: [value per dispatch]}} from a rocprofv3 CSV."""
    out = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            k = r["Kernel_Name"]
            out.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return out


def _find(d, key):
    hits = [k for k in d if key in k]
    if len(hits) != 1:
        raise SystemExit(f"expected one kernel matching {key!r}, found {hits}")
    return d[hits[0]]


def summarize_pmc(root):
    """Turn the FETCH_SIZE / WRITE_SIZE passes under `root` (subfolders
    copy_fetch, copy_write, {fp32,fp64}_fetch, {fp32,fp64}_write, each holding
    rocprofv3's *counter_collection.csv) into profiles/traffic_c4.json."""
    def load(sub):
        fs = glob.glob(os.path.join(root, sub, "**", "*counter_collection.csv"), recursive=True)
        if len(fs) != 1:
            raise SystemExit(f"{sub}: expected one counter CSV, found {fs}")
        return _counters(fs[0])
    kib = COPY_BYTES / 1024
    cf = _find(load("copy_fetch"), "copyBuffer")["FETCH_SIZE"]
    cw = _find(load("copy_write"), "copyBuffer")["WRITE_SIZE"]
    f_fetch = kib / (sum(cf) / len(cf))
    f_write = kib / (sum(cw) / len(cw))
    out = {"source_hash": sweep_source_hash(), "copy_bytes": COPY_BYTES,
           "fetch_factor": f_fetch, "write_factor": f_write,
           "copy_fetch_kib": sum(cf) / len(cf), "copy_write_kib": sum(cw) / len(cw)}
    for kind, tname in (("fp32", "sweep_kernel<float"), ("fp64", "sweep_kernel<double")):
        fe, wr = load(kind + "_fetch"), load(kind + "_write")
        # the operator applications are the last `applications` dispatches
        # (set-up runs the FP64 sweep and the finalize pass once before them)
        with open(os.path.join(root, kind + "_fetch.log")) as fh:
            n = [json.loads(ln) for ln in fh if ln.startswith('{"op"')][0]["applications"]
        rec = {"applications": n}
        total = 0.0
        for short, key in (("sweep", tname), ("finalize", "finalize_kernel")):
            fk = _find(fe, key)["FETCH_SIZE"][-n:]
            wk = _find(wr, key)["WRITE_SIZE"][-n:]
            fkib, wkib = sum(fk) / len(fk), sum(wk) / len(wk)
            b = 1024 * (fkib * f_fetch + wkib * f_write)
            rec[short] = {"dispatches": len(fk), "fetch_kib": fkib, "write_kib": wkib,
                          "hbm_bytes": b}
            total += b
        rec["hbm_bytes_per_launch"] = total
        out[kind] = rec
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def summarize_valu(root):
    """Turn the SQ counter passes fp32_sq and fp64_sq under `root` (each a
    rocprofv3 --pmc run of --op-only fp32 / fp64 with SQ_INSTS_VALU, its log
    beside it as fp32_sq.log / fp64_sq.log) into profiles/sweep_valu_c4.json."""
    out = {"source_hash": sweep_source_hash(), "simds": SIMDS, "clock_hz": CLOCK_HZ,
           "cycles_per_valu": VALU_CYCLES}
    for kind, tname in (("fp32", "sweep_kernel<float"), ("fp64", "sweep_kernel<double")):
        fs = glob.glob(os.path.join(root, kind + "_sq", "**", "*counter_collection.csv"),
                       recursive=True)
        if len(fs) != 1:
            raise SystemExit(f"{kind}_sq: expected one counter CSV, found {fs}")
        with open(os.path.join(root, kind + "_sq.log")) as fh:
            n = [json.loads(ln) for ln in fh if ln.startswith('{"op"')][0]["applications"]
        c = _find(_counters(fs[0]), tname)
        v = c["SQ_INSTS_VALU"][-n:]
        w = c["SQ_WAVES"][-n:] if "SQ_WAVES" in c else [0.0]
        out[kind] = {"applications": n, "valu_insts_per_launch": sum(v) / len(v),
                     "waves_per_launch": sum(w) / len(w)}
    with open(VALU_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


def op_bytes(p, plan, coef_mode, s):
    """Algorithmic bytes of one operator application with the sweep in a
    coefficient mode (0: (E, w) pairs streamed, 1: w streamed, 2: both
    computed): the step coefficients the mode streams per ray-interval (2 s,
    s or 0 bytes, s = 4 or 8), per ray the quadrature weight (8 bytes) and,
    for the derived modes, kappa (8) or kappa and 1 / kappa (16), per depth
    point dtau (8, derived modes), and sigma read and sigma_out written
    (FP64, 16 bytes per unknown)."""
    n_rays = p.n_atm * (p.n_mu // 2) * p.n_nu
    coef = {0: 2 * s, 1: s, 2: 0}[coef_mode] * plan["intervals"]
    ray = {0: 8, 1: 16, 2: 24}[coef_mode] * n_rays
    dep = 0 if coef_mode == 0 else 8 * int(np.sum(p.ns))
    return float(coef + ray + dep) + 16.0 * p.n_unknowns


def time_ops(torch, fn, v, out, n):
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(5):
        fn(v, out)
    e0.record(s)
    for _ in range(n):
        fn(v, out)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / n  # ms per application


def time_solves(torch, h, x0, kind, steps, warmup):
    """Wall time of `steps` solves after `warmup` ones; the last solve's x."""
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
    return time.perf_counter() - t0, info, x


def copy_bandwidth(torch, nbytes=1 << 30, reps=20):
    """Device-to-device copy rate (bytes read + written per second)."""
    x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        y.copy_(x)
    e1.record(s)
    e1.synchronize()
    return 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9


def host_cpu():
    """Model name of this host's CPU (from /proc/cpuinfo) and its core count."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def _cpu_prepare(sl):
    """The oracle's dense A of one slab (column by column from its operator),
    the LU solution of A x = b, A's 2-norm condition number and the Jacobi
    diagonal -- untimed preparation."""
    from oracle import oracle as O
    A = O.assemble(sl)
    b = O.rhs(sl)
    return dict(b=b, x_lu=np.linalg.solve(A, b), kappa=float(np.linalg.cond(A)),
                dinv=1.0 / np.diag(A).copy())


def _cpu_solve(args):
    """One timed FP64 Jacobi-GMRES(30) solve of a slab by the oracle."""
    from oracle import oracle as O
    sl, b, dinv = args
    t0 = time.perf_counter()
    x, info = O.gmres(sl, b=b, dinv=dinv, tol=RTOL, restart=30)
    return dict(t=time.perf_counter() - t0, x=x, iterations=info[0]["iterations"])


def cpu_baseline(p, n_multi=16, n_single=4):
    """The FP64 oracle's Jacobi-GMRES(30) on a sample of the batch's slabs,
    timed on one core (n_single slabs in this process) and on several
    (n_multi slabs, one process per slab, up to one GPU's share of host
    cores).  Runs before the GPU is touched: the worker processes are forked
    from a process that has not initialized it."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    idx = [int(i) for i in np.linspace(0, p.n_atm - 1, n_multi).round().astype(int)]
    slabs = [p.slab(i) for i in idx]
    workers = max(1, min(n_multi, CPU_SHARE, os.cpu_count() or 1))
    with ProcessPoolExecutor(workers, mp_context=mp.get_context("fork")) as ex:
        prep = list(ex.map(_cpu_prepare, slabs))
        jobs = [(sl, pr["b"], pr["dinv"]) for sl, pr in zip(slabs, prep)]
        t0 = time.perf_counter()
        sol = list(ex.map(_cpu_solve, jobs))
        wall = time.perf_counter() - t0
    single = [_cpu_solve(j) for j in jobs[:n_single]]
    t1 = sum(r["t"] for r in single)
    model, ncpu = host_cpu()
    its = sum(r["iterations"] for r in sol)
    return dict(idx=idx, prep=prep, sol=sol, line=dict(
        value=len(idx) / wall, unit="solves/s", cores=workers, kind="oracle",
        single_core_value=n_single / t1, host=model, host_cores=ncpu,
        sample=f"{len(idx)} of the 512 slabs (indices {idx}, Ns {[int(p.ns[i]) for i in idx]}), "
               f"each one FP64 Jacobi-GMRES(30) solve to 1e-9 by the oracle ({its} iterations), "
               f"one process per slab on {workers} cores: {wall:.1f} s wall; the first "
               f"{n_single} of them one after another on one core: {t1:.1f} s.  Jacobi "
               f"diagonal, right-hand side, and the LU solutions and condition numbers "
               f"of the oracle's assembled A computed before the timed region"))


def routes(steps):
    """The rows beside the hot path, timed on the GPU (one JSON line): the
    dense route (assembly, LU, SOR/SSOR-GMRES) on the 512-slab batch, the
    DELO-parabolic operator and solve, the field-unknown system and the
    frequency-redistribution system; plus the
    unpreconditioned GMRES counts of both formulations on the paper's grids."""
    import torch
    from paper_2110_11873_amd import binding as B
    from paper_2110_11873_amd import workloads as W

    torch.cuda.set_device(0)
    out = {"mode": "routes"}

    def ev_ms(fn, n):
        fn()
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(n):
            fn()
        e1.record(s)
        e1.synchronize()
        return e0.elapsed_time(e1) / n

    p = W.config4(512)
    x0 = torch.from_numpy(W.initial_guess(p)).cuda()
    with B.setup(p, autotune=True) as h:
        A = h.assemble()
        out["c4_assemble_ms"] = ev_ms(lambda: h.assemble(A), steps)
        out["c4_assembled_GB"] = A.numel() * 8 / 1e9
        del A
        torch.cuda.empty_cache()
        x = torch.zeros_like(x0)
        t0 = time.perf_counter()
        _, info = h.solve_lu(x)
        out["c4_lu_first_call_ms"] = 1e3 * (time.perf_counter() - t0)
        out["c4_lu_relres_max"] = max(i.relres for i in info)
        out["c4_lu_solve_ms"] = ev_ms(lambda: h.solve_lu(x), steps)
    for name, pc in (("sor", B.RT_PC_SOR), ("ssor", B.RT_PC_SSOR)):
        with B.setup(p, autotune=True, precond=pc, rtol=1e-10, precision=B.RT_PREC_MIXED) as h:
            dt, info, _ = time_solves(torch, h, x0, "gmres", max(1, steps // 2), 1)
            out[f"c4_{name}_gmres_mixed_ms"] = 1e3 * dt / max(1, steps // 2)
            out[f"c4_{name}_gmres_iterations_max"] = max(i.iterations for i in info)
            v = torch.from_numpy(W.random_vector(p.n_unknowns, 0)).cuda()
            out[f"c4_{name}_apply_ms"] = ev_ms(lambda: h.precond_apply(v), steps)

    q = W.config2("delo_parabolic")
    xq = torch.from_numpy(W.initial_guess(q)).cuda()
    with B.setup(q, rtol=1e-10) as h:
        vq = torch.from_numpy(W.random_vector(q.n_unknowns, 0)).cuda()
        out["c2_parabolic_matvec_us"] = 1e3 * ev_ms(lambda: h.apply_op(vq), 50)
        dt, info, _ = time_solves(torch, h, xq, "gmres", steps, 1)
        out["c2_parabolic_gmres_ms"] = 1e3 * dt / steps
        out["c2_parabolic_gmres_iterations"] = info[0].iterations
    pp = p.with_(formal_solver=W.FS_DELO_PARABOLIC)
    with B.setup(pp) as h:
        v = torch.from_numpy(W.random_vector(p.n_unknowns, 0)).cuda()
        out["c4_parabolic_matvec_ms"] = ev_ms(lambda: h.apply_op(v), 5)

    q = W.config2()
    with B.setup(q, rtol=1e-10, restart=30, maxit=20000) as h:
        f = torch.from_numpy(np.random.default_rng(0).uniform(-1, 1, h.field_size())).cuda()
        out["c2_field_size"] = f.numel()
        out["c2_field_matvec_us"] = 1e3 * ev_ms(lambda: h.apply_op_field(f), 50)
        If = torch.zeros_like(f)
        t0 = time.perf_counter()
        _, info = h.solve_field_gmres(If)
        torch.cuda.synchronize()
        out["c2_field_gmres_ms"] = 1e3 * (time.perf_counter() - t0)
        out["c2_field_gmres_iterations"] = info[0].iterations
        out["c2_field_gmres_relres"] = info[0].relres
    # frequency redistribution (256 depths, 32 mu, 256 nu, gamma = 0.5)
    p5, R5 = W.config5()
    with B.setup(p5, rtol=1e-9, restart=30, maxit=5000) as h:
        h.set_redistribution(R5)
        v = torch.from_numpy(np.random.default_rng(0).uniform(-1, 1, h.prd_size())).cuda()
        o5 = torch.empty_like(v)
        out["c5_prd_size"] = v.numel()
        out["c5_prd_matvec_us"] = 1e3 * ev_ms(lambda: h.apply_op_prd(v, o5), 50)
        x5 = torch.zeros_like(v)
        h.solve_prd_gmres(x5)  # first call sets up the workspace and diagonal
        x5.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = h.solve_prd_gmres(x5)
        torch.cuda.synchronize()
        out["c5_prd_gmres_ms"] = 1e3 * (time.perf_counter() - t0)
        out["c5_prd_gmres_iterations"] = info[0].iterations
        out["c5_prd_gmres_relres"] = info[0].relres
        out["c5_prd_bf16x3_matvec_us"] = 1e3 * ev_ms(lambda: h.apply_op_prd_bf16x3(v, o5), 50)
    # the mixed solve: FP64 refinement around BF16x3 inner GMRES
    with B.setup(p5, rtol=1e-9, restart=30, maxit=5000, precision=B.RT_PREC_MIXED) as h:
        h.set_redistribution(R5)
        x5 = torch.zeros(h.prd_size(), dtype=torch.float64, device="cuda")
        h.solve_prd_gmres(x5)
        x5.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = h.solve_prd_gmres(x5)
        torch.cuda.synchronize()
        out["c5_prd_mixed_ms"] = 1e3 * (time.perf_counter() - t0)
        out["c5_prd_mixed_iterations"] = info[0].iterations
        out["c5_prd_mixed_outer_steps"] = info[0].outer_steps
        out["c5_prd_mixed_relres"] = info[0].relres
    counts = {"ns": [], "sigma_gmres": [], "field_gmres": []}
    for ns in (20, 40, 60, 80, 100, 120, 140):
        r = W.paper_replica(ns, scale="integrated", normalize=False)
        with B.setup(r, rtol=1e-6, restart=RT_MAX_RESTART_USED, maxit=1000) as h:
            # the library's sigma solvers are always preconditioned; the
            # unpreconditioned sigma counts beside these are the paper's (which
            # the oracle reproduces exactly)
            If = torch.zeros(h.field_size(), dtype=torch.float64, device="cuda")
            _, info = h.solve_field_gmres(If)
        counts["ns"].append(ns)
        counts["field_gmres"].append(info[0].iterations)
    counts["sigma_gmres"] = [28, 48, 68, 87, 104, 120, 134]  # Table tab:no_prec, GMRES row
    out["replica_unpreconditioned_gmres"] = counts
    print(json.dumps(out), flush=True)
    return 0


MODE_NAMES = {0: "pairs", 1: "stream_w", 2: "recompute"}
MODE_OPTION = {0: 1, 1: 2, 2: 3}  # kernel coefficient mode -> rt_options.coef_mode


def normwise(ref, v, y):
    """||y - ref||_inf / (||v||_inf + ||v - ref||_inf): the operator error
    relative to its two terms (sigma_in and xi J Lambda T sigma_in)."""
    return float(np.abs(y - ref).max() / (np.abs(v).max() + np.abs(v - ref).max()))


# FP32 (and FP64) vector peak with packed FP32 instructions off (as this
# library is built): 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
ALU_PEAK_TFLOPS = 78.6
# algorithmic flops of one ray-interval (both directions, both sources) by
# coefficient mode: recurrences 4 FMA and quadrature 4 FMA (16), w (S_u - S_k)
# for the two sources (2); E = 1 - w d with d = kappa dtau (3, w streamed);
# d, exp(-d), w = (1 - E) / d (5, recomputed)
FLOPS_PER_INTERVAL = {0: 18, 1: 21, 2: 23}


def roofline_alu(flops, us, kname, traffic):
    a = flops / (us * 1e-6) / 1e12
    return {"bound": "alu", "achieved": a, "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": a / ALU_PEAK_TFLOPS, "traffic": traffic,
            "kernel": kname + " + rt::finalize_kernel", "flops_per_launch": flops,
            "launch_us": us}


def roofline_hbm(bytes_, us, kname, traffic):
    a = bytes_ / (us * 1e-6) / 1e9
    return {"bound": "hbm", "achieved": a, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": a / HBM_PEAK_GBS, "traffic": traffic, "kernel": kname + " + rt::finalize_kernel",
            "bytes_per_launch": bytes_, "launch_us": us}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--matvecs", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--op-only", choices=["fp32", "fp64", "prd", "prd_bf16", "lu"])
    ap.add_argument("--coef-mode", type=int, default=0,
                    help="with --op-only: rt_options.coef_mode (0 = the tuned plan's)")
    ap.add_argument("--copy-calib", action="store_true")
    ap.add_argument("--summarize-pmc", metavar="DIR")
    ap.add_argument("--summarize-valu", metavar="DIR")
    ap.add_argument("--routes", action="store_true",
                    help="time the dense, DELO-parabolic and field-unknown routes instead")
    args = ap.parse_args()
    if args.summarize_pmc:
        return summarize_pmc(args.summarize_pmc)
    if args.summarize_valu:
        return summarize_valu(args.summarize_valu)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the slabs of the batch are independent (a multi-GPU "
              "run would split them with no communication), so only N=1 is run here.",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calib:
        return copy_calib()
    if args.op_only:
        return op_only(args.op_only, args.matvecs, args.coef_mode)
    if args.routes:
        return routes(args.steps)

    from oracle import oracle as O
    from paper_2110_11873_amd import workloads as W
    p = W.config4(512)
    cpu = None
    if not args.no_cpu_baseline:
        # before anything touches the GPU (the worker processes are forked)
        cpu = cpu_baseline(p)
        print(json.dumps(dict(stage="cpu baseline done", **{k: cpu["line"][k] for k in (
            "value", "single_core_value", "cores")})), file=sys.stderr, flush=True)

    import torch
    from paper_2110_11873_amd import binding as B

    torch.cuda.set_device(0)
    out = {}
    x0 = torch.from_numpy(W.initial_guess(p)).cuda()
    v = torch.from_numpy(W.random_vector(p.n_unknowns, 0)).cuda()
    y = torch.empty_like(v)
    with B.setup(p, rtol=RTOL, restart=30, maxit=20000, precision=B.RT_PREC_MIXED,
                 autotune=True) as h:
        plan = h.plan_info()
        cfg32, cfg64 = h.sweep_config(True), h.sweep_config(False)
        o = h.effective_options()
        out["launch_plan"] = {"mixed": dict(chunk=plan["chunk"], sweep_waves=cfg32["waves"],
                                            prefetch=o.prefetch, wave_batches=o.wave_batches,
                                            coef_mode=o.coef_mode,
                                            fp32_sweep=MODE_NAMES[cfg32["coef_mode"]],
                                            fp64_sweep=MODE_NAMES[cfg64["coef_mode"]],
                                            status=h.tuned_plan_status())}
        kname32 = h.sweep_kernel_name(True)
        dt, info, xg = time_solves(torch, h, x0, "gmres", args.steps, args.warmup)
        value = p.n_atm * args.steps / dt
        ms_step = 1e3 * dt / args.steps
        st = [i.status for i in info]
        out["mixed_converged"] = sum(s == "converged" for s in st)
        out["mixed_relres_max"] = max(i.relres for i in info)
        out["mixed_outer_steps_max"] = max(i.outer_steps for i in info)
        out["mixed_iterations_max"] = max(i.iterations for i in info)
        x_mixed = xg.cpu().numpy()
        t32 = time_ops(torch, h.apply_op_fp32, v, y, args.matvecs)
        y32 = y.cpu().numpy()
    cm32 = cfg32["coef_mode"]
    out["matvecs_per_s_fp32"] = 1e3 / t32
    out["matvec_us_fp32"] = t32 * 1e3
    out["sweep_plan"] = plan

    # the operator in every coefficient mode, with the tuned plan otherwise
    modes = {}
    for cm in (0, 1, 2):
        with B.setup(p, chunk=plan["chunk"], sweep_waves=cfg32["waves"],
                     wave_batches=o.wave_batches, coef_mode=MODE_OPTION[cm]) as hm:
            u32 = time_ops(torch, hm.apply_op_fp32, v, y, max(20, args.matvecs // 3)) * 1e3
            u64 = time_ops(torch, hm.apply_op, v, y, max(20, args.matvecs // 3)) * 1e3
        m32, m64 = op_bytes(p, plan, cm, 4), op_bytes(p, plan, cm, 8)
        fl = FLOPS_PER_INTERVAL[cm] * plan["intervals"]
        modes[MODE_NAMES[cm]] = {"fp32_us": u32, "fp64_us": u64,
                                 "fp32_bytes": m32, "fp64_bytes": m64,
                                 "fp32_hbm_frac": m32 / (u32 * 1e-6) / 1e9 / HBM_PEAK_GBS,
                                 "fp64_hbm_frac": m64 / (u64 * 1e-6) / 1e9 / HBM_PEAK_GBS,
                                 "flops": fl,
                                 "fp32_alu_frac": fl / (u32 * 1e-6) / 1e12 / ALU_PEAK_TFLOPS,
                                 "fp64_alu_frac": fl / (u64 * 1e-6) / 1e12 / ALU_PEAK_TFLOPS}
    out["coef_modes"] = modes

    # the same mixed solve with every GMRES cycle replayed from a HIP graph
    # (options.graphs), beside the eager launches `value` is measured with
    if not args.no_extras:
        with B.setup(p, rtol=RTOL, restart=30, maxit=20000, precision=B.RT_PREC_MIXED,
                     autotune=True, graphs=1) as hg:
            ng = max(2, args.steps // 2)
            dtg, infog, _ = time_solves(torch, hg, x0, "gmres", ng, 1)
            out["mixed_graph_replay_solves_per_s"] = p.n_atm * ng / dtg
            out["mixed_graph_replay_relres_max"] = max(i.relres for i in infog)

    with B.setup(p, rtol=RTOL, restart=30, maxit=20000, autotune=True) as h:
        cm64 = h.sweep_config(False)["coef_mode"]
        kname64 = h.sweep_kernel_name(False)
        out["launch_plan"]["fp64"] = dict(chunk=h.plan_info()["chunk"],
                                          sweep_waves=h.sweep_config(False)["waves"],
                                          coef_mode=h.effective_options().coef_mode,
                                          fp64_sweep=MODE_NAMES[cm64],
                                          status=h.tuned_plan_status())
        n64 = max(2, args.steps // 2)
        dt64, info64, xg64 = time_solves(torch, h, x0, "gmres", n64, 1)
        out["fp64_solves_per_s"] = p.n_atm * n64 / dt64
        out["fp64_converged"] = sum(i.status == "converged" for i in info64)
        out["fp64_iterations_max"] = max(i.iterations for i in info64)
        x_fp64 = xg64.cpu().numpy()
        t64 = time_ops(torch, h.apply_op, v, y, args.matvecs)
    out["matvecs_per_s_fp64"] = 1e3 / t64
    out["matvec_us_fp64"] = t64 * 1e3
    if cm64 == 2:
        out["roofline_fp64"] = roofline_alu(FLOPS_PER_INTERVAL[2] * plan["intervals"], t64 * 1e3,
                                            kname64, measured_traffic("fp64"))
    else:
        out["roofline_fp64"] = roofline_hbm(op_bytes(p, plan, cm64, 8), t64 * 1e3, kname64,
                                            measured_traffic("fp64"))
    out["roofline_fp64"]["coef_mode"] = MODE_NAMES[cm64]
    out["roofline_fp64"]["valu_issue_frac"] = valu_issue_frac("fp64", t64 * 1e3)
    out["mixed_over_fp64"] = value / out["fp64_solves_per_s"]
    out["hbm_copy_GBs"] = copy_bandwidth(torch)  # measured, beside the 8 TB/s datasheet peak

    # errors against the FP64 oracle on sampled slabs of the batch
    sl = O._slices(p)
    vh = v.cpu().numpy()
    errs = []
    for i in (0, 123, 300, 511):
        ref = O.apply_slab(p, i, vh[sl[i]])
        errs.append(normwise(ref, vh[sl[i]], y32[sl[i]]))
    out["fp32_op_error_c4"] = max(errs)
    if cpu is not None:
        rr, fe_m, fe_64, fe_o, kap = [], [], [], [], []
        for i, pr, so in zip(cpu["idx"], cpu["prep"], cpu["sol"]):
            b = pr["b"]
            rr.append(np.linalg.norm(b - O.apply_slab(p, i, x_mixed[sl[i]])) / np.linalg.norm(b))
            nl = np.linalg.norm(pr["x_lu"])
            fe_m.append(np.linalg.norm(x_mixed[sl[i]] - pr["x_lu"]) / nl)
            fe_64.append(np.linalg.norm(x_fp64[sl[i]] - pr["x_lu"]) / nl)
            fe_o.append(np.linalg.norm(so["x"] - pr["x_lu"]) / nl)
            kap.append(pr["kappa"])
        out["mixed_oracle_relres_max"] = float(max(rr))
        out["forward_error_c4"] = {
            "slabs": cpu["idx"], "kappa2_max": float(max(kap)), "kappa2_min": float(min(kap)),
            "mixed_max": float(max(fe_m)), "fp64_max": float(max(fe_64)),
            "oracle_gmres_max": float(max(fe_o)),
            "what": "||x - x_LU|| / ||x_LU||, x_LU the LU solution of the oracle's assembled A "
                    "(FP64, LAPACK); kappa2 its 2-norm condition number"}

    if not args.no_extras:
        # one 1024-point atmosphere (32 mu, 201 nu), FP32 inner GMRES(30) + FP64
        # refinement to 1e-10, against the oracle
        q3 = W.config3()
        x03 = torch.from_numpy(W.initial_guess(q3)).cuda()
        with B.setup(q3, rtol=1e-10, restart=30, maxit=20000, precision=B.RT_PREC_MIXED,
                     autotune=True) as h:
            d, inf, x3 = time_solves(torch, h, x03, "gmres", 3, 1)
            out["c3_mixed_solves_per_s"] = 3 / d
            out["c3_mixed_iterations"] = inf[0].iterations
            out["c3_mixed_outer_steps"] = inf[0].outer_steps
            v3 = W.random_vector(q3.n_unknowns, 1)
            y3 = h.apply_op_fp32(torch.from_numpy(v3).cuda()).cpu().numpy()
            out["c3_matvec_us_fp32"] = 1e3 * time_ops(
                torch, h.apply_op_fp32, torch.from_numpy(v3).cuda(),
                torch.empty(q3.n_unknowns, dtype=torch.float64, device="cuda"), 100)
        with B.setup(q3, rtol=1e-10, restart=30, maxit=20000, autotune=True) as h:
            d, inf, _ = time_solves(torch, h, x03, "gmres", 3, 1)
            out["c3_fp64_solves_per_s"] = 3 / d
        b3 = O.rhs(q3)
        x3h = x3.cpu().numpy()
        out["c3_mixed_oracle_relres"] = float(np.linalg.norm(b3 - O.apply(q3, x3h)) /
                                              np.linalg.norm(b3))
        out["fp32_op_error_c3"] = normwise(O.apply(q3, v3), v3, y3)

        # the tiny configuration: forward error against LU with kappa
        q1 = W.config1()
        A1 = O.assemble(q1)
        b1 = O.rhs(q1)
        xlu = np.linalg.solve(A1, b1)
        with B.setup(q1, rtol=1e-10, precision=B.RT_PREC_MIXED) as h:
            x1 = torch.from_numpy(W.initial_guess(q1)).cuda()
            h.solve_gmres(x1)
            x1 = x1.cpu().numpy()
        out["forward_error_c1"] = {"mixed": float(np.linalg.norm(x1 - xlu) / np.linalg.norm(xlu)),
                                   "kappa2": float(np.linalg.cond(A1)),
                                   "relres": float(np.linalg.norm(b1 - A1 @ x1) / np.linalg.norm(b1))}

        # the single paper-shaped slab (Ns = 200, 20 mu, 101 nu), FP64
        q = W.config2("delo_linear")
        xq = torch.from_numpy(W.initial_guess(q)).cuda()
        with B.setup(q, rtol=1e-10, restart=30) as h:
            d, inf, _ = time_solves(torch, h, xq, "gmres", 20, 3)
            out["c2_gmres_solves_per_s"] = 20 / d
            out["c2_gmres_iterations"] = inf[0].iterations
            d, inf, _ = time_solves(torch, h, xq, "bicgstab", 10, 2)
            out["c2_bicgstab_solves_per_s"] = 10 / d
            out["c2_bicgstab_iterations"] = inf[0].iterations
            vq = torch.from_numpy(W.random_vector(q.n_unknowns, 0)).cuda()
            out["c2_matvec_us"] = 1e3 * time_ops(torch, h.apply_op, vq, torch.empty_like(vq), 500)
        with B.setup(q, rtol=1e-10, maxit=200000) as h:
            d, inf, _ = time_solves(torch, h, xq, "richardson", 3, 1)
            out["c2_richardson_solves_per_s"] = 3 / d
            out["c2_richardson_iterations"] = inf[0].iterations

    if cm32 == 2:
        roof = roofline_alu(FLOPS_PER_INTERVAL[2] * plan["intervals"], t32 * 1e3, kname32,
                            measured_traffic("fp32"))
    else:
        roof = roofline_hbm(op_bytes(p, plan, cm32, 4), t32 * 1e3, kname32,
                            measured_traffic("fp32"))
    roof["coef_mode"] = MODE_NAMES[cm32]
    # the sweep's VALU issue time (counters of the same sources) over the
    # operator's measured time: what holds the kernel when the bytes do not
    roof["valu_issue_frac"] = valu_issue_frac("fp32", t32 * 1e3)
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
        "dtype": "f32/f64 mixed",
        "data": "synthetic",
        "config": {"workload": "512 uneven isothermal slabs (Ns 64..512), 16 mu x 101 nu, "
                               "Jacobi-GMRES(30), FP32 sweeps + FP64 refinement to 1e-9",
                   "n_slabs": 512, "ns_range": [64, 512], "n_mu": 16, "n_nu": 101,
                   "formal_solver": "DELO-linear", "restart": 30, "rtol": RTOL,
                   "seed": W.SEED_BASE + 4},
        "roofline": roof,
    }
    line.update(out)
    if cpu is not None:
        line["cpu_baseline"] = cpu["line"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
