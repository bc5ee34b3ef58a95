"""Autotuner of the sweep's launch plan.

The formal-solver sweep has five launch parameters that change its speed but
not its result (beyond rounding): the chunk length L (and with it the chunk
count per ray and the rays per wavefront), the wavefronts per workgroup,
whether a wavefront loads its next ray batch while sweeping the current one,
the ray batches per wavefront (which sets the workgroups per direction), and
where the step coefficients come from (streamed (E, w) pairs, streamed w
with E derived, or both computed in the sweep).  This module times every
candidate's operator on the current GPU for one problem shape, then times a
full solve with the few fastest and keeps the plan whose solve is fastest:

    python -m paper_2110_11873_amd.autotune --config batch512   # tune, store

Plans are stored under the key the library computes for a problem
(rt_plan_key: architecture, precision, formal solver, directions,
frequencies, slabs, deepest slab, a hash of the depth counts), together with
the hash of the sweep sources of the library that measured them.  Two files
next to this module: tuned_plans.json holds every entry with its timing
table; tuned_plans.txt, regenerated from it, is the one-line-per-plan index
the library itself reads when options.autotune is set (so a C caller of
rt_setup gets the same plan as binding.setup(..., autotune=True)).
RT_TUNE_CACHE names another JSON file (its .txt beside it).
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuned_plans.json")
TUNED_FIELDS = ("chunk", "sweep_waves", "prefetch", "wave_batches", "coef_mode")
# share of operator applications done in FP32 by a mixed-precision solve
# (inner GMRES steps against outer residuals), used to weigh the two timings
MIXED_FP32_SHARE = 0.9
# coefficient modes (rt.h RT_COEF_*): pairs, stream w, recompute, and
# recompute in FP32 with w streamed in FP64
COEF_PAIRS, COEF_STREAM_W, COEF_RECOMPUTE, COEF_RECOMPUTE_FP32 = 1, 2, 3, 4


def cache_path():
    return os.environ.get("RT_TUNE_CACHE", DEFAULT_CACHE)


def index_path(json_path):
    return os.path.splitext(json_path)[0] + ".txt"


def gpu_arch():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def shape_key(prob, mixed, arch):
    """The library's key of this problem shape (rt_plan_key)."""
    from . import binding as B
    return B.plan_key(prob, mixed, arch)


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def entry(prob, mixed, arch=None, path=None):
    """The stored entry (options, timings, source hash) for this shape, or None."""
    arch = arch or gpu_arch()
    return _load(path or cache_path()).get(shape_key(prob, mixed, arch))


def lookup(prob, mixed, arch=None, path=None):
    """Stored best options (a dict over TUNED_FIELDS) for this shape, or None."""
    ent = entry(prob, mixed, arch, path)
    return None if ent is None else {k: int(ent["options"][k]) for k in TUNED_FIELDS}


def candidates(prob, mixed=True):
    """Launch plans worth timing for this problem: every coefficient mode
    (the FP32-only recompute mode only where FP32 sweeps run), chunk lengths
    that cover the deepest slab, 4 or 8 waves (8 compiled for chunks up to
    8), prefetch where compiled (pairs, chunks up to 8), and 0 (automatic), 8
    or 16 ray batches per wave (also 1, 2 and 4 for a handful of slabs)."""
    ns_max = int(max(prob.ns))
    chunks = [L for L in (4, 8, 16, 32) if 64 * L >= ns_max - 1][:3]
    modes = [COEF_PAIRS, COEF_STREAM_W, COEF_RECOMPUTE] + ([COEF_RECOMPUTE_FP32] if mixed else [])
    # a handful of slabs: also one to four batches per wave (many workgroups
    # per slab, the chip filled by one slab's rays)
    nbs = (0, 8, 16) if len(prob.ns) > 8 else (0, 1, 2, 4, 8, 16)
    out = []
    for cm in modes:
        for L in chunks:
            for waves in ((4, 8) if L <= 8 else (4,)):
                for pf in ((1, 2) if (L <= 8 and cm == COEF_PAIRS) else (1,)):
                    for nb in nbs:
                        out.append(dict(chunk=L, sweep_waves=waves, prefetch=pf,
                                        wave_batches=nb, coef_mode=cm))
    return out


def _time_apply(torch, h, fp32, v, y, n):
    f = h.apply_op_fp32 if fp32 else h.apply_op
    for _ in range(3):
        f(v, y)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(n):
        f(v, y)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / n * 1e3  # microseconds per application


def _time_solve(torch, h, x0, reps):
    x = x0.clone()
    h.solve_gmres(x)  # first call: workspace
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        x.copy_(x0)
        h.solve_gmres(x)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps * 1e3  # ms per solve


def tune(prob, mixed, reps=20, verbose=False, cands=None, solve_top=4, solve_kw=None,
         solve_reps=3):
    """Time every candidate plan's operator, then a full GMRES solve with the
    `solve_top` cheapest; return (best options, table of timings)."""
    import torch
    from . import binding as B
    from . import workloads as W
    v = torch.from_numpy(W.random_vector(prob.n_unknowns, 0)).cuda()
    y = torch.empty_like(v)
    x0 = torch.from_numpy(W.initial_guess(prob)).cuda()
    w32 = MIXED_FP32_SHARE if mixed else 0.0
    prec = B.RT_PREC_MIXED if mixed else B.RT_PREC_FP64
    skw = {**dict(restart=30, rtol=1e-9, maxit=20000), **(solve_kw or {})}
    table = []
    for c in (cands or candidates(prob, mixed)):
        with B.setup(prob, **c) as h:
            t64 = _time_apply(torch, h, False, v, y, reps)
            t32 = _time_apply(torch, h, True, v, y, reps) if mixed else None
        cost = w32 * t32 + (1 - w32) * t64 if mixed else t64
        table.append(dict(options=c, us_fp64=round(t64, 2),
                          us_fp32=None if t32 is None else round(t32, 2), cost=round(cost, 2)))
        if verbose:
            print(json.dumps(table[-1]), flush=True)
    ranked = sorted(table, key=lambda r: r["cost"])
    for r in ranked[:solve_top]:
        with B.setup(prob, precision=prec, **skw, **r["options"]) as h:
            r["solve_ms"] = round(_time_solve(torch, h, x0, solve_reps), 3)
        if verbose:
            print(json.dumps(dict(solve=r)), flush=True)
    timed = [r for r in table if "solve_ms" in r]
    best = min(timed, key=lambda r: r["solve_ms"]) if timed else ranked[0]
    return best["options"], table


def write_index(path=None):
    """Regenerate the plan index the library reads from the JSON cache."""
    path = path or cache_path()
    cache = _load(path)
    lines = ["# launch plans for rt_setup with options.autotune (written by "
             "paper_2110_11873_amd.autotune from tuned_plans.json)",
             "# key chunk sweep_waves prefetch wave_batches coef_mode source_hash"]
    for key in sorted(cache):
        o, src = cache[key]["options"], cache[key].get("source_hash", "unknown")
        lines.append(" ".join([key] + [str(int(o[f])) for f in TUNED_FIELDS] + [src]))
    with open(index_path(path), "w") as fh:
        fh.write("\n".join(lines) + "\n")


def store(prob, mixed, options, table, arch=None, path=None, source_hash=None):
    from . import binding as B
    path = path or cache_path()
    arch = arch or gpu_arch()
    cache = _load(path)
    cache[shape_key(prob, mixed, arch)] = {
        "options": {k: int(options[k]) for k in TUNED_FIELDS},
        "timings_us": table,
        "ranked_by": "solve time of the fastest operators" if any(
            "solve_ms" in r for r in table) else "operator time",
        "source_hash": source_hash or B.sweep_source_hash(),
        "tuned": time.strftime("%Y-%m-%d"),
    }
    with open(path, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    write_index(path)


def _configs():
    """name -> (problem maker, solve options of the configuration)."""
    from . import workloads as W
    return {"batch512": (lambda: W.config4(512), dict(rtol=1e-9)),
            "slab200": (lambda: W.config2(), dict(rtol=1e-10)),
            "slab1024": (lambda: W.config3(), dict(rtol=1e-10))}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--config", choices=sorted(_configs()), action="append", required=True)
    ap.add_argument("--precision", choices=["fp64", "mixed", "both"], default="both")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--solve-top", type=int, default=4)
    ap.add_argument("--solve-reps", type=int, default=3)
    ap.add_argument("--cache", default=None)
    args = ap.parse_args(argv)
    modes = {"fp64": [False], "mixed": [True], "both": [False, True]}[args.precision]
    for name in args.config:
        make, skw = _configs()[name]
        prob = make()
        for mixed in modes:
            best, table = tune(prob, mixed, reps=args.reps, verbose=True,
                               solve_top=args.solve_top, solve_kw=skw,
                               solve_reps=args.solve_reps)
            store(prob, mixed, best, table, path=args.cache)
            print(json.dumps(dict(config=name, mixed=mixed, best=best)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
