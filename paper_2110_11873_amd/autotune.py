"""Autotuner of the sweep's launch plan.

The formal-solver sweep has four launch parameters that change its speed but
not its result: the chunk length L (and with it the chunk count per ray and
the rays per wavefront), the wavefronts per workgroup, whether a wavefront
loads its next ray batch while sweeping the current one, and the ray batches
per wavefront (which sets the workgroups per direction).  This module times
the candidates on the current GPU for one problem shape, keeps the fastest,
and remembers it in a JSON cache keyed by the shape and the GPU
architecture:

    python -m paper_2110_11873_amd.autotune --config batch512   # tune, store

`lookup` returns the stored options for a problem (or None), and
`binding.setup(..., autotune=True)` applies them.  The cache shipped with the
package lives next to this file (tuned_plans.json); RT_TUNE_CACHE names
another.
"""
import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuned_plans.json")
TUNED_FIELDS = ("chunk", "sweep_waves", "prefetch", "wave_batches")
# share of operator applications done in FP32 by a mixed-precision solve
# (inner GMRES steps against outer residuals), used to weigh the two timings
MIXED_FP32_SHARE = 0.9


def cache_path():
    return os.environ.get("RT_TUNE_CACHE", DEFAULT_CACHE)


def gpu_arch():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def shape_key(prob, mixed, arch):
    """The problem features the launch plan depends on."""
    ns = [int(n) for n in prob.ns]
    digest = hashlib.sha1(",".join(map(str, ns)).encode()).hexdigest()[:12]
    return "|".join(map(str, (arch, "mixed" if mixed else "fp64", prob.formal_solver,
                              len(prob.mu), len(prob.w_nu), len(ns), max(ns), digest)))


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def lookup(prob, mixed, arch=None, path=None):
    """Stored best options (a dict over TUNED_FIELDS) for this shape, or None."""
    arch = arch or gpu_arch()
    ent = _load(path or cache_path()).get(shape_key(prob, mixed, arch))
    return None if ent is None else {k: int(ent["options"][k]) for k in TUNED_FIELDS}


def candidates(prob):
    """Launch plans worth timing for this problem."""
    ns_max = int(max(prob.ns))
    chunks = [L for L in (4, 8, 16, 32) if 64 * L >= ns_max - 1][:3]
    out = []
    for L in chunks:
        for waves in ((4, 8) if L <= 8 else (4,)):
            for pf in ((1, 2) if L <= 8 else (1,)):
                for nb in (0, 8, 16):
                    out.append(dict(chunk=L, sweep_waves=waves, prefetch=pf, wave_batches=nb))
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


def tune(prob, mixed, reps=20, verbose=False, cands=None):
    """Time every candidate plan; return (best options, table of timings)."""
    import torch
    from . import binding as B
    from . import workloads as W
    v = torch.from_numpy(W.random_vector(prob.n_unknowns, 0)).cuda()
    y = torch.empty_like(v)
    w32 = MIXED_FP32_SHARE if mixed else 0.0
    table = []
    for c in (cands or candidates(prob)):
        with B.setup(prob, **c) as h:
            t64 = _time_apply(torch, h, False, v, y, reps)
            t32 = _time_apply(torch, h, True, v, y, reps) if mixed else None
        cost = w32 * t32 + (1 - w32) * t64 if mixed else t64
        table.append(dict(options=c, us_fp64=round(t64, 2),
                          us_fp32=None if t32 is None else round(t32, 2), cost=round(cost, 2)))
        if verbose:
            print(json.dumps(table[-1]), flush=True)
    best = min(table, key=lambda r: r["cost"])
    return best["options"], table


def store(prob, mixed, options, table, arch=None, path=None):
    path = path or cache_path()
    arch = arch or gpu_arch()
    cache = _load(path)
    cache[shape_key(prob, mixed, arch)] = {
        "options": {k: int(options[k]) for k in TUNED_FIELDS},
        "timings_us": table,
        "tuned": time.strftime("%Y-%m-%d"),
    }
    with open(path, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)


def _configs():
    from . import workloads as W
    return {"batch512": lambda: W.config4(512), "slab200": lambda: W.config2(),
            "slab1024": lambda: W.config3()}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--config", choices=sorted(_configs()), action="append", required=True)
    ap.add_argument("--precision", choices=["fp64", "mixed", "both"], default="both")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--cache", default=None)
    args = ap.parse_args(argv)
    modes = {"fp64": [False], "mixed": [True], "both": [False, True]}[args.precision]
    for name in args.config:
        prob = _configs()[name]()
        for mixed in modes:
            best, table = tune(prob, mixed, reps=args.reps, verbose=True)
            store(prob, mixed, best, table, path=args.cache)
            print(json.dumps(dict(config=name, mixed=mixed, best=best)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
