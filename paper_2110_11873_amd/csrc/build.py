"""Build librt.so (the gfx950 library behind include/rt.h) with hipcc.

    python -m paper_2110_11873_amd.csrc.build      # or: python build.py

Compiles every .hip file of this directory for gfx950 only, one process per
file in parallel (objects under paper_2110_11873_amd/_build/), and links them
into paper_2110_11873_amd/librt.so.  Packed FP32 instructions are disabled for the
device code (-packed-fp32-ops); hipcc's host pass warns that it does not know
the feature, which is harmless.
"""
import hashlib
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(PKG, "librt.so")
SOURCES = ["rt_api.hip", "rt_sweep.hip", "rt_sweep_f32.hip", "rt_sweep_f64.hip",
           "rt_sweep_f32_w.hip", "rt_sweep_f64_w.hip", "rt_sweep_f32_rc.hip", "rt_sweep_f64_rc.hip",
           "rt_krylov.hip",
           "rt_assemble.hip", "rt_dense.hip", "rt_raysweep.hip", "rt_field.hip",
           "rt_fieldsolve.hip", "rt_prd.hip", "rt_noalloc.hip"]
OBJDIR = os.path.join(PKG, "_build")
# the sources of the sweep's kernels and launchers: their hash is built into
# the library, and stored launch plans and counter readings are trusted only
# while it is unchanged
SWEEP_SOURCES = ["rt_sweep_kernel.h", "rt_sweep.hip", "rt_sweep_f32.hip", "rt_sweep_f64.hip",
                 "rt_sweep_f32_w.hip", "rt_sweep_f64_w.hip", "rt_sweep_f32_rc.hip",
                 "rt_sweep_f64_rc.hip", "rt_coef.h"]


def sweep_source_hash() -> str:
    h = hashlib.sha256()
    for f in SWEEP_SOURCES:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]

FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = [ln for ln in (r.stdout + r.stderr).splitlines()
             if ln.strip() and "packed-fp32-ops" not in ln and "warning generated" not in ln]
    return r.returncode, "\n".join(noise)


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJDIR, exist_ok=True)
    tag = f".{os.getpid()}"
    objs = [os.path.join(OBJDIR, os.path.splitext(src)[0] + tag + ".o") for src in SOURCES]
    define = f'-DRT_SWEEP_SOURCE_HASH="{sweep_source_hash()}"'
    cmds = [[hipcc, *FLAGS, define, "-I", INCLUDE, "-I", HERE, "-c", os.path.join(HERE, src), "-o",
             obj] for src, obj in zip(SOURCES, objs)]
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda c: _run(c, verbose), cmds))
    failed = [(c, msg) for c, (rc, msg) in zip(cmds, results) if rc != 0]
    for c, msg in failed:
        sys.stderr.write(msg + "\n")
    if verbose:
        for _, msg in results:
            if msg:
                print(msg)
    tmp = OUT + f".tmp{os.getpid()}"
    rc, msg = (1, "") if failed else _run(
        [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
    for o in objs:
        if os.path.exists(o):
            os.remove(o)
    if failed:
        raise RuntimeError("hipcc failed building librt.so")
    if rc != 0:
        sys.stderr.write(msg + "\n")
        raise RuntimeError("linking librt.so failed")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
