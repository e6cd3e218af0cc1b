"""Build libvpp.so (HIP kernels + C ABI) in-tree for gfx950 with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libvpp.so")
LIB_DEBUG = os.path.join(HERE, "libvpp_debug.so")
# the apply kernels: one unit per precision and degree, so that the
# template-heavy units compile in parallel
APPLY_UNITS = [f"apply_{p}_k{k}.hip" for p in ("f64", "f32") for k in (2, 3, 4)]
SOURCES = [*APPLY_UNITS, "apply_f64.hip", "apply_f32.hip", "apply_misc.hip", "blas.hip", "adjoint.hip",
           "closest_point.hip", "levelset.hip", "noalloc.hip", "amr.hip", "api.cpp"]
# the sources whose code changes under VPP_BOUNDS_CHECK (the instrumented
# kernels and the entry point that reads their counters); the debug library
# links the release objects of the others
DEBUG_SOURCES = [*APPLY_UNITS, "apply_misc.hip", "api.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-munsafe-fp-atomics",
         # packed FP32 VALU forms stay off (plain FP32 ops only)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def _compile(job) -> str:
    src, debug = job
    out = os.path.join(OUT, "debug") if debug else OUT
    obj = os.path.join(out, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *(["-DVPP_BOUNDS_CHECK"] if debug else []), "-x", "hip", "-c", os.path.join(SRC, src),
           "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}{' (debug)' if debug else ''}:\n{r.stderr}")
    return obj


def _link(objs, lib: str) -> None:
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)


def build(verbose: bool = True) -> str:
    """Compile every source (always) and link libvpp.so and its bounds-checked
    twin libvpp_debug.so (the same sources with VPP_BOUNDS_CHECK)."""
    os.makedirs(os.path.join(OUT, "debug"), exist_ok=True)
    # the slow template-heavy units first, so that they overlap
    jobs = [(src, True) for src in DEBUG_SOURCES] + [(src, False) for src in SOURCES]
    with cf.ThreadPoolExecutor(max(1, min(len(jobs), os.cpu_count() or 1))) as ex:
        objs = dict(zip(jobs, ex.map(_compile, jobs)))
    _link([objs[(src, False)] for src in SOURCES], LIB)
    _link([objs[(src, src in DEBUG_SOURCES)] for src in SOURCES], LIB_DEBUG)
    if verbose:
        print(f"built {LIB} and {LIB_DEBUG}")
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
