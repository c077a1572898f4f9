"""Builds libtbs.so (HIP for gfx950) in-tree with hipcc.

    python paper_1904_03057_amd/build.py [--jobs N] [--save-temps]

Every source is compiled on each call (object files go to paper_1904_03057_amd/_build/); the
shared library is written next to this file.  No GPU is needed to build.
"""
import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtbs.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# (source, object name, extra defines): the stencil kernels compile once per degree and boundary
# condition from one instantiation unit, in parallel with the rest
STENCIL_UNITS = [("stencil_inst.hip", "stencil_n%d_%s" % (n, b.lower()), ["-DTBS_DEGREE=%d" % n, "-DTBS_BC=BC_%s" % b])
                 for n in (5, 4, 3, 2, 1) for b in ("ROBIN", "DIRICHLET", "PERIODIC")]
SOURCES = STENCIL_UNITS + [(f, f, []) for f in ("stencil.hip", "vector.hip", "net.hip", "transfer.hip",
                                                "varcoef.hip", "api.cpp")]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "-Wno-unused-variable", "-Wno-unused-but-set-variable",
    # packed FP32 instructions stay off (plain scalar FP32 is what the kernels are written for)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(os.path.dirname(HERE), "include"),
]


def _compile(unit, extra):
    src, name, defs = unit
    obj = os.path.join(BUILD, name + ".o")
    cmd = [HIPCC] + FLAGS + defs + extra + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), p.stdout, p.stderr))
    return obj


def build(jobs=None, save_temps=False, verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    extra = ["-save-temps=obj"] if save_temps else []
    jobs = jobs or min(os.cpu_count() or 8, 16, len(SOURCES))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, extra), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,-z,defs", "-o", tmp] + objs
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (p.stdout, p.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--save-temps", action="store_true")
    a = ap.parse_args()
    build(a.jobs, a.save_temps, verbose=True)
    sys.exit(0)
