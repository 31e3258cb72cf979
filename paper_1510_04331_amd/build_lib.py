"""Build libgraphic.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_1510_04331_amd.build_lib   (or call build()).
"""

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libgraphic.so")
BUILD = os.path.join(ROOT, "_build")

SOURCES = ["line_pass.hip", "median.hip", "aux_kernels.hip", "register.hip", "preprocess.hip", "quality.hip",
           "graphic.cpp"]

ARCH = os.environ.get("GRAPHIC_OFFLOAD_ARCH", "gfx950")

# Packed-FP32 instructions are disabled for the device code: hipcc -O3 would
# otherwise form them from ordinary float code.
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
DEVICE = ["-x", "hip", "--offload-arch=" + ARCH, "-Xclang", "-target-feature",
          "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics"]


def _hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src, verbose, defines=()):
    tag = "_".join(d.replace("=", "") for d in defines)
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + (("_" + tag) if tag else "") + ".o")
    cmd = [_hipcc()] + COMMON + DEVICE + ["-D" + d for d in defines] + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (src, r.stdout, r.stderr))
    return obj


# Measurement programs (not part of the library): built next to it.
EXPERIMENTS = {"dft32_mfma": "experiments/dft32_mfma.hip"}


def _build_experiment(name, verbose):
    exe = os.path.join(HERE, name)
    cmd = [_hipcc()] + [f for f in COMMON if f != "-fPIC"] + DEVICE[2:] + \
        [os.path.join(CSRC, EXPERIMENTS[name]), "-o", exe + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (name, r.stdout, r.stderr))
    os.replace(exe + ".tmp", exe)
    return exe


def build(verbose=False, jobs=4, out=None, defines=()):
    """Compile every source and link libgraphic.so next to this file (or to
    ``out``), with optional extra ``-D`` definitions; also build the
    measurement programs."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        exps = [ex.submit(_build_experiment, n, verbose) for n in EXPERIMENTS] if out is None else []
        objs = list(ex.map(lambda s: _compile(s, verbose, defines), SOURCES))
        for f in exps:
            f.result()
    lib = out or LIB
    tmp = lib + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
