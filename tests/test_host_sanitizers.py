"""Host code of the library under AddressSanitizer and UndefinedBehaviorSanitizer.

graphic.cpp (argument checks, geometry and flag validation, workspace and
batch planning, status strings) is compiled with both sanitizers on its host
side only (device code is unchanged), linked with the library's other objects
into the C driver tests/host_sanitize/abi_checks.c, and run on the CPU: the
driver exercises every host-only path of the C ABI, including sizes at and
beyond the limits.  The run must end cleanly, with no sanitizer report and no
leak.  Needs the objects of a normal build (``__graft_entry__.build()``).
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1510_04331_amd", "csrc")
BUILD = os.path.join(ROOT, "_build")
OUT = os.path.join(BUILD, "host_sanitize")
OTHER = ["line_pass", "median", "aux_kernels", "register", "preprocess", "quality"]


def _tool(*cands):
    for c in cands:
        if c and os.path.exists(c):
            return c
    return None


HIPCC = _tool(shutil.which("hipcc"), "/opt/rocm/bin/hipcc")
CLANG = _tool("/opt/rocm/llvm/bin/clang")
CLANGXX = _tool("/opt/rocm/llvm/bin/clang++")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-2000:], r.stderr[-4000:])


def test_abi_host_paths_are_clean_under_asan_and_ubsan():
    if not (HIPCC and CLANG and CLANGXX):
        pytest.skip("ROCm compilers not found")
    objs = [os.path.join(BUILD, o + ".o") for o in OTHER]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("library objects not built (run __graft_entry__.build())")
    os.makedirs(OUT, exist_ok=True)
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    lib_obj = os.path.join(OUT, "graphic_san.o")
    # host side only: each sanitizer flag follows -Xarch_host
    _run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "-Wno-unused-value"] + inc +
         ["-x", "hip", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-Xarch_host", "-fno-omit-frame-pointer",
          "-c", os.path.join(CSRC, "graphic.cpp"), "-o", lib_obj])
    drv_obj = os.path.join(OUT, "abi_checks.o")
    san = "-fsanitize=address,undefined"
    _run([CLANG, "-O1", "-g", san, "-fno-omit-frame-pointer", "-I" + os.path.join(ROOT, "include"),
          "-c", os.path.join(ROOT, "tests", "host_sanitize", "abi_checks.c"), "-o", drv_obj])
    exe = os.path.join(OUT, "abi_checks")
    _run([CLANGXX, san, "-o", exe, drv_obj, lib_obj] + objs +
         ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-6000:]
    assert "abi host checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-6000:]
