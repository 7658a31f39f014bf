"""Build libabp.so (HIP, gfx950) in-tree with hipcc.

Every source under csrc/ is compiled to an object in _build/ (in parallel)
and linked into paper_1609_09833_amd/libabp.so. No torch headers or
libraries are involved: the library's interface is the C-ABI in include/abp.h.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libabp.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# No fast-math: the compensated sums rely on IEEE evaluation order.
# Packed FP32 instructions are disabled for all device code.
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
          f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


# Per-source flags. grid.hip: the MFMA deposit keeps its accumulators in
# ordinary VGPRs (the VGPR form of the MFMA instructions); with AGPR
# accumulators the compiler copies all of them in and out on every iteration.
EXTRA = {"grid.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def sources():
    out = []
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".cpp")):
            out.append(os.path.join(CSRC, name))
    return out


def _compile(src, build_dir=BUILD, extra=()):
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *COMMON, *EXTRA.get(os.path.basename(src), []), *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-fp32 feature and says so; drop that line
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in (r.stderr or "").splitlines() if noise not in l and "(ignoring feature)" not in l)
    return src, obj, r.returncode, err


def build(verbose: bool = True, lib_path: str = LIB, extra=(), build_dir: str = BUILD) -> str:
    """Compile and link. `extra` adds compiler flags (e.g. -D overrides of tile
    constants) and `lib_path`/`build_dir` redirect the outputs, for variants."""
    os.makedirs(build_dir, exist_ok=True)
    srcs = sources()
    jobs = min(len(srcs), max(1, (os.cpu_count() or 4)), 16)
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for src, obj, rc, err in ex.map(lambda s: _compile(s, build_dir, tuple(extra)), srcs):
            if err.strip() and verbose:
                print(err, file=sys.stderr)
            if rc != 0:
                raise RuntimeError(f"hipcc failed on {src}")
            objs.append(obj)
    tmp = lib_path + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Wl,-soname,libabp.so", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        print(r.stderr, file=sys.stderr)
        raise RuntimeError("link of libabp.so failed")
    os.replace(tmp, lib_path)
    if lib_path == LIB:
        build_driver()
    return lib_path


DRIVER_SRC = os.path.join(PKG, "examples", "abp_serve_driver.cpp")
DRIVER = os.path.join(PKG, "examples", "libabp_serve_driver.so")


def build_driver() -> str:
    """The serving load generator (a client of the C-ABI, not part of the
    library): plain C++ against include/abp.h, linked to libabp.so."""
    tmp = DRIVER + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread", "-Wall", "-I", INCLUDE, DRIVER_SRC,
           "-L", PKG, "-labp", "-Wl,-rpath,$ORIGIN/..", "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        print(r.stderr, file=sys.stderr)
        raise RuntimeError("build of the serving driver failed")
    os.replace(tmp, DRIVER)
    return DRIVER


if __name__ == "__main__":
    print(build())
