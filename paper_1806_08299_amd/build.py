"""Build libwavett.so (the C-ABI library) for gfx950 with hipcc.

Every translation unit is compiled in parallel into _build/, then linked into
``paper_1806_08299_amd/libwavett.so``.  Flags that matter for results:

* ``-ffp-contract=off``: no implicit fused multiply-adds, so the per-point
  arithmetic is exactly the sequence written in wave_device.h in every kernel
  (the time-tiled sweep must be bitwise identical to the untiled one);
* ``-Xclang -target-feature -Xclang -packed-fp32-ops``: no packed FP32 ops;
* no fast-math of any kind.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libwavett.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-fPIC", "-std=c++17", "--offload-arch=" + ARCH, "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]


def sources():
    srcs = [os.path.join(CSRC, "wave_api.cpp")]
    srcs += [os.path.join(CSRC, "wave_r%d_%s%d.hip" % (r, k, m)) for r in range(1, 9) for k in "mb" for m in range(3)]
    srcs += [os.path.join(CSRC, "wave_r%d_m3.hip" % r) for r in range(1, 9)]   # explicit diffusion
    srcs += [os.path.join(CSRC, "wave_r%d_m4.hip" % r) for r in range(1, 9)]   # two-level diffusion
    return srcs


def _headers(with_abi: bool):
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".h", ".inc"))]
    if with_abi:   # only the host unit includes the public header
        inc = os.path.join(ROOT, "include")
        hs += [os.path.join(inc, f) for f in os.listdir(inc) if f.endswith(".h")]
    return hs


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if incremental and os.path.exists(obj):
        newest = max(os.path.getmtime(f) for f in _headers(src.endswith(".cpp")) + [src, __file__])
        if os.path.getmtime(obj) > newest:
            return obj
    cmd = [HIPCC, "-c", "-x", "hip", src, "-o", obj] + FLAGS
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout, r.stderr))
    return obj


def build(jobs: int = 0, verbose: bool = True, incremental: bool = False) -> str:
    """Compile every translation unit (incremental=True: only those older
    than their sources or any header) and link libwavett.so."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    srcs = sources()
    # largest units first (unrolled register rings: radius 4, 3, 2, then the rest)
    cost = {"wave_r4": 0, "wave_r3": 1, "wave_r2": 2}
    srcs.sort(key=lambda s: cost.get(os.path.basename(s)[:7], 3))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda f: _compile(f, incremental), srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB, file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build(incremental="--incremental" in sys.argv)
