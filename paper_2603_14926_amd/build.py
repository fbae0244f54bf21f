"""Build libmpx.so (the HIP library for gfx950) in-tree.

Every HIP translation unit is compiled with
  -ffp-contract=off              no implicit fusing of a*b+c (TwoProd's fma is
                                 the only fused operation, and it is explicit)
  -fno-gpu-flush-denormals-to-zero  IEEE binary32 behaviour for float-float
  -Xclang -target-feature -Xclang -packed-fp32-ops
                                 no packed FP32 instructions
and the units are linked into paper_2603_14926_amd/libmpx.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libmpx.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    "-ffp-contract=off", "-fno-fast-math", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    f"-I{os.path.join(ROOT, 'include')}",
]


# Per-file flags.  The Ozaki slice GEMM keeps its MFMA accumulators in
# ordinary VGPRs (the accumulator-register form made the compiler copy every
# accumulator in and out of AGPRs on each loop iteration).
FILE_FLAGS = {"mpx_ozaki.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str, extra, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *FILE_FLAGS.get(os.path.basename(src), []), *extra, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, flush=True)
    return obj


# Host-sanitised variant of the library (AddressSanitizer and
# UndefinedBehaviorSanitizer on the host code only; the device code is the
# same as the product's), for the CPU tests of argument checking, plan
# construction and the tune cache.  Load it with the compiler's ASan runtime
# preloaded.  Not the product: the binding loads it only when MPX_LIBRARY
# names it.
ASAN_DIR = os.path.join(BUILD, "asan")
ASAN_LIB = os.path.join(ASAN_DIR, "libmpx_host_asan.so")
ASAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile_asan(src: str) -> str:
    obj = os.path.join(ASAN_DIR, os.path.basename(src) + ".o")
    cmd = [HIPCC, "-O1", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-ffp-contract=off",
           "-fno-fast-math", "-fno-gpu-flush-denormals-to-zero",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           f"-I{os.path.join(ROOT, 'include')}", *FILE_FLAGS.get(os.path.basename(src), []),
           *ASAN_FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc (host ASan) failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, extra=(), asan: bool = True) -> str:
    """Compile every csrc/*.hip for gfx950 and link libmpx.so (and, with
    asan, the host-sanitised test variant); returns the library's path."""
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(ASAN_DIR, exist_ok=True)
    srcs = sources()
    workers = min(2 * len(srcs), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        futs = [ex.submit(_compile, s, list(extra), verbose) for s in srcs]
        afuts = [ex.submit(_compile_asan, s) for s in srcs] if asan else []
        objs = [f.result() for f in futs]
        aobjs = [f.result() for f in afuts]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    if asan:
        subprocess.check_call([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *ASAN_FLAGS,
                               *aobjs, "-o", ASAN_LIB + ".tmp"])
        os.replace(ASAN_LIB + ".tmp", ASAN_LIB)
    return LIB


if __name__ == "__main__":
    extra = []
    if "--resource-usage" in sys.argv:
        extra = ["-Rpass-analysis=kernel-resource-usage"]
    print(build(verbose="-v" in sys.argv or bool(extra), extra=extra, asan=not extra))
