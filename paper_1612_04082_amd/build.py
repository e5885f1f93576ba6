"""Build libkfmm.so (HIP for gfx950 + host C++) in-tree with hipcc.

Every HIP source is compiled with packed FP32 instructions disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops); the compiler still vectorises ordinary code.
gemm.hip (the FP64 translation GEMMs) selects the VGPR form of the MFMA instructions
(-amdgpu-mfma-vgpr-form): with the accumulators in AGPRs the compiler copied every accumulator out of and
back into AGPRs around each LDS stage of those loops.  The FP32 M2L kernel (gemm_f32.hip) keeps the
default form, which measured faster for it.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libkfmm.so")
ARCH = os.environ.get("KFMM_ARCH", "gfx950")

SOURCES = ["tree.hip", "gemm.hip", "gemm_f32.hip", "gemm_h3.hip", "split_h3.hip", "fmm.hip", "bem.hip", "precond.hip",
           "nearfield.hip", "alg1.hip", "learn.hip", "operators.cpp", "capi.cpp"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-Wno-unused-result", "-I", os.path.join(HERE, "..", "include")]


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c


EXTRA = {"gemm.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]}


def _compile(src):
    obj = os.path.join(BUILD, src + ".o")
    extra = EXTRA.get(src, [])
    cmd = [_hipcc()] + COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    workers = min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8")))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr[-4000:])
    os.replace(tmp, LIB)
    if verbose:
        print(LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
