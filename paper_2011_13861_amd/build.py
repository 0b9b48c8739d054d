"""Compiles the HIP/C++ sources under csrc/ into lib/libklmf.so for gfx950.

Every source with device code is compiled by hipcc (device code for gfx950 only) with
packed FP32 instructions disabled; the host-only sources (setup, dense eigensolver) are
compiled as plain C++; everything is linked into one shared library exposing the C ABI of
include/kl.h.  The issue-rate microbenchmark ubench/rates.hip is built next to it as
lib/klrates.
"""

import concurrent.futures
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "lib")
LIB = os.path.join(OUT_DIR, "libklmf.so")
OBJ_DIR = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(ROOT, "include"), "-Wno-unused-command-line-argument"]


# host-only sources (no device code): plain C++ through the same compiler, so that they may
# carry x86 function multiversioning; `omp simd` reductions are honoured (no OpenMP runtime)
CLANG = os.environ.get("KL_HOST_CXX", "/opt/rocm/lib/llvm/bin/clang++")
HOST_ONLY = ("dense_eig.cpp", "setup.cpp")


def _compile(src):
    obj = os.path.join(OBJ_DIR, os.path.basename(src) + ".o")
    if os.path.basename(src) in HOST_ONLY:
        cmd = [CLANG, "-O3", "-std=c++17", "-fPIC", "-fopenmp-simd", "-x", "c++", "-D__HIP_PLATFORM_AMD__",
               "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), "-c", src, "-o", obj]
    else:
        cmd = [HIPCC] + COMMON + ["-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr[-6000:]))
    return obj


def build(verbose=False):
    os.makedirs(OUT_DIR, exist_ok=True)
    os.makedirs(OBJ_DIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    jobs = min(8, len(srcs), os.cpu_count() or 1)
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs + [
        "-L/opt/rocm/lib", "-pthread", "-Wl,-rpath,/opt/rocm/lib", "-Wl,--no-undefined"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr[-4000:])
    os.replace(tmp, LIB)
    # the issue-rate microbenchmark that prices the covariance kernel's roofline
    rates = os.path.join(OUT_DIR, "klrates")
    cmd = [HIPCC] + COMMON + ["-o", rates + ".tmp", os.path.join(HERE, "ubench", "rates.hip")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for ubench/rates.hip:\n%s" % r.stderr[-4000:])
    os.replace(rates + ".tmp", rates)
    if verbose:
        print("built", LIB, "and", rates)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
