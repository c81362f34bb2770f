"""Build librlbm.so (HIP kernels for gfx950 + host C ABI) in-tree with hipcc."""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "librlbm.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("RLBM_OFFLOAD_ARCH", "gfx950")

# packed FP32 instructions are disabled for all device code
COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{INCLUDE}", f"-I{CSRC}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose_resources=False):
    os.makedirs(BUILD, exist_ok=True)
    k_obj = os.path.join(BUILD, "kernels.o")
    h_obj = os.path.join(BUILD, "rlbm.o")
    extra = ["-Rpass-analysis=kernel-resource-usage"] if verbose_resources else []
    _run([HIPCC, f"--offload-arch={ARCH}", *COMMON, *extra, "-c",
          os.path.join(CSRC, "kernels.hip"), "-o", k_obj])
    _run([HIPCC, f"--offload-arch={ARCH}", *COMMON, "-c", "-x", "hip",
          os.path.join(CSRC, "rlbm.cpp"), "-o", h_obj])
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", k_obj, h_obj, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose_resources="-v" in sys.argv)
