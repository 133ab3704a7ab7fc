"""Build libcastfem.so (gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libcastfem.so")
BUILD = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function", "-I" + CSRC]
DEVICE = ["-x", "hip", "--offload-arch=" + ARCH, "-munsafe-fp-atomics",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST = ["-x", "hip", "--offload-arch=" + ARCH, "--offload-host-only", "-fopenmp"]

SOURCES = [("kernels.hip", DEVICE), ("apparent.hip", DEVICE), ("varprops.hip", DEVICE), ("surrogate.hip", DEVICE),
           ("capi.cpp", HOST),
           ("prep.cpp", HOST),
           ("surrogate.cpp", HOST)]


def build(verbose=True):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src, flags in SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        cmd = [HIPCC] + COMMON + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = OUT + ".tmp%d" % os.getpid()
    link = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-fopenmp", "-o", tmp] + objs + [
        "-Wl,-rpath,/opt/rocm/lib/llvm/lib", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
