"""Build libmrab.so (gfx950 HIP kernels + C++ host runtime) in-tree.

hipcc --offload-arch=gfx950 -O3 -std=c++17 -fPIC, packed-FP32 instructions
disabled for the device code.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmrab.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("MRAB_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
          "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = False) -> str:
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    src = os.path.join(HERE, "csrc")
    objs = []
    for name in ("kernels.hip", "adjoint.hip"):
        o = os.path.join(bdir, name + ".o")
        _run([HIPCC] + COMMON + DEVICE + ["-c", os.path.join(src, name), "-o", o], verbose)
        objs.append(o)
    o = os.path.join(bdir, "runtime.o")
    _run([HIPCC] + COMMON + ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-c",
                             os.path.join(src, "runtime.cpp"),
                             "-o", o], verbose)
    objs.append(o)
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs, verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
