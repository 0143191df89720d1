"""Build libstc.so in-tree: the host analyser and plan persistence (g++) and
the HIP runtime and kernels (hipcc, gfx950)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libstc.so")
BUILD = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("STC_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-mllvm", "-amdgpu-mfma-vgpr-form",
             "-Wall", "-Wno-unused-result"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    ana_o = os.path.join(BUILD, "analyse.o")
    rt_o = os.path.join(BUILD, "runtime.o")
    per_o = os.path.join(BUILD, "persist.o")
    for src, obj in (("analyse.cpp", ana_o), ("persist.cpp", per_o)):
        _run(["g++", "-O2", "-std=c++17", "-fPIC", "-pthread", "-Wall", "-c", os.path.join(CSRC, src),
              "-o", obj], verbose)
    _run([HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, "runtime.hip"), "-o", rt_o], verbose)
    tmp = OUT + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "-pthread", f"--offload-arch={ARCH}", rt_o, ana_o, per_o, "-o", tmp],
         verbose)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
