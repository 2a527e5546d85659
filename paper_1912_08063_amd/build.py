"""Build libfwi.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1912_08063_amd.build      # or paper_1912_08063_amd.build.build()
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libfwi.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["fwi_kernels.hip", "fwi_runtime.cpp", "revolve.cpp"]
# packed-fp32 instructions are disabled: hand-written or generated
# v_pk_{add,mul,fma}_f32 are avoided on this target.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", INCLUDE, "-I", CSRC]


def build(verbose=False, out=None, extra=None):
    """Compile every source and link libfwi.so (or `out`).  `extra` (or the
    environment variable FWI_HIPCC_FLAGS) adds compiler flags, e.g. -D options."""
    extra = list(extra or []) + os.environ.get("FWI_HIPCC_FLAGS", "").split()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(objdir, src + ".o")
        if src.endswith(".hip"):
            cmd = [HIPCC] + COMMON + DEVICE_FLAGS + extra + ["-x", "hip", "-c", path, "-o", obj]
        else:   # host-only C++ (HIP runtime API only)
            cmd = [HIPCC] + COMMON + ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
                                      "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    lib = out or LIB
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
