"""The library's host code (validation, layout, revolve schedules and launch
plans) under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

fwi_runtime.cpp and revolve.cpp are compiled with g++ and
-fsanitize=address,undefined, linked with the (uninstrumented) kernel object
of the regular build into a separate shared library, and the whole CPU ABI
test module runs against it in a child process (FWI_LIBRARY selects the
build; the sanitizer runtime is preloaded, since the Python interpreter is
not instrumented).  Any invalid access, leak-free use after free, overflow or
undefined operation aborts the child and fails this test.  No GPU is used:
the ABI tests call only host-side entry points and argument checks.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1912_08063_amd")
CSRC = os.path.join(PKG, "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]


def _sanitized_library(out_dir):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not available")
    kernels = os.path.join(PKG, "_build", "fwi_kernels.hip.o")
    if not os.path.exists(kernels):
        from paper_1912_08063_amd import build
        build.build()
    objs = [kernels]
    for src in ("fwi_runtime.cpp", "revolve.cpp"):
        obj = os.path.join(out_dir, src + ".san.o")
        subprocess.run([gxx, "-O1", "-g", "-std=c++17", "-fPIC"] + SAN +
                       ["-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
                        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                        "-c", os.path.join(CSRC, src), "-o", obj], check=True)
        objs.append(obj)
    lib = os.path.join(out_dir, "libfwi_san.so")
    subprocess.run([gxx, "-shared", "-fPIC"] + SAN + ["-o", lib] + objs +
                   ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64"], check=True)
    return lib


def test_abi_tests_pass_under_asan_and_ubsan(tmp_path):
    lib = _sanitized_library(str(tmp_path))
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True, check=True).stdout
    assert "__asan_report_load" in syms and "__ubsan_handle" in syms   # instrumented
    asan = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True,
                          text=True, check=True).stdout.strip()
    env = dict(os.environ, FWI_LIBRARY=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    p = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_cpu.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = p.stdout[-4000:] + p.stderr[-4000:]
    assert p.returncode == 0, out
    assert "passed" in p.stdout and "ERROR: AddressSanitizer" not in out
    assert "runtime error" not in out
