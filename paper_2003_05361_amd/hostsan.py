"""Host-sanitizer build of libras.so, for checking the host code on the CPU.

    python -m paper_2003_05361_amd.hostsan      # prints how to run the CPU tests with it

The host sources (partitioner, overlap, sparse ordering and factorisation, stop
rule, C-ABI and upload) are compiled by ROCm's clang as plain host C++ with
AddressSanitizer and UndefinedBehaviorSanitizer (every undefined-behaviour
report is fatal); the device code object is the one the normal build made
(paper_2003_05361_amd/_build/kernels.o), so run the normal build first.  The
result is paper_2003_05361_amd/_lib/libras_hostsan.so.  Python is not
instrumented, so the sanitizer runtime is preloaded and leak checking is off
(the interpreter keeps its own allocations to the end).  GPU code is not
instrumented: the library is for the CPU tests (-m "not gpu").
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

from .build import BUILD, CSRC, LIBDIR, ROOT

CLANG = "/opt/rocm/llvm/bin/clang++"
LIB = os.path.join(LIBDIR, "libras_hostsan.so")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-shared-libasan"]
FLAGS = ["-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer", "-ffp-contract=off",
         "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]
HOST_SOURCES = ("plan", "sparse", "control", "api")


def runtime() -> str:
    """clang's shared sanitizer runtime, to preload into the interpreter."""
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not found:
        raise RuntimeError("clang's AddressSanitizer runtime not found under /opt/rocm/llvm")
    return found[-1]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"build step failed ({p.returncode}): {' '.join(cmd)}\n{p.stdout}")


def build() -> str:
    kernels = os.path.join(BUILD, "kernels.o")
    if not os.path.exists(kernels):
        raise RuntimeError("kernels.o missing: run python -m paper_2003_05361_amd.build first")
    objs = [os.path.join(BUILD, f"hostsan_{f}.o") for f in HOST_SOURCES]
    jobs = [[CLANG, *FLAGS, *SAN, "-c", os.path.join(CSRC, f + ".cpp"), "-o", o]
            for f, o in zip(HOST_SOURCES, objs)]
    with cf.ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        list(ex.map(_run, jobs))
    os.makedirs(LIBDIR, exist_ok=True)
    _run([CLANG, "-shared", *SAN, "-o", LIB, *objs, kernels, "-L/opt/rocm/lib", "-lamdhip64", "-lpthread",
          "-Wl,-rpath,/opt/rocm/lib"])
    return LIB


def env() -> dict:
    """Environment that runs Python against the sanitizer build."""
    e = dict(os.environ)
    e.update(LD_PRELOAD=runtime(), ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
             UBSAN_OPTIONS="print_stacktrace=1", RAS_LIBRARY=LIB)
    return e


if __name__ == "__main__":
    lib = build()
    e = env()
    print(lib)
    print(f"LD_PRELOAD={e['LD_PRELOAD']} ASAN_OPTIONS={e['ASAN_OPTIONS']} UBSAN_OPTIONS={e['UBSAN_OPTIONS']} "
          f"RAS_LIBRARY={lib} python -m pytest tests -q -m 'not gpu'")
    sys.exit(0)
