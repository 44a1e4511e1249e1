"""Build the native library libras.so (host setup in C++, kernels in HIP for gfx950).

    python -m paper_2003_05361_amd.build        # or paper_2003_05361_amd.build.build()

Objects go to paper_2003_05361_amd/_build/, the library to paper_2003_05361_amd/_lib/.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "libras.so")
ROOT = os.path.dirname(HERE)

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# hipcc's host pass warns about the device-only feature below; that is harmless
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"build step failed ({p.returncode}): {' '.join(cmd)}\n{p.stdout}")
    return p.stdout


def _stale(cmd) -> bool:
    """A compile step is stale when its object is older than its source or any header."""
    out = cmd[cmd.index("-o") + 1]
    src = cmd[cmd.index("-c") + 1]
    if not os.path.exists(out):
        return True
    deps = [src] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    deps.append(os.path.join(ROOT, "include", "ras.h"))
    return any(os.path.getmtime(d) > os.path.getmtime(out) for d in deps)


def build(verbose: bool = False, force: bool = True) -> str:
    """Compile every source (force) or only the stale ones, then link libras.so."""
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(LIBDIR, exist_ok=True)
    jobs = [
        # host setup: plain IEEE arithmetic (no contraction) keeps the partitioner bit-exact
        (["g++", *COMMON, "-ffp-contract=off", "-c", os.path.join(CSRC, "plan.cpp"), "-o",
          os.path.join(BUILD, "plan.o")]),
        (["g++", *COMMON, "-ffp-contract=off", "-c", os.path.join(CSRC, "sparse.cpp"), "-o",
          os.path.join(BUILD, "sparse.o")]),
        (["g++", *COMMON, "-c", os.path.join(CSRC, "control.cpp"), "-o", os.path.join(BUILD, "control.o")]),
        ([HIPCC, *COMMON, "-ffp-contract=off", "-c", os.path.join(CSRC, "api.cpp"), "-o",
          os.path.join(BUILD, "api.o")]),
        ([HIPCC, *COMMON, f"--offload-arch={ARCH}", *DEVICE_FLAGS, "-x", "hip", "-c",
          os.path.join(CSRC, "kernels.hip"), "-o", os.path.join(BUILD, "kernels.o")]),
    ]
    if not force:
        jobs = [j for j in jobs if _stale(j)]
    with cf.ThreadPoolExecutor(max_workers=5) as ex:
        outs = list(ex.map(_run, jobs))
    if verbose:
        for o in outs:
            sys.stdout.write(o)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp,
          os.path.join(BUILD, "plan.o"), os.path.join(BUILD, "sparse.o"), os.path.join(BUILD, "control.o"),
          os.path.join(BUILD, "api.o"),
          os.path.join(BUILD, "kernels.o"),
          "-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, force="--changed" not in sys.argv))
