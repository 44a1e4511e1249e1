"""The C ABI from a plain C caller, with no Python between it and the library:
tests/c_abi_consumer.c includes include/ras.h, is compiled by gcc, linked to the
built libras.so, and checks the host-only entry points (plan, index sets,
communication volume, band factors, stop rule, argument and pattern errors)
against values it computes from their definitions."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2003_05361_amd", "_lib")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_c_caller_of_the_host_entry_points(tmp_path):
    assert os.path.exists(os.path.join(LIBDIR, "libras.so")), "build the library first"
    exe = str(tmp_path / "c_abi_consumer")
    cc = subprocess.run(["gcc", "-std=c11", "-O1", "-Wall", "-Wextra", "-Werror", f"-I{os.path.join(ROOT, 'include')}",
                         os.path.join(ROOT, "tests", "c_abi_consumer.c"), "-o", exe, f"-L{LIBDIR}", "-lras",
                         f"-Wl,-rpath,{LIBDIR}", "-lm"], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert cc.returncode == 0, cc.stdout
    run = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=120)
    assert run.returncode == 0, run.stdout
    assert "c consumer ok" in run.stdout
