"""The boundary from plain C: a C11 program that includes only
include/nbs.h and links libnbs.so compiles, runs on the host (host-only
plan, no GPU) and sees the documented counts and errors."""
import os
import subprocess

import pytest

from paper_1604_07983_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_plain_c_consumer(tmp_path):
    if not os.path.exists(binding._LIB_PATH):
        pytest.skip("libnbs.so is not built")
    exe = str(tmp_path / "abi_host")
    libdir = os.path.dirname(binding._LIB_PATH)
    subprocess.check_call(["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "c", "abi_host.c"), "-L", libdir, "-lnbs",
                           "-Wl,-rpath," + libdir, "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "abi_host: ok" in out.stdout
