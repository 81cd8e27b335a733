"""Host code under the address and undefined-behaviour sanitizers (no GPU):
the channel compiler and the plan's host-only paths (built with g++ against
stand-ins for the kernel launchers) through the C ABI, and the oracle's C
entry points (built with gcc).  A sanitizer report fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1604_07983_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")


def _run(exe):
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    text = out.stdout + out.stderr
    assert out.returncode == 0, text[-4000:]
    assert "AddressSanitizer" not in text and "runtime error" not in text, text[-4000:]
    return text


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_plan_host_paths_under_sanitizers(tmp_path):
    exe = str(tmp_path / "plan_host_checks")
    objs = []
    for src, lang in ((os.path.join(CSRC, "compiler.cpp"), "c++"), (os.path.join(CSRC, "plan.cpp"), "c++"),
                      (os.path.join(ROOT, "tests", "c", "kernel_stubs.cpp"), "c++"),
                      (os.path.join(ROOT, "tests", "c", "plan_host_checks.c"), "c")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        comp = ["g++", "-std=c++17"] if lang == "c++" else ["gcc", "-std=c11"]
        subprocess.check_call(comp + SAN + ["-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
                                            "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", src, "-o", obj])
        objs.append(obj)
    subprocess.check_call(["g++"] + SAN + objs + ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib",
                                                  "-o", exe])
    assert "plan_host_checks: ok" in _run(exe)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_host_checks")
    subprocess.check_call(["gcc", "-std=gnu11", "-fopenmp"] + SAN +
                          ["-I", os.path.join(ROOT, "oracle"), os.path.join(ROOT, "oracle", "nbs_oracle.c"),
                           os.path.join(ROOT, "tests", "c", "oracle_host_checks.c"), "-lm", "-o", exe])
    assert "oracle_host_checks: ok" in _run(exe)
