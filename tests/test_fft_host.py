"""The in-house FFT's Stockham stages (fft.hpp), built for the host, against numpy."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "fft_host.cpp")
LIB = os.path.join(ROOT, "tests", "_build", "libfft_host.so")


@pytest.fixture(scope="module")
def fftlib():
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    deps = [SRC] + [os.path.join(ROOT, "paper_1604_07983_amd", "csrc", h) for h in ("fft.hpp", "fft_reg.hpp")]
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(d) for d in deps):
        subprocess.check_call(["hipcc", "-O2", "-std=c++17", "-fPIC", "-shared", "-x", "c++",
                               "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-I", os.path.join(ROOT, "paper_1604_07983_amd", "csrc"),
                               "-o", LIB, SRC])
    lib = ctypes.CDLL(LIB)
    lib.fft_line_host.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    lib.fft_reg_line_host.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    lib.twiddle_max_err.argtypes = [ctypes.c_int]
    lib.twiddle_max_err.restype = ctypes.c_double
    return lib


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 8, 12, 16, 20, 24, 30, 32, 40, 48, 60, 64, 96, 120, 128])
@pytest.mark.parametrize("sign", [-1, 1])
def test_stockham_matches_numpy(fftlib, n, sign):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    buf = np.ascontiguousarray(x.astype(np.complex128))
    assert fftlib.fft_line_host(buf.ctypes.data, n, sign) > 0
    want = np.fft.fft(x) if sign < 0 else np.fft.ifft(x) * n
    np.testing.assert_allclose(buf, want, rtol=0, atol=1e-13 * np.sqrt(n) * np.abs(want).max())


def test_rejects_unsupported_sizes(fftlib):
    buf = np.zeros(7, dtype=np.complex128)
    assert fftlib.fft_line_host(buf.ctypes.data, 7, -1) == -1


REG_SIZES = [2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 32, 40, 48]


@pytest.mark.parametrize("n", REG_SIZES)
@pytest.mark.parametrize("sign", [-1, 1])
def test_register_fft_matches_numpy(fftlib, n, sign):
    rng = np.random.default_rng(100 + n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    buf = np.ascontiguousarray(x.astype(np.complex128))
    assert fftlib.fft_reg_line_host(buf.ctypes.data, n, sign) == 1
    want = np.fft.fft(x) if sign < 0 else np.fft.ifft(x) * n
    np.testing.assert_allclose(buf, want, rtol=0, atol=1e-14 * np.sqrt(n) * np.abs(want).max())


@pytest.mark.parametrize("n", REG_SIZES + [96, 128])
def test_compile_time_twiddles(fftlib, n):
    assert fftlib.twiddle_max_err(n) <= 2.3e-16  # about one ulp at 1
