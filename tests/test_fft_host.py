"""The library's FFT passes (Stockham, radices 2-16), compiled for the host from
the same header as the GPU kernels, against numpy's FFT."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def lib():
    d = tempfile.mkdtemp()
    so = os.path.join(d, "fft_host_check.so")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-o", so,
                           os.path.join(HERE, "native", "fft_host_check.cpp")])
    L = ctypes.CDLL(so)
    L.fft_lines_host.restype = ctypes.c_int
    return L


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 30, 36, 40, 45, 48, 64, 72, 80, 96, 100, 160, 192])
@pytest.mark.parametrize("direction", [-1, 1])
def test_stockham_matches_numpy(lib, N, direction):
    rng = np.random.default_rng(N)
    nl = 3
    x = rng.standard_normal((nl, N)) + 1j * rng.standard_normal((nl, N))
    out = np.empty_like(x)
    rc = lib.fft_lines_host(N, direction, nl, x.ctypes.data_as(ctypes.c_void_p), out.ctypes.data_as(ctypes.c_void_p))
    assert rc == 0
    ref = np.fft.fft(x, axis=1) if direction < 0 else np.fft.ifft(x, axis=1) * N
    assert np.max(np.abs(out - ref)) < 1e-13 * N


def test_unsupported_length_is_rejected(lib):
    x = np.zeros(7, dtype=np.complex128)
    assert lib.fft_lines_host(7, -1, 1, x.ctypes.data_as(ctypes.c_void_p), x.ctypes.data_as(ctypes.c_void_p)) == -1


def _reg_sizes(L):
    buf = (ctypes.c_int * 64)()
    n = L.fft_reg_sizes(buf, 64)
    return [buf[i] for i in range(min(n, 64))]


def test_register_lengths_match_numpy(lib):
    """Every length with a register-resident kernel, both directions, on random lines
    (the transform is linear, so three random lines per length cover every output)."""
    sizes = _reg_sizes(lib)
    assert sizes and 48 in sizes and 16 in sizes
    for N in sizes:
        rng = np.random.default_rng(1000 + N)
        for direction in (-1, 1):
            for _ in range(3):
                x = rng.standard_normal(N) + 1j * rng.standard_normal(N)
                out = np.empty_like(x)
                rc = lib.fft_reg_host(N, direction, x.ctypes.data_as(ctypes.c_void_p),
                                      out.ctypes.data_as(ctypes.c_void_p))
                assert rc == 0
                ref = np.fft.fft(x) if direction < 0 else np.fft.ifft(x) * N
                assert np.max(np.abs(out - ref)) < 1e-13 * N, (N, direction)


def test_register_unsupported_length_is_rejected(lib):
    x = np.zeros(7, dtype=np.complex128)
    assert lib.fft_reg_host(7, -1, x.ctypes.data_as(ctypes.c_void_p), x.ctypes.data_as(ctypes.c_void_p)) == -1
