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


def _f32_bias(lib, fn, N, direction, nlines=4000, seed=7):
    """Mean over random lines of (|X_32|^2 - |X|^2)/|X|^2 per output bin, weighted by |X|^2, and the
    statistical noise of that mean; X the exact transform (numpy, FP64) of the same FP32 input."""
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal((nlines, N)) + 1j * rng.standard_normal((nlines, N))).astype(np.complex64)
    out = np.empty_like(x)
    rc = fn(N, direction, nlines, x.ctypes.data_as(ctypes.c_void_p), out.ctypes.data_as(ctypes.c_void_p))
    assert rc == 0
    xd = x.astype(np.complex128)
    ref = np.fft.fft(xd, axis=1) if direction < 0 else np.fft.ifft(xd, axis=1) * N
    a64 = np.abs(ref) ** 2
    rel = (np.abs(out.astype(np.complex128)) ** 2 - a64) / a64
    w = a64 / a64.sum(axis=0, keepdims=True)
    bias = (rel * w).sum(axis=0)
    noise = np.sqrt(((rel - bias) ** 2 * w * w).sum(axis=0))
    return bias, noise, np.max(np.abs(out - ref)) / np.max(np.abs(ref))


@pytest.mark.parametrize("N", [40, 48, 160])
def test_fp32_transforms_carry_no_systematic_bias(lib, N):
    """FP32 transforms multiply by roots of unity held as two floats (the value and its remainder): their
    outputs then carry the rounding of the arithmetic alone, which averages over lines, and no systematic
    shift of |X|^2 from rounded constants. The mean over 4000 random lines stays within a few standard
    errors of zero, and far below the ~1e-7 that singly rounded FP32 constants produce."""
    fns = [lib.fft_lines_host_f32]
    if N in _reg_sizes(lib):
        fns.append(lib.fft_reg_host_f32)
    for fn in fns:
        fn.restype = ctypes.c_int
        for direction in (-1, 1):
            bias, noise, err = _f32_bias(lib, fn, N, direction)
            assert err < 1e-6
            assert np.max(np.abs(bias)) < 2e-8, (fn.__name__, direction, np.max(np.abs(bias)))
            assert np.median(np.abs(bias) / noise) < 3.0
