"""The oracle's own discrete Fourier transform (test infrastructure only).

``X[k] = sum_n x[n] exp(-2 pi i n k / M)`` along one axis, vectorised over the
others.  Powers of two use an iterative radix-2 decimation-in-time
Cooley-Tukey transform; any other length uses Bluestein's chirp-z identity
``n k = (n^2 + k^2 - (k - n)^2) / 2``, which turns the DFT into a circular
convolution of power-of-two length evaluated with the radix-2 transform.
"""
from __future__ import annotations

import numpy as np


def _is_pow2(n: int) -> bool:
    return n > 0 and (n & (n - 1)) == 0


def _bit_reverse(n: int) -> np.ndarray:
    bits = n.bit_length() - 1
    idx = np.arange(n)
    rev = np.zeros(n, dtype=np.int64)
    for b in range(bits):
        rev |= ((idx >> b) & 1) << (bits - 1 - b)
    return rev


def _radix2_last(x: np.ndarray, sign: int) -> np.ndarray:
    """Radix-2 DIT FFT along the last axis (length a power of two)."""
    n = x.shape[-1]
    y = x[..., _bit_reverse(n)].astype(np.complex128, copy=True)
    size = 2
    while size <= n:
        half = size // 2
        w = np.exp(sign * 2j * np.pi * np.arange(half) / size)
        y = y.reshape(y.shape[:-1] + (n // size, size))
        even = y[..., :half].copy()
        odd = y[..., half:] * w
        y[..., :half] = even + odd
        y[..., half:] = even - odd
        y = y.reshape(y.shape[:-2] + (n,))
        size *= 2
    return y


def _bluestein_last(x: np.ndarray, sign: int) -> np.ndarray:
    n = x.shape[-1]
    L = 1
    while L < 2 * n - 1:
        L *= 2
    k = np.arange(n)
    chirp = np.exp(sign * 1j * np.pi * (k * k % (2 * n)) / n)       # exp(sign*i*pi*k^2/n)
    a = np.zeros(x.shape[:-1] + (L,), dtype=np.complex128)
    a[..., :n] = x * chirp
    b = np.zeros(L, dtype=np.complex128)
    b[:n] = np.conj(chirp)
    b[L - n + 1:] = np.conj(chirp[1:][::-1])
    A = _radix2_last(a, -1)
    B = _radix2_last(b, -1)
    c = _radix2_last(A * B, +1) / L
    return c[..., :n] * chirp


def fft(x: np.ndarray, axis: int = -1, inverse: bool = False) -> np.ndarray:
    """DFT along ``axis``; the inverse includes the 1/M factor."""
    x = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, -1)
    n = x.shape[-1]
    sign = 1 if inverse else -1
    y = _radix2_last(x, sign) if _is_pow2(n) else _bluestein_last(x, sign)
    if inverse:
        y = y / n
    return np.moveaxis(y, -1, axis)


def fftn(x: np.ndarray, axes=(-3, -2, -1), inverse: bool = False) -> np.ndarray:
    for ax in axes:
        x = fft(x, axis=ax, inverse=inverse)
    return x
