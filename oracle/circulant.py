"""Block-circulant preconditioner of ``I - M_eps N`` (test infrastructure only).

Section V-D of the paper preconditions GMRES with the block-circulant matrix W
closest to ``I - M_eps N`` in the Frobenius norm, circulant along one or more of
the three Toeplitz levels (the conclusion names "one or more levels").  The
reading taken here: circulant along the waveguide axis (the third level),
dense within a cross-section, and restricted to the support of the contrast in
all three axes, since the operator is the identity on every other voxel:

* columns: the voxel columns S where chi is non-zero on some slice;
* slices: a window of P consecutive slices starting at z0 that covers every
  slice where chi is non-zero on S, with P the smallest length >= that extent
  whose prime factors are 2, 3, 5 (P <= n3; otherwise P = n3), and z0 as small
  a shift of the first such slice as keeps the window inside the grid.

With blocks ``A_{i,j} = delta_ij I - D_i N_{i-j}`` (window slices i, j; D_i the
contrast of slice z0 + i on S, N_m the cross-section block of N at z-offset m),
the Frobenius-nearest block circulant averages the blocks of every wrapped
diagonal (i - j) mod P = k:

    W_k = delta_k0 I - (1/P) [ (sum_{i >= k} D_i) N_k + (sum_{i < k} D_i) N_{k - P} ]

and is block-diagonalised by the DFT along the window.  Every voxel outside
S x window keeps the identity.
"""
from __future__ import annotations

import numpy as np

from . import fft as _fft
from .green import COMPONENTS, parity


def support_columns(chi: np.ndarray) -> np.ndarray:
    """Cross-section voxels (i1, i2) where the contrast is non-zero on some slice, (|S|, 2)."""
    return np.argwhere(np.any(chi != 0, axis=2))


def smooth_length(n: int) -> int:
    """Smallest integer >= n whose prime factors are 2, 3 and 5."""
    m = max(n, 1)
    while True:
        v = m
        for p in (2, 3, 5):
            while v % p == 0:
                v //= p
        if v == 1:
            return m
        m += 1


def support_window(chi: np.ndarray) -> tuple:
    """(z0, P): the slice window of the preconditioner (module docstring)."""
    n3 = chi.shape[2]
    on = np.nonzero(np.any(chi != 0, axis=(0, 1)))[0]
    if len(on) == 0:
        return 0, n3
    first, last = int(on[0]), int(on[-1])
    P = smooth_length(last - first + 1)
    if P > n3:
        return 0, n3
    return min(first, n3 - P), P


def _N_block(table: np.ndarray, S: np.ndarray, m3: int) -> np.ndarray:
    """Cross-section block of N at z-offset m3 on S: shape (3|S|, 3|S|), index (a*|S| + p)."""
    s = len(S)
    d1 = S[:, None, 0] - S[None, :, 0]
    d2 = S[:, None, 1] - S[None, :, 1]
    out = np.zeros((3 * s, 3 * s), dtype=np.complex128)
    for ci, (a, b) in enumerate(COMPONENTS):
        blk = table[ci][np.abs(d1), np.abs(d2), abs(m3)].copy()
        sgn = np.ones_like(d1, dtype=np.float64)
        if parity(a, b, 0) < 0:
            sgn = sgn * np.where(d1 < 0, -1.0, 1.0)
        if parity(a, b, 1) < 0:
            sgn = sgn * np.where(d2 < 0, -1.0, 1.0)
        if parity(a, b, 2) < 0 and m3 < 0:
            sgn = -sgn
        blk = blk * sgn
        out[a * s:(a + 1) * s, b * s:(b + 1) * s] = blk
        out[b * s:(b + 1) * s, a * s:(a + 1) * s] = blk
    return out


def dense_A_on_support(table: np.ndarray, chi: np.ndarray, S: np.ndarray) -> np.ndarray:
    """I - D N restricted to S x window in slice-major order: block (i, j) of size 3|S|."""
    z0, n3 = support_window(chi)
    s = len(S)
    m = 3 * s
    A = np.zeros((n3 * m, n3 * m), dtype=np.complex128)
    for i in range(n3):
        Di = np.tile(chi[S[:, 0], S[:, 1], z0 + i], 3)
        for j in range(n3):
            blk = -Di[:, None] * _N_block(table, S, i - j)
            if i == j:
                blk = blk + np.eye(m)
            A[i * m:(i + 1) * m, j * m:(j + 1) * m] = blk
    return A


def optimal_blocks(table: np.ndarray, chi: np.ndarray, S: np.ndarray) -> np.ndarray:
    """W_k, k < P, shape (P, 3|S|, 3|S|) (the formula in the module docstring)."""
    z0, n3 = support_window(chi)
    s = len(S)
    m = 3 * s
    D = np.stack([np.tile(chi[S[:, 0], S[:, 1], z0 + i], 3) for i in range(n3)])   # (P, m)
    W = np.zeros((n3, m, m), dtype=np.complex128)
    for k in range(n3):
        up = D[k:].sum(axis=0)
        lo = D[:k].sum(axis=0)
        W[k] = -(up[:, None] * _N_block(table, S, k)) / n3
        if k > 0:
            W[k] -= (lo[:, None] * _N_block(table, S, k - n3)) / n3
        if k == 0:
            W[k] += np.eye(m)
    return W


def block_circulant_dense(W: np.ndarray) -> np.ndarray:
    """Dense matrix of the block circulant with first block column W_k."""
    n3, m, _ = W.shape
    C = np.zeros((n3 * m, n3 * m), dtype=np.complex128)
    for i in range(n3):
        for j in range(n3):
            C[i * m:(i + 1) * m, j * m:(j + 1) * m] = W[(i - j) % n3]
    return C


def spectrum_inverse(W: np.ndarray) -> np.ndarray:
    """Inverses of the DFT blocks What_f = sum_k W_k e^{-2 pi i f k / n3}."""
    What = _fft.fft(W, axis=0)
    return np.linalg.inv(What)


def apply(Winv_hat: np.ndarray, S: np.ndarray, r: np.ndarray, window: tuple) -> np.ndarray:
    """z = W^{-1} r on S x window (window = support_window(chi)), identity elsewhere.
    r: (3, n1, n2, n3)."""
    z0, P = window
    z = r.copy()
    s = len(S)
    R = np.concatenate([r[a][S[:, 0], S[:, 1], z0:z0 + P] for a in range(3)], axis=0)   # (3|S|, P)
    Rh = _fft.fft(R, axis=1)
    Zh = np.einsum("fij,jf->if", Winv_hat, Rh)
    Z = _fft.fft(Zh, axis=1, inverse=True)
    for a in range(3):
        z[a][S[:, 0], S[:, 1], z0:z0 + P] = Z[a * s:(a + 1) * s]
    return z


def frequency_block(table: np.ndarray, chi: np.ndarray, S: np.ndarray, f: int) -> np.ndarray:
    """One DFT block What_f = sum_k W_k exp(-2 pi i f k / P), accumulated one W_k at a
    time (for full-size grids whose P blocks do not fit in memory together)."""
    z0, n3 = support_window(chi)
    s = len(S)
    m = 3 * s
    D = np.stack([np.tile(chi[S[:, 0], S[:, 1], z0 + i], 3) for i in range(n3)])
    suffix = np.cumsum(D[::-1], axis=0)[::-1]            # suffix[k] = sum_{i >= k} D_i
    total = suffix[0]
    out = np.eye(m, dtype=np.complex128)
    for k in range(n3):
        ph = np.exp(-2j * np.pi * ((f * k) % n3) / n3)
        Wk = -(suffix[k][:, None] * _N_block(table, S, k)) / n3
        if k > 0:
            Wk -= ((total - suffix[k])[:, None] * _N_block(table, S, k - n3)) / n3
        out += ph * Wk
    return out
