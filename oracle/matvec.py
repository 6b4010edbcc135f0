"""Matrix-vector product of the discrete J-VIE operator ``I - M_eps N`` (test infrastructure).

Section III-A: with material constant per voxel the discrete J-VIE is
``(I - M_eps N) w_e = c_e M_eps e_inc`` (restated in Section V-D), where M_eps is
diagonal with entries ``(eps_r - 1)/eps_r`` (Section III) and N is the Toeplitz
Galerkin matrix of ``curl curl S``.  The constant c_e is dropped (the system is
linear and the right-hand side is built by the caller).

Vector layout: complex array of shape (3, n1, n2, n3), component-major, C order.
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np

from . import fft as _fft
from .green import COMPONENTS, parity


def contrast(eps: np.ndarray, eps_b: float) -> np.ndarray:
    """M_eps on a voxel: (eps_r - 1)/eps_r with eps_r = eps/eps_b (background scaled to 1,
    Section II)."""
    eps_r = np.asarray(eps, dtype=np.complex128) / eps_b
    return (eps_r - 1.0) / eps_r


def rhs_from_field(eps: np.ndarray, eps_b: float, e_inc: np.ndarray, h: float) -> np.ndarray:
    """b = M_eps e_inc with (e_inc)_i = <E_inc, P_i> taken at the voxel centre:
    h^{3/2} E_inc(r_i) (Section III-A, P_i = h^{-3/2} on V_i)."""
    return (h ** 1.5) * contrast(eps, eps_b)[None] * e_inc


def signed_table(table: np.ndarray) -> np.ndarray:
    """Full 3x3 tensor for every signed offset m in (-n, n): shape (3, 3, 2n1-1, 2n2-1, 2n3-1),
    index m + n - 1.  Negative offsets by the per-axis parity of each component."""
    _, n1, n2, n3 = table.shape
    out = np.empty((3, 3, 2 * n1 - 1, 2 * n2 - 1, 2 * n3 - 1), dtype=np.complex128)
    idx = [np.abs(np.arange(-nn + 1, nn)) for nn in (n1, n2, n3)]
    neg = [np.arange(-nn + 1, nn) < 0 for nn in (n1, n2, n3)]
    for ci, (a, b) in enumerate(COMPONENTS):
        blk = table[ci][np.ix_(idx[0], idx[1], idx[2])].copy()
        for d in range(3):
            if parity(a, b, d) < 0:
                shape = [1, 1, 1]
                shape[d] = -1
                blk *= np.where(neg[d], -1.0, 1.0).reshape(shape)
        out[a, b] = blk
        out[b, a] = blk
    return out


def apply_N_direct(table: np.ndarray, x: np.ndarray) -> np.ndarray:
    """(N x)_i^a = sum_j sum_b N^{ab}(i - j) x_j^b, one output voxel at a time."""
    _, n1, n2, n3 = table.shape
    T = signed_table(table)
    out = np.zeros_like(x, dtype=np.complex128)
    jj = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij"), 0)
    for i1 in range(n1):
        for i2 in range(n2):
            for i3 in range(n3):
                o1 = i1 - jj[0] + n1 - 1
                o2 = i2 - jj[1] + n2 - 1
                o3 = i3 - jj[2] + n3 - 1
                blk = T[:, :, o1, o2, o3]                      # (3,3,n1,n2,n3)
                out[:, i1, i2, i3] = np.einsum("abxyz,bxyz->a", blk, x)
    return out


def matvec_direct(table: np.ndarray, chi: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y = x - chi * (N x) by the direct Toeplitz sum."""
    return x - chi[None] * apply_N_direct(table, x)


def dense_N(table: np.ndarray) -> np.ndarray:
    """Assembled 3N x 3N matrix of N in the (3, n1, n2, n3) flattening."""
    _, n1, n2, n3 = table.shape
    N = n1 * n2 * n3
    T = signed_table(table)
    ii = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij"), 0).reshape(3, -1)
    o = [ii[d][:, None] - ii[d][None, :] + (n1, n2, n3)[d] - 1 for d in range(3)]
    A = np.empty((3 * N, 3 * N), dtype=np.complex128)
    for a in range(3):
        for b in range(3):
            A[a * N:(a + 1) * N, b * N:(b + 1) * N] = T[a, b][o[0], o[1], o[2]]
    return A


def dense_A(table: np.ndarray, chi: np.ndarray) -> np.ndarray:
    """I - M_eps N assembled densely."""
    N = dense_N(table)
    c = np.tile(chi.reshape(-1), 3)
    return np.eye(N.shape[0], dtype=np.complex128) - c[:, None] * N


# ---------------------------------------------------------------------------
# FFT form: circulant embedding of the Toeplitz table (the matvec in O(N log N)).
# ---------------------------------------------------------------------------

def circulant_size(n: Tuple[int, int, int]) -> Tuple[int, int, int]:
    return tuple(2 * nn for nn in n)


def embed(table: np.ndarray, M: Tuple[int, int, int]) -> np.ndarray:
    """Circulant C^{ab}[k], k in [0, M): k_d < n_d holds offset k_d, k_d > M_d - n_d holds
    offset k_d - M_d, every other slot is zero.  Shape (6, M1, M2, M3)."""
    _, n1, n2, n3 = table.shape
    n = (n1, n2, n3)
    if any(M[d] < 2 * n[d] - 1 for d in range(3)):
        raise ValueError("circulant too small for the Toeplitz offsets")
    out = np.zeros((6,) + tuple(M), dtype=np.complex128)
    sel, src, sgn = [], [], []
    for d in range(3):
        k = np.arange(M[d])
        off = np.where(k < n[d], k, k - M[d])
        ok = (k < n[d]) | (k > M[d] - n[d])
        sel.append(k[ok])
        src.append(np.abs(off[ok]))
        sgn.append(off[ok] < 0)
    for ci, (a, b) in enumerate(COMPONENTS):
        blk = table[ci][np.ix_(src[0], src[1], src[2])].copy()
        for d in range(3):
            if parity(a, b, d) < 0:
                shape = [1, 1, 1]
                shape[d] = -1
                blk *= np.where(sgn[d], -1.0, 1.0).reshape(shape)
        out[ci][np.ix_(sel[0], sel[1], sel[2])] = blk
    return out


def spectrum(table: np.ndarray, M: Tuple[int, int, int] | None = None) -> np.ndarray:
    """G_hat^{ab} = DFT3(C^{ab}), shape (6, M1, M2, M3), with the oracle's own FFT."""
    if M is None:
        M = circulant_size(table.shape[1:])
    return _fft.fftn(embed(table, M))


def apply_N_fft(spec: np.ndarray, x: np.ndarray) -> np.ndarray:
    """N x via zero padding, forward DFT, 3x3 product, inverse DFT and crop."""
    M = spec.shape[1:]
    n = x.shape[1:]
    xp = np.zeros((3,) + tuple(M), dtype=np.complex128)
    xp[:, :n[0], :n[1], :n[2]] = x
    X = _fft.fftn(xp)
    G = {}
    for ci, (a, b) in enumerate(COMPONENTS):
        G[(a, b)] = G[(b, a)] = spec[ci]
    U = np.empty_like(X)
    for a in range(3):
        U[a] = G[(a, 0)] * X[0] + G[(a, 1)] * X[1] + G[(a, 2)] * X[2]
    u = _fft.fftn(U, inverse=True)
    return u[:, :n[0], :n[1], :n[2]]


def matvec_fft(spec: np.ndarray, chi: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y = x - chi * (N x) with the FFT form of N."""
    return x - chi[None] * apply_N_fft(spec, x)


class Operator:
    """The oracle's operator A = I - M_eps N for one grid, kappa and contrast."""

    def __init__(self, table: np.ndarray, chi: np.ndarray):
        self.table = table
        self.chi = np.asarray(chi, dtype=np.complex128)
        self.n = table.shape[1:]
        self.spec = spectrum(table)

    def __call__(self, x: np.ndarray) -> np.ndarray:
        return matvec_fft(self.spec, self.chi, x.reshape((3,) + tuple(self.n))).reshape(x.shape)


def kappa_of(h: float, k0: float, eps_b: float) -> float:
    """Background wavenumber times voxel size: k_b h = k0 sqrt(eps_b) h (Section II scaling)."""
    return k0 * math.sqrt(eps_b) * h
