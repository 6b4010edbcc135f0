"""The JM-VIE with electric and magnetic currents (test infrastructure).

Test infrastructure (see the package docstring): never used by the product path.

Section III writes the coupled system ``(I - M T) (J, M) = C M (E_inc, H_inc)``
with ``T = [[N, -c_e K], [c_m K, N]]``, ``K = curl S``, ``N = curl curl S`` and the
diagonal multipliers ``M_eps = (eps_r - 1)/eps_r``, ``M_mu = (mu_r - 1)/mu_r``;
Section III-A discretises it with the same normalised voxel indicators
``P_i = h^{-3/2} 1_{V_i}`` as the J-VIE, which makes K block Toeplitz too.

Galerkin entries of K.  ``(curl (phi e_b))_a = eps_{akb} d_k phi``, so with
``Phi_j = int_{V_j} G`` and the divergence theorem on the testing voxel,
``<K P_j e_b, P_i e_a> = h^{-3} eps_{akb} [int_{face +k of V_i} Phi_j - int_{face -k} Phi_j]``.
Integrating over the difference vector d = r - r' (h = 1) this is
``K^{ab}(m) = eps_{akb} Q_k(m)`` with

    Q_k(m) = int G(d) [1_{[m_k, m_k+1]} - 1_{[m_k-1, m_k]}](d_k) prod_{l != k} (1 - |d_l - m_l|) dd,

a signed unit step along k and the tent weight along the two other axes: the
same lattice boxes as the orthogonal-face term of N.  K^{aa} = 0, K^{ba} = -K^{ab};
Q_k is odd in m_k and even in the other offsets.

Units.  N is dimensionless and K has the unit of length: K = h K^ with K^ the
table above at h = 1.  Writing the magnetic unknowns in impedance units,
``w_m = eta w~_m``, the coupling blocks become ``-j kappa K^`` and ``+j kappa K^``
(kappa = k h, Section II's background scaling gives k = k_b, eta = eta_b) in the
paper's exp(+j omega t); the conjugate system used throughout this package
(exp(-i omega t)) is

    T~ = [[N, i kappa K^], [-i kappa K^, N]],
    y_e = x_e - M_eps (N x_e + i kappa K^ x_m),
    y_m = x_m - M_mu  (-i kappa K^ x_e + N x_m).

The right-hand side is ``h^{3/2} (M_eps e_inc, M_mu eta h_inc)`` (the common factor
c_e dropped as for the J-VIE), with ``eta H = curl E / (i k)`` for exp(-i omega t).

Vectors: complex arrays of shape (6, n1, n2, n3): electric components 0..2,
magnetic components 3..5.
"""
from __future__ import annotations

import math
from typing import Iterable, Tuple

import numpy as np

from . import fft as _fft
from .green import _tent_boxes, box_integrals
from .matvec import apply_N_fft, apply_N_direct, dense_N, spectrum

# order of the 3 unique entries of the antisymmetric tensor K^{ab}
KCOMPONENTS = ((0, 1), (0, 2), (1, 2))


def curl_Q(k: int, m: np.ndarray, kappa: float) -> np.ndarray:
    """Q_k(m) for offsets m (K, 3) at h = 1 (module docstring)."""
    m = np.asarray(m, dtype=np.int64).reshape(-1, 3)
    K = m.shape[0]
    perp = [l for l in range(3) if l != k]
    los, als, bes = [], [], []
    for lk, sk in ((m[:, k], 1.0), (m[:, k] - 1, -1.0)):
        for l0, a0, b0 in _tent_boxes(m[:, perp[0]]):
            for l1, a1, b1 in _tent_boxes(m[:, perp[1]]):
                lo = np.empty((K, 3), np.int64)
                al = np.zeros((K, 3))
                be = np.zeros((K, 3))
                lo[:, k], al[:, k] = lk, sk
                lo[:, perp[0]], al[:, perp[0]], be[:, perp[0]] = l0, a0, b0
                lo[:, perp[1]], al[:, perp[1]], be[:, perp[1]] = l1, a1, b1
                los.append(lo), als.append(al), bes.append(be)
    vals = box_integrals(np.concatenate(los), np.concatenate(als), np.concatenate(bes), kappa)
    return vals.reshape(8, K).sum(axis=0)


def levi_civita(a: int, k: int, b: int) -> int:
    if len({a, k, b}) < 3:
        return 0
    return 1 if (a, k, b) in ((0, 1, 2), (1, 2, 0), (2, 0, 1)) else -1


def galerkin_K(m: np.ndarray, kappa: float) -> np.ndarray:
    """K^{ab}(m) at h = 1 for the components KCOMPONENTS, shape (3, K)."""
    m = np.asarray(m, dtype=np.int64).reshape(-1, 3)
    out = np.empty((3, m.shape[0]), dtype=np.complex128)
    for ci, (a, b) in enumerate(KCOMPONENTS):
        k = 3 - a - b
        out[ci] = levi_civita(a, k, b) * curl_Q(k, m, kappa)
    return out


def curl_parity(a: int, b: int, d: int) -> int:
    """Sign of K^{ab} when the offset along axis d is negated: odd along the third axis."""
    return -1 if d == 3 - a - b else 1


def curl_table(n: Iterable[int], kappa: float) -> np.ndarray:
    """K^{ab}(m) for 0 <= m_d < n_d: shape (3, n1, n2, n3), components KCOMPONENTS."""
    n1, n2, n3 = n
    g = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij"), -1)
    return galerkin_K(g.reshape(-1, 3), kappa).reshape(3, n1, n2, n3)


def signed_curl(ktable: np.ndarray) -> np.ndarray:
    """Full antisymmetric tensor for every signed offset: (3, 3, 2n1-1, 2n2-1, 2n3-1)."""
    _, n1, n2, n3 = ktable.shape
    out = np.zeros((3, 3, 2 * n1 - 1, 2 * n2 - 1, 2 * n3 - 1), dtype=np.complex128)
    idx = [np.abs(np.arange(-nn + 1, nn)) for nn in (n1, n2, n3)]
    neg = [np.arange(-nn + 1, nn) < 0 for nn in (n1, n2, n3)]
    for ci, (a, b) in enumerate(KCOMPONENTS):
        blk = ktable[ci][np.ix_(idx[0], idx[1], idx[2])].copy()
        for d in range(3):
            if curl_parity(a, b, d) < 0:
                shape = [1, 1, 1]
                shape[d] = -1
                blk *= np.where(neg[d], -1.0, 1.0).reshape(shape)
        out[a, b] = blk
        out[b, a] = -blk
    return out


def apply_K_direct(ktable: np.ndarray, x: np.ndarray) -> np.ndarray:
    """(K^ x)_i^a = sum_j sum_b K^{ab}(i - j) x_j^b, one output voxel at a time."""
    _, n1, n2, n3 = ktable.shape
    T = signed_curl(ktable)
    out = np.zeros_like(x, dtype=np.complex128)
    jj = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij"), 0)
    for i1 in range(n1):
        for i2 in range(n2):
            for i3 in range(n3):
                blk = T[:, :, i1 - jj[0] + n1 - 1, i2 - jj[1] + n2 - 1, i3 - jj[2] + n3 - 1]
                out[:, i1, i2, i3] = np.einsum("abxyz,bxyz->a", blk, x)
    return out


def dense_K(ktable: np.ndarray) -> np.ndarray:
    """Assembled 3N x 3N matrix of K^ in the (3, n1, n2, n3) flattening."""
    _, n1, n2, n3 = ktable.shape
    N = n1 * n2 * n3
    T = signed_curl(ktable)
    ii = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij"), 0).reshape(3, -1)
    o = [ii[d][:, None] - ii[d][None, :] + (n1, n2, n3)[d] - 1 for d in range(3)]
    A = np.empty((3 * N, 3 * N), dtype=np.complex128)
    for a in range(3):
        for b in range(3):
            A[a * N:(a + 1) * N, b * N:(b + 1) * N] = T[a, b][o[0], o[1], o[2]]
    return A


def curl_spectrum(ktable: np.ndarray, M: Tuple[int, int, int] | None = None) -> np.ndarray:
    """DFT3 of the circulant embedding of K^{ab} (slots k_d < n_d hold offset k_d,
    k_d > M_d - n_d offset k_d - M_d, the rest zero): shape (3, M1, M2, M3)."""
    _, n1, n2, n3 = ktable.shape
    n = (n1, n2, n3)
    if M is None:
        M = tuple(2 * nn for nn in n)
    emb = np.zeros((3,) + tuple(M), dtype=np.complex128)
    sel, src, sgn = [], [], []
    for d in range(3):
        k = np.arange(M[d])
        off = np.where(k < n[d], k, k - M[d])
        ok = (k < n[d]) | (k > M[d] - n[d])
        sel.append(k[ok])
        src.append(np.abs(off[ok]))
        sgn.append(off[ok] < 0)
    for ci, (a, b) in enumerate(KCOMPONENTS):
        blk = ktable[ci][np.ix_(src[0], src[1], src[2])].copy()
        for d in range(3):
            if curl_parity(a, b, d) < 0:
                shape = [1, 1, 1]
                shape[d] = -1
                blk *= np.where(sgn[d], -1.0, 1.0).reshape(shape)
        emb[ci][np.ix_(sel[0], sel[1], sel[2])] = blk
    return _fft.fftn(emb)


def apply_K_fft(kspec: np.ndarray, x: np.ndarray) -> np.ndarray:
    """K^ x via zero padding, forward DFT, antisymmetric 3x3 product, inverse DFT, crop."""
    M = kspec.shape[1:]
    n = x.shape[1:]
    xp = np.zeros((3,) + tuple(M), dtype=np.complex128)
    xp[:, :n[0], :n[1], :n[2]] = x
    X = _fft.fftn(xp)
    Kab = {}
    for ci, (a, b) in enumerate(KCOMPONENTS):
        Kab[(a, b)] = kspec[ci]
        Kab[(b, a)] = -kspec[ci]
    U = np.zeros_like(X)
    for a in range(3):
        for b in range(3):
            if a != b:
                U[a] += Kab[(a, b)] * X[b]
    u = _fft.fftn(U, inverse=True)
    return u[:, :n[0], :n[1], :n[2]]


def jm_matvec(spec: np.ndarray, kspec: np.ndarray, chi_e: np.ndarray, chi_m: np.ndarray, kappa: float,
              x: np.ndarray) -> np.ndarray:
    """y = (I - M T~) x for x of shape (6, n1, n2, n3) (module docstring)."""
    xe, xm = x[:3], x[3:]
    ye = xe - chi_e[None] * (apply_N_fft(spec, xe) + 1j * kappa * apply_K_fft(kspec, xm))
    ym = xm - chi_m[None] * (-1j * kappa * apply_K_fft(kspec, xe) + apply_N_fft(spec, xm))
    return np.concatenate([ye, ym])


def jm_matvec_direct(table: np.ndarray, ktable: np.ndarray, chi_e: np.ndarray, chi_m: np.ndarray, kappa: float,
                     x: np.ndarray) -> np.ndarray:
    """The same product by direct Toeplitz sums (small grids)."""
    xe, xm = x[:3], x[3:]
    ye = xe - chi_e[None] * (apply_N_direct(table, xe) + 1j * kappa * apply_K_direct(ktable, xm))
    ym = xm - chi_m[None] * (-1j * kappa * apply_K_direct(ktable, xe) + apply_N_direct(table, xm))
    return np.concatenate([ye, ym])


def dense_JM(table: np.ndarray, ktable: np.ndarray, chi_e: np.ndarray, chi_m: np.ndarray,
             kappa: float) -> np.ndarray:
    """I - M T~ assembled densely (6N x 6N)."""
    Nd = dense_N(table)
    Kd = dense_K(ktable)
    T = np.block([[Nd, 1j * kappa * Kd], [-1j * kappa * Kd, Nd]])
    c = np.concatenate([np.tile(chi_e.reshape(-1), 3), np.tile(chi_m.reshape(-1), 3)])
    return np.eye(T.shape[0], dtype=np.complex128) - c[:, None] * T


def magnetic_contrast(mu_r: np.ndarray) -> np.ndarray:
    """M_mu on a voxel: (mu_r - 1)/mu_r (Section III; the background has mu_r = 1)."""
    mu_r = np.asarray(mu_r, dtype=np.complex128)
    return (mu_r - 1.0) / mu_r


class JMOperator:
    """The oracle's JM operator I - M T~ for one grid, kappa and pair of contrasts,
    acting on flat vectors of 6N values."""

    def __init__(self, table: np.ndarray, ktable: np.ndarray, chi_e: np.ndarray, chi_m: np.ndarray,
                 kappa: float):
        self.n = table.shape[1:]
        self.spec = spectrum(table)
        self.kspec = curl_spectrum(ktable)
        self.chi_e = np.asarray(chi_e, dtype=np.complex128)
        self.chi_m = np.asarray(chi_m, dtype=np.complex128)
        self.kappa = kappa

    def __call__(self, x: np.ndarray) -> np.ndarray:
        y = jm_matvec(self.spec, self.kspec, self.chi_e, self.chi_m, self.kappa,
                      x.reshape((6,) + tuple(self.n)))
        return y.reshape(x.shape)
