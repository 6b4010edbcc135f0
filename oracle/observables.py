"""Observables computed from the solved currents (test infrastructure only)."""
from __future__ import annotations

import numpy as np


def field_from_current(w: np.ndarray, eps: np.ndarray, eps_b: float, h: float) -> np.ndarray:
    """E in each voxel from its current weight: J = c_e (eps_r - 1) E (Section III) with
    J = w h^{-3/2} on the voxel; c_e dropped.  Background voxels (eps_r = 1) carry no
    current and get NaN."""
    eps_r = np.asarray(eps, dtype=np.complex128) / eps_b
    with np.errstate(divide="ignore", invalid="ignore"):
        return w / ((h ** 1.5) * (eps_r - 1.0))[None]


def reflection(E_ref: np.ndarray, E_L: np.ndarray) -> float:
    """R = ||E_ref - E_L||^2 / ||E_ref||^2 over a sampled line (Section V-A); uniform
    samples, so the L2 integrals reduce to sums."""
    d = np.asarray(E_ref) - np.asarray(E_L)
    return float(np.sum(np.abs(d) ** 2) / np.sum(np.abs(E_ref) ** 2))


def total_field(w: np.ndarray, Nw: np.ndarray, e_inc: np.ndarray, eps: np.ndarray, eps_b: float,
                h: float) -> np.ndarray:
    """E on every voxel, background included, from the currents w and N w.

    The volume integral equation E = E_inc + (k^2 + grad div) S[(eps_r - 1) E] with
    N = curl curl S = (k^2 + grad div) S + I gives eps_r E = E_inc + N J for
    J = (eps_r - 1) E (Section III).  In the normalised voxel basis (Section III-A,
    P_i = h^{-3/2} on V_i, e_inc sampled at the centre) the coefficient of eps_r E
    is h^{3/2} e_inc + N w, hence E = (h^{3/2} e_inc + N w) / (h^{3/2} eps_r)."""
    eps_r = np.asarray(eps, dtype=np.complex128) / eps_b
    return ((h ** 1.5) * e_inc + Nw) / ((h ** 1.5) * eps_r)[None]


def slice_transmission(E_slice: np.ndarray, h: float) -> float:
    """T = integral of |E|^2 over a voxel-wide cross-section (Section V, Bragg grating):
    the sum over the slice's voxels of |E|^2 h^2."""
    return float(np.sum(np.abs(E_slice) ** 2) * h * h)
