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
