"""Seeded synthetic inputs for the voxel J-VIE: geometry, permittivity, incident fields.

This module is shared by the oracle and by the GPU path.  It builds the *inputs*
of the method only -- per-voxel relative permittivity arrays, incident-field
samples at voxel centres and seeded random right-hand sides -- and holds none of
the method's arithmetic (no contrast, no Green's function, no operator).

Conventions (Section II and Section III of the paper):

* Lengths are in micrometres.  The background (cladding) is silica with relative
  permittivity ``eps_b``; the paper rescales to a unit background, which the
  solver does by using the background wavenumber ``k_b = k0*sqrt(eps_b)`` and the
  relative contrast ``eps/eps_b``.
* Voxel (i1, i2, i3) occupies ``[i*h, (i+1)*h)`` per axis, centre ``h*(i+1/2)``.
  The third axis (n3, fastest in memory) is the waveguide axis.
* Time dependence ``exp(-i*omega*t)``: a passive absorber has ``Im eps >= 0``.
  The paper writes ``exp(+j*omega*t)`` and ``eps' - j*eps''``; the two systems are
  complex conjugates of each other, so every real observable is identical.
* Absorber profile (Section IV-A): conductivity ``sigma0 * s(u)``, ``s(u) = u**d``,
  with ``u`` the distance from the absorber's inner interface divided by its
  length ``L``, sampled at voxel centres (material is constant per voxel,
  Section III-A).  Inside the absorber ``eps = eps_core + 1j*sigma_max*u**d``.
* ``sigma_max`` for a prescribed round-trip reflection ``R_rt`` follows the
  round-trip estimate of Section IV-C with the unmatched factor D = 2 and
  eta = 1, written in dimensionless form
  ``sigma_max = -(d+1) ln(R_rt) sqrt(eps_core) / (D * eta * k0 * L)``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence, Tuple

import numpy as np

LAMBDA0 = 1.55                      # free-space wavelength, um (Section II)
K0 = 2.0 * math.pi / LAMBDA0        # free-space wavenumber, 1/um
EPS_B = 2.085                       # silica, 1.444**2 rounded (Section II)
EPS_SI = 12.11                      # silicon at 1.55 um (lambda_Si = 446 nm, Section II-A)


def sigma_max_for(r_rt: float, d: int, length_um: float, eps_core: float = EPS_SI,
                  k0: float = K0, D: float = 2.0, eta: float = 1.0) -> float:
    """Absorber strength giving round-trip reflection ``r_rt`` (Section IV-C, eq. for sigma0).

    The paper's ``p+1`` is the profile degree plus one.  With ``eps''`` equal to
    ``sigma0 s / (omega eps0)`` the dimensionless strength is returned.
    """
    return -(d + 1) * math.log(r_rt) * math.sqrt(eps_core) / (D * eta * k0 * length_um)


@dataclasses.dataclass
class Waveguide:
    """A straight rectangular-core waveguide on a voxel grid, absorbers at both ends."""
    n: Tuple[int, int, int]
    h: float
    core_x: Tuple[int, int]          # voxel index range [lo, hi) along axis 1
    core_y: Tuple[int, int]          # voxel index range [lo, hi) along axis 2
    core_z: Tuple[int, int]          # voxel index range [lo, hi) along axis 3 (incl. absorbers)
    n_abs: int                       # absorber length in voxels at each end of the core
    d: int                           # monomial degree of the profile
    sigma_max: float
    eps_core: float = EPS_SI
    eps_b: float = EPS_B
    k0: float = K0
    # optional sidewall roughness: per-z integer offsets of the two x-sidewalls
    rough_lo: Optional[np.ndarray] = None
    rough_hi: Optional[np.ndarray] = None
    # which ends of the core carry an absorber: "both", or "right" (high-z end
    # only, as for the directional source of Section V-A)
    ends: str = "both"
    # magnetic conductivity alongside the electric one, impedance matched
    # (Section IV-B: mu'' = eps''/eps' in the absorber); False keeps mu_r = 1
    magnetic: bool = False
    # length (voxels) and strength of the low-z absorber when they differ from the
    # high-z one (None: n_abs and sigma_max); used with ends == "both"
    n_abs_left: Optional[int] = None
    sigma_left: Optional[float] = None

    def __post_init__(self):
        if self.ends not in ("both", "right"):
            raise ValueError("ends must be 'both' or 'right'")

    @property
    def N(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    def _left(self) -> int:
        if self.ends != "both":
            return 0
        return self.n_abs if self.n_abs_left is None else self.n_abs_left

    def absorber_u(self) -> np.ndarray:
        """u in (0,1) per z index (0 outside absorbers); u grows toward the domain end."""
        n3 = self.n[2]
        u = np.zeros(n3)
        z0, z1 = self.core_z
        Ll, L = self._left(), self.n_abs
        for k in range(z0, z0 + Ll):             # left absorber: inner interface at z0+Ll
            u[k] = (z0 + Ll - k - 0.5) / Ll
        for k in range(z1 - L, z1):              # right absorber: inner interface at z1-L
            u[k] = (k - (z1 - L) + 0.5) / L
        return u

    def in_absorber(self) -> np.ndarray:
        n3 = self.n[2]
        m = np.zeros(n3, dtype=bool)
        z0, z1 = self.core_z
        m[z0:z0 + self._left()] = True
        if self.n_abs > 0:
            m[z1 - self.n_abs:z1] = True
        return m

    def absorber_sigma(self) -> np.ndarray:
        """sigma_max per z index (that of the absorber the index lies in, 0 elsewhere)."""
        sig = np.where(self.in_absorber(), self.sigma_max, 0.0)
        if self.sigma_left is not None:
            z0 = self.core_z[0]
            sig[z0:z0 + self._left()] = self.sigma_left
        return sig

    def lossless_range(self) -> Tuple[int, int]:
        """z index range [lo, hi) of the core outside the absorbers."""
        z0, z1 = self.core_z
        return (z0 + self._left(), z1 - self.n_abs)

    def core_mask(self) -> np.ndarray:
        n1, n2, n3 = self.n
        mask = np.zeros(self.n, dtype=bool)
        x0, x1 = self.core_x
        y0, y1 = self.core_y
        z0, z1 = self.core_z
        if self.rough_lo is None:
            mask[x0:x1, y0:y1, z0:z1] = True
        else:
            for k in range(z0, z1):
                lo = min(max(x0 + int(self.rough_lo[k]), 0), n1)
                hi = min(max(x1 + int(self.rough_hi[k]), lo), n1)
                mask[lo:hi, y0:y1, k] = True
        return mask

    def eps(self) -> np.ndarray:
        """Relative permittivity per voxel, complex128 array of shape n (C order)."""
        eps = np.full(self.n, self.eps_b, dtype=np.complex128)
        mask = self.core_mask()
        u = self.absorber_u()
        absz = self.in_absorber()
        prof = np.where(absz, u ** self.d if self.d > 0 else 1.0, 0.0)
        prof = np.where(absz, prof, 0.0)
        core_val = self.eps_core + 1j * self.absorber_sigma() * prof   # per z
        eps[mask] = np.broadcast_to(core_val, self.n)[mask]
        return eps

    def mu(self) -> np.ndarray:
        """Relative permeability per voxel: 1 everywhere, except, when the absorber is
        magnetic, 1 + i eps''/eps' in its core voxels (exp(-i omega t) sign), so that
        mu_r/eps_r stays 1/eps_core and the absorber's impedance matches the core's."""
        mu = np.ones(self.n, dtype=np.complex128)
        if not self.magnetic:
            return mu
        eps = self.eps()
        lossy = self.core_mask() & (eps.imag != 0)
        mu[lossy] = 1.0 + 1j * eps.imag[lossy] / eps.real[lossy]
        return mu

    def core_axis(self) -> Tuple[int, int]:
        """(i1, i2) indices of the voxel column on the core's centre line."""
        return ((self.core_x[0] + self.core_x[1]) // 2, (self.core_y[0] + self.core_y[1]) // 2)


def centred_range(n: int, w: int) -> Tuple[int, int]:
    """Index range of width w centred in [0,n); the lower index gets the smaller margin."""
    lo = (n - w) // 2
    return lo, lo + w


def dipole_field(n: Sequence[int], h: float, r0: Sequence[float], p: Sequence[complex],
                 k: float) -> np.ndarray:
    """Electric field of a point dipole p at r0 in a homogeneous medium, at voxel centres.

    Textbook radiating-dipole field (exp(-i omega t)), constant prefactor dropped:
    ``E = e^{ikr} [ k^2 (p - n(n.p)) / r + (3 n(n.p) - p)(1/r^3 - i k / r^2) ]``.
    Returns shape (3, n1, n2, n3) complex128.  r0 must not coincide with a centre.
    """
    n1, n2, n3 = n
    c = [h * (np.arange(nn) + 0.5) for nn in (n1, n2, n3)]
    X, Y, Z = np.meshgrid(c[0] - r0[0], c[1] - r0[1], c[2] - r0[2], indexing="ij")
    r = np.sqrt(X * X + Y * Y + Z * Z)
    if np.any(r == 0):
        raise ValueError("dipole coincides with a voxel centre")
    nx, ny, nz = X / r, Y / r, Z / r
    p = np.asarray(p, dtype=np.complex128)
    ndp = nx * p[0] + ny * p[1] + nz * p[2]
    ph = np.exp(1j * k * r)
    far = k * k / r
    near = 1.0 / r ** 3 - 1j * k / r ** 2
    out = np.empty((3, n1, n2, n3), dtype=np.complex128)
    for a, na in enumerate((nx, ny, nz)):
        out[a] = ph * (far * (p[a] - na * ndp) + near * (3.0 * na * ndp - p[a]))
    return out


def complex_source_dipole_field(n: Sequence[int], h: float, r0: Sequence[float], p: Sequence[complex],
                                k: float, shift: Sequence[float]) -> np.ndarray:
    """Field of a dipole p at the complex location r0 + i*shift, at voxel centres.

    The dipole field above continued analytically to a complex source point
    (Section II: the source is moved off the real axis so that it radiates a
    beam).  With ``d = r - r0 - i*shift`` the distance is ``R = sqrt(d.d)`` on the
    principal branch (Re R >= 0), ``n = d/R``, and the textbook expression is
    evaluated with these complex values.  For ``exp(-i omega t)`` a shift of +b
    along an axis makes a beam travelling in the +axis direction (the paper's
    -j*b for ``exp(+j omega t)``).  Away from the disc |rho| <= |shift| in the
    plane through r0 normal to the shift (where R is 0 on the rim and changes
    branch inside) the field solves the same Maxwell equations as a real dipole.
    Returns shape (3, n1, n2, n3) complex128.
    """
    n1, n2, n3 = n
    c = [h * (np.arange(nn) + 0.5) for nn in (n1, n2, n3)]
    s = np.asarray(shift, dtype=float)
    X, Y, Z = np.meshgrid(c[0] - r0[0] - 1j * s[0], c[1] - r0[1] - 1j * s[1], c[2] - r0[2] - 1j * s[2],
                          indexing="ij")
    r = np.sqrt(X * X + Y * Y + Z * Z)              # principal branch, Re >= 0
    if np.any(np.abs(r) < 1e-12 * h):
        raise ValueError("a voxel centre lies on the complex source's branch rim")
    nx, ny, nz = X / r, Y / r, Z / r
    p = np.asarray(p, dtype=np.complex128)
    ndp = nx * p[0] + ny * p[1] + nz * p[2]
    ph = np.exp(1j * k * r)
    far = k * k / r
    near = 1.0 / r ** 3 - 1j * k / r ** 2
    out = np.empty((3, n1, n2, n3), dtype=np.complex128)
    for a, na in enumerate((nx, ny, nz)):
        out[a] = ph * (far * (p[a] - na * ndp) + near * (3.0 * na * ndp - p[a]))
    return out


def complex_source_dipole_hfield(n: Sequence[int], h: float, r0: Sequence[float], p: Sequence[complex],
                                 k: float, shift: Sequence[float]) -> np.ndarray:
    """eta H of the same complex-source dipole, in the units of complex_source_dipole_field:
    ``eta H = k^2 (n x p) e^{ikR}/R (1 - 1/(ikR))`` (the textbook magnetic field of a
    radiating dipole, continued to the complex source point; ``curl E = i k eta H`` for
    exp(-i omega t)).  Returns shape (3, n1, n2, n3) complex128."""
    n1, n2, n3 = n
    c = [h * (np.arange(nn) + 0.5) for nn in (n1, n2, n3)]
    s = np.asarray(shift, dtype=float)
    X, Y, Z = np.meshgrid(c[0] - r0[0] - 1j * s[0], c[1] - r0[1] - 1j * s[1], c[2] - r0[2] - 1j * s[2],
                          indexing="ij")
    r = np.sqrt(X * X + Y * Y + Z * Z)              # principal branch, Re >= 0
    if np.any(np.abs(r) < 1e-12 * h):
        raise ValueError("a voxel centre lies on the complex source's branch rim")
    nv = (X / r, Y / r, Z / r)
    p = np.asarray(p, dtype=np.complex128)
    amp = k * k * np.exp(1j * k * r) / r * (1.0 - 1.0 / (1j * k * r))
    cross = (nv[1] * p[2] - nv[2] * p[1], nv[2] * p[0] - nv[0] * p[2], nv[0] * p[1] - nv[1] * p[0])
    return np.stack([amp * cc for cc in cross])


def gaussian_rhs(n: Sequence[int], seed: int = 0) -> np.ndarray:
    """Seeded complex Gaussian vector of shape (3, n1, n2, n3)."""
    z = np.random.default_rng(seed).standard_normal((3, n[0], n[1], n[2], 2))
    return np.ascontiguousarray(z[..., 0] + 1j * z[..., 1])


def gaussian_process_offsets(n3: int, sigma: float, corr: float, seed: int) -> np.ndarray:
    """Stationary Gaussian sequence with covariance sigma^2 exp(-dz^2/corr^2), rounded.

    Drawn by a Cholesky factor of the covariance matrix (jitter 1e-10) from a
    seeded standard normal vector, then rounded to integer voxel offsets.
    """
    z = np.arange(n3)
    C = sigma ** 2 * np.exp(-((z[:, None] - z[None, :]) ** 2) / corr ** 2)
    Lc = np.linalg.cholesky(C + 1e-10 * np.eye(n3))
    g = Lc @ np.random.default_rng(seed).standard_normal(n3)
    return np.rint(g).astype(np.int64)


# ---------------------------------------------------------------------------
# Workload recipes.  Every geometry is parametric and synthetic.
# ---------------------------------------------------------------------------

def strip_small(d: int = 2, sigma_max: float = 2.0) -> Waveguide:
    """8x8x32 voxels, h = 50 nm, 4x4-voxel core along z, 8-voxel absorbers at each end."""
    n = (8, 8, 32)
    return Waveguide(n=n, h=0.05, core_x=(2, 6), core_y=(2, 6), core_z=(0, 32), n_abs=8,
                     d=d, sigma_max=sigma_max)


def strip_small_dipole_rhs_field(wg: Waveguide) -> np.ndarray:
    """z-dipole on the core centre line at the plane where the lossless core starts."""
    r0 = (wg.h * 4, wg.h * 4, wg.h * wg.n_abs)
    kb = wg.k0 * math.sqrt(wg.eps_b)
    return dipole_field(wg.n, wg.h, r0, (0, 0, 1), kb)


def strip_long(d: int = 2, n3: int = 512, n_abs: int = 80, r_rt: float = 1e-10,
               sigma_max: Optional[float] = None) -> Waveguide:
    """32x32xn3 voxels, h = 25 nm, 20x9-voxel core (500x225 nm), absorbers of n_abs voxels."""
    n = (32, 32, n3)
    h = 0.025
    if sigma_max is None:
        sigma_max = sigma_max_for(r_rt, d, n_abs * h)
    return Waveguide(n=n, h=h, core_x=centred_range(32, 20), core_y=centred_range(32, 9),
                     core_z=(0, n3), n_abs=n_abs, d=d, sigma_max=sigma_max)


def transverse_dipole_field(wg: Waveguide, offset_um: Optional[float] = None) -> np.ndarray:
    """x-polarised dipole on the core centre line, a quarter silicon wavelength after
    the left absorber, snapped to a voxel face (Section II)."""
    lam_si = LAMBDA0 / math.sqrt(wg.eps_core)
    if offset_um is None:
        offset_um = lam_si / 4.0
    z_face = wg.core_z[0] + wg.n_abs + int(round(offset_um / wg.h))
    cx = 0.5 * (wg.core_x[0] + wg.core_x[1])
    cy = 0.5 * (wg.core_y[0] + wg.core_y[1])
    # centre line; if it falls on a voxel centre shift to the nearest face
    rx = cx * wg.h if (cx % 1) == 0 else math.floor(cx) * wg.h
    ry = cy * wg.h if (cy % 1) == 0 else math.floor(cy) * wg.h
    r0 = (rx, ry, z_face * wg.h)
    kb = wg.k0 * math.sqrt(wg.eps_b)
    return dipole_field(wg.n, wg.h, r0, (1, 0, 0), kb)


def strip_family(length_um: float, d: int, r_rt: float = 1e-10, core_len: int = 152,
                 h: float = 0.025) -> Waveguide:
    """Absorber-length family: lossless core of core_len voxels, absorbers of L at both ends,
    n3 rounded up to a multiple of 64 with background voxels split between the ends."""
    n_abs = int(round(length_um / h))
    used = core_len + 2 * n_abs
    n3 = ((used + 63) // 64) * 64
    z0 = (n3 - used) // 2
    sig = sigma_max_for(r_rt, d, n_abs * h)
    return Waveguide(n=(32, 32, n3), h=h, core_x=centred_range(32, 20),
                     core_y=centred_range(32, 9), core_z=(z0, z0 + used), n_abs=n_abs, d=d,
                     sigma_max=sig)


def rough_strip(seed: int, n3: int = 256, n_abs: int = 40, d: int = 2,
                sigma_vox: float = 1.0, corr_vox: float = 8.0) -> Waveguide:
    """32x32xn3 strip with seeded Gaussian-correlated x-sidewall roughness over the lossless part."""
    wg = strip_long(d=d, n3=n3, n_abs=n_abs, r_rt=1e-10)
    lo = gaussian_process_offsets(n3, sigma_vox, corr_vox, 2 * seed)
    hi = gaussian_process_offsets(n3, sigma_vox, corr_vox, 2 * seed + 1)
    absz = wg.in_absorber()
    lo[absz] = 0
    hi[absz] = 0
    wg.rough_lo, wg.rough_hi = lo, hi
    return wg


H_PAPER = 0.05 / 3.0                 # 50/3 nm voxels (Section II-A)
STRIP_LEN = 810                      # 13.5 um lossless strip in voxels (Section II-A)


def strip_paper(length_um: float, d: int, r_rt: float = 1e-10, magnetic: bool = False) -> Waveguide:
    """The strip of Section II-A: a 500 x 200 nm silicon core 13.5 um long in silica,
    voxels of 50/3 nm (30 x 12 across, 810 along), with one absorber of length
    length_um appended at the far end (Section V-A).  The grid is the core itself.
    With magnetic=True the absorber is impedance matched and its strength takes the
    factor D = 4 of the round-trip estimate (Section IV-C) instead of 2."""
    n_abs = int(round(length_um / H_PAPER))
    n3 = STRIP_LEN + n_abs
    sig = sigma_max_for(r_rt, d, n_abs * H_PAPER, D=4.0 if magnetic else 2.0)
    return Waveguide(n=(30, 12, n3), h=H_PAPER, core_x=(0, 30), core_y=(0, 12), core_z=(0, n3), n_abs=n_abs,
                     d=d, sigma_max=sig, ends="right", magnetic=magnetic)


def strip_paper_source_h(wg: Waveguide) -> np.ndarray:
    """eta H of strip_paper_source (the magnetic right-hand side of the JM-VIE)."""
    lam_si = LAMBDA0 / math.sqrt(wg.eps_core)
    r0 = (0.5 * wg.n[0] * wg.h, 0.5 * wg.n[1] * wg.h, wg.core_z[0] * wg.h + lam_si / 4.0)
    kb = wg.k0 * math.sqrt(wg.eps_b)
    return complex_source_dipole_hfield(wg.n, wg.h, r0, (1, 0, 0), kb, (0.0, 0.0, lam_si))


def strip_paper_source(wg: Waveguide) -> np.ndarray:
    """Incident field of Section II: a dipole across the strip's width (the dominant TE
    mode's polarisation) on the centre line, a quarter silicon wavelength from the
    near end, at the complex location shifted by one silicon wavelength along the
    guide (a beam travelling away from the near end)."""
    lam_si = LAMBDA0 / math.sqrt(wg.eps_core)
    r0 = (0.5 * wg.n[0] * wg.h, 0.5 * wg.n[1] * wg.h, wg.core_z[0] * wg.h + lam_si / 4.0)
    kb = wg.k0 * math.sqrt(wg.eps_b)
    return complex_source_dipole_field(wg.n, wg.h, r0, (1, 0, 0), kb, (0.0, 0.0, lam_si))


# ---- Bragg grating (Section II-B, transmission study of Section V) ----------------
BRAGG_H = 0.02                       # 20 nm voxels: the 500 x 220 nm section exactly
BRAGG_PERIOD = 16                    # 320 nm period in voxels, half wide, half narrow
BRAGG_TAIL = 20                      # uniform voxels between the grating and the far absorber


def bragg_grating(lambda0_um: float = LAMBDA0, periods: int = 100, lead_periods: int = 10, d: int = 2,
                  r_rt: float = 1e-10, absorber_um: float = 2.2) -> Waveguide:
    """The Bragg grating of Section II-B on 20 nm voxels: a 500 x 220 nm silicon strip
    whose width steps between W + dW and W - dW (dW = 40 nm, one voxel per sidewall)
    every half period (period 320 nm, wide half first) over `periods` periods, after
    a uniform lead-in of `lead_periods` periods and followed by BRAGG_TAIL uniform
    voxels; quadratic (degree d) absorbers of absorber_um on both ends, strength
    from r_rt at this wavelength (Section IV-C).  The grid is the wide section's
    bounding box, 27 x 11 voxels across; the permittivities do not depend on the
    wavelength (silicon's dispersion is not given)."""
    h = BRAGG_H
    n_abs = int(round(absorber_um / h))
    n3 = 2 * n_abs + (lead_periods + periods) * BRAGG_PERIOD + BRAGG_TAIL
    k0 = 2.0 * math.pi / lambda0_um
    lo = np.zeros(n3, dtype=np.int64)
    hi = np.zeros(n3, dtype=np.int64)
    g0 = n_abs + lead_periods * BRAGG_PERIOD
    half = BRAGG_PERIOD // 2
    for p in range(periods):
        a = g0 + p * BRAGG_PERIOD
        lo[a:a + half], hi[a:a + half] = -1, 1                        # wide: 27 voxels
        lo[a + half:a + 2 * half], hi[a + half:a + 2 * half] = 1, -1  # narrow: 23 voxels
    sig = sigma_max_for(r_rt, d, n_abs * h, k0=k0)
    return Waveguide(n=(27, 11, n3), h=h, core_x=(1, 26), core_y=(0, 11), core_z=(0, n3), n_abs=n_abs, d=d,
                     sigma_max=sig, k0=k0, rough_lo=lo, rough_hi=hi, ends="both")


def bragg_grating_range(wg: Waveguide) -> Tuple[int, int]:
    """z index range [lo, hi) of the corrugated part."""
    nz = np.nonzero(wg.rough_lo)[0]
    return int(nz[0]), int(nz[-1]) + 1


def bragg_slice(wg: Waveguide) -> int:
    """z index of the transmission slice: the middle of the uniform tail between the
    grating's end and the far absorber."""
    return wg.lossless_range()[1] - BRAGG_TAIL // 2


def bragg_source(wg: Waveguide) -> np.ndarray:
    """The strip's complex-source dipole (strip_paper_source) placed a quarter silicon
    wavelength after the near absorber's inner interface, at the grid's wavelength."""
    lam0 = 2.0 * math.pi / wg.k0
    lam_si = lam0 / math.sqrt(wg.eps_core)
    z0 = wg.lossless_range()[0] * wg.h + lam_si / 4.0
    r0 = (0.5 * wg.n[0] * wg.h, 0.5 * wg.n[1] * wg.h, z0)
    kb = wg.k0 * math.sqrt(wg.eps_b)
    return complex_source_dipole_field(wg.n, wg.h, r0, (1, 0, 0), kb, (0.0, 0.0, lam_si))


def bragg_slow_light(lambda0_um: float, absorber_periods: int, lossless_periods: int = 20, lead_periods: int = 10,
                     d: int = 2, r_rt: float = 1e-10, corrugated: bool = True,
                     left_absorber_um: float = 2.2) -> Waveguide:
    """The "infinite" Bragg grating of Section V: after a uniform lead-in of
    `lead_periods` periods (behind a uniform absorber of left_absorber_um) the grating
    of Section II-B runs for `lossless_periods` periods and then continues, with the
    same corrugation, through an absorber of `absorber_periods` periods (degree d,
    strength from r_rt for its own length).  corrugated=False gives the uniform
    500 x 220 nm strip with the same lengths, the reference case of Section V-A."""
    h = BRAGG_H
    n_left = int(round(left_absorber_um / h))
    n_abs = absorber_periods * BRAGG_PERIOD
    g0 = n_left + lead_periods * BRAGG_PERIOD
    n3 = g0 + lossless_periods * BRAGG_PERIOD + n_abs
    k0 = 2.0 * math.pi / lambda0_um
    lo = np.zeros(n3, dtype=np.int64)
    hi = np.zeros(n3, dtype=np.int64)
    if corrugated:
        half = BRAGG_PERIOD // 2
        for a in range(g0, n3, BRAGG_PERIOD):
            lo[a:a + half], hi[a:a + half] = -1, 1
            lo[a + half:a + 2 * half], hi[a + half:a + 2 * half] = 1, -1
    return Waveguide(n=(27, 11, n3), h=h, core_x=(1, 26), core_y=(0, 11), core_z=(0, n3), n_abs=n_abs, d=d,
                     sigma_max=sigma_max_for(r_rt, d, n_abs * h, k0=k0), k0=k0, rough_lo=lo, rough_hi=hi,
                     ends="both", n_abs_left=n_left, sigma_left=sigma_max_for(r_rt, d, n_left * h, k0=k0))

