"""The Bragg grating of Section II-B (geometry, source, band-gap read-out) and the
oracle's total-field observable, pinned against the quasi-static dipole field."""
import math

import numpy as np
import pytest

from oracle import green, matvec as mv, observables
from paper_1803_06237_amd import experiments, inputs


def test_grating_geometry_follows_section_ii_b():
    wg = inputs.bragg_grating()
    assert wg.h == 0.02 and wg.n == (27, 11, 2000) and wg.n[2] <= 2048
    assert wg.n_abs == 110 and wg.ends == "both" and wg.d == 2            # 2.2 um quadratic absorbers
    g0, g1 = inputs.bragg_grating_range(wg)
    assert (g0, g1) == (110 + 10 * 16, 110 + 110 * 16)                    # 10-period lead-in, 100 periods
    assert wg.lossless_range() == (110, 1890)
    z = inputs.bragg_slice(wg)
    assert g1 <= z < wg.lossless_range()[1]                              # after the grating, before the absorber
    m = wg.core_mask()
    assert m[:, :, :].any(axis=(0, 1)).all()                              # the core runs the whole length
    widths = m[:, 5, :].sum(axis=0)
    assert (m.sum(axis=1) == 11 * m[:, 0, :]).all()                      # 220 nm: all 11 voxels in y
    assert (widths[:g0] == 25).all() and (widths[g1:] == 25).all()       # W = 500 nm
    per = widths[g0:g1].reshape(100, 16)
    assert (per[:, :8] == 27).all() and (per[:, 8:] == 23).all()          # W +- dW, dW = 40 nm, 320 nm period
    # the sidewalls move symmetrically: the corrugated core stays centred
    cols = np.nonzero(m[:, 5, g0])[0], np.nonzero(m[:, 5, g0 + 8])[0]
    assert (cols[0][0], cols[0][-1]) == (0, 26) and (cols[1][0], cols[1][-1]) == (2, 24)


def test_grating_materials_and_absorbers():
    for lam in (1.52, 1.57):
        wg = inputs.bragg_grating(lam)
        assert abs(wg.k0 - 2 * math.pi / lam) < 1e-15
        assert abs(wg.sigma_max - inputs.sigma_max_for(1e-10, 2, 2.2, k0=wg.k0)) < 1e-12
        eps = wg.eps()
        lo, hi = wg.lossless_range()
        core = wg.core_mask()
        assert np.all(eps[core][..., None].imag >= 0)
        assert np.all(eps[:, :, lo:hi][core[:, :, lo:hi]] == inputs.EPS_SI)
        assert np.all(eps[~core] == inputs.EPS_B)
        assert eps[13, 5, 0].imag > eps[13, 5, 100].imag > 0                # grows toward both ends
        assert eps[13, 5, 1999].imag > eps[13, 5, 1899].imag > 0
    # the permittivities do not depend on the wavelength; the absorber strength does
    a, b = inputs.bragg_grating(1.52).eps(), inputs.bragg_grating(1.57).eps()
    assert np.array_equal(a.real, b.real) and not np.array_equal(a.imag, b.imag)


def test_grating_source_is_the_strips_complex_dipole():
    wg = inputs.bragg_grating(1.55)
    e = inputs.bragg_source(wg)
    assert e.shape == (3,) + wg.n and np.isfinite(e).all()
    lam_si = 1.55 / math.sqrt(inputs.EPS_SI)
    z0 = 110 * 0.02 + lam_si / 4
    r0 = (13.5 * 0.02, 5.5 * 0.02, z0)
    kb = wg.k0 * math.sqrt(inputs.EPS_B)
    want = inputs.complex_source_dipole_field(wg.n, wg.h, r0, (1, 0, 0), kb, (0, 0, lam_si))
    assert np.abs(e - want).max() <= 1e-12 * np.abs(want).max()
    # a beam toward +z: stronger a few wavelengths downstream than upstream
    i = int(round(z0 / wg.h))
    assert np.abs(e[0, 13, 5, i + 40]) > 3 * np.abs(e[0, 13, 5, i - 40])


def test_band_gap_read_out():
    lam = np.arange(1520.0, 1570.5, 1.0)
    T = 1.0 - 0.9 * np.exp(-((lam - 1545.0) / 8.0) ** 2)
    g = experiments.band_gap(lam, T)
    assert g["lambda_min_nm"] == 1545.0 and abs(g["T_min_over_max"] - 0.1 / T.max()) < 1e-12
    # T < max/2 where 0.9 exp(-x^2) > 1 - max/2
    half = 8.0 * math.sqrt(-math.log((1 - T.max() / 2) / 0.9))
    assert abs(g["gap_width_nm"] - 2 * half) <= 2.0 and abs(g["gap_centre_nm"] - 1545.0) <= 0.5
    assert not g["gap_open_at_range_end"]
    flat = experiments.band_gap(lam, np.ones_like(lam))
    assert "gap_width_nm" not in flat


@pytest.mark.parametrize("h", [1.0, 0.05, 0.02])
@pytest.mark.parametrize("comp", [0, 2])
def test_total_field_outside_a_small_voxel_is_its_dipole_field(comp, h):
    """One silicon voxel of edge h in a uniform field, kh -> 0: in the background voxels
    along z the scattered field is the quasi-static dipole field (3 n (n.p) - p)/(4 pi r^3)
    of p = (eps_r - 1) E_in h^3 at r = m h; a uniformly polarised cube has no quadrupole
    moment, so the difference falls as (h/r)^4.  Neither E_in nor the field at r = m h
    may depend on h (scale invariance at fixed kh), which pins the powers of h that the
    normalised basis P_i = h^{-3/2} 1_{V_i} (Section III-A) brings into the right-hand
    side, the field read-out inside the voxel and the total field outside it."""
    eps_b, eps_s, kh = 2.085, 12.11, 1e-3
    n = (1, 1, 7)
    T = green.green_table(n, kh)
    eps = np.full(n, eps_b, complex)
    eps[0, 0, 0] = eps_s
    A = mv.dense_A(T, mv.contrast(eps, eps_b))
    e = np.zeros((3,) + n, complex)
    e[comp] = 1.0
    w = np.linalg.solve(A, mv.rhs_from_field(eps, eps_b, e, h).ravel()).reshape((3,) + n)
    E = observables.total_field(w, mv.apply_N_direct(T, w), e, eps, eps_b, h)
    # inside the dielectric voxel the two read-outs agree (w = M (e_inc + N w))
    E_in = observables.field_from_current(w, eps, eps_b, h)[:, 0, 0, 0]
    assert np.abs(E[:, 0, 0, 0] - E_in).max() < 1e-13
    # Clausius-Mossotti value inside, independent of h
    er = eps_s / eps_b
    assert abs(E_in[comp] - 3.0 / (er + 2.0)) < 5 * kh ** 2
    p = (er - 1.0) * E_in                # times h^3, which cancels against r^3 = (m h)^3
    nv = np.array([0.0, 0.0, 1.0])
    errs = []
    for m in range(2, 7):
        Es = (3 * nv * (nv @ p) - p) / (4 * math.pi * m ** 3)
        err = np.abs((E[:, 0, 0, m] - e[:, 0, 0, m]) - Es).max() / np.abs(Es).max()
        assert err < 0.5 / m ** 4, (m, err)
        errs.append(err)
    assert errs[-1] < errs[1] / 10


def test_total_field_without_scatterer_is_the_incident_field():
    n = (2, 2, 3)
    eps = np.full(n, 2.085, complex)
    rng = np.random.default_rng(0)
    e = rng.standard_normal((3,) + n) + 1j * rng.standard_normal((3,) + n)
    E = observables.total_field(np.zeros_like(e), np.zeros_like(e), e, eps, 2.085, 0.02)
    assert np.abs(E - e).max() < 1e-15
    assert abs(observables.slice_transmission(e[:, :, :, 1], 0.02)
               - 4e-4 * np.sum(np.abs(e[:, :, :, 1]) ** 2)) < 1e-15


def test_slow_light_geometry():
    """The grating continues, in phase, through an absorber of its own shape; the
    lossless part and the left absorber do not depend on the absorber's length."""
    ref = inputs.bragg_slow_light(1.52, 90)
    assert ref.n == (27, 11, 2030) and ref.n[2] <= 2048
    for P in (3, 5, 10, 20, 40, 90):
        wg = inputs.bragg_slow_light(1.52, P)
        assert wg.lossless_range() == (110, 590) and wg.n_abs == 16 * P
        assert abs(wg.sigma_left - inputs.sigma_max_for(1e-10, 2, 2.2, k0=wg.k0)) < 1e-12
        assert abs(wg.sigma_max - inputs.sigma_max_for(1e-10, 2, 0.32 * P, k0=wg.k0)) < 1e-12
        widths = wg.core_mask()[:, 5, :].sum(axis=0)
        assert (widths[:270] == 25).all()
        per = widths[270:].reshape(-1, 16)
        assert (per[:, :8] == 27).all() and (per[:, 8:] == 23).all()    # through the absorber too
        eps = wg.eps()
        assert np.array_equal(eps[:, :, :590], ref.eps()[:, :, :590])   # left absorber and lossless part
        assert (eps[13, 5, 110:590].imag == 0).all() and (eps[13, 5, 590:].imag > 0).all()
        flat = inputs.bragg_slow_light(1.52, P, corrugated=False)
        assert (flat.core_mask()[:, 5, :].sum(axis=0) == 25).all()
        assert np.array_equal(flat.eps()[13, 5], eps[13, 5])            # same absorber profile on the axis
