"""Pins of the inputs of the strip reflection study (Sections II and V-A): the
complex-source dipole that launches a beam, the single-ended absorber and the
strip recipe.  These are inputs, not the method; they are checked against the
Maxwell equations, the closed-form directivity of a complex source point and
the geometry the paper states."""
import math

import numpy as np
import pytest

from paper_1803_06237_amd import inputs


def test_zero_shift_is_the_real_dipole():
    n, h = (4, 3, 5), 0.05
    r0, p, k = (0.1, 0.05, 0.125), (0.3, -1.0, 0.5j), 7.0
    a = inputs.complex_source_dipole_field(n, h, r0, p, k, (0.0, 0.0, 0.0))
    b = inputs.dipole_field(n, h, r0, p, k)
    assert np.allclose(a, b, rtol=1e-14, atol=0)


@pytest.mark.parametrize("p", [(1.0, 0.0, 0.0), (0.2, 0.7j, -0.4)])
def test_complex_source_field_solves_maxwell(p):
    """Ahead of the source (away from the branch disc) the field is divergence free and
    satisfies the vector Helmholtz equation lap E + k^2 E = 0 (second-order differences
    on a fine grid, relative error O((kh)^2))."""
    k, b, h = 10.0, 0.3, 0.002
    n = (9, 9, 9)
    r0 = (4.5 * h + 0.01, 4.5 * h - 0.02, -0.45)
    E = inputs.complex_source_dipole_field(n, h, r0, p, k, (0.0, 0.0, b))
    c = (slice(1, -1),) * 3

    def d(f, ax):
        sl_p = [slice(1, -1)] * 3
        sl_m = [slice(1, -1)] * 3
        sl_p[ax] = slice(2, None)
        sl_m[ax] = slice(None, -2)
        return (f[tuple(sl_p)] - f[tuple(sl_m)]) / (2 * h)

    def lap(f):
        out = -6.0 * f[c]
        for ax in range(3):
            sl_p = [slice(1, -1)] * 3
            sl_m = [slice(1, -1)] * 3
            sl_p[ax] = slice(2, None)
            sl_m[ax] = slice(None, -2)
            out = out + f[tuple(sl_p)] + f[tuple(sl_m)]
        return out / h ** 2

    scale = k * k * np.max(np.abs(E))
    div = sum(d(E[a], a) for a in range(3))
    assert np.max(np.abs(div)) < 1e-3 * k * np.max(np.abs(E))   # |div E| << k |E|
    for a in range(3):
        res = lap(E[a]) + k * k * E[a][c]
        assert np.max(np.abs(res)) < 1e-2 * scale


def test_complex_source_beams_forward_with_the_closed_form_directivity():
    """On the axis of a complex source point r0 + i b z, the forward and backward fields
    at the same distance differ by exp(2 k b) up to O(1/(kR)) near-field terms."""
    k, b = 10.0, 0.25
    h = 0.05
    far = 40 * b
    # one-voxel grids whose centre sits on the axis at +far and at -far from the source
    fwd = inputs.complex_source_dipole_field((1, 1, 1), h, (0.5 * h, 0.5 * h, 0.5 * h - far), (1, 0, 0), k,
                                             (0, 0, b))[0, 0, 0, 0]
    bwd = inputs.complex_source_dipole_field((1, 1, 1), h, (0.5 * h, 0.5 * h, 0.5 * h + far), (1, 0, 0), k,
                                             (0, 0, b))[0, 0, 0, 0]
    ratio = abs(fwd) / abs(bwd)
    assert abs(ratio / math.exp(2 * k * b) - 1) < 3.0 / (k * far)


def test_single_ended_absorber_profile():
    wg = inputs.Waveguide(n=(2, 2, 20), h=0.05, core_x=(0, 2), core_y=(0, 2), core_z=(0, 20), n_abs=5, d=2,
                          sigma_max=3.0, ends="right")
    u = wg.absorber_u()
    assert np.all(u[:15] == 0)
    assert np.allclose(u[15:], (np.arange(5) + 0.5) / 5)
    assert wg.lossless_range() == (0, 15)
    eps = wg.eps()
    assert np.allclose(eps[1, 1, 15:], inputs.EPS_SI + 3.0j * u[15:] ** 2)
    assert np.all(eps[:, :, :15] == inputs.EPS_SI)
    both = inputs.Waveguide(n=(2, 2, 20), h=0.05, core_x=(0, 2), core_y=(0, 2), core_z=(0, 20), n_abs=5, d=2,
                            sigma_max=3.0)
    assert both.lossless_range() == (5, 15) and both.absorber_u()[0] > 0
    with pytest.raises(ValueError):
        inputs.Waveguide(n=(2, 2, 20), h=0.05, core_x=(0, 2), core_y=(0, 2), core_z=(0, 20), n_abs=5, d=2,
                         sigma_max=3.0, ends="left")


def test_paper_strip_recipe():
    """500 x 200 nm core, 13.5 um long, 50/3 nm voxels (Section II-A), one absorber of L
    at the far end with the strength of the round-trip estimate (Section IV-C)."""
    for L in (0.45, 4.5, 9.45):
        wg = inputs.strip_paper(L, 2, 1e-25)
        assert wg.n == (30, 12, 810 + round(L * 60))
        assert abs(30 * wg.h - 0.5) < 1e-12 and abs(12 * wg.h - 0.2) < 1e-12 and abs(810 * wg.h - 13.5) < 1e-9
        assert wg.lossless_range() == (0, 810)
        assert wg.sigma_max == pytest.approx(inputs.sigma_max_for(1e-25, 2, round(L * 60) * wg.h))
        assert np.all(wg.eps()[:, :, :810] == inputs.EPS_SI)
    wg = inputs.strip_paper(0.45, 1, 1e-10)
    e = inputs.strip_paper_source(wg)
    axis = np.abs(e[0, 15, 6])
    lam = inputs.LAMBDA0 / math.sqrt(inputs.EPS_SI)
    k_src = int(lam / 4 / wg.h)                       # last voxel before the source plane
    # the beam goes toward the absorber: far more field ahead of the source than behind
    assert axis[k_src + 1] > 50 * axis[k_src]
    assert np.argmax(axis) == k_src + 1


def test_length_for_reflection_interpolates_in_log_log():
    from paper_1803_06237_amd import experiments as ex
    # R = L^-4 crosses 1e-8 at L = 100 exactly: bracketed, and extrapolated
    L = [10.0, 50.0, 200.0]
    R = [x ** -4 for x in L]
    assert ex.length_for_reflection(L, R) == pytest.approx(100.0, rel=1e-12)
    assert ex.length_for_reflection(L[:2], R[:2]) == pytest.approx(100.0, rel=1e-12)
    assert ex.length_for_reflection([1.0, 2.0], [1e-3, 1e-2]) is None
    assert ex.length_for_reflection([1.0, 2.0], [1e-9, 1e-10]) == 1.0


def test_strip_axis_field_is_the_mean_of_the_four_centre_columns():
    from paper_1803_06237_amd import experiments as ex
    wg = inputs.strip_paper(0.45, 2)
    w = np.zeros((3,) + wg.n, dtype=np.complex128)
    for k, (a, b) in enumerate([(14, 5), (14, 6), (15, 5), (15, 6)]):
        w[:, a, b, :] = k + 1
    E = ex.strip_axis_field(wg, w)
    assert E.shape == (3, 810)
    want = 2.5 / (wg.h ** 1.5 * (inputs.EPS_SI / inputs.EPS_B - 1.0))
    assert np.allclose(E, want, rtol=1e-14)


def test_reflection_analysis_on_exact_power_laws():
    """R = c L^-2(d+1): the fitted slope is exact, the window drops the points near the
    reference and under the floor, and the R = 1e-8 length is interpolated or extrapolated."""
    from paper_1803_06237_amd import experiments as ex
    lam = ex.LAMBDA_SI
    L = [0.45 * k for k in range(1, 21)]
    for d, c in ((0, 1e-2), (2, 3e-5)):
        R = [c * x ** (-2 * (d + 1)) for x in L]
        a = ex.analyse_reflection(L, R, d, 1e-25, 9.45)
        assert a["slope"] == pytest.approx(-2 * (d + 1), rel=1e-10)
        exact = (c / 1e-8) ** (1 / (2 * (d + 1))) / lam
        assert a["length_lambda"] == pytest.approx(exact, rel=1e-9)
        assert a["method"] == ("extrapolated" if exact * lam > 9.45 / 2 else "interpolated")
        if a["method"] == "extrapolated":
            assert a["length_lambda_predicted_slope"] == pytest.approx(exact, rel=1e-9)
    # points beyond half the reference length are not used: a fake drop there changes nothing
    R = [1e-2 * x ** -2 for x in L]
    R2 = list(R)
    R2[-1] = 1e-12
    assert ex.analyse_reflection(L, R2, 0, 1e-25, 9.45) == ex.analyse_reflection(L, R, 0, 1e-25, 9.45)


@pytest.mark.parametrize("shift", [0.0, 0.3])
def test_magnetic_field_is_the_curl_of_the_electric_field(shift):
    """curl E = i k eta H (exp(-i omega t)) by central differences ahead of the source."""
    k, h = 10.0, 0.002
    n = (9, 9, 9)
    r0 = (4.5 * h + 0.01, 4.5 * h - 0.02, -0.45)
    p = (0.2, 0.7j, -0.4)
    E = inputs.complex_source_dipole_field(n, h, r0, p, k, (0.0, 0.0, shift))
    H = inputs.complex_source_dipole_hfield(n, h, r0, p, k, (0.0, 0.0, shift))

    def d(f, ax):
        sp = [slice(1, -1)] * 3
        sm = [slice(1, -1)] * 3
        sp[ax] = slice(2, None)
        sm[ax] = slice(None, -2)
        return (f[tuple(sp)] - f[tuple(sm)]) / (2 * h)

    curl = [d(E[2], 1) - d(E[1], 2), d(E[0], 2) - d(E[2], 0), d(E[1], 0) - d(E[0], 1)]
    c = (slice(1, -1),) * 3
    scale = k * np.max(np.abs(H))
    for a in range(3):
        assert np.max(np.abs(curl[a] - 1j * k * H[a][c])) < 1e-3 * scale


def test_matched_absorber_permeability():
    """mu'' = eps''/eps' in the absorber (Section IV-B) and D = 4 in the strength."""
    wg = inputs.strip_paper(0.9, 2, 1e-25, magnetic=True)
    eps, mu = wg.eps(), wg.mu()
    assert np.all(mu[:, :, :810] == 1)
    assert np.allclose(mu[:, :, 810:], 1 + 1j * eps[:, :, 810:].imag / inputs.EPS_SI, rtol=1e-15, atol=0)
    assert np.allclose(mu[:, :, 810:] / eps[:, :, 810:], 1 / inputs.EPS_SI, rtol=1e-14, atol=0)
    e_only = inputs.strip_paper(0.9, 2, 1e-25)
    assert wg.sigma_max == pytest.approx(0.5 * e_only.sigma_max, rel=1e-14)
    assert np.all(e_only.mu() == 1)
