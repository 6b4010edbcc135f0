"""Pins of the oracle's JM-VIE (Section III: K = curl S and the coupled operator)
against facts outside its own code: the point curl of the Green function far
away, scipy's adaptive quadrature, the symmetry of the curl's Galerkin matrix,
direct Toeplitz sums, and the duality of Maxwell's equations (exchanging the
electric and magnetic roles maps solutions to solutions)."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import green, jm
from oracle import matvec as mv
from oracle import solve

KAPPA = 0.3
RNG = np.random.default_rng(11)


def _cvec(shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


def _point_curl(m, kappa):
    """(curl (G e_b))_a at the point m = (grad G x e_b)_a for the components
    KCOMPONENTS, with grad G = G (i kappa - 1/R) m / R."""
    R = np.linalg.norm(m)
    grad = np.exp(1j * kappa * R) / (4 * math.pi * R) * (1j * kappa - 1.0 / R) * m / R
    return np.array([np.cross(grad, np.eye(3)[b])[a] for a, b in jm.KCOMPONENTS])


def _far_errors(kappa, smoothed):
    errs = []
    for t in (2, 4, 8, 16):
        m = np.array([[t, 2 * t, 3 * t]])
        K = jm.galerkin_K(m, kappa)[:, 0]
        P = _point_curl(m[0].astype(float), kappa)
        if smoothed:
            nhat = m[0] / np.linalg.norm(m[0])
            P = P * np.prod(np.sinc(kappa * nhat / (2 * math.pi)) ** 2)   # numpy sinc(x) = sin(pi x)/(pi x)
        errs.append(np.max(np.abs(K - P)) / np.max(np.abs(P)))
    return errs, [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


def test_static_far_field_is_the_point_curl_with_fourth_order_error():
    """At kappa = 0, K^{ab}(m) is eps_{akb} d_k (1/(4 pi R)) averaged over the voxel pair.
    The signed unit step is the derivative of the tent, so the average is a tent along
    every axis; its second moments are isotropic and 1/R is harmonic, so the first
    correction is of fourth order: the relative error falls like R^-4."""
    errs, rates = _far_errors(0.0, False)
    assert all(3.6 < r < 4.4 for r in rates), (errs, rates)
    assert errs[-1] < 1e-6


def test_dynamic_far_field_is_the_smoothed_point_curl():
    """For kappa > 0 the same tent smoothing multiplies the outgoing wave exp(i kappa n.d)
    by prod_l sinc^2(kappa n_l / 2) (about 1 - kappa^2/12): with that factor the relative
    error is small and falls with the distance; without it, it stays near kappa^2/12."""
    errs, rates = _far_errors(KAPPA, True)
    assert all(e2 < e1 for e1, e2 in zip(errs, errs[1:])) and rates[-1] > 0.8, (errs, rates)
    assert errs[-1] < 1e-6
    raw, _ = _far_errors(KAPPA, False)
    assert abs(raw[-1] / (KAPPA ** 2 / 12) - 1) < 0.01


def _scipy_Q(k, m, kappa):
    """Q_k(m) by nested adaptive quadrature over the 8 unit boxes of its weight."""
    perp = [l for l in range(3) if l != k]
    total = 0j
    for lk, sk in ((m[k], 1.0), (m[k] - 1, -1.0)):
        for s0 in (0, 1):
            for s1 in (0, 1):
                los = {k: lk}
                w = {}
                for l, s in zip(perp, (s0, s1)):
                    los[l] = m[l] - 1 if s == 0 else m[l]
                ranges = [(los[d], los[d] + 1) for d in range(3)]

                def f(x0, x1, x2):
                    x = (x0, x1, x2)
                    r = math.sqrt(x0 * x0 + x1 * x1 + x2 * x2)
                    g = np.exp(1j * kappa * r) / (4 * math.pi * r)
                    wt = sk
                    for l in perp:
                        wt *= 1.0 - abs(x[l] - m[l])
                    return g * wt
                re = integrate.nquad(lambda *x: f(*x).real, ranges, opts={"epsabs": 1e-13, "epsrel": 1e-11})[0]
                im = integrate.nquad(lambda *x: f(*x).imag, ranges, opts={"epsabs": 1e-13, "epsrel": 1e-11})[0]
                total += re + 1j * im
    return total


@pytest.mark.parametrize("k,m", [(0, (2, 1, 1)), (1, (1, 2, 3))])
def test_spot_entries_match_adaptive_quadrature(k, m):
    got = jm.curl_Q(k, np.array([m]), KAPPA)[0]
    want = _scipy_Q(k, m, KAPPA)
    assert abs(got - want) < 1e-9 * abs(want), (got, want)


def test_parity_by_recomputing_negative_offsets():
    ms = np.array([[1, 2, 3], [0, 1, 2], [2, 0, 1], [1, 1, 0]])
    for ci, (a, b) in enumerate(jm.KCOMPONENTS):
        base = jm.galerkin_K(ms, KAPPA)[ci]
        for d in range(3):
            flip = ms.copy()
            flip[:, d] *= -1
            got = jm.galerkin_K(flip, KAPPA)[ci]
            assert np.allclose(got, jm.curl_parity(a, b, d) * base, atol=1e-14, rtol=1e-12)
    # the entries odd along their axis vanish at zero offset there
    assert np.allclose(jm.curl_Q(2, np.array([[1, 2, 0]]), KAPPA), 0, atol=1e-15)


def test_galerkin_matrix_of_the_curl_is_symmetric():
    """<K P_j e_b, P_i e_a> = <K P_i e_a, P_j e_b>: antisymmetric components with odd
    parity give a symmetric matrix (the curl is symmetric under the bilinear form)."""
    Kt = jm.curl_table((3, 2, 4), KAPPA)
    Kd = jm.dense_K(Kt)
    assert np.allclose(Kd, Kd.T, atol=1e-15, rtol=0)
    assert np.abs(Kd).max() > 1e-2


def test_direct_sum_equals_fft_product():
    n = (3, 2, 5)
    T = green.green_table(n, KAPPA)
    Kt = jm.curl_table(n, KAPPA)
    x = _cvec((3,) + n)
    assert np.allclose(jm.apply_K_direct(Kt, x), jm.apply_K_fft(jm.curl_spectrum(Kt), x), atol=1e-13, rtol=0)
    chi_e = _cvec(n)
    chi_m = _cvec(n)
    x6 = _cvec((6,) + n)
    a = jm.jm_matvec_direct(T, Kt, chi_e, chi_m, KAPPA, x6)
    b = jm.jm_matvec(mv.spectrum(T), jm.curl_spectrum(Kt), chi_e, chi_m, KAPPA, x6)
    assert np.allclose(a, b, atol=1e-12, rtol=0)
    D = jm.dense_JM(T, Kt, chi_e, chi_m, KAPPA)
    assert np.allclose(D @ x6.ravel(), a.ravel(), atol=1e-12, rtol=0)


def _swap(x6):
    """Duality J(x_e, x_m) = (x_m, -x_e)."""
    return np.concatenate([x6[3:], -x6[:3]])


def test_duality_exchanges_electric_and_magnetic_roles():
    """Maxwell's equations are invariant under E -> eta H, eta H -> -E with eps <-> mu, so
    A(eps, mu) maps to A(mu, eps) under J: A(mu, eps) J x = J A(eps, mu) x; with eps = mu
    the operator commutes with J.  A wrong sign on either coupling block breaks it."""
    n = (3, 3, 4)
    T = green.green_table(n, KAPPA)
    Kt = jm.curl_table(n, KAPPA)
    spec, kspec = mv.spectrum(T), jm.curl_spectrum(Kt)
    chi_e, chi_m = _cvec(n), _cvec(n)
    x6 = _cvec((6,) + n)
    lhs = jm.jm_matvec(spec, kspec, chi_m, chi_e, KAPPA, _swap(x6))
    rhs = _swap(jm.jm_matvec(spec, kspec, chi_e, chi_m, KAPPA, x6))
    assert np.allclose(lhs, rhs, atol=1e-13, rtol=0)
    lhs = jm.jm_matvec(spec, kspec, chi_e, chi_e, KAPPA, _swap(x6))
    rhs = _swap(jm.jm_matvec(spec, kspec, chi_e, chi_e, KAPPA, x6))
    assert np.allclose(lhs, rhs, atol=1e-13, rtol=0)
    # the coupling is really present
    assert np.abs(jm.jm_matvec(spec, kspec, chi_e, chi_m, KAPPA, x6)[:3]
                  - mv.matvec_fft(spec, chi_e, x6[:3])).max() > 1e-3


def test_without_magnetic_contrast_it_is_the_j_vie():
    n = (3, 2, 4)
    T = green.green_table(n, KAPPA)
    Kt = jm.curl_table(n, KAPPA)
    chi_e = _cvec(n)
    x6 = _cvec((6,) + n)
    x6[3:] = 0
    y = jm.jm_matvec(mv.spectrum(T), jm.curl_spectrum(Kt), chi_e, np.zeros(n), KAPPA, x6)
    assert np.allclose(y[:3], mv.matvec_fft(mv.spectrum(T), chi_e, x6[:3]), atol=1e-13, rtol=0)
    assert np.all(y[3:] == 0)


def test_gmres_solves_the_jm_system():
    n = (3, 2, 6)
    T = green.green_table(n, KAPPA)
    Kt = jm.curl_table(n, KAPPA)
    eps_r = 1 + 4 * RNG.random(n) + 0.5j * RNG.random(n)
    mu_r = 1 + 0.3j * RNG.random(n)
    chi_e = mv.contrast(eps_r, 1.0)
    chi_m = jm.magnetic_contrast(mu_r)
    op = jm.JMOperator(T, Kt, chi_e, chi_m, KAPPA)
    b = _cvec((6,) + n).ravel()
    x, info = solve.gmres(op, b, tol=1e-10, restart=200)
    assert info.converged
    D = jm.dense_JM(T, Kt, chi_e, chi_m, KAPPA)
    assert np.linalg.norm(x - np.linalg.solve(D, b)) <= 1e-8 * np.linalg.norm(x)
