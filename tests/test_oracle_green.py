"""Pins of the oracle's Galerkin table against facts fixed by the mathematics.

Each test would fail for a plausible slip in the oracle (a dropped term, a
wrong sign or index, a transposed operand, an under-resolved quadrature).
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

from oracle import green

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "constants.json")))
ZERO = np.zeros((1, 3), dtype=np.int64)


def test_static_volume_self_term_closed_form():
    v = green.volume_V(ZERO, 0.0)[0]
    assert abs(4 * math.pi * v - GOLD["cube_inverse_distance"]["value"]) < 2e-14
    assert v.imag == 0.0


def test_static_same_face_closed_form():
    for a in range(3):
        g = green.face_g(a, np.array([0]), np.array([[0, 0]]), 0.0)[0]
        assert abs(4 * math.pi * g - GOLD["square_inverse_distance"]["value"]) < 2e-14


def test_cube_depolarisation():
    for a in range(3):
        f = green.face_F_diag(a, ZERO, 0.0)[0]
        assert abs(f - GOLD["cube_depolarisation"]["value"]) < 1e-14
    N = green.galerkin_N(ZERO, 0.0)[:, 0]
    for ci, (a, b) in enumerate(green.COMPONENTS):
        assert abs(N[ci] - (2.0 / 3.0 if a == b else 0.0)) < 1e-14


@pytest.mark.parametrize("kappa", [0.1463, 0.2927, 1.3])
def test_dynamic_self_term_by_cubic_symmetry(kappa):
    V0 = green.volume_V(ZERO, kappa)[0]
    N = green.galerkin_N(ZERO, kappa)[:, 0]
    for ci, (a, b) in enumerate(green.COMPONENTS):
        want = (2.0 / 3.0) * (1 + kappa ** 2 * V0) if a == b else 0.0
        assert abs(N[ci] - want) < 1e-14


def test_small_kh_expansion_of_volume_self_term():
    """4 pi V(0) = 1.88231... + i k - (Robbins/2) k^2 - i k^3/12 + O(k^4) (h = 1):
    e^{ikR}/R = 1/R + ik - k^2 R/2 - i k^3 R^2/6 + ..., with mean R the Robbins
    constant and mean R^2 = 1/2 over pairs of points of the unit cube."""
    c0 = GOLD["cube_inverse_distance"]["value"]
    rob = GOLD["robbins_constant"]["value"]
    for k in (1e-2, 2e-2, 4e-2):
        v = 4 * math.pi * green.volume_V(ZERO, k)[0]
        approx = c0 + 1j * k - 0.5 * rob * k * k - 1j * k ** 3 / 12
        assert abs(v - approx) < 0.2 * k ** 4 + 1e-14


KAP = 0.2927
OFFSETS = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [1, 0, 1], [1, 1, 1],
                    [2, 0, 0], [2, 1, 0], [2, 2, 1], [0, 3, 5], [4, 1, 7], [7, 7, 31], [0, 0, 12]])


def test_trace_identity_ties_faces_to_volume():
    """sum_a F^{aa}(m) = delta_m0 + kappa^2 V(m) because div grad S = -k^2 S - I."""
    N = green.galerkin_N(OFFSETS, KAP)
    V = green.volume_V(OFFSETS, KAP)
    tr = N[0] + N[3] + N[5]
    want = 2.0 * np.all(OFFSETS == 0, axis=1) + 2.0 * KAP * KAP * V
    assert np.max(np.abs(tr - want)) < 2e-15


def test_symmetry_and_parity_from_direct_integration():
    """F^{ab} = F^{ba}; negating the offset along axis d multiplies N^{ab} by -1
    exactly when one of a, b is d.  Both sides are integrated directly."""
    rng = np.random.default_rng(3)
    ms = rng.integers(-4, 5, size=(12, 3))
    for a in range(3):
        for b in range(3):
            if a == b:
                base = green.face_F_diag(a, ms, KAP)
            else:
                base = green.face_F_offdiag(a, b, ms, KAP)
                swapped = green.face_F_offdiag(b, a, ms, KAP)
                assert np.max(np.abs(base - swapped)) < 1e-15
            for d in range(3):
                mflip = ms.copy()
                mflip[:, d] *= -1
                flip = green.face_F_diag(a, mflip, KAP) if a == b else green.face_F_offdiag(a, b, mflip, KAP)
                assert np.max(np.abs(flip - green.parity(a, b, d) * base)) < 1e-15
    V = green.volume_V(ms, KAP)
    assert np.max(np.abs(green.volume_V(-ms, KAP) - V)) < 1e-16


def _dyadic_far(m, kappa):
    """(kappa^2 delta_ab + d_a d_b) G at m, G = e^{i kappa R}/(4 pi R), in COMPONENTS order."""
    m = np.asarray(m, dtype=float)
    R = np.linalg.norm(m)
    n = m / R
    G = np.exp(1j * kappa * R) / (4 * math.pi * R)
    p = 1j * kappa - 1.0 / R
    out = []
    for a, b in green.COMPONENTS:
        dab = 1.0 if a == b else 0.0
        dd = G * ((dab - n[a] * n[b]) * p / R + n[a] * n[b] * (p * p + 1.0 / R ** 2))
        out.append(kappa ** 2 * dab * G + dd)
    return np.array(out)


def test_far_field_is_the_dyadic_green_function():
    """Away from the source the Galerkin entry is the averaged point value of
    (k^2 + grad grad)G.  Averaging over two voxels convolves with a tent of second
    moment 1/6 per axis, so the leading correction is (1/12) Laplacian = -k^2/12
    (the kernel solves the Helmholtz equation there); the static remainder is
    O((h/R)^4) because the Laplacian of the static kernel vanishes."""
    for m in ([0, 0, 10], [0, 0, 20], [0, 0, 40], [10, 20, 30], [3, 25, 11], [60, 0, 0]):
        R = np.linalg.norm(m)
        N0 = green.galerkin_N(np.array([m]), 0.0)[:, 0]
        F0 = _dyadic_far(m, 0.0)
        rel0 = np.max(np.abs(N0 - F0)) / np.max(np.abs(F0))
        assert rel0 * R ** 4 < 0.5, (m, rel0)
        N = green.galerkin_N(np.array([m]), KAP)[:, 0]
        F = _dyadic_far(m, KAP)
        rel = np.max(np.abs(N - (1 - KAP ** 2 / 12) * F)) / np.max(np.abs(F))
        assert rel < 0.01 * KAP ** 4 + 0.5 / R ** 4, (m, rel)
        # without the moment correction the error is the full k^2/12
        assert abs(np.max(np.abs(N - F)) / np.max(np.abs(F)) - KAP ** 2 / 12) < 0.05 * KAP ** 2 / 12
    # the static remainder really is fourth order along an axis
    r20 = np.max(np.abs(green.galerkin_N(np.array([[0, 0, 20]]), 0.0)[:, 0] - _dyadic_far([0, 0, 20], 0.0)))
    r40 = np.max(np.abs(green.galerkin_N(np.array([[0, 0, 40]]), 0.0)[:, 0] - _dyadic_far([0, 0, 40], 0.0)))
    f20 = np.max(np.abs(_dyadic_far([0, 0, 20], 0.0)))
    f40 = np.max(np.abs(_dyadic_far([0, 0, 40], 0.0)))
    assert 15.0 < (r20 / f20) / (r40 / f40) < 17.0


def _adaptive_box(fun, ranges):
    re = integrate.nquad(lambda *x: fun(*x).real, ranges, opts={"epsabs": 1e-15, "epsrel": 1e-13})[0]
    im = integrate.nquad(lambda *x: fun(*x).imag, ranges, opts={"epsabs": 1e-15, "epsrel": 1e-13})[0]
    return re + 1j * im


def _G(x, y, z, k=KAP):
    r = math.sqrt(x * x + y * y + z * z)
    return np.exp(1j * k * r) / (4 * math.pi * r)


def test_spot_entries_against_adaptive_integration():
    """Non-singular entries integrated with scipy's adaptive quadrature on each box."""
    # g_0(1, (0, 0)): square face at unit distance
    want = 0
    for y0 in (-1, 0):
        for z0 in (-1, 0):
            want += _adaptive_box(lambda y, z: _G(1.0, y, z) * (1 - abs(y)) * (1 - abs(z)),
                                  [[y0, y0 + 1], [z0, z0 + 1]])
    got = green.face_g(0, np.array([1]), np.array([[0, 0]]), KAP)[0]
    assert abs(got - want) < 1e-13
    # F^{01} at m = (2, 1, 3): orthogonal faces, signed steps in a and b, tent in c
    m = (2, 1, 3)
    want = 0
    for la, sa in ((m[0], 1), (m[0] - 1, -1)):
        for lb, sb in ((m[1] - 1, 1), (m[1], -1)):
            for lc in (m[2] - 1, m[2]):
                want += sa * sb * _adaptive_box(
                    lambda x, y, z: _G(x, y, z) * (1 - abs(z - m[2])),
                    [[la, la + 1], [lb, lb + 1], [lc, lc + 1]])
    got = green.face_F_offdiag(0, 1, np.array([m]), KAP)[0]
    assert abs(got - want) < 1e-13


def test_quadrature_is_converged():
    """Raising every Gauss-Legendre and Duffy order changes no entry by more than 1e-15."""
    base = green.galerkin_N(OFFSETS, KAP)
    old = (green._TOL_DIGITS, green.Q_SINGULAR)
    try:
        green._TOL_DIGITS, green.Q_SINGULAR = 23.0, 22
        green.q_for_distance.cache_clear()
        fine = green.galerkin_N(OFFSETS, KAP)
    finally:
        green._TOL_DIGITS, green.Q_SINGULAR = old
        green.q_for_distance.cache_clear()
    assert np.max(np.abs(fine - base)) < 1e-15


def test_table_entries_match_pointwise_evaluation():
    T = green.green_table((3, 4, 5), KAP)
    ms = np.array([[2, 3, 4], [0, 1, 0], [1, 0, 3]])
    N = green.galerkin_N(ms, KAP)
    for j, m in enumerate(ms):
        assert np.max(np.abs(T[:, m[0], m[1], m[2]] - N[:, j])) == 0.0
    # signed lookup honours parity
    assert green.entry(T, 0, 1, (-1, 2, 0)) == -T[1, 1, 2, 0]
    assert green.entry(T, 2, 0, (1, 0, -3)) == -T[2, 1, 0, 3]
    assert green.entry(T, 1, 1, (-2, -3, -4)) == T[3, 2, 3, 4]


def test_table_in_worker_processes_equals_the_serial_table():
    for n, kap in (((5, 2, 7), 0.3), ((4, 3, 3), 1.1)):
        a = green.green_table(n, kap)
        b = green.green_table(n, kap, workers=3)
        assert np.abs(a - b).max() <= 1e-15 * np.abs(a).max()
