"""Pins of the oracle's FFT, matvec, solvers and observables."""
import math

import numpy as np
import pytest

from oracle import fft, green, matvec as mv, observables, solve
from paper_1803_06237_amd import inputs

KAP = 0.2927
RNG = np.random.default_rng(11)


def _cvec(shape, rng=RNG):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("n", [1, 2, 8, 64, 6, 12, 30, 97])
def test_own_fft_matches_library(n):
    x = _cvec((3, 4, n))
    assert np.max(np.abs(fft.fft(x) - np.fft.fft(x))) < 1e-13 * max(1, n)
    assert np.max(np.abs(fft.fft(x, inverse=True) - np.fft.ifft(x))) < 1e-14 * max(1, n)


@pytest.fixture(scope="module")
def small():
    n = (3, 4, 6)
    T = green.green_table(n, KAP)
    chi = _cvec(n)
    return n, T, chi


def test_direct_sum_equals_fft_matvec(small):
    n, T, chi = small
    for M in (mv.circulant_size(n), (5, 8, 11), (8, 9, 16)):   # any M >= 2n-1 embeds exactly
        spec = mv.spectrum(T, M)
        x = _cvec((3,) + n)
        yd = mv.matvec_direct(T, chi, x)
        yf = mv.matvec_fft(spec, chi, x)
        assert np.linalg.norm(yd - yf) / np.linalg.norm(yd) < 1e-13


def test_zero_contrast_is_identity_bit_exact(small):
    n, T, _ = small
    x = _cvec((3,) + n)
    spec = mv.spectrum(T)
    y = mv.matvec_fft(spec, np.zeros(n, complex), x)
    assert np.array_equal(y, x)


def test_delta_input_gives_toeplitz_column(small):
    """x = unit vector at (voxel j, component b): (N x)_i^a = N^{ab}(i - j), with the
    entries evaluated directly at the signed offsets."""
    n, T, _ = small
    spec = mv.spectrum(T)
    j = (1, 2, 4)
    for b in range(3):
        x = np.zeros((3,) + n, complex)
        x[(b,) + j] = 1.0
        col = mv.apply_N_fft(spec, x)
        ii = np.stack(np.meshgrid(*[np.arange(k) for k in n], indexing="ij"), -1).reshape(-1, 3)
        offs = ii - np.array(j)
        direct = np.empty((3, offs.shape[0]), complex)
        for a in range(3):
            if a == b:
                direct[a] = np.where(np.all(offs == 0, axis=1), 1.0, 0.0) + KAP ** 2 * green.volume_V(offs, KAP) \
                    - green.face_F_diag(a, offs, KAP)
            else:
                direct[a] = -green.face_F_offdiag(a, b, offs, KAP)
        assert np.max(np.abs(col.reshape(3, -1) - direct)) < 1e-14


def test_reciprocity_and_linearity(small):
    n, T, chi = small
    spec = mv.spectrum(T)
    u, v = _cvec((3,) + n), _cvec((3,) + n)
    Nu, Nv = mv.apply_N_fft(spec, u), mv.apply_N_fft(spec, v)
    assert abs(np.sum(u * Nv) - np.sum(v * Nu)) < 1e-13 * np.linalg.norm(u) * np.linalg.norm(Nv)
    a, b = 0.3 - 1.2j, -2.0 + 0.5j
    y = mv.matvec_fft(spec, chi, a * u + b * v)
    y2 = a * mv.matvec_fft(spec, chi, u) + b * mv.matvec_fft(spec, chi, v)
    assert np.linalg.norm(y - y2) / np.linalg.norm(y) < 1e-14


def test_dense_assembly_matches_direct_sum(small):
    n, T, chi = small
    x = _cvec((3,) + n)
    A = mv.dense_A(T, chi)
    y = mv.matvec_direct(T, chi, x)
    assert np.linalg.norm(A @ x.ravel() - y.ravel()) / np.linalg.norm(y) < 1e-14
    Nd = mv.dense_N(T)
    assert np.max(np.abs(Nd - Nd.T)) < 1e-15       # complex symmetric (odd entries at m_d = 0 are quadrature zeros)


@pytest.mark.parametrize("h", [1.0, 0.05, 0.02])
def test_single_voxel_clausius_mossotti(h):
    """One small voxel of edge h in a uniform incident field: E_in/E_inc -> 3/(eps_r + 2)
    as kh -> 0, whatever h.  With kh fixed, Maxwell's equations are invariant under a
    change of length scale, so the field may not depend on h; the normalised basis
    P_i = h^{-3/2} 1_{V_i} (Section III-A) puts h^{3/2} into the right-hand side and
    takes it out again in the field read-out, and a mismatch between the two shows
    here as a power of h."""
    eps_b = 2.085
    for eps in (12.11, 4.0 + 1.0j):
        for kh in (1e-3, 1e-4):
            T = green.green_table((1, 1, 1), kh)
            chi = mv.contrast(np.full((1, 1, 1), eps), eps_b)
            A = mv.dense_A(T, chi)
            e_inc = np.zeros((3, 1, 1, 1), complex)
            e_inc[2] = 1.0
            b = mv.rhs_from_field(np.full((1, 1, 1), eps), eps_b, e_inc, h)
            w = np.linalg.solve(A, b.ravel()).reshape(3, 1, 1, 1)
            E = observables.field_from_current(w, np.full((1, 1, 1), eps), eps_b, h)
            er = eps / eps_b
            assert abs(E[2, 0, 0, 0] - 3.0 / (er + 2.0)) < 5 * kh ** 2
            assert abs(E[0, 0, 0, 0]) < 1e-15


def test_contrast_of_background_is_zero():
    eps = np.array([2.085, 12.11, 12.11 + 3j])
    chi = mv.contrast(eps, 2.085)
    assert chi[0] == 0
    assert abs(chi[1] - (1 - 2.085 / 12.11)) < 1e-16


# --------------------------------------------------------------------------- solvers

@pytest.fixture(scope="module")
def waveguide_system():
    wg = inputs.Waveguide(n=(3, 3, 10), h=0.05, core_x=(1, 2), core_y=(0, 3), core_z=(0, 10),
                          n_abs=3, d=2, sigma_max=2.0)
    kap = mv.kappa_of(wg.h, wg.k0, wg.eps_b)
    T = green.green_table(wg.n, kap)
    chi = mv.contrast(wg.eps(), wg.eps_b)
    return wg, T, chi


def test_lu_and_gmres_agree(waveguide_system):
    wg, T, chi = waveguide_system
    A = mv.dense_A(T, chi)
    b = inputs.gaussian_rhs(wg.n, 0).ravel()
    x_lu = solve.solve_lu(A, b)
    assert np.linalg.norm(A @ x_lu - b) / np.linalg.norm(b) < 1e-14
    op = mv.Operator(T, chi)
    for restart in (5, 200):
        x, info = solve.gmres(op, b, tol=1e-8, restart=restart)
        assert info.converged and info.rel_res_true <= 1e-8
        kappa_A = np.linalg.cond(A)
        assert np.linalg.norm(x - x_lu) / np.linalg.norm(x_lu) < 10 * kappa_A * 1e-8


def test_gmres_history_is_the_krylov_minimum(waveguide_system):
    wg, T, chi = waveguide_system
    op = mv.Operator(T, chi)
    b = inputs.gaussian_rhs(wg.n, 1).ravel()
    _, info = solve.gmres(op, b, tol=1e-14, restart=400, maxit=15)
    brute = solve.krylov_min_residual(op, b, 15)
    hist = np.array(info.history[:15])
    # the brute force forms b - A Q y explicitly, so its absolute error is ~1e-15
    assert np.max(np.abs(hist - brute) / (brute + 1e-5)) < 1e-10, (hist, brute)


def test_gmres_finite_termination():
    n = (1, 1, 3)        # 9 unknowns
    T = green.green_table(n, KAP)
    chi = _cvec(n) * 0.5
    op = mv.Operator(T, chi)
    b = _cvec((3,) + n).ravel()
    x, info = solve.gmres(op, b, tol=1e-13, restart=9, maxit=9)
    assert info.iters <= 9 and info.rel_res_true < 1e-12


def test_fgmres_with_exact_preconditioner_converges_in_one_step(waveguide_system):
    wg, T, chi = waveguide_system
    A = mv.dense_A(T, chi)
    Ainv = np.linalg.inv(A)
    op = mv.Operator(T, chi)
    b = inputs.gaussian_rhs(wg.n, 2).ravel()
    x, info = solve.fgmres(op, b, tol=1e-10, restart=10, precond=lambda v: Ainv @ v)
    assert info.iters == 1 and info.rel_res_true < 1e-12


def test_paper_time_convention_is_the_conjugate_system(waveguide_system):
    """With exp(+j omega t) the kernel is e^{-jkR} and absorbers have eps' - j eps'':
    the system is the complex conjugate, so the currents are conjugated."""
    wg, T, chi = waveguide_system
    kap = mv.kappa_of(wg.h, wg.k0, wg.eps_b)
    Tp = green.green_table(wg.n, -kap)
    chip = mv.contrast(np.conj(wg.eps()), wg.eps_b)
    b = inputs.gaussian_rhs(wg.n, 4).ravel()
    x = solve.solve_lu(mv.dense_A(T, chi), b)
    xp = solve.solve_lu(mv.dense_A(Tp, chip), np.conj(b))
    assert np.linalg.norm(xp - np.conj(x)) / np.linalg.norm(x) < 1e-13


def test_reflection_definition():
    e = _cvec(50)
    assert observables.reflection(e, e) == 0.0
    assert abs(observables.reflection(e, 0.9 * e) - 0.01) < 1e-15


def test_input_recipes():
    wg = inputs.strip_long(d=1)
    assert abs(wg.sigma_max - 2 * 4.942) < 2e-3
    u = wg.absorber_u()
    assert np.allclose(u[:80], (80 - np.arange(80) - 0.5) / 80)
    assert np.allclose(u[-80:], (np.arange(80) + 0.5) / 80)
    eps = wg.eps()
    assert eps[0, 0, 0] == inputs.EPS_B and eps[16, 15, 256] == inputs.EPS_SI
    assert [inputs.strip_family(L, 2).n[2] for L in (0.5, 1, 2, 4, 8)] == [192, 256, 320, 512, 832]
    r = inputs.rough_strip(3)
    assert r.core_mask().sum() > 0
