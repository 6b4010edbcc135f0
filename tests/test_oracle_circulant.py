"""Pins of the oracle's block-circulant preconditioner (Section V-D) against facts
that do not depend on its code: the independently pinned dense operator, the
first-order optimality of a Frobenius least-squares fit, T. Chan's closed form
for a Toeplitz matrix, and the DFT diagonalisation of a block circulant."""
import numpy as np
import pytest

from oracle import circulant as circ
from oracle import green, matvec as mv
from oracle import solve
from paper_1803_06237_amd import inputs

RNG = np.random.default_rng(5)
KAPPA = 0.31


def _case(n=(3, 3, 7), cols=((0, 0), (1, 1), (2, 1), (1, 2)), z_varying=True):
    """Contrast on a few cross-section columns, varying along z (an absorber-like ramp) or not."""
    chi = np.zeros(n, dtype=np.complex128)
    for (i1, i2) in cols:
        base = 2.0 + 0.3 * i1 - 0.2j * i2
        ramp = 1.0 + 0.4j * np.linspace(0, 1, n[2]) ** 2 if z_varying else np.ones(n[2])
        chi[i1, i2, :] = base * ramp
    table = green.green_table(n, KAPPA)
    return table, chi


def _support_perm(n, S, window=None):
    """Rows of the (3, n1, n2, n3) flattening in the slice-major support order (i3, a, p),
    i3 over the window (z0, P) (default: all slices)."""
    n1, n2, n3 = n
    z0, P = window if window is not None else (0, n3)
    idx = []
    for i3 in range(z0, z0 + P):
        for a in range(3):
            for (i1, i2) in S:
                idx.append(((a * n1 + i1) * n2 + i2) * n3 + i3)
    return np.array(idx)


def test_support_operator_is_the_dense_operator_restricted():
    table, chi = _case()
    S = circ.support_columns(chi)
    A = mv.dense_A(table, chi)
    perm = _support_perm(chi.shape, S)
    assert np.allclose(circ.dense_A_on_support(table, chi, S), A[np.ix_(perm, perm)], atol=1e-14, rtol=0)


@pytest.mark.parametrize("z_varying", [False, True])
def test_blocks_satisfy_frobenius_normal_equations(z_varying):
    """W minimises ||A - circ(W)||_F over block circulants iff, for every k, the blocks of
    A on the wrapped diagonal k sum to n3 W_k.  A comes from the dense operator."""
    table, chi = _case(z_varying=z_varying)
    n3 = chi.shape[2]
    S = circ.support_columns(chi)
    m = 3 * len(S)
    A = mv.dense_A(table, chi)
    perm = _support_perm(chi.shape, S)
    As = A[np.ix_(perm, perm)]
    W = circ.optimal_blocks(table, chi, S)
    for k in range(n3):
        acc = np.zeros((m, m), dtype=np.complex128)
        for i in range(n3):
            j = (i - k) % n3
            acc += As[i * m:(i + 1) * m, j * m:(j + 1) * m]
        assert np.allclose(acc / n3, W[k], atol=1e-14, rtol=0)
    # and any block-circulant perturbation increases the distance
    C = circ.block_circulant_dense(W)
    base = np.linalg.norm(As - C)
    for _ in range(3):
        E = RNG.standard_normal(W.shape) + 1j * RNG.standard_normal(W.shape)
        assert np.linalg.norm(As - circ.block_circulant_dense(W + 1e-3 * E)) > base


def test_uniform_contrast_reduces_to_chans_optimal_circulant():
    """With chi constant along z, each Toeplitz level t_k of a fixed (p, q) entry maps to
    ((n - k) t_k + k t_{k-n}) / n (T. Chan, SIAM J. Sci. Stat. Comput. 9, 1988)."""
    table, chi = _case(z_varying=False)
    n3 = chi.shape[2]
    S = circ.support_columns(chi)
    s = len(S)
    W = circ.optimal_blocks(table, chi, S)
    T = mv.signed_table(table)                    # (3, 3, 2n1-1, 2n2-1, 2n3-1), offset + n - 1
    n1, n2, _ = chi.shape
    for k in range(n3):
        for (pi, p) in enumerate(S):
            for (qi, q) in enumerate(S):
                d1, d2 = p[0] - q[0] + n1 - 1, p[1] - q[1] + n2 - 1
                dp = chi[p[0], p[1], 0]
                for a in range(3):
                    for b in range(3):
                        tk = T[a, b, d1, d2, k + n3 - 1]
                        tkn = T[a, b, d1, d2, k - n3 + n3 - 1] if k > 0 else 0.0
                        want = ((n3 - k) * tk + k * tkn) / n3
                        want = (1.0 if (k == 0 and a == b and pi == qi) else 0.0) - dp * want
                        assert abs(W[k, a * s + pi, b * s + qi] - want) < 1e-14


def test_fft_apply_solves_the_block_circulant():
    table, chi = _case()
    n = chi.shape
    S = circ.support_columns(chi)
    W = circ.optimal_blocks(table, chi, S)
    Winv = circ.spectrum_inverse(W)
    r = RNG.standard_normal((3,) + n) + 1j * RNG.standard_normal((3,) + n)
    z = circ.apply(Winv, S, r, circ.support_window(chi))
    perm = _support_perm(n, S)
    zs = np.linalg.solve(circ.block_circulant_dense(W), r.ravel()[perm])
    assert np.allclose(z.ravel()[perm], zs, atol=1e-12, rtol=0)
    outside = np.ones(3 * np.prod(n), dtype=bool)
    outside[perm] = False
    assert np.array_equal(z.ravel()[outside], r.ravel()[outside])


def test_zero_contrast_gives_identity():
    n = (2, 3, 5)
    table = green.green_table(n, KAPPA)
    chi = np.zeros(n, dtype=np.complex128)
    chi[1, 1, :] = 0.0
    chi[0, 0, 2] = 1e-300          # a single column with a negligible contrast
    S = circ.support_columns(chi)
    W = circ.optimal_blocks(table, chi, S)
    assert np.allclose(W[0], np.eye(3 * len(S)), atol=1e-290)
    assert np.allclose(W[1:], 0, atol=1e-290)


def test_preconditioner_cuts_iterations_and_keeps_the_solution():
    """Right-preconditioned FGMRES reaches the same 1e-8 solution in fewer iterations on a
    small absorbing guide, and its count does not grow with the length."""
    counts = {}
    for n3 in (32, 64):
        wg = inputs.Waveguide(n=(6, 6, n3), h=0.05, core_x=(1, 5), core_y=(2, 4), core_z=(0, n3), n_abs=8,
                              d=2, sigma_max=2.0)
        kap = mv.kappa_of(wg.h, wg.k0, wg.eps_b)
        table = green.green_table(wg.n, kap)
        chi = mv.contrast(wg.eps(), wg.eps_b)
        op = mv.Operator(table, chi)
        S = circ.support_columns(chi)
        Winv = circ.spectrum_inverse(circ.optimal_blocks(table, chi, S))
        b = mv.rhs_from_field(wg.eps(), wg.eps_b, inputs.gaussian_rhs(wg.n, 1), wg.h).ravel()
        win = circ.support_window(chi)
        pc = lambda v: circ.apply(Winv, S, v.reshape((3,) + wg.n), win).ravel()
        x0, i0 = solve.gmres(op, b, tol=1e-8, restart=400)
        x1, i1 = solve.fgmres(op, b, tol=1e-8, restart=400, precond=pc)
        assert i0.converged and i1.converged
        assert np.linalg.norm(x1 - x0) <= 1e-6 * np.linalg.norm(x0)
        counts[n3] = (i0.iters, i1.iters)
    for n3, (plain, pre) in counts.items():
        assert pre < plain / 2, counts
    assert counts[64][1] <= counts[32][1] + 3, counts


def test_single_frequency_block_matches_the_fft_of_all_blocks():
    table, chi = _case()
    S = circ.support_columns(chi)
    W = circ.optimal_blocks(table, chi, S)
    What = np.fft.fft(W, axis=0)                  # library DFT, independent of the oracle's FFT
    for f in (0, 1, 4):
        assert np.allclose(circ.frequency_block(table, chi, S, f), What[f], atol=1e-13, rtol=0)


def test_smooth_lengths_and_windows():
    assert [circ.smooth_length(n) for n in (1, 7, 8, 59, 97, 472, 625, 832)] == [1, 8, 8, 60, 100, 480, 625, 864]
    chi = np.zeros((2, 2, 12), dtype=np.complex128)
    chi[0, 1, 3:9] = 1.5
    assert circ.support_window(chi) == (3, 6)
    chi = np.zeros((2, 2, 10), dtype=np.complex128)
    chi[1, 0, 3:10] = 1.0                     # extent 7 -> P = 8, shifted to fit: z0 = 2
    assert circ.support_window(chi) == (2, 8)
    chi = np.zeros((2, 2, 7), dtype=np.complex128)
    chi[0, 0, :] = 1.0                        # extent 7 -> 8 > n3: the whole grid
    assert circ.support_window(chi) == (0, 7)
    assert circ.support_window(np.zeros((2, 2, 5))) == (0, 5)


def test_window_blocks_satisfy_normal_equations_and_apply_is_identity_outside():
    """Contrast on slices 3..8 of 12 (window (3, 6)): the blocks are the Frobenius fit of
    the dense operator restricted to S x window, and W^{-1} leaves other voxels alone."""
    n = (3, 2, 12)
    table = green.green_table(n, KAPPA)
    chi = np.zeros(n, dtype=np.complex128)
    chi[0, 0, 3:9] = 2.0 + 0.3j * np.arange(6)
    chi[1, 1, 4:9] = 1.5
    S = circ.support_columns(chi)
    win = circ.support_window(chi)
    assert win == (3, 6)
    P, m = win[1], 3 * len(S)
    perm = _support_perm(n, S, win)
    As = mv.dense_A(table, chi)[np.ix_(perm, perm)]
    W = circ.optimal_blocks(table, chi, S)
    assert W.shape == (P, m, m)
    for k in range(P):
        acc = sum(As[i * m:(i + 1) * m, ((i - k) % P) * m:(((i - k) % P) + 1) * m] for i in range(P))
        assert np.allclose(acc / P, W[k], atol=1e-14, rtol=0)
    r = RNG.standard_normal((3,) + n) + 1j * RNG.standard_normal((3,) + n)
    z = circ.apply(circ.spectrum_inverse(W), S, r, win)
    outside = np.ones(3 * np.prod(n), dtype=bool)
    outside[perm] = False
    assert np.array_equal(z.ravel()[outside], r.ravel()[outside])
    zs = np.linalg.solve(circ.block_circulant_dense(W), r.ravel()[perm])
    assert np.allclose(z.ravel()[perm], zs, atol=1e-12, rtol=0)


def test_background_slices_do_not_dilute_the_preconditioner():
    """A guide whose core stops short of both grid ends converges as fast as the same
    core filling the grid (the window drops the background slices)."""
    its = []
    for n3, core_z in ((40, (0, 40)), (52, (6, 46))):
        wg = inputs.Waveguide(n=(6, 6, n3), h=0.05, core_x=(1, 5), core_y=(2, 4), core_z=core_z, n_abs=8,
                              d=2, sigma_max=2.0)
        kap = mv.kappa_of(wg.h, wg.k0, wg.eps_b)
        table = green.green_table(wg.n, kap)
        chi = mv.contrast(wg.eps(), wg.eps_b)
        op = mv.Operator(table, chi)
        S = circ.support_columns(chi)
        win = circ.support_window(chi)
        Winv = circ.spectrum_inverse(circ.optimal_blocks(table, chi, S))
        b = mv.rhs_from_field(wg.eps(), wg.eps_b, inputs.gaussian_rhs(wg.n, 2), wg.h).ravel()
        pc = lambda v: circ.apply(Winv, S, v.reshape((3,) + wg.n), win).ravel()
        x, info = solve.fgmres(op, b, tol=1e-8, restart=400, precond=pc)
        assert info.converged
        its.append(info.iters)
    assert its[1] <= its[0] + 2, its
