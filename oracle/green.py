"""Galerkin entries of the Green-tensor operator N for piecewise-constant voxel bases.

Test infrastructure (see the package docstring): never used by the product path.

Section III-A of the paper expands the current in normalised voxel indicators
``P_i = h^{-3/2} 1_{V_i}`` and tests with the same functions, so the operator
``N = curl curl S`` (Section III, with ``S f = int G f``) becomes the matrix
``N_ij = <N P_j, P_i>``.  On a uniform grid the entry depends only on the index
offset ``m = i - j`` (block Toeplitz, 6 unique symmetric components).  The paper
does not say how these integrals are evaluated; this module writes them out from
the definitions.

Derivation used here (time dependence exp(-i omega t), G(R) = e^{ikR}/(4 pi R)):

* ``curl curl = grad div - Laplacian`` and ``Laplacian(S f) = -k^2 S f - f``, so
  ``N f = grad div S f + k^2 S f + f``.
* Identity part: ``<P_j, P_i> = delta_ij``.
* Volume part: ``V(m) = h^{-3} int_{V_i} int_{V_j} G`` which, after integrating
  over the difference vector, is ``h^{-3} int_{[-h,h]^3} G(mh + s) prod_d (h - |s_d|) ds``.
* grad-div part: by the divergence theorem on both voxels,
  ``<d_a d_b S 1_{V_j}, 1_{V_i}> = - sum_faces n_a n'_b int int G``, so it reduces
  to face-face integrals ``F^{ab}(m) = h^{-3} sum n_a n'_b int_{f_i} int_{f_j} G``.
  For a == b the faces are parallel and ``F^{aa}(m) = h^{-3}[2 g_a(m_a) -
  g_a(m_a+1) - g_a(m_a-1)]`` with ``g_a(mu) = int_{[-h,h]^2} G(mu h e_a + m_perp h
  + t) prod (h - |t_d|) dt``.  For a != b (third axis c) the faces are orthogonal
  and the integral is over (Delta_a, Delta_b, t) with signed unit steps in a, b
  and the tent weight in c.
* ``N^{ab}(m) = delta_ab (delta_{m0} + k^2 V(m)) - F^{ab}(m)``.

Everything is made dimensionless with h = 1 and ``kappa = k h``; the table
depends on kappa and m only.

Quadrature.  Each integral is split into lattice-aligned unit boxes on which
its weight is a polynomial.  The integrand is singular only at the origin,
which is then a vertex of a box (this happens for |m|_inf <= 1); such boxes use
a Duffy (pyramid) map at that vertex, which cancels the 1/R singularity and
leaves an analytic integrand.  All other boxes are at distance >= 1 from the
origin and use tensor Gauss-Legendre of an order chosen from that distance via
the Bernstein-ellipse convergence rate of the nearest singularity.
"""
from __future__ import annotations

import functools
import math
from typing import Dict, Iterable, Tuple

import numpy as np

FOUR_PI = 4.0 * math.pi
_TOL_DIGITS = 17.0        # target: each box integral accurate to ~1e-17 relative to its scale


@functools.lru_cache(maxsize=None)
def gauss_legendre01(q: int) -> Tuple[np.ndarray, np.ndarray]:
    """Gauss-Legendre nodes and weights on [0, 1] (library routine)."""
    x, w = np.polynomial.legendre.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def bernstein_rho(dist: float) -> float:
    """Smallest Bernstein-ellipse parameter of 1/R along any axis-parallel unit segment
    of a unit box whose distance from the singular point is ``dist``.

    A segment s in [s0, s0+1] at transverse distance r has its singularity at
    s = +-i r; in the interval's normalised coordinate t = 2(s - s0) - 1 this is
    t* = -1 - 2 s0 + 2 i r with s0^2 + r^2 >= dist^2.  The worst case over the
    angle gives the rate.
    """
    best = math.inf
    for th in np.linspace(0.0, 0.5 * math.pi, 181):
        s0, r = dist * math.cos(th), dist * math.sin(th)
        t = complex(-1.0 - 2.0 * s0, 2.0 * r)
        root = np.sqrt(t * t - 1.0)
        rho = max(abs(t + root), abs(t - root))
        best = min(best, rho)
    return best


@functools.lru_cache(maxsize=None)
def q_for_distance(dist_sq: int) -> int:
    """Gauss-Legendre order for a unit box at squared distance ``dist_sq`` (>= 1)."""
    rho = min(bernstein_rho(math.sqrt(dist_sq)), 60.0)   # the oscillation e^{ik R} caps the usable ellipse
    q = int(math.ceil(_TOL_DIGITS * math.log(10.0) / (2.0 * math.log(rho))))
    return max(4, min(q, 24))


Q_SINGULAR = 16   # Duffy order per dimension; the mapped integrand is analytic (rho ~ 4.6)


def _green(x: np.ndarray, y: np.ndarray, z: np.ndarray, kappa: float) -> np.ndarray:
    r = np.sqrt(x * x + y * y + z * z)
    return np.exp(1j * kappa * r) / (FOUR_PI * r)


def _tensor_nodes(q: int, D: int) -> Tuple[np.ndarray, np.ndarray]:
    x, w = gauss_legendre01(q)
    grids = np.meshgrid(*([x] * D), indexing="ij")
    wts = functools.reduce(np.multiply.outer, [w] * D)
    return np.stack([g.ravel() for g in grids], axis=-1), wts.ravel()


@functools.lru_cache(maxsize=None)
def duffy_nodes(q: int, D: int) -> Tuple[np.ndarray, np.ndarray]:
    """Nodes xi in [0,1]^D and weights for integrands singular like 1/|xi| at xi = 0.

    [0,1]^D is split into D pyramids by the index p of the largest coordinate;
    on pyramid p, xi_p = u and the others are u*v_k, Jacobian u^(D-1).
    """
    (uvw, w) = _tensor_nodes(q, D)
    pts, wts = [], []
    u = uvw[:, 0]
    jac = u ** (D - 1)
    for p in range(D):
        xi = np.empty_like(uvw)
        xi[:, p] = u
        others = [k for k in range(D) if k != p]
        for j, k in enumerate(others):
            xi[:, k] = u * uvw[:, 1 + j]
        pts.append(xi)
        wts.append(w * jac)
    return np.concatenate(pts), np.concatenate(wts)


@functools.lru_cache(maxsize=None)
def tensor_nodes(q: int, D: int) -> Tuple[np.ndarray, np.ndarray]:
    return _tensor_nodes(q, D)


def box_integrals(lo: np.ndarray, alpha: np.ndarray, beta: np.ndarray, kappa: float,
                  fixed: np.ndarray | None = None, fixed_axis: int | None = None,
                  chunk_points: int = 4_000_000) -> np.ndarray:
    """Integrals of G(x) * prod_d (alpha_d + beta_d (x_d - lo_d)) over unit boxes.

    ``lo``: (K, D) integer lower corners of the boxes, D = 3, or D = 2 with the
    remaining coordinate ``x[fixed_axis] = fixed`` (K,) held fixed.
    ``alpha``, ``beta``: (K, D) coefficients of the weight, linear in the local
    coordinate t = x - lo in [0,1] per axis.
    """
    lo = np.asarray(lo, dtype=np.int64)
    K, D = lo.shape
    out = np.zeros(K, dtype=np.complex128)
    if K == 0:
        return out
    if D == 2:
        fixed = np.asarray(fixed, dtype=np.int64)
    # squared distance from origin to each box (integer arithmetic)
    near = np.where(lo > 0, lo, np.where(lo + 1 < 0, -(lo + 1), 0))
    dist_sq = (near * near).sum(axis=1)
    if D == 2:
        dist_sq = dist_sq + fixed * fixed
    singular = dist_sq == 0
    groups: Dict[int, np.ndarray] = {}
    qs = np.zeros(K, dtype=np.int64)
    for ds in np.unique(dist_sq[~singular]):
        qs[dist_sq == ds] = q_for_distance(int(ds))
    for q in np.unique(qs[~singular]):
        groups[int(q)] = np.nonzero((~singular) & (qs == q))[0]
    jobs = [(idx, tensor_nodes(q, D), False) for q, idx in groups.items()]
    if singular.any():
        jobs.append((np.nonzero(singular)[0], duffy_nodes(Q_SINGULAR, D), True))
    for idx, (xi, w), is_sing in jobs:
        P = xi.shape[0]
        step = max(1, chunk_points // P)
        for s in range(0, idx.size, step):
            sel = idx[s:s + step]
            l = lo[sel][:, None, :].astype(np.float64)             # (k,1,D)
            if is_sing:
                # vertex at the origin: box [lo, lo+1] with lo in {-1, 0}; x = sgn * xi
                sgn = np.where(lo[sel] == 0, 1.0, -1.0)[:, None, :]
                x = sgn * xi[None, :, :]
            else:
                x = l + xi[None, :, :]
            t = x - l                                                 # local coordinate in [0,1]
            wfun = np.prod(alpha[sel][:, None, :] + beta[sel][:, None, :] * t, axis=2)
            if D == 3:
                g = _green(x[..., 0], x[..., 1], x[..., 2], kappa)
            else:
                f = fixed[sel][:, None].astype(np.float64) * np.ones((1, P))
                cols = [None, None, None]
                free = [k for k in range(3) if k != fixed_axis]
                cols[fixed_axis] = f
                cols[free[0]] = x[..., 0]
                cols[free[1]] = x[..., 1]
                g = _green(cols[0], cols[1], cols[2], kappa)
            out[sel] = (g * wfun) @ w
    return out


# ---------------------------------------------------------------------------
# The three kinds of Galerkin integral, vectorised over offsets m (K, 3).
# ---------------------------------------------------------------------------

def _tent_boxes(mc: np.ndarray):
    """The two unit intervals of the tent weight (1 - |x - mc|) on [mc-1, mc+1]:
    yields (lo, alpha, beta) with the weight linear in t = x - lo."""
    return [(mc - 1, 0.0, 1.0), (mc, 1.0, -1.0)]


def volume_V(m: np.ndarray, kappa: float) -> np.ndarray:
    """V(m) = int_{[-1,1]^3} G(m + s) prod_d (1 - |s_d|) ds  (h = 1)."""
    m = np.asarray(m, dtype=np.int64).reshape(-1, 3)
    K = m.shape[0]
    los, als, bes = [], [], []
    for s0 in range(2):
        for s1 in range(2):
            for s2 in range(2):
                lo = np.empty((K, 3), np.int64)
                al = np.empty((K, 3))
                be = np.empty((K, 3))
                for d, s in enumerate((s0, s1, s2)):
                    l, a, b = _tent_boxes(m[:, d])[s]
                    lo[:, d], al[:, d], be[:, d] = l, a, b
                los.append(lo), als.append(al), bes.append(be)
    vals = box_integrals(np.concatenate(los), np.concatenate(als), np.concatenate(bes), kappa)
    return vals.reshape(8, K).sum(axis=0)


def face_g(a: int, mu: np.ndarray, mperp: np.ndarray, kappa: float) -> np.ndarray:
    """g_a(mu, m_perp) = int_{[-1,1]^2} G(mu e_a + m_perp + t) prod (1 - |t_d|) dt.

    ``mperp`` is (K, 2): the offsets along the two axes other than a, in order."""
    mu = np.asarray(mu, dtype=np.int64).reshape(-1)
    mperp = np.asarray(mperp, dtype=np.int64).reshape(-1, 2)
    K = mu.size
    los, als, bes, fx = [], [], [], []
    for s0 in range(2):
        for s1 in range(2):
            lo = np.empty((K, 2), np.int64)
            al = np.empty((K, 2))
            be = np.empty((K, 2))
            for d, s in enumerate((s0, s1)):
                l, aa, bb = _tent_boxes(mperp[:, d])[s]
                lo[:, d], al[:, d], be[:, d] = l, aa, bb
            los.append(lo), als.append(al), bes.append(be), fx.append(mu)
    vals = box_integrals(np.concatenate(los), np.concatenate(als), np.concatenate(bes), kappa,
                         fixed=np.concatenate(fx), fixed_axis=a)
    return vals.reshape(4, K).sum(axis=0)


def face_F_diag(a: int, m: np.ndarray, kappa: float) -> np.ndarray:
    """F^{aa}(m) = 2 g_a(m_a) - g_a(m_a + 1) - g_a(m_a - 1)  (parallel faces)."""
    m = np.asarray(m, dtype=np.int64).reshape(-1, 3)
    others = [k for k in range(3) if k != a]
    mperp = m[:, others]
    g0 = face_g(a, m[:, a], mperp, kappa)
    gp = face_g(a, m[:, a] + 1, mperp, kappa)
    gm = face_g(a, m[:, a] - 1, mperp, kappa)
    return 2.0 * g0 - gp - gm


def face_F_offdiag(a: int, b: int, m: np.ndarray, kappa: float) -> np.ndarray:
    """F^{ab}(m), a != b: orthogonal faces.

    int_{-1}^{1} (1-|t|) [int_{m_a}^{m_a+1} - int_{m_a-1}^{m_a}] dDa
                         [int_{m_b-1}^{m_b} - int_{m_b}^{m_b+1}] dDb  G(Da e_a + Db e_b + (m_c+t) e_c)
    """
    m = np.asarray(m, dtype=np.int64).reshape(-1, 3)
    c = 3 - a - b
    K = m.shape[0]
    los, als, bes = [], [], []
    a_parts = [(m[:, a], 1.0), (m[:, a] - 1, -1.0)]
    b_parts = [(m[:, b] - 1, 1.0), (m[:, b], -1.0)]
    for la, sa in a_parts:
        for lb, sb in b_parts:
            for lc, ac, bc in _tent_boxes(m[:, c]):
                lo = np.empty((K, 3), np.int64)
                al = np.zeros((K, 3))
                be = np.zeros((K, 3))
                lo[:, a], lo[:, b], lo[:, c] = la, lb, lc
                al[:, a], al[:, b] = sa, sb
                al[:, c], be[:, c] = ac, bc
                los.append(lo), als.append(al), bes.append(be)
    vals = box_integrals(np.concatenate(los), np.concatenate(als), np.concatenate(bes), kappa)
    return vals.reshape(8, K).sum(axis=0)


# component order of the 6 unique entries of the symmetric tensor
COMPONENTS = ((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))


def galerkin_N(m: np.ndarray, kappa: float) -> np.ndarray:
    """N^{ab}(m) for the 6 components (order COMPONENTS), shape (6, K).

    ``N^{ab}(m) = delta_ab (delta_{m0} + kappa^2 V(m)) - F^{ab}(m)`` (h = 1)."""
    m = np.asarray(m, dtype=np.int64).reshape(-1, 3)
    V = volume_V(m, kappa)
    is0 = np.all(m == 0, axis=1).astype(np.float64)
    out = np.empty((6, m.shape[0]), dtype=np.complex128)
    for ci, (a, b) in enumerate(COMPONENTS):
        if a == b:
            out[ci] = is0 + kappa * kappa * V - face_F_diag(a, m, kappa)
        else:
            out[ci] = -face_F_offdiag(a, b, m, kappa)
    return out


def parity(a: int, b: int, d: int) -> int:
    """Sign picked up by N^{ab} when the offset along axis d is negated:
    -1 iff exactly one of a, b equals d (the tensor is even in |m| otherwise)."""
    return -1 if ((a == d) != (b == d)) else 1


def _galerkin_chunk(args):
    m, kappa = args
    return galerkin_N(m, kappa)


def green_table(n: Iterable[int], kappa: float, workers: int = 1) -> np.ndarray:
    """Toeplitz table N^{ab}(m) for all non-negative offsets 0 <= m_d < n_d.

    Returns complex128 array of shape (6, n1, n2, n3) (components in COMPONENTS order).
    Entries for negative offsets follow from ``parity``.  workers > 1 evaluates
    slices of offsets along the first axis in that many processes; every entry is
    computed by the same code either way (the vectorised quadrature sums may round
    differently in the last bit with the batch size; tests check agreement to 1e-15)."""
    n1, n2, n3 = n
    g = np.stack(np.meshgrid(np.arange(n1), np.arange(n2), np.arange(n3), indexing="ij"), -1)
    if workers <= 1 or n1 < 2:
        vals = galerkin_N(g.reshape(-1, 3), kappa)
        return vals.reshape(6, n1, n2, n3)
    import concurrent.futures as cf
    import multiprocessing as mp
    jobs = [(g[i].reshape(-1, 3), kappa) for i in range(n1)]
    with cf.ProcessPoolExecutor(max_workers=min(workers, n1), mp_context=mp.get_context("fork")) as ex:
        parts = list(ex.map(_galerkin_chunk, jobs))
    return np.stack([p.reshape(6, n2, n3) for p in parts], axis=1)


def entry(table: np.ndarray, a: int, b: int, m: Tuple[int, int, int]) -> complex:
    """N^{ab}(m) for a signed offset m from a non-negative-offset table."""
    lo, hi = min(a, b), max(a, b)
    ci = COMPONENTS.index((lo, hi))
    s = 1
    for d in range(3):
        if m[d] < 0:
            s *= parity(a, b, d)
    return s * table[ci, abs(m[0]), abs(m[1]), abs(m[2])]
