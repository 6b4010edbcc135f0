"""Solvers for the discrete J-VIE (test infrastructure only).

Section V-D: only matrix-vector products with ``I - M_eps N`` are needed, and
the paper solves with GMRES to a tolerance of 1e-8 (Section V).  The paper does
not say relative to what; the oracle reads it as the 2-norm residual relative
to ||b|| with a zero initial guess, confirmed on the true residual.

* ``solve_lu``  -- dense LU (LAPACK via numpy), the textbook special case.
* ``gmres``     -- restarted GMRES(m): Arnoldi with classical Gram-Schmidt applied
                   twice (CGS2), complex Givens rotations on the Hessenberg matrix.
* ``fgmres``    -- flexible GMRES with a (possibly varying) right preconditioner.
* ``krylov_min_residual`` -- min over x in x0 + K_j(A, r0) of ||b - A x|| by
                   Householder QR of the Krylov basis and least squares.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional

import numpy as np


def solve_lu(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    return np.linalg.solve(A, b)


@dataclasses.dataclass
class SolveInfo:
    iters: int = 0
    restarts: int = 0
    converged: bool = False
    rel_res_true: float = np.inf
    history: List[float] = dataclasses.field(default_factory=list)   # estimated rel. residual per iteration


def _givens(a: complex, b: complex):
    """Rotation [[c, s], [-conj(s), c]] with c real that maps (a, b) to (r, 0)."""
    if b == 0:
        return 1.0, 0.0 + 0.0j, a
    if a == 0:
        return 0.0, 1.0 + 0.0j, b
    t = np.hypot(abs(a), abs(b))
    ph = a / abs(a)
    return abs(a) / t, ph * np.conj(b) / t, ph * t


def fgmres(A: Callable[[np.ndarray], np.ndarray], b: np.ndarray, tol: float = 1e-8,
           restart: int = 50, maxit: int = 10000, x0: Optional[np.ndarray] = None,
           precond: Optional[Callable[[np.ndarray], np.ndarray]] = None):
    """Flexible GMRES(m); with ``precond=None`` this is plain GMRES(m).

    Stops when the relative residual estimate |g_{j+1}|/||b|| <= tol and the true
    relative residual ||b - A x||/||b|| <= tol; otherwise restarts from x."""
    b = np.asarray(b, dtype=np.complex128).ravel()
    n = b.size
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128).ravel()
    bnorm = np.linalg.norm(b)
    info = SolveInfo()
    if bnorm == 0:
        info.converged, info.rel_res_true = True, 0.0
        return np.zeros_like(b), info
    r = b - A(x)
    beta = np.linalg.norm(r)
    while info.iters < maxit:
        if beta / bnorm <= tol:
            info.converged = True
            break
        m = restart
        V = np.zeros((m + 1, n), dtype=np.complex128)
        Z = np.zeros((m, n), dtype=np.complex128) if precond is not None else None
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(m):
            z = precond(V[j]) if precond is not None else V[j]
            if Z is not None:
                Z[j] = z
            w = A(z)
            # classical Gram-Schmidt, twice
            h = V[:j + 1].conj() @ w
            w = w - V[:j + 1].T @ h
            h2 = V[:j + 1].conj() @ w
            w = w - V[:j + 1].T @ h2
            h = h + h2
            hn = np.linalg.norm(w)
            H[:j + 1, j] = h
            H[j + 1, j] = hn
            if hn != 0:
                V[j + 1] = w / hn
            for i in range(j):
                a_, b_ = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a_ + sn[i] * b_
                H[i + 1, j] = -np.conj(sn[i]) * a_ + cs[i] * b_
            c, s, rr = _givens(H[j, j], H[j + 1, j])
            cs[j], sn[j] = c, s
            H[j, j], H[j + 1, j] = rr, 0.0
            g[j + 1] = -np.conj(s) * g[j]
            g[j] = c * g[j]
            info.iters += 1
            j_done = j + 1
            est = abs(g[j + 1]) / bnorm
            info.history.append(est)
            if est <= tol or hn == 0 or info.iters >= maxit:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        basis = Z if Z is not None else V
        x = x + basis[:j_done].T @ y
        r = b - A(x)
        beta = np.linalg.norm(r)
        info.restarts += 1
    info.rel_res_true = float(np.linalg.norm(b - A(x)) / bnorm)
    info.converged = info.rel_res_true <= tol
    return x, info


def gmres(A, b, tol=1e-8, restart=50, maxit=10000, x0=None):
    return fgmres(A, b, tol=tol, restart=restart, maxit=maxit, x0=x0, precond=None)


def krylov_min_residual(A: Callable[[np.ndarray], np.ndarray], b: np.ndarray, jmax: int) -> np.ndarray:
    """min_{x in K_j(A, b)} ||b - A x|| / ||b|| for j = 1..jmax (x0 = 0).

    The basis is grown one vector at a time, each step re-orthonormalised with a
    Householder QR (numpy.linalg.qr) of all columns; the minimisation is a dense
    least-squares solve."""
    b = np.asarray(b, dtype=np.complex128).ravel()
    bn = np.linalg.norm(b)
    Q = (b / bn)[:, None]
    out = []
    for j in range(1, jmax + 1):
        AQ = np.stack([A(Q[:, i]) for i in range(Q.shape[1])], axis=1)
        y, *_ = np.linalg.lstsq(AQ, b, rcond=None)
        out.append(np.linalg.norm(b - AQ @ y) / bn)
        nxt = A(Q[:, -1])
        Q, _ = np.linalg.qr(np.concatenate([Q, nxt[:, None]], axis=1))
    return np.array(out)
