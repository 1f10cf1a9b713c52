"""Section 5 of the paper in plain FP64: the preconditioner quality of
assumption (4) and the quantities of Theorems 1 and 2.  TEST INFRASTRUCTURE
ONLY.

Definitions used (A SPD, T the SMG V-cycle, possibly nonsymmetric):
* ||x||_{A^{-1}} = sqrt(x' A^{-1} x); the induced operator norm satisfies
  ||M||_{A^{-1}} = ||A^{-1/2} M A^{1/2}||_2.
* Assumption (4): ||I - A T||_{A^{-1}} <= delta < 1; scaling T by c,
  delta(c) = ||I - c A T||_{A^{-1}}, and delta_min = min_c delta(c) is the
  scaling-free measure (PSD and PCG are invariant to scaling T).
* Bound (3): one PSD step contracts ||r||_{A^{-1}} by at most delta(c) for
  every c (the step's exact line search absorbs the scaling).
* Theorem 2 (T SPD): with c chosen so that max Lambda(c T A) + min
  Lambda(c T A) = 2, delta = (kappa - 1)/(kappa + 1), kappa = kappa(T A), and
  ||I - c T A||_{T^{-1}} gives the same number.

Two tiers: dense matrices (grids up to about 8^3: A from the C oracle's
stencil applied to the identity, T likewise from its V-cycle), and power
iterations that only apply A, T and T's transpose to vectors (any size).
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O


def dense_operator(apply, n):
    """The matrix of a linear map given on vectors (column j = apply(e_j))."""
    return np.stack([apply(e) for e in np.eye(n)], axis=1)


def dense_pair(shape, c, pre, post):
    n = int(np.prod(shape))
    A = dense_operator(lambda v: O.matvec(v, shape, c), n)
    S = O.SMG(shape, c, pre, post)
    T = dense_operator(S.apply, n)
    return A, T


def _sqrt_and_inv_sqrt(A):
    w, V = np.linalg.eigh(0.5 * (A + A.T))
    return (V * np.sqrt(w)) @ V.T, (V / np.sqrt(w)) @ V.T


def delta_dense(A, T, c):
    """||I - c A T||_{A^{-1}} = ||A^{-1/2} (I - c A T) A^{1/2}||_2."""
    Ah, Aih = _sqrt_and_inv_sqrt(A)
    M = np.eye(A.shape[0]) - c * (A @ T)
    return float(np.linalg.norm(Aih @ M @ Ah, 2))


def delta_min_dense(A, T, lo=0.2, hi=3.0):
    """(c, min_c delta(c)); delta(c) is convex in c."""
    from scipy.optimize import minimize_scalar
    r = minimize_scalar(lambda cc: delta_dense(A, T, cc), bounds=(lo, hi), method="bounded",
                        options={"xatol": 1e-10})
    return float(r.x), float(r.fun)


def spectrum_dense(A, T):
    """Extreme eigenvalues of T A for SPD T, from the similar symmetric matrix
    A^{1/2} T A^{1/2} (a nonsymmetric eigensolver loses accuracy on the large
    cluster of eigenvalues near 1 that a good multigrid cycle produces)."""
    assert np.abs(T - T.T).max() <= 1e-12 * np.abs(T).max()
    Ah, _ = _sqrt_and_inv_sqrt(A)
    w = np.linalg.eigvalsh(Ah @ (0.5 * (T + T.T)) @ Ah)
    return float(w[0]), float(w[-1])


def norm_t_inv(A, T, c):
    """||I - c T A||_{T^{-1}} = ||T^{-1/2} (I - c T A) T^{1/2}||_2 (T SPD), Theorem 2's form."""
    Th, Tih = _sqrt_and_inv_sqrt(T)
    M = np.eye(A.shape[0]) - c * (T @ A)
    return float(np.linalg.norm(Tih @ M @ Th, 2))


def delta_power(shape, c_grid, S, St, c, v0, iters):
    """delta(c) by power iteration on E# E in the A inner product, E = I - c T A,
    E# = I - c T^T A (St applies T^T); the same steps as the library's estimate:
    u = E v with ||v||_A = 1 gives delta^2 ~ (u, A u); then v = E# u, normalised."""
    A = lambda x: O.matvec(x, shape, c_grid)
    v = np.array(v0, dtype=np.float64)
    w = A(v)
    s = 1.0 / np.sqrt(v @ w)
    v, w = v * s, w * s
    q = 0.0
    for it in range(iters):
        u = v - c * S.apply(w)
        au = A(u)
        q = float(u @ au)
        if it + 1 == iters:
            break
        v = u - c * St.apply(au)
        w = A(v)
        yy = float(v @ w)
        if not yy > 0.0:
            break
        s = 1.0 / np.sqrt(yy)
        v, w = v * s, w * s
    return float(np.sqrt(abs(q)))


def spectrum_power(shape, c_grid, S, v0, iters):
    """(lambda_min, lambda_max) of T A for SPD T: power iteration on T A, then
    on lambda_max I - T A, in the A inner product (Rayleigh quotients)."""
    A = lambda x: O.matvec(x, shape, c_grid)

    def power(shift):
        v = np.array(v0, dtype=np.float64)
        w = A(v)
        s = 1.0 / np.sqrt(v @ w)
        v, w = v * s, w * s
        q = 0.0
        for it in range(iters):
            t = S.apply(w)
            q = shift - float(w @ t)
            if it + 1 == iters:
                break
            v = shift * v - t
            w = A(v)
            yy = float(v @ w)
            if not yy > 0.0:
                break
            s = 1.0 / np.sqrt(yy)
            v, w = v * s, w * s
        return q

    lmax = -power(0.0)
    return lmax - power(lmax), lmax
