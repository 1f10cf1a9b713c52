"""LOBPCG oracle (Section 4: the m smallest eigenpairs of the model Laplacian,
preconditioned by SMG).  TEST INFRASTRUCTURE ONLY.

The paper runs BLOPEX's LOBPCG; this is the published locally optimal block
preconditioned conjugate gradient method (Knyazev 2001) written from its
definition, in FP64, with the small dense steps done by NumPy (Cholesky,
symmetric eigensolver) and the operator and preconditioner applied column by
column through the C oracle:

1. orthonormalise the initial block X (Cholesky QR, twice) and take Ritz
   pairs of X^T A X;
2. each iteration: residuals R = A X - X diag(theta); columns whose relative
   residual ||r_i|| / (|theta_i| ||x_i||) exceeds rtol are active; the
   preconditioned residuals W = T R_active and the previous directions
   P_active extend the trial basis S = [X, W, P];
3. S is orthonormalised (Cholesky QR twice; if S^T S is numerically singular,
   P and then W directions are dropped through an eigen-decomposition of the
   Gram matrix), the same transform is applied to A S, and the m smallest
   Ritz pairs of S^T A S give the new X, A X and the new directions P (the
   W and P parts of the Ritz vectors).

Converged columns stay in X and in the Rayleigh-Ritz basis but generate no
new directions ("soft locking").
"""
from __future__ import annotations

import numpy as np


def _cholqr(S, AS):
    """Orthonormalise the columns of S (and transform A S alike); None if singular."""
    for _ in range(2):
        G = S.T @ S
        G = 0.5 * (G + G.T)
        try:
            L = np.linalg.cholesky(G)
        except np.linalg.LinAlgError:
            return None
        if np.linalg.cond(L) ** 2 > 1e14:
            return None
        Linv_T = np.linalg.inv(L).T
        S = S @ Linv_T
        AS = AS @ Linv_T
    return S, AS


def _svqb(S, AS, drop=1e-12):
    """Eigen-based orthonormalisation keeping directions above a relative threshold."""
    G = S.T @ S
    d = np.sqrt(np.abs(np.diag(G)))
    d[d == 0] = 1.0
    Gs = G / d[:, None] / d[None, :]
    w, V = np.linalg.eigh(0.5 * (Gs + Gs.T))
    keep = w > drop * w.max()
    T = (V[:, keep] / np.sqrt(w[keep])) / d[:, None]
    return S @ T, AS @ T


def lobpcg(apply_A, apply_T, X0: np.ndarray, rtol=1e-8, max_iter=500, history=None):
    """X0: (m, n) array, one initial vector per row.  apply_A/apply_T map an
    (k, n) block to an (k, n) block.  Returns (theta, X (m, n), iters, res)."""
    X = np.array(X0, dtype=np.float64).T.copy()          # n x m, columns are vectors
    n, m = X.shape
    AX = apply_A(X.T).T
    out = _cholqr(X, AX)
    if out is None:
        X, AX = _svqb(X, AX)
    else:
        X, AX = out
    G = X.T @ AX
    theta, C = np.linalg.eigh(0.5 * (G + G.T))
    X, AX = X @ C, AX @ C
    P = AP = None
    it = 0
    res = None
    for it in range(max_iter + 1):
        R = AX - X * theta[None, :]
        res = np.linalg.norm(R, axis=0) / (np.abs(theta) * np.linalg.norm(X, axis=0))
        if history is not None:
            history.append((theta.copy(), res.copy()))
        active = np.nonzero(res > rtol)[0]
        if active.size == 0 or it == max_iter:
            break
        W = apply_T(R[:, active].T).T
        W = W / np.linalg.norm(W, axis=0)[None, :]      # unit columns: keeps S^T S well scaled
        AW = apply_A(W.T).T
        blocks, ablocks = [X, W], [AX, AW]
        if P is not None:
            pn = np.linalg.norm(P[:, active], axis=0)[None, :]
            blocks.append(P[:, active] / pn)
            ablocks.append(AP[:, active] / pn)
        S, AS = np.hstack(blocks), np.hstack(ablocks)
        out = _cholqr(S, AS)
        if out is None and P is not None:          # drop P
            out = _cholqr(np.hstack(blocks[:2]), np.hstack(ablocks[:2]))
        if out is None:
            S, AS = _svqb(S, AS)
        else:
            S, AS = out
        G = S.T @ AS
        w, C = np.linalg.eigh(0.5 * (G + G.T))
        theta, Cm = w[:m], C[:, :m]
        Xn, AXn = S @ Cm, AS @ Cm
        # new directions: the part of the Ritz vectors outside span(X) basis columns
        P = S[:, m:] @ Cm[m:, :]
        AP = AS[:, m:] @ Cm[m:, :]
        X, AX = Xn, AXn
    return theta, X.T.copy(), it, res
