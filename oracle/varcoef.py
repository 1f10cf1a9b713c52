"""Variable-coefficient SMG in plain FP64 with explicit sparse matrices.
TEST INFRASTRUCTURE ONLY.

The paper runs SMG, which was designed for general structured-grid problems
(Section 1, Schaffer's semicoarsening multigrid), on the constant 7-point
Laplacian.  This oracle extends the constant-coefficient reading of the C
oracle to a general symmetric 7-point operator given per point:
    (A x)_p = diag_p x_p - sum over axes e of (a_e[p] x_{p+e} + a_e[p-e] x_{p-e}),
with a_e[p] = 0 where p+e leaves the brick.  Everything below is a definition
written with scipy.sparse matrices, so a reader can check each step:

* 3D hierarchy: z-semicoarsening by two (coarse planes = odd fine planes),
  prolongation P with one weight per point of every even (F) plane for each
  of its C-plane neighbours, coarse operator P^T A P (Galerkin).
* Interpolation weights.  "linear": 1/2 from each neighbouring C-plane.
  "operator": from the collapsed couplings of the F-point's row to the two
  planes, a = -(sum of the row's entries in the plane below) and b = -(sum in
  the plane above), weights a/(a+b) and b/(a+b) (a flux-matching choice that
  follows jumps of the coefficient across planes).  An F-plane with a single
  C-neighbour takes 1/2 from it (as linear interpolation does), and a point
  whose collapsed couplings are not both positive falls back to 1/2 each.
* Plane solve: one 2D V-cycle of the plane's own operator A[k, k] built by the
  same rules in y with x-lines, whose line blocks are solved exactly.
* Relaxation, V-cycle and smoothing order exactly as in the constant case:
  correction form, pre F then C, post C then F, x = 0 at the start of every
  level, coarsest 3D level one plane solve, coarsest 2D level one line solve.

With constant coefficients and "linear" weights every operator equals the C
oracle's (a pin); "operator" weights equal 1/2 there too on bricks whose nz
(and ny) are 2^m or 2^m - 1.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def operator(shape, diag, ax, ay, az) -> sp.csr_matrix:
    """The sparse matrix of the 7-point operator (index i + nx (j + ny k))."""
    nx, ny, nz = shape
    n = nx * ny * nz
    idx = np.arange(n)
    i = idx % nx
    j = (idx // nx) % ny
    k = idx // (nx * ny)
    rows, cols, vals = [idx], [idx], [np.asarray(diag, dtype=np.float64)]
    for a, ok, step in ((ax, i < nx - 1, 1), (ay, j < ny - 1, nx), (az, k < nz - 1, nx * ny)):
        a = np.asarray(a, dtype=np.float64)
        p = idx[ok]
        rows += [p, p + step]
        cols += [p + step, p]
        vals += [-a[p], -a[p]]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def _blocks(n_outer: int, m: int):
    """Index ranges of the n_outer blocks (planes or lines) of m points."""
    return [np.arange(b * m, (b + 1) * m) for b in range(n_outer)]


def prolongation(A: sp.csr_matrix, n_outer: int, m: int, weights: str) -> sp.csr_matrix:
    """Semicoarsening prolongation along the outer index of A (blocks of m
    points): coarse block K sits on fine block 2K+1; fine block 2K gets w_dn
    times coarse K-1 and w_up times coarse K (per point)."""
    nc = n_outer // 2
    A = A.tocsr()
    rows, cols, vals = [], [], []
    for f in range(n_outer):
        fi = np.arange(f * m, (f + 1) * m)
        if f % 2 == 1:
            K = f // 2
            rows.append(fi)
            cols.append(K * m + np.arange(m))
            vals.append(np.ones(m))
            continue
        has_dn = f - 1 >= 0
        has_up = f + 1 < n_outer
        if not has_dn and not has_up:
            continue
        wdn = np.full(m, 0.5 if has_dn else 0.0)
        wup = np.full(m, 0.5 if has_up else 0.0)
        if weights == "operator" and has_dn and has_up:
            a = -np.asarray(A[fi][:, (f - 1) * m:f * m].sum(axis=1)).ravel()
            b = -np.asarray(A[fi][:, (f + 1) * m:(f + 2) * m].sum(axis=1)).ravel()
            ok = (a > 0) & (b > 0)
            wdn = np.where(ok, a / np.where(ok, a + b, 1.0), 0.5)
            wup = np.where(ok, b / np.where(ok, a + b, 1.0), 0.5)
        if has_dn:
            rows.append(fi)
            cols.append((f // 2 - 1) * m + np.arange(m))
            vals.append(wdn)
        if has_up:
            rows.append(fi)
            cols.append((f // 2) * m + np.arange(m))
            vals.append(wup)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n_outer * m, nc * m))


class Hier2D:
    """2D semicoarsening hierarchy of a plane operator Q (ny lines of nx points)."""

    def __init__(self, Q: sp.csr_matrix, nx: int, ny: int, weights: str):
        self.nx = nx
        self.ops, self.P, self.ny = [Q.tocsr()], [], [ny]
        while self.ny[-1] > 1:
            P = prolongation(self.ops[-1], self.ny[-1], nx, weights)
            self.P.append(P)
            self.ops.append((P.T @ self.ops[-1] @ P).tocsr())
            self.ny.append(self.ny[-1] // 2)
        # the line blocks of each colour, factorised once (exact line solves)
        self.lu = []
        for Ql, nyl in zip(self.ops, self.ny):
            per = []
            for colour in (0, 1):
                ids = np.concatenate([np.arange(j * nx, (j + 1) * nx) for j in range(colour, nyl, 2)]) \
                    if colour < nyl else np.zeros(0, dtype=np.int64)
                per.append((ids, spla.splu(Ql[ids][:, ids].tocsc()) if ids.size else None))
            self.lu.append(per)

    def sweep(self, l, colour, b, x):
        ids, lu = self.lu[l][colour]
        if lu is None:
            return
        r = b - self.ops[l] @ x
        x[ids] += lu.solve(r[ids])

    def vcycle(self, l, b, pre, post, order=0):
        Q = self.ops[l]
        if self.ny[l] == 1:
            return spla.spsolve(Q.tocsc(), b) if Q.shape[0] > 1 else b / Q.toarray()[0, 0]
        first, second = (0, 1) if order == 0 else (1, 0)
        x = np.zeros_like(b)
        for _ in range(pre):
            self.sweep(l, first, b, x)
            self.sweep(l, second, b, x)
        P = self.P[l]
        x += P @ self.vcycle(l + 1, P.T @ (b - Q @ x), pre, post, order)
        for _ in range(post):
            self.sweep(l, second, b, x)
            self.sweep(l, first, b, x)
        return x


class VarSMG:
    """The SMG V-cycle preconditioner T of a variable-coefficient 7-point operator."""

    def __init__(self, shape, diag, ax, ay, az, pre=1, post=1, ipre=-1, ipost=-1, order=0, weights="operator"):
        self.shape = tuple(int(v) for v in shape)
        nx, ny, nz = self.shape
        self.pre, self.post = pre, post
        self.ipre = pre if ipre < 0 else ipre
        self.ipost = post if ipost < 0 else ipost
        self.order = order
        self.weights = weights
        self.A = operator(self.shape, diag, ax, ay, az)
        m = nx * ny
        self.ops, self.P, self.nz = [self.A], [], [nz]
        while self.nz[-1] > 1:
            P = prolongation(self.ops[-1], self.nz[-1], m, weights)
            self.P.append(P)
            self.ops.append((P.T @ self.ops[-1] @ P).tocsr())
            self.nz.append(self.nz[-1] // 2)
        self.planes = []
        for Al, nzl in zip(self.ops, self.nz):
            self.planes.append([Hier2D(Al[blk][:, blk], nx, ny, weights) for blk in _blocks(nzl, m)])

    def _sweep(self, l, colour, b, x):
        m = self.shape[0] * self.shape[1]
        r = b - self.ops[l] @ x
        for k in range(colour, self.nz[l], 2):
            s = slice(k * m, (k + 1) * m)
            x[s] += self.planes[l][k].vcycle(0, r[s], self.ipre, self.ipost, self.order)

    def _vcycle(self, l, b):
        if self.nz[l] == 1:
            return self.planes[l][0].vcycle(0, b, self.ipre, self.ipost, self.order)
        first, second = (0, 1) if self.order == 0 else (1, 0)
        x = np.zeros_like(b)
        for _ in range(self.pre):
            self._sweep(l, first, b, x)
            self._sweep(l, second, b, x)
        P = self.P[l]
        x += P @ self._vcycle(l + 1, P.T @ (b - self.ops[l] @ x))
        for _ in range(self.post):
            self._sweep(l, second, b, x)
            self._sweep(l, first, b, x)
        return x

    def apply(self, r):
        return self._vcycle(0, np.asarray(r, dtype=np.float64).ravel())

    def matvec(self, x):
        return self.A @ np.asarray(x, dtype=np.float64).ravel()


def krylov(method: str, b, A_apply, T_apply, x0=None, rtol=1e-8, max_iter=500):
    """Algorithm 1 of Section 2 with beta from equation (1) ("pcg"), (2)
    ("fpcg", r_{k-1} stored) or 0 ("psd"); stops when ||r_k||_2 <= rtol ||b||_2.
    Returns (x, iterations, relative residual history, status 0/1)."""
    b = np.asarray(b, dtype=np.float64).ravel()
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64).ravel()
    r = b - A_apply(x)
    bden = np.linalg.norm(b) or 1.0
    rels = [np.linalg.norm(r) / bden]
    p = r_prev = None
    sr_prev = 0.0
    k = 0
    while k < max_iter and rels[-1] > rtol:
        s = T_apply(r)
        sr = float(s @ r)
        if k == 0 or method == "psd":
            p = s.copy()
        else:
            num = sr if method == "pcg" else sr - float(s @ r_prev)
            p = s + (num / sr_prev) * p
        q = A_apply(p)
        alpha = sr / float(p @ q)
        r_prev = r
        x = x + alpha * p
        r = r - alpha * q
        sr_prev = sr
        rels.append(np.linalg.norm(r) / bden)
        k += 1
    return x, k, np.array(rels), 0 if rels[-1] <= rtol else 1
