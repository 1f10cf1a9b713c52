"""Definitional forms of the method's objects with explicit sparse/dense matrices.

TEST INFRASTRUCTURE ONLY.  These are slow, tiny-grid restatements written
straight from the definitions, used to pin the C oracle:

* the model operator of Section 2 as a Kronecker sum, its closed-form
  eigenpairs and its exact inverse by the three-dimensional sine transform;
* semicoarsening prolongations P (coarse points on odd fine indices, linear
  weights 1/2 on the even neighbours) and Galerkin coarse operators formed as
  explicit products P^T A P;
* the SMG V-cycle read as in the C oracle, but written with explicit matrix
  slices and dense solves instead of stencil recurrences.
"""
from __future__ import annotations

import numpy as np
import scipy.fft
import scipy.sparse as sp


def tri(n: int) -> sp.csr_matrix:
    """T = tridiag(-1, 2, -1) of order n (Dirichlet second difference)."""
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")


def laplacian(shape, c=(1.0, 1.0, 1.0)) -> sp.csr_matrix:
    """A = cx*Tx (+) cy*Ty (+) cz*Tz with x fastest: I_z (x) I_y (x) Tx etc."""
    nx, ny, nz = shape
    Ix, Iy, Iz = sp.identity(nx), sp.identity(ny), sp.identity(nz)
    A = (c[0] * sp.kron(Iz, sp.kron(Iy, tri(nx)))
         + c[1] * sp.kron(Iz, sp.kron(tri(ny), Ix))
         + c[2] * sp.kron(tri(nz), sp.kron(Iy, Ix)))
    return A.tocsr()


def eig1(n: int, a: int, h_scale: float = 1.0):
    """a-th (1-based) eigenpair of tridiag(-1,2,-1) of order n."""
    t = np.arange(1, n + 1)
    v = np.sin(a * np.pi * t / (n + 1))
    lam = 4.0 * np.sin(a * np.pi / (2 * (n + 1))) ** 2
    return lam * h_scale, v


def eigenvalues(shape, c=(1.0, 1.0, 1.0)) -> np.ndarray:
    """All eigenvalues of A, ascending, with multiplicity."""
    nx, ny, nz = shape
    lx = c[0] * 4 * np.sin(np.arange(1, nx + 1) * np.pi / (2 * (nx + 1))) ** 2
    ly = c[1] * 4 * np.sin(np.arange(1, ny + 1) * np.pi / (2 * (ny + 1))) ** 2
    lz = c[2] * 4 * np.sin(np.arange(1, nz + 1) * np.pi / (2 * (nz + 1))) ** 2
    return np.sort((lz[:, None, None] + ly[None, :, None] + lx[None, None, :]).reshape(-1))


def smallest_eigenvalues(shape, c, m: int) -> np.ndarray:
    """The m smallest eigenvalues without forming all n of them (uses a bounded index box)."""
    nx, ny, nz = shape
    kx, ky, kz = min(nx, m), min(ny, m), min(nz, m)
    lx = c[0] * 4 * np.sin(np.arange(1, kx + 1) * np.pi / (2 * (nx + 1))) ** 2
    ly = c[1] * 4 * np.sin(np.arange(1, ky + 1) * np.pi / (2 * (ny + 1))) ** 2
    lz = c[2] * 4 * np.sin(np.arange(1, kz + 1) * np.pi / (2 * (nz + 1))) ** 2
    return np.sort((lz[:, None, None] + ly[None, :, None] + lx[None, None, :]).reshape(-1))[:m]


def eigenvector(shape, abc) -> np.ndarray:
    """Closed-form eigenvector with mode numbers (a, b, c), flattened x fastest."""
    nx, ny, nz = shape
    a, b, cc = abc
    vx = np.sin(a * np.pi * np.arange(1, nx + 1) / (nx + 1))
    vy = np.sin(b * np.pi * np.arange(1, ny + 1) / (ny + 1))
    vz = np.sin(cc * np.pi * np.arange(1, nz + 1) / (nz + 1))
    return (vz[:, None, None] * vy[None, :, None] * vx[None, None, :]).reshape(-1)


def eigenvalue_of(shape, c, abc) -> float:
    nx, ny, nz = shape
    a, b, cc = abc
    return (c[0] * 4 * np.sin(a * np.pi / (2 * (nx + 1))) ** 2
            + c[1] * 4 * np.sin(b * np.pi / (2 * (ny + 1))) ** 2
            + c[2] * 4 * np.sin(cc * np.pi / (2 * (nz + 1))) ** 2)


def dst_solve(b: np.ndarray, shape, c=(1.0, 1.0, 1.0)) -> np.ndarray:
    """x = A^{-1} b by diagonalising A with the type-I sine transform in each axis."""
    nx, ny, nz = shape
    B = b.reshape(nz, ny, nx)
    Bh = scipy.fft.dstn(B, type=1, norm="ortho")
    lx = c[0] * 4 * np.sin(np.arange(1, nx + 1) * np.pi / (2 * (nx + 1))) ** 2
    ly = c[1] * 4 * np.sin(np.arange(1, ny + 1) * np.pi / (2 * (ny + 1))) ** 2
    lz = c[2] * 4 * np.sin(np.arange(1, nz + 1) * np.pi / (2 * (nz + 1))) ** 2
    lam = lz[:, None, None] + ly[None, :, None] + lx[None, None, :]
    return scipy.fft.idstn(Bh / lam, type=1, norm="ortho").reshape(-1)


def prolongation_1d(n: int) -> sp.csr_matrix:
    """P (n by n//2): coarse K -> fine 2K+1 with weight 1, fine 2K and 2K+2 with 1/2."""
    nc = n // 2
    rows, cols, vals = [], [], []
    for K in range(nc):
        for f, w in ((2 * K, 0.5), (2 * K + 1, 1.0), (2 * K + 2, 0.5)):
            if f < n:
                rows.append(f); cols.append(K); vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, nc))


def prolongation_z(shape) -> sp.csr_matrix:
    nx, ny, nz = shape
    return sp.kron(prolongation_1d(nz), sp.identity(nx * ny)).tocsr()


def prolongation_y(nx: int, ny: int) -> sp.csr_matrix:
    return sp.kron(prolongation_1d(ny), sp.identity(nx)).tocsr()


class ExplicitSMG:
    """SMG V-cycle with explicit Galerkin products and dense block solves (tiny grids)."""

    def __init__(self, shape, c=(1.0, 1.0, 1.0), pre=1, post=1, ipre=None, ipost=None, order=0):
        self.shape = tuple(shape)
        nx, ny, nz = shape
        self.nx, self.ny = nx, ny
        self.pre, self.post = pre, post
        self.ipre = pre if ipre is None else ipre
        self.ipost = post if ipost is None else ipost
        self.order = order
        self.A = [laplacian(shape, c)]
        self.P = []
        self.nz = [nz]
        while self.nz[-1] > 1:
            P = prolongation_z((nx, ny, self.nz[-1]))
            self.P.append(P)
            self.A.append((P.T @ self.A[-1] @ P).tocsr())
            self.nz.append(self.nz[-1] // 2)
        self.pl = nx * ny
        # plane hierarchies: per level, per plane, list of 2D operators and prolongations
        self.plane = []
        for l, A in enumerate(self.A):
            planes = []
            for k in range(self.nz[l]):
                blk = A[k * self.pl:(k + 1) * self.pl, k * self.pl:(k + 1) * self.pl].tocsr()
                Q, Py, nyl = [blk], [], [ny]
                while nyl[-1] > 1:
                    P2 = prolongation_y(nx, nyl[-1])
                    Py.append(P2)
                    Q.append((P2.T @ Q[-1] @ P2).tocsr())
                    nyl.append(nyl[-1] // 2)
                planes.append((Q, Py, nyl))
            self.plane.append(planes)

    def _colours(self):
        first = 0 if self.order == 0 else 1
        return first, 1 - first

    def _v2(self, Q, Py, nyl, l, b):
        nx = self.nx
        if nyl[l] == 1:
            return np.linalg.solve(Q[l].toarray(), b)
        x = np.zeros_like(b)
        f, s = self._colours()

        def sweep(col):
            for j in range(col, nyl[l], 2):
                sl = slice(j * nx, (j + 1) * nx)
                r = (b - Q[l] @ x)[sl]
                x[sl] += np.linalg.solve(Q[l][sl, sl].toarray(), r)

        for _ in range(self.ipre):
            sweep(f); sweep(s)
        xc = self._v2(Q, Py, nyl, l + 1, Py[l].T @ (b - Q[l] @ x))
        x += Py[l] @ xc
        for _ in range(self.ipost):
            sweep(s); sweep(f)
        return x

    def plane_solve(self, l, k, b):
        Q, Py, nyl = self.plane[l][k]
        return self._v2(Q, Py, nyl, 0, b)

    def _v3(self, l, b):
        if self.nz[l] == 1:
            return self.plane_solve(l, 0, b)
        A, pl = self.A[l], self.pl
        x = np.zeros_like(b)
        f, s = self._colours()

        def sweep(col):
            r = b - A @ x
            for k in range(col, self.nz[l], 2):
                sl = slice(k * pl, (k + 1) * pl)
                x[sl] += self.plane_solve(l, k, r[sl])

        for _ in range(self.pre):
            sweep(f); sweep(s)
        xc = self._v3(l + 1, self.P[l].T @ (b - A @ x))
        x += self.P[l] @ xc
        for _ in range(self.post):
            sweep(s); sweep(f)
        return x

    def apply(self, r):
        return self._v3(0, np.asarray(r, dtype=np.float64).reshape(-1))

    def dense(self) -> np.ndarray:
        n = self.A[0].shape[0]
        return np.column_stack([self.apply(e) for e in np.eye(n)])
