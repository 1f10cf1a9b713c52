"""Pins of the LOBPCG oracle (Section 4) against what the mathematics fixes:
closed-form Dirichlet eigenvalues (with multiplicity), eigenvectors spanning
the closed-form eigenspaces, orthonormal Ritz vectors, monotone Ritz values
(Courant-Fischer: the trial subspace always contains the previous X), and the
Section 4 observation that dropping post-smoothing costs some extra iterations.
"""
import numpy as np
import pytest

import synth
from oracle import definitional as D
from oracle import lobpcg as LB
from oracle import oracle as O


def _run(n, m, pp, seed=3, rtol=1e-8, max_iter=300, history=None):
    shape, c = (n, n, n), ((n + 1.0) ** 2,) * 3
    S = O.SMG(shape, c, *pp)
    A = lambda Y: np.stack([O.matvec(y, shape, c) for y in Y])
    T = lambda Y: np.stack([S.apply(y) for y in Y])
    return LB.lobpcg(A, T, synth.block(n ** 3, m, seed), rtol=rtol, max_iter=max_iter, history=history)


def _eigvecs_upto(n, lam_max, c):
    """Orthonormal closed-form eigenvectors with eigenvalue <= lam_max."""
    shape = (n, n, n)
    vs = []
    for a in range(1, n + 1):
        for b in range(1, n + 1):
            for cc in range(1, n + 1):
                if D.eigenvalue_of(shape, c, (a, b, cc)) <= lam_max * (1 + 1e-12):
                    v = D.eigenvector(shape, (a, b, cc))
                    vs.append(v / np.linalg.norm(v))
    return np.array(vs)


@pytest.mark.parametrize("n,m,pp", [(8, 1, (1, 0)), (10, 4, (1, 1)), (12, 10, (1, 0)), (12, 16, (1, 0)),
                                    (12, 16, (1, 1))])
def test_eigenpairs_match_closed_form(n, m, pp):
    c = ((n + 1.0) ** 2,) * 3
    h = []
    theta, X, it, res = _run(n, m, pp, history=h)
    ex = D.smallest_eigenvalues((n, n, n), c, m)
    assert np.max(np.abs(theta - ex) / ex) <= 1e-10
    assert res.max() <= 1e-8
    assert np.abs(X @ X.T - np.eye(m)).max() <= 1e-12
    # Ritz values never increase (span of the old X is inside the new trial basis)
    ths = np.array([t for t, _ in h])
    assert np.all(np.diff(ths, axis=0) <= 1e-12 * ths[0][None, :])
    # X lies in the span of the closed-form eigenvectors up to lambda_m, whole cluster included
    V = _eigvecs_upto(n, ex[-1], c)
    assert V.shape[0] >= m
    resid = X.T - V.T @ (V @ X.T)
    assert np.linalg.norm(resid, axis=0).max() <= 1e-7


def test_dense_eigensolver_agrees_on_tiny_grid():
    n, m = 6, 5
    c = (49.0,) * 3
    theta, X, _, _ = _run(n, m, (1, 1))
    lam = np.linalg.eigvalsh(D.laplacian((n, n, n), c).toarray())[:m]
    assert np.allclose(theta, lam, rtol=1e-11)


def test_no_post_smoothing_costs_iterations_but_converges():
    """Section 4: without post-relaxation LOBPCG needs more, but not vastly more, iterations."""
    it11 = _run(16, 16, (1, 1))[2]
    it10 = _run(16, 16, (1, 0))[2]
    assert it11 < it10 <= 2 * it11
