"""Pins of the oracle's model operator and line solver (Section 2 model problem).

The oracle's stencil loop is checked against two definitions that share none
of its code: the Kronecker-sum matrix and the closed-form Dirichlet
eigenpairs; its Thomas line solve against a dense LAPACK solve.
"""
import numpy as np
import pytest

from oracle import definitional as D
from oracle import oracle as O

SHAPES = [(1, 1, 1), (5, 1, 1), (1, 6, 1), (1, 1, 7), (4, 5, 6), (9, 3, 2), (8, 8, 8)]


@pytest.mark.parametrize("shape", SHAPES)
def test_matvec_equals_kronecker_sum(shape):
    c = (1.0, 2.5, 0.75)
    x = np.random.default_rng(1).standard_normal(np.prod(shape))
    y = O.matvec(x, shape, c)
    ref = D.laplacian(shape, c) @ x
    assert np.allclose(y, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("shape,abc", [((7, 6, 5), (1, 1, 1)), ((7, 6, 5), (3, 2, 4)),
                                       ((16, 16, 16), (1, 2, 3)), ((10, 1, 3), (10, 1, 2))])
def test_matvec_closed_form_eigenpairs(shape, abc):
    n = shape[0]
    c = ((n + 1) ** 2,) * 3
    v = D.eigenvector(shape, abc)
    lam = D.eigenvalue_of(shape, c, abc)
    Av = O.matvec(v, shape, c)
    assert np.linalg.norm(Av - lam * v) <= 1e-13 * lam * np.linalg.norm(v)


def test_dst_solve_equals_dense_solve():
    shape, c = (5, 4, 6), (1.0, 1.7, 0.4)
    b = np.random.default_rng(2).standard_normal(np.prod(shape))
    x = D.dst_solve(b, shape, c)
    ref = np.linalg.solve(D.laplacian(shape, c).toarray(), b)
    assert np.allclose(x, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 257])
@pytest.mark.parametrize("a,b", [(1.0, 2.0), (3.5, 0.1), (1.0, 0.0), (0.0, 2.0)])
def test_line_solve_equals_dense(n, a, b):
    f = np.random.default_rng(n).standard_normal(n)
    u = O.line_solve(a, b, f)
    M = a * D.tri(n).toarray() + b * np.eye(n)
    ref = np.linalg.solve(M, f)
    cond = np.linalg.cond(M)
    assert np.linalg.norm(u - ref) <= 1e-15 * cond * np.linalg.norm(ref) + 1e-300
