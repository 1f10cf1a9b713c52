"""Pins of the oracle's SMG preconditioner (Section 3 reading; Section 1 symmetry claims).

* Galerkin scalars against explicit sparse products P^T A P (3D levels and
  the 2D hierarchies of every plane), plus a hand-derived worked example.
* The whole V-cycle against an explicit-matrix restatement on tiny odd and
  even bricks, for several smoothing counts and both colour orders.
* Operator properties the paper states or relies on: the preconditioner is
  fixed and linear; balanced smoothing gives a symmetric positive definite
  operator, removing post-smoothing makes it nonsymmetric.
* Special cases: one x-line (the cycle is an exact solve); one plane (the
  cycle is one 2D plane cycle); the V-cycle is a convergent iteration whose
  rate does not degrade with refinement.
"""
import numpy as np
import pytest

from oracle import definitional as D
from oracle import oracle as O

TINY = [(4, 4, 4), (5, 4, 3), (3, 5, 9), (6, 7, 8), (1, 1, 6), (7, 1, 1), (2, 9, 1), (8, 8, 8)]


def _block(M, i, j, n):
    return M[i * n:(i + 1) * n, j * n:(j + 1) * n].toarray()


@pytest.mark.parametrize("shape", [(4, 5, 8), (3, 3, 9), (5, 4, 7), (2, 2, 16)])
def test_galerkin_3d_scalars_equal_explicit_ptap(shape):
    c = (1.3, 0.6, 2.2)
    S = O.SMG(shape, c, 1, 1)
    E = D.ExplicitSMG(shape, c, 1, 1)
    nx, ny, _ = shape
    pl = nx * ny
    T2 = (c[0] * np.kron(np.eye(ny), D.tri(nx).toarray())
          + c[1] * np.kron(D.tri(ny).toarray(), np.eye(nx)))
    assert S.nlevels() == len(E.A)
    for l, A in enumerate(E.A):
        nz = S.level_nz(l)
        assert nz == E.nz[l]
        for K in range(nz):
            a, b, g, d = S.plane_coef(l, K)
            assert np.allclose(_block(A, K, K, pl), a * T2 + b * np.eye(pl), rtol=0, atol=1e-14)
            if K + 1 < nz:
                assert np.allclose(_block(A, K, K + 1, pl), g * T2 + d * np.eye(pl), rtol=0, atol=1e-14)
                assert np.allclose(_block(A, K + 1, K, pl), g * T2 + d * np.eye(pl), rtol=0, atol=1e-14)
            for K2 in range(K + 2, nz):
                assert np.abs(_block(A, K, K2, pl)).max() == 0.0


@pytest.mark.parametrize("shape", [(5, 8, 3), (4, 7, 4), (3, 16, 2)])
def test_galerkin_2d_scalars_equal_explicit_ptap(shape):
    c = (0.9, 1.4, 1.1)
    S = O.SMG(shape, c, 1, 1)
    E = D.ExplicitSMG(shape, c, 1, 1)
    nx = shape[0]
    Tx = D.tri(nx).toarray()
    for l in range(S.nlevels()):
        for K in range(S.level_nz(l)):
            Q, _, nyl = E.plane[l][K]
            assert S.plane_nlevels(l, K) == len(Q)
            for l2, Ql in enumerate(Q):
                assert S.plane_level_ny(l, K, l2) == nyl[l2]
                for j in range(nyl[l2]):
                    a, b, cc, d = S.line_coef(l, K, l2, j)
                    assert np.allclose(_block(Ql, j, j, nx), a * Tx + b * np.eye(nx), atol=1e-14, rtol=0)
                    if j + 1 < nyl[l2]:
                        assert np.allclose(_block(Ql, j, j + 1, nx), cc * Tx + d * np.eye(nx),
                                           atol=1e-14, rtol=0)


def test_galerkin_worked_example_unit_coefficients():
    """c = 1, nz = 32.  By hand from D^c = 1/4 D + D + 1/4 D + O + O with
    D = T2 + 2I, O = -I: interior coarse plane 1.5*T2 + 1*I (diagonal 7);
    the last coarse plane lacks fine plane 32, giving 1.25*T2 + 1.5*I
    (diagonal 6.5); couplings 1/2(-I) + 1/4(T2 + 2I) + 1/2(-I) = 0.25*T2 - 0.5*I.
    Every interior row of the coarse operator sums to zero, like the Laplacian."""
    S = O.SMG((8, 8, 32), (1.0, 1.0, 1.0), 1, 1)
    assert S.level_nz(1) == 16
    for K in range(15):
        assert np.array_equal(S.plane_coef(1, K), [1.5, 1.0, 0.25, -0.5])
    assert np.array_equal(S.plane_coef(1, 15)[:2], [1.25, 1.5])
    # row sum of an interior row away from in-plane boundaries: T2 rows sum to 0
    a, b, g, d = S.plane_coef(1, 7)
    assert b + 2 * d == 0.0


@pytest.mark.parametrize("shape", TINY)
@pytest.mark.parametrize("pp", [(1, 1), (1, 0), (2, 1), (0, 1), (1, 2)])
def test_vcycle_equals_explicit_matrix_cycle(shape, pp):
    c = (1.0, 1.9, 0.6)
    S = O.SMG(shape, c, *pp)
    E = D.ExplicitSMG(shape, c, *pp)
    r = np.random.default_rng(7).standard_normal(np.prod(shape))
    a, b = S.apply(r), E.apply(r)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()


@pytest.mark.parametrize("shape", [(5, 6, 7), (8, 8, 8)])
def test_vcycle_colour_order_and_inner_counts(shape):
    c = (1.0, 1.0, 1.0)
    for kw in [dict(order=1), dict(ipre=1, ipost=1, pre=1, post=0), dict(ipre=2, ipost=0, pre=1, post=1)]:
        pre, post = kw.pop("pre", 1), kw.pop("post", 0)
        S = O.SMG(shape, c, pre, post, kw.get("ipre", -1), kw.get("ipost", -1), kw.get("order", 0))
        E = D.ExplicitSMG(shape, c, pre, post, kw.get("ipre"), kw.get("ipost"), kw.get("order", 0))
        r = np.random.default_rng(3).standard_normal(np.prod(shape))
        a, b = S.apply(r), E.apply(r)
        assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()


@pytest.mark.parametrize("n", [8, 16, 24])
def test_balanced_cycle_is_symmetric(n):
    shape, c = (n, n, n), ((n + 1) ** 2,) * 3
    S = O.SMG(shape, c, 1, 1)
    g = np.random.default_rng(n)
    u, v = g.standard_normal(n ** 3), g.standard_normal(n ** 3)
    uBv, vBu = u @ S.apply(v), v @ S.apply(u)
    assert abs(uBv - vBu) <= 1e-12 * abs(uBv)
    assert u @ S.apply(u) > 0


@pytest.mark.parametrize("n", [16, 32])
def test_no_post_smoothing_is_nonsymmetric(n):
    shape, c = (n, n, n), ((n + 1) ** 2,) * 3
    S = O.SMG(shape, c, 1, 0)
    g = np.random.default_rng(n)
    u, v = g.standard_normal(n ** 3), g.standard_normal(n ** 3)
    uBv, vBu = u @ S.apply(v), v @ S.apply(u)
    assert abs(uBv - vBu) > 1e-3 * abs(uBv)


def test_cycle_is_linear():
    shape, c = (9, 7, 10), (1.0, 1.0, 1.0)
    for pp in [(1, 1), (1, 0)]:
        S = O.SMG(shape, c, *pp)
        g = np.random.default_rng(5)
        u, v = g.standard_normal(np.prod(shape)), g.standard_normal(np.prod(shape))
        lhs = S.apply(2.5 * u - 0.75 * v)
        rhs = 2.5 * S.apply(u) - 0.75 * S.apply(v)
        assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(rhs).max()


def test_dense_balanced_preconditioner_is_spd_and_unbalanced_is_not_symmetric():
    shape, c = (5, 5, 5), (36.0, 36.0, 36.0)
    S11, S10 = O.SMG(shape, c, 1, 1), O.SMG(shape, c, 1, 0)
    I = np.eye(125)
    B11 = np.column_stack([S11.apply(e) for e in I])
    B10 = np.column_stack([S10.apply(e) for e in I])
    assert np.abs(B11 - B11.T).max() <= 1e-12 * np.abs(B11).max()
    assert np.linalg.eigvalsh(0.5 * (B11 + B11.T)).min() > 0
    assert np.abs(B10 - B10.T).max() > 1e-3 * np.abs(B10).max()


def test_single_line_brick_is_exact_solve():
    shape, c = (17, 1, 1), (4.0, 1.0, 1.0)
    b = np.random.default_rng(0).standard_normal(17)
    for pp in [(1, 1), (1, 0), (0, 1)]:
        x = O.SMG(shape, c, *pp).apply(b)
        assert np.allclose(x, D.dst_solve(b, shape, c), rtol=1e-13, atol=1e-14)


def test_single_plane_brick_is_one_plane_cycle():
    shape, c = (6, 9, 1), (1.0, 2.0, 3.0)
    S = O.SMG(shape, c, 1, 0)
    b = np.random.default_rng(1).standard_normal(54)
    assert np.array_equal(S.apply(b), S.plane_solve(0, 0, b))
    E = D.ExplicitSMG(shape, c, 1, 0)
    assert np.allclose(S.plane_solve(0, 0, b), E.plane_solve(0, 0, b), rtol=1e-13, atol=1e-14)


def _rho_power(S, shape, c, iters=30):
    """Estimate the spectral radius of I - B A by power iteration."""
    x = np.random.default_rng(11).standard_normal(np.prod(shape))
    rho = 0
    for _ in range(iters):
        y = x - S.apply(O.matvec(x, shape, c))
        rho = np.linalg.norm(y) / np.linalg.norm(x)
        x = y / np.linalg.norm(y)
    return rho


def test_cycle_contracts_independently_of_h():
    rates = []
    for n in (8, 16, 32):
        shape, c = (n, n, n), ((n + 1) ** 2,) * 3
        rates.append(_rho_power(O.SMG(shape, c, 1, 1), shape, c))
    assert max(rates) < 0.5
    assert rates[-1] < rates[0] + 0.15
