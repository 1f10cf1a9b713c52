"""Pins of the Section 5 oracle (dense tier against the paper's statements and
linear algebra; power-iteration tier against the dense tier)."""
import numpy as np
import pytest

import synth
from oracle import definitional as D
from oracle import oracle as O
from oracle import theory as TH

SHAPES = [(5, 4, 3), (6, 6, 6)]


@pytest.mark.parametrize("shape", SHAPES)
def test_transposed_cycle_swaps_pre_and_post(shape):
    """T(pre, post)^T = T(post, pre): the post-sweeps run the pre-sweeps'
    adjoint order and restriction is the transpose of prolongation (Section 1)."""
    c = (1.0, 1.3, 0.7)
    for pre, post in [(1, 0), (2, 1)]:
        _, T = TH.dense_pair(shape, c, pre, post)
        _, Tt = TH.dense_pair(shape, c, post, pre)
        assert np.abs(T.T - Tt).max() <= 1e-14 * np.abs(T).max()


@pytest.mark.parametrize("shape", SHAPES)
def test_theorem2_prescaling(shape):
    """Balanced SMG is SPD; with c = 2/(lambda_min + lambda_max) of T A the
    three numbers of Theorem 2 coincide: ||I - c A T||_{A^{-1}},
    ||I - c T A||_{T^{-1}} and (kappa - 1)/(kappa + 1); and that c minimises delta."""
    c = tuple((v + 1.0) ** 2 for v in shape)
    A, T = TH.dense_pair(shape, c, 1, 1)
    assert np.abs(T - T.T).max() <= 1e-13 * np.abs(T).max()
    assert np.linalg.eigvalsh(0.5 * (T + T.T)).min() > 0
    lmin, lmax = TH.spectrum_dense(A, T)
    w = np.sort(np.linalg.eigvals(T @ A).real)         # the same spectrum, less accurately
    assert w[0] == pytest.approx(lmin, rel=1e-6) and w[-1] == pytest.approx(lmax, rel=1e-6)
    cs = 2.0 / (lmin + lmax)
    kappa = lmax / lmin
    want = (kappa - 1.0) / (kappa + 1.0)
    assert TH.delta_dense(A, T, cs) == pytest.approx(want, rel=1e-10)
    assert TH.norm_t_inv(A, T, cs) == pytest.approx(want, rel=1e-10)
    cmin, dmin = TH.delta_min_dense(A, T)
    # the minimiser sits at a kink of max|1 - c lambda|: a scalar search finds it to ~1e-7
    assert dmin == pytest.approx(want, rel=1e-6) and cmin == pytest.approx(cs, rel=1e-6)
    assert want < 1.0


@pytest.mark.parametrize("pp", [(1, 1), (1, 0)])
def test_bound3_holds_for_psd(pp):
    """Bound (3): every PSD step contracts ||r||_{A^{-1}} by at most
    min_c ||I - c A T||_{A^{-1}} < 1, with or without post-smoothing."""
    shape = (6, 6, 6)
    c = tuple((v + 1.0) ** 2 for v in shape)
    A, T = TH.dense_pair(shape, c, *pp)
    _, dmin = TH.delta_min_dense(A, T)
    assert dmin < 1.0
    b = synth.rhs(*shape, seed=4)
    xs = np.linalg.solve(A, b)
    S = O.SMG(shape, c, *pp)
    prev = None
    for k in range(6):
        x = O.krylov(O.PSD, b, shape, c, S, rtol=0.0, max_iter=k, history=False).x
        e = xs - x
        ea = np.sqrt(e @ A @ e)
        if prev is not None and prev > 1e-12 * np.sqrt(xs @ A @ xs):
            assert ea <= dmin * prev * (1 + 1e-10)
        prev = ea


@pytest.mark.parametrize("pp", [(1, 1), (1, 0)])
def test_power_iteration_reaches_dense_delta(pp):
    """The power-iteration estimate increases to the dense operator norm."""
    shape = (6, 5, 4)
    c = tuple((v + 1.0) ** 2 for v in shape)
    A, T = TH.dense_pair(shape, c, *pp)
    S, St = O.SMG(shape, c, *pp), O.SMG(shape, c, pp[1], pp[0])
    v0 = synth.uniform_pm1(3, int(np.prod(shape)))
    for cc in (0.8, 1.0, 1.3):
        exact = TH.delta_dense(A, T, cc)
        ests = [TH.delta_power(shape, c, S, St, cc, v0, it) for it in (5, 40, 400)]
        assert all(e <= exact * (1 + 1e-12) for e in ests)
        assert ests[0] <= ests[1] * (1 + 1e-12) <= ests[2] * (1 + 1e-12)
        assert ests[2] == pytest.approx(exact, rel=2e-5)     # slow near a cluster of eigenvalues


def test_power_iteration_reaches_dense_spectrum():
    shape = (6, 5, 4)
    c = tuple((v + 1.0) ** 2 for v in shape)
    A, T = TH.dense_pair(shape, c, 1, 1)
    lmin, lmax = TH.spectrum_dense(A, T)
    v0 = synth.uniform_pm1(5, int(np.prod(shape)))
    plo, phi = TH.spectrum_power(shape, c, O.SMG(shape, c, 1, 1), v0, 600)
    assert phi == pytest.approx(lmax, rel=1e-4)     # lambda_max sits in a cluster: slow
    assert plo == pytest.approx(lmin, rel=1e-4)
    assert plo >= lmin * (1 - 1e-10) and phi <= lmax * (1 + 1e-12)
