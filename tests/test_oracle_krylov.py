"""Pins of the oracle's Algorithm 1 (Section 2) and of the paper's observations (Sections 3 and 5).

* Without preconditioning, beta from (1) and from (2) give the same CG
  (Section 2, Figure 2), which ends, up to rounding, within as many steps as
  the right-hand side has distinct eigen-components.
* Theorem 1 (Section 5): one PSD step contracts the A^{-1}-norm of the
  residual by exactly sin of the A^{-1}-angle between r and A T r.
* Local optimality (Section 5): a flexible-PCG step is never worse in the
  A-norm of the error than a PSD step from the same iterate.
* The iterates converge to the exact solution given by the sine transform.
* Section 3 observations: with balanced SMG the two PCG variants coincide and
  PSD needs a few more steps; without post-smoothing the standard PCG stalls
  while flexible PCG and PSD stay close.  The paper's printed Figure 5 and
  Figure 7 data show the same relations (golden fixtures).
"""
import os

import numpy as np
import pytest

import synth
from oracle import definitional as D
from oracle import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _problem(n, seed=1):
    shape = (n, n, n)
    c = ((n + 1) ** 2,) * 3
    return shape, c, synth.rhs(n, n, n, seed)


def test_unpreconditioned_beta1_equals_beta2():
    shape, c, b = _problem(12)
    r1 = O.krylov(O.PCG, b, shape, c, None, rtol=1e-10, max_iter=200)
    r2 = O.krylov(O.FPCG, b, shape, c, None, rtol=1e-10, max_iter=200)
    assert r1.status == 0 and r2.status == 0
    assert r1.iters == r2.iters
    assert np.allclose(r1.hist, r2.hist, rtol=1e-6, atol=1e-14)
    assert np.linalg.norm(r1.x - r2.x) <= 1e-8 * np.linalg.norm(r1.x)


def test_unpreconditioned_cg_finite_termination():
    """4^3 cube, c = 1: A has as many distinct eigenvalues as distinct sums
    s(a)+s(b)+s(c); CG must reach the rounding level by that step."""
    shape, c = (4, 4, 4), (1.0, 1.0, 1.0)
    lam = D.eigenvalues(shape, c)
    distinct = np.unique(np.round(lam, 10)).size
    b = synth.rhs(4, 4, 4, 3)
    r = O.krylov(O.PCG, b, shape, c, None, rtol=0.0, max_iter=distinct)
    assert r.hist[distinct] < 1e-14
    assert r.hist[distinct - 1] > 1e-9   # not converged one step earlier


def test_psd_theorem1_identity():
    shape, c, b = _problem(10, seed=4)
    for pp in [(1, 1), (1, 0)]:
        S = O.SMG(shape, c, *pp)
        for k in range(4):
            xk = O.krylov(O.PSD, b, shape, c, S, rtol=0.0, max_iter=k).x
            xk1 = O.krylov(O.PSD, b, shape, c, S, rtol=0.0, max_iter=k + 1).x
            rk = b - O.matvec(xk, shape, c)
            rk1 = b - O.matvec(xk1, shape, c)
            nk = rk @ D.dst_solve(rk, shape, c)
            nk1 = rk1 @ D.dst_solve(rk1, shape, c)
            s = S.apply(rk)
            As = O.matvec(s, shape, c)
            # cos = |r'Tr| / (||r||_{A^-1} ||A T r||_{A^-1}),  ||A s||^2_{A^-1} = s'As
            cos2 = (rk @ s) ** 2 / (nk * (s @ As))
            assert abs(nk1 / nk - (1.0 - cos2)) <= 1e-10 * max(1e-3, nk1 / nk)


def test_fpcg_locally_optimal_vs_psd_step():
    shape, c, b = _problem(10, seed=5)
    xs = D.dst_solve(b, shape, c)
    S = O.SMG(shape, c, 1, 0)

    def enorm(e):
        return np.sqrt(e @ O.matvec(e, shape, c))

    for k in range(1, 6):
        xk = O.krylov(O.FPCG, b, shape, c, S, rtol=0.0, max_iter=k).x
        xk1 = O.krylov(O.FPCG, b, shape, c, S, rtol=0.0, max_iter=k + 1).x
        rk = b - O.matvec(xk, shape, c)
        s = S.apply(rk)
        alpha = (s @ rk) / (s @ O.matvec(s, shape, c))
        assert enorm(xs - xk1) <= enorm(xs - (xk + alpha * s)) * (1 + 1e-10)


@pytest.mark.parametrize("method", [O.PCG, O.FPCG, O.PSD])
def test_solution_matches_sine_transform(method):
    shape, c, b = _problem(16, seed=6)
    S = O.SMG(shape, c, 1, 1)
    r = O.krylov(method, b, shape, c, S, rtol=1e-10, max_iter=100)
    assert r.status == 0 and r.true_rel <= 2e-10
    xs = D.dst_solve(b, shape, c)
    assert np.linalg.norm(r.x - xs) <= 1e-7 * np.linalg.norm(xs)


@pytest.mark.parametrize("n", [16, 32])
def test_section3_observations(n):
    shape, c, b = _problem(n)
    S11, S10 = O.SMG(shape, c, 1, 1), O.SMG(shape, c, 1, 0)
    pcg11 = O.krylov(O.PCG, b, shape, c, S11)
    fpcg11 = O.krylov(O.FPCG, b, shape, c, S11)
    psd11 = O.krylov(O.PSD, b, shape, c, S11)
    pcg10 = O.krylov(O.PCG, b, shape, c, S10, max_iter=100)
    fpcg10 = O.krylov(O.FPCG, b, shape, c, S10)
    psd10 = O.krylov(O.PSD, b, shape, c, S10)
    # balanced: the two PCG variants coincide up to rounding
    assert pcg11.iters == fpcg11.iters
    assert np.linalg.norm(pcg11.x - fpcg11.x) <= 1e-9 * np.linalg.norm(pcg11.x)
    # PSD needs only a few more steps (Section 3: "only 2-3 more")
    assert 1 <= psd11.iters - pcg11.iters <= 3
    # no post-smoothing: standard PCG stalls, flexible PCG and PSD stay close
    assert pcg10.status == 1 and pcg10.rel > 1e-6
    assert fpcg10.status == 0 and psd10.status == 0
    assert 0 <= psd10.iters - fpcg10.iters <= 2
    assert 1 <= fpcg10.iters - fpcg11.iters <= 6
    for r in (pcg11, fpcg11, psd11, fpcg10, psd10):
        assert r.true_rel <= 1.5e-8


def test_paper_figures_show_the_same_relations():
    """The paper's own printed data obey the relations checked above."""
    h = np.loadtxt(os.path.join(GOLDEN, "paper_fig5_history.txt"))
    pcg1, psd, pcg2 = h[:, 1], h[:, 2], h[:, 3]
    assert pcg1[-1] > 1e-2 and psd[-1] < 1e-15 and np.nanmin(pcg2) < 1e-15
    it = np.loadtxt(os.path.join(GOLDEN, "paper_fig7_iterations.txt"))
    psd10, fpcg10, pcg11, fpcg11 = it[:, 1], it[:, 2], it[:, 3], it[:, 4]
    assert np.array_equal(pcg11, fpcg11)
    assert np.all((psd10 - fpcg10 >= 0) & (psd10 - fpcg10 <= 2))
    assert np.all((fpcg10 - fpcg11 >= 1) & (fpcg10 - fpcg11 <= 6))


def test_history_c_norm_starts_at_one_for_zero_guess():
    shape, c, b = _problem(8)
    r = O.krylov(O.FPCG, b, shape, c, O.SMG(shape, c, 1, 0))
    assert abs(r.histC[0] - 1.0) < 1e-14
    assert r.hist[0] == pytest.approx(1.0, abs=1e-15)


def test_cnorm_stopping_without_preconditioner_is_2norm_stopping():
    """With T = I the C-norm ratio sqrt|(T r, r)| / sqrt|(T b, b)| is the
    2-norm ratio, so both stopping rules end at the same step; with SMG the
    C-norm history starts at sqrt|(T r_0, r_0)| / sqrt|(T b, b)| (= 1 for x0 = 0)."""
    shape, c, b = _problem(12, seed=6)
    r2 = O.krylov(O.PCG, b, shape, c, None, rtol=1e-7, max_iter=200)
    rc = O.krylov(O.PCG, b, shape, c, None, rtol=1e-7, max_iter=200, stop="c")
    assert r2.status == 0 and rc.status == 0 and r2.iters == rc.iters
    assert np.allclose(rc.histC, r2.hist[:len(rc.histC)], rtol=1e-12, atol=0)
    S = O.SMG(shape, c, 1, 0)
    f = O.krylov(O.FPCG, b, shape, c, S, rtol=1e-7, stop="c")
    assert f.status == 0 and f.histC[0] == pytest.approx(1.0, rel=1e-14)
    assert f.histC[-1] <= 1e-7 < f.histC[-2]
    # a random x0: the first ratio is |(T r0, r0)|^(1/2) / |(T b, b)|^(1/2)
    x0 = synth.uniform_pm1(8, b.size)
    g = O.krylov(O.FPCG, b, shape, c, S, x0=x0, rtol=1e-7, stop="c")
    r0 = b - O.matvec(x0, shape, c)
    want = np.sqrt(abs(S.apply(r0) @ r0) / abs(S.apply(b) @ b))
    assert g.histC[0] == pytest.approx(want, rel=1e-12)
