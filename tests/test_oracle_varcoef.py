"""Pins of the variable-coefficient SMG oracle (oracle/varcoef.py).

* With constant coefficients it is the C oracle's V-cycle (an independent
  implementation of the constant-coefficient reading), for every smoothing
  knob, colour order and both interpolations.
* The Galerkin coarse operators have the stencils the method relies on:
  symmetric, 15-point on 3D levels (5 in-plane points on 3 planes), 9-point
  on 2D levels, and the interpolation weights are a partition of unity.
* With balanced smoothing the preconditioner is symmetric positive definite
  (1e-12), and T(pre, post)^T = T(post, pre).
* Exactness: a brick of one line is solved exactly.
* It converges on jumping and anisotropic coefficients, and follows
  Algorithm 1: with T = I its PCG and FPCG are the same CG.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import oracle as O
from oracle import varcoef as V


def _problem(shape, kind, seed=7, c=(1.0, 1.0, 1.0)):
    return synth.diffusion_stencil(shape, *synth.conductivity(shape, kind, seed), c=c)


@pytest.mark.parametrize("shape", [(5, 4, 3), (9, 7, 6), (12, 10, 13), (1, 6, 5), (7, 1, 4)])
@pytest.mark.parametrize("weights", ["linear", "operator"])
def test_constant_coefficients_reduce_to_the_scalar_oracle(shape, weights):
    c = (1.0, 2.0, 0.5)
    coef = _problem(shape, "const", c=c)
    r = synth.rhs(*shape, 3)
    for pp, order in [((1, 1), 0), ((1, 0), 0), ((2, 1), 1), ((0, 1), 0), ((1, 0), 1)]:
        s = V.VarSMG(shape, *coef, *pp, order=order, weights=weights).apply(r)
        ref = O.SMG(shape, c, *pp, -1, -1, order).apply(r)
        assert np.abs(s - ref).max() <= 1e-13 * np.abs(ref).max(), (pp, order)


def test_operator_matches_the_model_problem():
    shape, c = (6, 5, 4), (1.0, 2.0, 0.5)
    A = V.operator(shape, *_problem(shape, "const", c=c))
    x = synth.rhs(*shape, 1)
    assert np.abs(A @ x - O.matvec(x, shape, c)).max() <= 1e-14 * np.abs(A @ x).max()


def _offsets(A, shape):
    nx, ny, _ = shape
    A = A.tocoo()
    d = A.col - A.row
    ri, rj, rk = A.row % nx, (A.row // nx) % ny, A.row // (nx * ny)
    ci, cj, ck = A.col % nx, (A.col // nx) % ny, A.col // (nx * ny)
    return set(zip((ci - ri).tolist(), (cj - rj).tolist(), (ck - rk).tolist()))


@pytest.mark.parametrize("kind", ["layers", "aniso_layers", "lognormal"])
@pytest.mark.parametrize("weights", ["linear", "operator"])
def test_coarse_stencils(kind, weights):
    shape = (9, 8, 11)
    S = V.VarSMG(shape, *_problem(shape, kind), 1, 1, weights=weights)
    allowed3 = {(di, dj, dk) for dk in (-1, 0, 1) for di, dj in ((0, 0), (1, 0), (-1, 0), (0, 1), (0, -1))}
    for l, A in enumerate(S.ops):
        assert abs(A - A.T).max() <= 1e-12 * abs(A).max()
        offs = _offsets(A, (9, 8, S.nz[l]))
        assert offs <= allowed3
        if l >= 1 and S.nz[l] > 1:
            assert offs == allowed3            # the coarse levels fill all 15 points
    allowed2 = {(di, dj, 0) for di in (-1, 0, 1) for dj in (-1, 0, 1)}
    for planes in S.planes:
        for H in planes:
            for Q, nyl in zip(H.ops, H.ny):
                assert abs(Q - Q.T).max() <= 1e-12 * abs(Q).max()
                assert _offsets(Q, (9, nyl, 1)) <= allowed2
    for P in S.P:                             # interpolation weights sum to 1 on F-planes with two neighbours
        rs = np.asarray(P.sum(axis=1)).ravel()
        assert np.all((np.abs(rs - 1.0) <= 1e-14) | (np.abs(rs - 0.5) <= 1e-14))


def test_operator_weights_follow_a_jump():
    """On the fine level an F-point couples to each neighbouring plane through
    one z-face, so its weights are the face couplings' shares az_dn/(az_dn +
    az_up) and az_up/(az_dn + az_up): across a jump of the conductivity the
    better-connected plane dominates.  An F-plane with one C-neighbour takes 1/2."""
    shape = (4, 4, 5)
    kap = np.r_[np.ones(48), 1e3 * np.ones(32)]        # planes 0-2: 1, planes 3-4: 1000
    d, ax, ay, az = synth.diffusion_stencil(shape, kap, kap, kap)
    P = V.prolongation(V.operator(shape, d, ax, ay, az), 5, 16, "operator").toarray()
    a_dn, a_up = az[16:32], az[32:48]                  # faces 1-2 and 2-3
    assert np.allclose(P[32:48, 0:16].diagonal(), a_dn / (a_dn + a_up), rtol=1e-14)
    assert np.allclose(P[32:48, 16:32].diagonal(), a_up / (a_dn + a_up), rtol=1e-14)
    assert np.all(a_up > 1.9 * a_dn)
    assert np.allclose(P[0:16, 0:16].diagonal(), 0.5) and np.allclose(P[64:80, 16:32].diagonal(), 0.5)


@pytest.mark.parametrize("kind", ["layers", "lognormal"])
def test_balanced_cycle_is_spd_and_transposes(kind):
    shape = (6, 5, 7)
    coef = _problem(shape, kind)
    n = int(np.prod(shape))
    E = np.eye(n)
    S11, S10, S01 = (V.VarSMG(shape, *coef, *pp) for pp in ((1, 1), (1, 0), (0, 1)))
    B11 = np.stack([S11.apply(e) for e in E], axis=1)
    assert np.abs(B11 - B11.T).max() <= 1e-12 * np.abs(B11).max()
    assert np.linalg.eigvalsh(0.5 * (B11 + B11.T)).min() > 0
    B10 = np.stack([S10.apply(e) for e in E], axis=1)
    B01 = np.stack([S01.apply(e) for e in E], axis=1)
    assert np.abs(B10.T - B01).max() <= 1e-12 * np.abs(B10).max()
    assert np.abs(B10 - B10.T).max() > 1e-3 * np.abs(B10).max()     # without post-smoothing: nonsymmetric
    # linearity
    u, v = synth.rhs(*shape, 1), synth.rhs(*shape, 2)
    S = V.VarSMG(shape, *coef, 1, 0)
    assert np.allclose(S.apply(2 * u - 3 * v), 2 * S.apply(u) - 3 * S.apply(v), rtol=0, atol=1e-12 * np.abs(S.apply(u)).max())


def test_single_line_brick_is_solved_exactly():
    shape = (17, 1, 1)
    coef = _problem(shape, "lognormal")
    A = V.operator(shape, *coef).toarray()
    b = synth.rhs(*shape, 4)
    for pp in [(1, 1), (1, 0)]:
        x = V.VarSMG(shape, *coef, *pp).apply(b)
        assert np.abs(A @ x - b).max() <= 1e-13 * np.abs(b).max()


@pytest.mark.parametrize("kind", ["layers", "aniso_layers", "lognormal"])
def test_flexible_pcg_converges(kind):
    shape = (16, 14, 17)
    coef = _problem(shape, kind)
    b = synth.rhs(*shape, 1)
    A = V.operator(shape, *coef)
    its = {}
    for w in ("linear", "operator"):
        S = V.VarSMG(shape, *coef, 1, 0, weights=w)
        x, k, rels, st = V.krylov("fpcg", b, S.matvec, S.apply)
        assert st == 0 and k <= 20
        assert np.linalg.norm(b - A @ x) <= 1.5e-8 * np.linalg.norm(b)
        its[w] = k
    if kind == "layers":
        assert its["operator"] <= its["linear"]


def test_unpreconditioned_beta1_equals_beta2():
    shape = (8, 7, 6)
    A = V.operator(shape, *_problem(shape, "lognormal"))
    b = synth.rhs(*shape, 2)
    x1, k1, h1, _ = V.krylov("pcg", b, lambda v: A @ v, lambda v: v, rtol=1e-10)
    x2, k2, h2, _ = V.krylov("fpcg", b, lambda v: A @ v, lambda v: v, rtol=1e-10)
    # the same CG up to rounding (which CG amplifies on this rough problem)
    assert k1 == k2 and np.allclose(h1[:8], h2[:8], rtol=1e-6, atol=1e-14)
    assert np.linalg.norm(x1 - x2) <= 1e-8 * np.linalg.norm(x1)
    xs = sp.linalg.spsolve(A.tocsc(), b)
    assert np.linalg.norm(x1 - xs) <= 1e-8 * np.linalg.norm(xs) * 1e2
