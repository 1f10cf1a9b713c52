"""GPU parity of Algorithm 1 (PCG with (1), FPCG with (2), PSD) against the FP64 oracle.

The GPU evaluates (s_k, r_k - r_{k-1}) as -alpha_{k-1}(s_k, A p_{k-1}) and
reduces in another order, so iterates agree with the oracle to rounding:
iteration counts must match within one step, both must reach the stated
relative residual, and the solutions must agree to 1e-6 relative (each is
within ~1e-8 * cond of the exact solution).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import definitional as D
from oracle import oracle as O

pytestmark = pytest.mark.gpu

METHODS = {"pcg": O.PCG, "fpcg": O.FPCG, "psd": O.PSD}


def _smg(shape, c, pre, post, **kw):
    from paper_1212_6680_amd.smg import SMG
    return SMG(shape, c, pre, post, **kw)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("pp", [(1, 1), (1, 0)])
@pytest.mark.parametrize("method", ["pcg", "fpcg", "psd"])
def test_krylov_parity_32(method, pp):
    n = 32
    shape, c = (n, n, n), ((n + 1.0) ** 2,) * 3
    b = synth.rhs(n, n, n, 1)
    G = _smg(shape, c, *pp)
    maxit = 100 if (method == "pcg" and pp == (1, 0)) else 500
    ref = O.krylov(METHODS[method], b, shape, c, O.SMG(shape, c, *pp), max_iter=maxit)
    x, info = getattr(G, method)(_dev(b), max_iter=maxit, history=True)
    x = x.cpu().numpy()
    if method == "pcg" and pp == (1, 0):
        # standard PCG stalls with the nonsymmetric preconditioner (Section 3)
        assert info.status == 1 and ref.status == 1
        assert info.rel_res > 1e-6 and ref.rel > 1e-6
        return
    assert info.status == 0 and ref.status == 0
    assert abs(info.iters - ref.iters) <= 1
    assert info.rel_res <= 1e-8 and info.true_rel_res <= 1.5e-8
    assert np.linalg.norm(x - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
    h = np.array(info.history)
    k = min(len(h), len(ref.hist))
    assert np.allclose(h[:k], ref.hist[:k], rtol=1e-4, atol=1e-12)
    assert np.allclose(info.history_c[:k - 1], ref.histC[:k - 1], rtol=1e-4, atol=1e-12)


def test_unpreconditioned_cg_parity():
    shape = (20, 18, 16)
    c = (1.0, 1.0, 1.0)
    b = synth.rhs(*shape, seed=9)
    G = _smg(shape, c, 1, 1)
    for method in ("pcg", "fpcg"):
        ref = O.krylov(METHODS[method], b, shape, c, None, rtol=1e-10, max_iter=400)
        x, info = getattr(G, method)(_dev(b), rtol=1e-10, max_iter=400, precond="none")
        assert info.status == 0 and abs(info.iters - ref.iters) <= 1
        assert np.linalg.norm(x.cpu().numpy() - ref.x) <= 1e-7 * np.linalg.norm(ref.x)


def test_solution_against_sine_transform():
    n = 48
    shape, c = (n, n, n), ((n + 1.0) ** 2,) * 3
    b = synth.rhs(n, n, n, 4)
    x, info = _smg(shape, c, 1, 0).fpcg(_dev(b), rtol=1e-11)
    xs = D.dst_solve(b, shape, c)
    assert info.status == 0
    assert np.linalg.norm(x.cpu().numpy() - xs) <= 1e-9 * np.linalg.norm(xs)


def test_nonzero_initial_guess_and_odd_brick():
    shape = (45, 38, 27)
    c = (46.0 ** 2, 39.0 ** 2, 28.0 ** 2)
    b = synth.rhs(*shape, seed=12)
    x0 = synth.uniform_pm1(13, np.prod(shape))
    ref = O.krylov(O.FPCG, b, shape, c, O.SMG(shape, c, 1, 0), x0=x0)
    x, info = _smg(shape, c, 1, 0).fpcg(_dev(b), _dev(x0.copy()))
    assert info.status == 0 and abs(info.iters - ref.iters) <= 1
    assert np.linalg.norm(x.cpu().numpy() - ref.x) <= 1e-6 * np.linalg.norm(ref.x)


def test_edge_cases():
    shape, c = (16, 16, 16), (1.0, 1.0, 1.0)
    G = _smg(shape, c, 1, 0)
    b = synth.rhs(*shape, seed=1)
    # max_iter = 0 and 1
    x, info = G.fpcg(_dev(b), max_iter=0)
    assert info.status == 1 and info.iters == 0 and float(x.abs().max()) == 0.0
    x, info = G.fpcg(_dev(b), max_iter=1)
    assert info.status == 1 and info.iters == 1
    # zero right-hand side: converged at once, x = 0
    x, info = G.fpcg(torch.zeros(16 ** 3, dtype=torch.float64, device="cuda"))
    assert info.status == 0 and info.iters == 0 and float(x.abs().max()) == 0.0
    # non-finite right-hand side is reported, not iterated on
    bn = b.copy()
    bn[77] = np.nan
    from paper_1212_6680_amd.smg import SMGError
    with pytest.raises(SMGError, match="non-finite"):
        G.fpcg(_dev(bn))


@pytest.mark.parametrize("method", ["fpcg", "pcg", "psd"])
def test_full_size_headline_solve(method):
    """256^3, c = 257^2, b from seed 2, x0 = 0: iteration count equals the
    oracle's within one and the true residual meets 1e-8."""
    n = 256
    shape, c = (n, n, n), ((n + 1.0) ** 2,) * 3
    b = synth.rhs(n, n, n, 2)
    pp = (1, 1) if method == "pcg" else (1, 0)
    ref = O.krylov(METHODS[method], b, shape, c, O.SMG(shape, c, *pp), history=False)
    x, info = getattr(_smg(shape, c, *pp), method)(_dev(b))
    assert info.status == 0 and ref.status == 0
    assert abs(info.iters - ref.iters) <= 1
    assert info.true_rel_res <= 1.5e-8
    xg = x.cpu().numpy()
    assert np.linalg.norm(xg - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
