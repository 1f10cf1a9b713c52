"""GPU parity of the Section 5 diagnostics: the power-iteration estimates of
delta(c) = ||I - c A T||_{A^{-1}} (assumption (4)) and of the extreme
eigenvalues of T A (Theorem 2) against the oracle's same iterations, step
count for step count; against dense linear algebra on a small grid; and the
paper's bound (3) on the GPU's own PSD steps."""
import numpy as np
import pytest
import torch

import synth
from oracle import definitional as D
from oracle import oracle as O
from oracle import theory as TH

pytestmark = pytest.mark.gpu


def _smg(shape, c, pre, post, **kw):
    from paper_1212_6680_amd.smg import SMG
    return SMG(shape, c, pre, post, **kw)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("pp", [(1, 0), (1, 1), (2, 1)])
def test_delta_power_matches_oracle(pp):
    shape = (24, 20, 18)
    c = tuple((v + 1.0) ** 2 for v in shape)
    v0 = synth.uniform_pm1(7, int(np.prod(shape)))
    G, Gt = _smg(shape, c, *pp), _smg(shape, c, pp[1], pp[0])
    S, St = O.SMG(shape, c, *pp), O.SMG(shape, c, pp[1], pp[0])
    for cc in (0.9, 1.2):
        ref = TH.delta_power(shape, c, S, St, cc, v0, 30)
        got = G.delta(cc, _dev(v0), iters=30, transpose=Gt)
        assert got == pytest.approx(ref, rel=1e-9), (cc, got, ref)
        assert 0.0 < got < 1.0


def test_spectrum_matches_oracle():
    shape = (24, 20, 18)
    c = tuple((v + 1.0) ** 2 for v in shape)
    v0 = synth.uniform_pm1(8, int(np.prod(shape)))
    lo, hi = _smg(shape, c, 1, 1).spectrum(_dev(v0), iters=30)
    rlo, rhi = TH.spectrum_power(shape, c, O.SMG(shape, c, 1, 1), v0, 30)
    assert hi == pytest.approx(rhi, rel=1e-10) and lo == pytest.approx(rlo, rel=1e-8)
    assert 0.0 < lo < hi <= 1.0 + 1e-12


@pytest.mark.parametrize("pp", [(1, 0), (1, 1)])
def test_delta_min_against_dense(pp):
    """On a 6^3 grid the GPU's minimised estimate approaches the dense
    min_c ||I - c A T||_{A^{-1}} from below."""
    shape = (6, 6, 6)
    c = tuple((v + 1.0) ** 2 for v in shape)
    A, T = TH.dense_pair(shape, c, *pp)
    cref, dref = TH.delta_min_dense(A, T)
    v0 = synth.uniform_pm1(9, int(np.prod(shape)))
    G, Gt = _smg(shape, c, *pp), _smg(shape, c, pp[1], pp[0])
    cb, d = G.delta_min(_dev(v0), 0.5, 2.0, 1e-6, iters=400, transpose=Gt)
    assert d <= dref * (1 + 1e-9) and d >= dref * (1 - 1e-3), (d, dref)
    assert cb == pytest.approx(cref, rel=1e-2)


def test_theorem2_prescaling_on_gpu():
    """Balanced SMG at 32^3: with c = 2/(lambda_min + lambda_max) from the GPU
    spectrum, the GPU's delta(c) equals (kappa - 1)/(kappa + 1) (Theorem 2),
    to the accuracy of the power iterations."""
    n = 32
    shape, c = (n, n, n), ((n + 1.0) ** 2,) * 3
    v0 = _dev(synth.uniform_pm1(10, n ** 3))
    G = _smg(shape, c, 1, 1)
    lo, hi = G.spectrum(v0, iters=150)
    cs = 2.0 / (lo + hi)
    kappa = hi / lo
    want = (kappa - 1.0) / (kappa + 1.0)
    d = G.delta(cs, v0, iters=150)
    print(f"lambda(TA) in [{lo:.6f}, {hi:.6f}], kappa {kappa:.4f}, delta {d:.5f} vs (k-1)/(k+1) {want:.5f}")
    assert d == pytest.approx(want, rel=0.03)
    assert want < 0.2


@pytest.mark.parametrize("pp", [(1, 0), (1, 1)])
def test_bound3_psd_steps_on_gpu(pp):
    """Bound (3) on the GPU's PSD steps at 32^3: every step contracts
    ||r||_{A^{-1}} (logged by the solver against the exact solution) by no
    more than the estimated min_c ||I - c A T||_{A^{-1}} (a lower estimate,
    so a small margin)."""
    n = 32
    shape, c = (n, n, n), ((n + 1.0) ** 2,) * 3
    b = synth.rhs(n, n, n, 11)
    xs = D.dst_solve(b, shape, c)
    G, Gt = _smg(shape, c, *pp), _smg(shape, c, pp[1], pp[0])
    _, dmin = G.delta_min(_dev(synth.uniform_pm1(12, n ** 3)), 0.5, 2.0, 1e-3, iters=60, transpose=Gt)
    _, info = G.psd(_dev(b), rtol=1e-10, xstar=_dev(xs))
    e = np.array(info.err_a)
    ok = e[:-1] > 1e-7
    ratio = e[1:][ok] / e[:-1][ok]
    print(pp, "delta_min", dmin, "PSD per-step", np.round(ratio, 4))
    assert dmin < 1.0
    assert np.all(ratio <= dmin * 1.05)
