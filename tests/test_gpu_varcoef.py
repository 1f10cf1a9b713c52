"""GPU parity of SMG for variable-coefficient 7-point operators against the
sparse-matrix oracle (oracle/varcoef.py).

* Setup: every 3D level's Galerkin operator P^T A P (15-point, per point) and
  every plane's 2D operators (9-point) equal the oracle's explicit sparse
  products entry by entry (1e-12 of the largest entry).
* The V-cycle equals the oracle's at 1e-12 (max norm, relative), on ragged
  bricks, lines of one to three waves' worth of points, every smoothing knob
  and both interpolations; with constant coefficients it equals the model
  problem's V-cycle of the constant-coefficient kernels.
* Krylov solves: iteration counts within one of the oracle's, solutions to
  1e-6; LOBPCG eigenvalues against a dense eigensolver to 1e-8.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import synth
from oracle import oracle as O
from oracle import varcoef as V

pytestmark = pytest.mark.gpu


def _coef(shape, kind, seed=7, c=(1.0, 1.0, 1.0)):
    return synth.diffusion_stencil(shape, *synth.conductivity(shape, kind, seed), c=c)


def _gpu(shape, coef, pre=1, post=1, **kw):
    from paper_1212_6680_amd.smg import SMG
    return SMG.variable(shape, *coef, pre, post, **kw)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _entries(A, nx, ny, nb, offsets):
    """A[p, p + o] for every point p of the nb blocks (0 where p + o leaves the grid)."""
    A = A.tocsr()
    n = nx * ny * nb
    idx = np.arange(n)
    i, j, k = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    out = []
    for di, dj, dk in offsets:
        ok = (i + di >= 0) & (i + di < nx) & (j + dj >= 0) & (j + dj < ny) & (k + dk >= 0) & (k + dk < nb)
        q = idx + di + nx * dj + nx * ny * dk
        v = np.zeros(n)
        v[ok] = np.asarray(A[idx[ok], q[ok]]).ravel()
        out.append(v)
    return np.stack(out)


OFF3 = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (-1, 0, 1), (0, 1, 1), (0, -1, 1)]
OFF2 = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0), (-1, 1, 0)]


@pytest.mark.parametrize("shape,kind", [((9, 8, 11), "layers"), ((13, 6, 7), "lognormal"), ((16, 16, 16), "aniso_layers"),
                                        ((70, 5, 9), "lognormal")])
@pytest.mark.parametrize("interp", ["linear", "operator"])
def test_setup_equals_explicit_galerkin_products(shape, kind, interp):
    coef = _coef(shape, kind)
    ref = V.VarSMG(shape, *coef, 1, 1, weights=interp)
    G = _gpu(shape, coef, interp=interp)
    nx, ny, nz = shape
    n3, n2 = G.levels()
    assert n3 == len(ref.ops) and n2 == len(ref.planes[0][0].ops)
    for l, A in enumerate(ref.ops):
        nzl = ref.nz[l]
        got = G.export(l, -1, nz_l=nzl).numpy().reshape(8, -1)
        want = _entries(A, nx, ny, nzl, OFF3)
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max(), l
        for l2, nyl in enumerate(ref.planes[l][0].ny):
            got2 = G.export(l, l2, nz_l=nzl, ny_l2=nyl).numpy().reshape(5, nzl, -1)
            for k in range(nzl):
                want2 = _entries(ref.planes[l][k].ops[l2], nx, nyl, 1, OFF2)
                assert np.abs(got2[:, k] - want2).max() <= 1e-12 * np.abs(want2).max(), (l, l2, k)


SHAPES = [(1, 1, 1), (1, 6, 5), (7, 1, 4), (5, 4, 3), (9, 8, 11), (33, 17, 9), (70, 9, 37), (130, 5, 6),
          (16, 16, 16), (20, 18, 33)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("kind", ["layers", "lognormal"])
def test_vcycle_parity(shape, kind):
    coef = _coef(shape, kind)
    r = synth.rhs(*shape, 21)
    for pp in [(1, 1), (1, 0)]:
        for interp in ("linear", "operator"):
            ref = V.VarSMG(shape, *coef, *pp, weights=interp).apply(r)
            s = _gpu(shape, coef, *pp, interp=interp).apply(_dev(r)).cpu().numpy()
            assert _relerr(s, ref) <= 1e-12, (pp, interp)


@pytest.mark.parametrize("kw", [dict(pre=2, post=1), dict(pre=0, post=1), dict(pre=1, post=0, order=1),
                                dict(pre=1, post=1, inner_pre=2, inner_post=0), dict(pre=1, post=0, inner_pre=1,
                                                                                     inner_post=1)])
def test_vcycle_knobs_parity(kw):
    shape = (37, 20, 23)
    coef = _coef(shape, "aniso_layers")
    pre, post = kw.pop("pre"), kw.pop("post")
    ref = V.VarSMG(shape, *coef, pre, post, kw.get("inner_pre", -1), kw.get("inner_post", -1), kw.get("order", 0))
    r = synth.rhs(*shape, 5)
    s = _gpu(shape, coef, pre, post, **kw).apply(_dev(r)).cpu().numpy()
    assert _relerr(s, ref.apply(r)) <= 1e-12


@pytest.mark.parametrize("pp", [(1, 1), (1, 0)])
def test_constant_coefficients_equal_the_model_kernels(pp):
    from paper_1212_6680_amd.smg import SMG
    shape, c = (40, 33, 29), (1.0, 2.0, 0.5)
    coef = _coef(shape, "const", c=c)
    r = _dev(synth.rhs(*shape, 6))
    a = _gpu(shape, coef, *pp, interp="operator").apply(r).cpu().numpy()
    b = SMG(shape, c, *pp).apply(r).cpu().numpy()
    assert _relerr(a, b) <= 1e-12


def test_matvec_parity():
    shape = (33, 20, 17)
    coef = _coef(shape, "lognormal")
    A = V.operator(shape, *coef)
    n = int(np.prod(shape))
    X = torch.zeros(2, n + 13, dtype=torch.float64)
    for j in range(2):
        X[j, :n] = torch.from_numpy(synth.rhs(*shape, 30 + j))
    Xd = X.cuda()
    Y = torch.full_like(Xd, 5.0)
    _gpu(shape, coef).matvec(Xd[:, :n], Y[:, :n])
    Y = Y.cpu().numpy()
    for j in range(2):
        ref = A @ X[j, :n].numpy()
        assert _relerr(Y[j, :n], ref) <= 1e-14
        assert np.all(Y[j, n:] == 5.0)


@pytest.mark.parametrize("method,pp", [("fpcg", (1, 0)), ("pcg", (1, 1)), ("psd", (1, 0)), ("fpcg", (1, 1))])
@pytest.mark.parametrize("kind", ["layers", "aniso_layers", "lognormal"])
def test_krylov_parity(method, pp, kind):
    shape = (24, 20, 33)
    coef = _coef(shape, kind)
    b = synth.rhs(*shape, 1)
    S = V.VarSMG(shape, *coef, *pp)
    xr, kr, rels, st = V.krylov(method, b, S.matvec, S.apply)
    x, info = getattr(_gpu(shape, coef, *pp), method)(_dev(b))
    assert st == 0 and info.status == 0
    assert abs(info.iters - kr) <= 1
    assert info.true_rel_res <= 1.5e-8
    assert np.linalg.norm(x.cpu().numpy() - xr) <= 1e-6 * np.linalg.norm(xr)


def test_lobpcg_with_variable_coefficients():
    shape = (12, 10, 9)
    coef = _coef(shape, "lognormal")
    A = V.operator(shape, *coef).toarray()
    ex = np.linalg.eigvalsh(A)[:4]
    n = int(np.prod(shape))
    G = _gpu(shape, coef, 1, 0, max_nrhs=5)
    lam, X, info = G.lobpcg(_dev(synth.block(n, 5, 3)), rtol=1e-9, max_iter=300, guard=1)
    assert info.status == 0
    assert np.max(np.abs(lam[:4] - ex) / ex) <= 1e-8


def test_paths_that_reject_variable_handles():
    from paper_1212_6680_amd.smg import SMGError, SMGBatch, Net
    shape = (8, 8, 8)
    G = _gpu(shape, _coef(shape, "layers"), 1, 0)
    r = _dev(synth.rhs(*shape, 1))
    with pytest.raises(SMGError):
        G.autotune(r)
    with pytest.raises(SMGError):
        SMGBatch([G], [r], [torch.empty_like(r)])
    net = Net(G.n, "f64", train=False)
    with pytest.raises(SMGError):
        G.fpcg_learned(net, r)
