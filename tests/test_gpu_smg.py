"""GPU parity of the SMG preconditioner and the 7-point operator against the FP64 oracle.

Every case is called through the C ABI (the ctypes binding) on seeded inputs
shared with the oracle.  Tolerance: the V-cycle is a fixed sequence of
well-conditioned FP64 operations (line solves of diagonally dominant SPD
tridiagonals, stencils with O(1) row sums relative to the diagonal); the GPU
evaluates the Thomas recurrences as lane scans and the prolongation sums in
another order, so results differ from the oracle by rounding only.  The bar
is a max-norm error of 1e-12 relative to the max-norm of the result.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import oracle as O

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _smg(shape, c, pre, post, **kw):
    from paper_1212_6680_amd.smg import SMG
    return SMG(shape, c, pre, post, **kw)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


SHAPES = [(1, 1, 1), (1, 1, 9), (7, 1, 1), (1, 6, 1), (5, 4, 3), (8, 8, 8), (16, 16, 16),
          (33, 17, 9), (65, 3, 5), (64, 64, 2), (130, 6, 7), (17, 40, 33), (32, 32, 32)]


@pytest.mark.parametrize("shape", SHAPES)
def test_matvec_parity(shape):
    n = shape[0]
    c = ((n + 1.0) ** 2, 1.7 * (shape[1] + 1) ** 2, 0.9 * (shape[2] + 1) ** 2)
    x = synth.rhs(*shape, seed=11)
    ref = O.matvec(x, shape, c)
    G = _smg(shape, c, 1, 1)
    y = G.matvec(_dev(x)).cpu().numpy()
    assert _relerr(y, ref) <= 1e-14


@pytest.mark.parametrize("shape,nrhs,pad", [((17, 40, 33), 3, 0), ((17, 40, 33), 3, 77), ((33, 17, 9), 67, 5),
                                            ((65, 40, 29), 67, 0), ((64, 64, 2), 3, 1), ((130, 64, 37), 5, 3)])
def test_matvec_block_parity(shape, nrhs, pad):
    """y = A x over nrhs columns with leading dimension N + pad (the LOBPCG
    block products): the column index and the z-chunking of the marching
    stencil (nz not a multiple of the chunk for these shapes) against the
    oracle column by column; the padding between columns is left untouched."""
    n = int(np.prod(shape))
    c = (1.3, 0.7, 2.1)
    ld = n + pad
    X = torch.zeros(nrhs, ld, dtype=torch.float64)
    for j in range(nrhs):
        X[j, :n] = torch.from_numpy(synth.rhs(*shape, seed=100 + j))
    Xd = X.cuda()
    Y = torch.full_like(Xd, 123.0)
    G = _smg(shape, c, 1, 1)
    G.matvec(Xd[:, :n], Y[:, :n])
    Y = Y.cpu().numpy()
    for j in range(nrhs):
        ref = O.matvec(X[j, :n].numpy(), shape, c)
        assert _relerr(Y[j, :n], ref) <= 1e-14, j
        assert np.all(Y[j, n:] == 123.0)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("pp", [(1, 1), (1, 0)])
def test_vcycle_parity(shape, pp):
    c = tuple((v + 1.0) ** 2 for v in shape)
    r = synth.rhs(*shape, seed=21)
    ref = O.SMG(shape, c, *pp).apply(r)
    s = _smg(shape, c, *pp).apply(_dev(r)).cpu().numpy()
    assert _relerr(s, ref) <= TOL


@pytest.mark.parametrize("kw", [dict(pre=2, post=1), dict(pre=0, post=1), dict(pre=1, post=2),
                                dict(pre=1, post=0, order=1), dict(pre=1, post=1, order=1),
                                dict(pre=1, post=0, inner_pre=1, inner_post=1),
                                dict(pre=1, post=1, inner_pre=2, inner_post=0),
                                dict(pre=0, post=0)])
def test_vcycle_knobs_parity(kw):
    shape = (37, 20, 23)
    c = (1.0, 2.0, 0.5)
    pre, post = kw.pop("pre"), kw.pop("post")
    ref = O.SMG(shape, c, pre, post, kw.get("inner_pre", -1), kw.get("inner_post", -1), kw.get("order", 0))
    r = synth.rhs(*shape, seed=5)
    s = _smg(shape, c, pre, post, **kw).apply(_dev(r)).cpu().numpy()
    assert _relerr(s, ref.apply(r)) <= TOL


def test_vcycle_max_line_length():
    shape = (512, 3, 4)
    c = (1.0, 1.0, 1.0)
    r = synth.rhs(*shape, seed=8)
    for pp in [(1, 1), (1, 0)]:
        ref = O.SMG(shape, c, *pp).apply(r)
        assert _relerr(_smg(shape, c, *pp).apply(_dev(r)).cpu().numpy(), ref) <= TOL


def test_batched_rhs_equal_single_rhs_bitwise():
    shape, c = (24, 20, 18), (1.0, 1.0, 1.0)
    R = np.stack([synth.rhs(*shape, seed=100 + i) for i in range(5)])
    G = _smg(shape, c, 1, 0, max_nrhs=5)
    Sb = G.apply(_dev(R)).cpu().numpy()
    for i in range(5):
        si = G.apply(_dev(R[i])).cpu().numpy()
        assert np.array_equal(Sb[i], si)
    # and with a leading dimension larger than n
    n = int(np.prod(shape))
    Rp = np.zeros((3, n + 64))
    Rp[:, :n] = R[:3]
    Sp = G.apply(_dev(Rp)[:, :n]).cpu().numpy()          # rows of a padded block: ld = n + 64
    assert np.array_equal(Sp, Sb[:3])


def test_repeatable_bitwise():
    shape, c = (40, 33, 29), (1.0, 1.0, 1.0)
    G = _smg(shape, c, 1, 1)
    r = _dev(synth.rhs(*shape, seed=3))
    a = G.apply(r).cpu().numpy()
    b = G.apply(r).cpu().numpy()
    assert np.array_equal(a, b)


def test_gpu_balanced_symmetric_unbalanced_not():
    n = 24
    shape, c = (n, n, n), ((n + 1.0) ** 2,) * 3
    u, v = synth.rhs(n, n, n, 1), synth.rhs(n, n, n, 2)
    for pp, sym in [((1, 1), True), ((1, 0), False)]:
        G = _smg(shape, c, *pp)
        uBv = u @ G.apply(_dev(v)).cpu().numpy()
        vBu = v @ G.apply(_dev(u)).cpu().numpy()
        if sym:
            assert abs(uBv - vBu) <= 1e-12 * abs(uBv)
        else:
            assert abs(uBv - vBu) > 1e-3 * abs(uBv)


@pytest.mark.parametrize("n", [256])
def test_vcycle_parity_full_size(n):
    """The benchmark's brick (256^3, c = 257^2, seed 2): one full V-cycle of each smoothing."""
    shape, c = (n, n, n), ((n + 1.0) ** 2,) * 3
    r = synth.rhs(n, n, n, 2)
    for pp in [(1, 0), (1, 1)]:
        ref = O.SMG(shape, c, *pp).apply(r)
        s = _smg(shape, c, *pp).apply(_dev(r)).cpu().numpy()
        assert _relerr(s, ref) <= TOL


FUSED_SHAPES = [(1, 1, 1), (9, 1, 1), (5, 4, 3), (16, 16, 16), (33, 17, 9), (64, 64, 2), (130, 6, 7),
                (17, 40, 33), (100, 70, 45), (256, 256, 4), (300, 11, 3), (64, 200, 5), (384, 30, 4), (512, 3, 4)]


@pytest.mark.parametrize("shape", FUSED_SHAPES)
@pytest.mark.parametrize("pp", [(1, 0), (1, 1), (2, 0), (0, 1)])
def test_fused_schedule_equals_stage_schedule_and_oracle(shape, pp):
    """The fused kernels (strip relax+restrict, LDS-resident coarse levels,
    prolongation chains) compute the same cycle as one launch per stage."""
    c = tuple((v + 1.0) ** 2 for v in shape)
    r = _dev(synth.rhs(*shape, seed=17))
    a = _smg(shape, c, *pp, kernel_mode=0).apply(r).cpu().numpy()
    b = _smg(shape, c, *pp, kernel_mode=1).apply(r).cpu().numpy()
    assert _relerr(a, b) <= TOL
    if np.prod(shape) <= 200000:
        ref = O.SMG(shape, c, *pp).apply(synth.rhs(*shape, seed=17))
        assert _relerr(a, ref) <= TOL


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_fused_schedule_low_precision(prec):
    shape = (96, 80, 40)
    c = tuple((v + 1.0) ** 2 for v in shape)
    r = _dev(synth.rhs(*shape, seed=18))
    for pp in [(1, 0), (1, 1)]:
        a = _smg(shape, c, *pp, precision=prec, kernel_mode=0).apply(r).cpu().numpy()
        b = _smg(shape, c, *pp, precision=prec, kernel_mode=1).apply(r).cpu().numpy()
        assert _relerr(a, b) <= (1e-5 if prec == "f32" else 3e-2)


@pytest.mark.parametrize("shape", [(64, 40, 24), (300, 33, 9)])
def test_autotuned_schedule_matches_oracle(shape):
    """The autotuner only changes the schedule (which 2D levels run in the LDS
    kernel, strip heights): the V-cycle stays the oracle's to 1e-12."""
    from paper_1212_6680_amd.smg import SMG
    c = (3.0, 2.0, 1.5)
    r = synth.rhs(*shape, seed=77)
    G = SMG(shape, c, 1, 0)
    info = G.autotune(torch.from_numpy(r).cuda(), reps=2)
    assert info.candidates >= 1 and info.best_ms <= info.default_ms
    s = G.apply(torch.from_numpy(r).cuda()).cpu().numpy()
    ref = O.SMG(shape, c, 1, 0).apply(r)
    assert np.linalg.norm(s - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("shape,nrhs", [((33, 45, 17), 1), ((70, 129, 9), 1), ((200, 31, 12), 1),
                                        ((256, 64, 8), 1), ((96, 57, 6), 3), ((300, 37, 6), 1),
                                        ((384, 48, 5), 2)])
@pytest.mark.parametrize("pp", [(1, 0), (1, 1)])
def test_marching_pre_smoothing(shape, nrhs, pp):
    """Pre-smoothing kernels that march runs of 2, 4 or 8 coarse lines per wave
    (forced on every level by a threshold of 1, mixed with single-line waves
    by a threshold of 5) give the V-cycle of single-line waves up to rounding
    (the same operations; the compiler may fuse a multiply-add differently),
    and the oracle's to 1e-12: odd and even line counts, runs cut by the end
    of a level, line widths of 1 to 4 points per lane (wider lines, 5 and 6
    points, take the LDS strip kernel either way), several right-hand sides."""
    c = tuple((v + 1.0) ** 2 for v in shape)
    n = int(np.prod(shape))
    r = np.stack([synth.rhs(*shape, seed=90 + i).reshape(-1) for i in range(nrhs)])
    G = _smg(shape, c, *pp, max_nrhs=nrhs)
    rd = _dev(r if nrhs > 1 else r[0])
    G.set_march(0)
    base = G.apply(rd).cpu().numpy()
    for mw in (1, 5):
        G.set_march(mw)
        s = G.apply(rd).cpu().numpy()
        d = float(np.abs(s - base).max() / np.abs(base).max())
        assert d <= 1e-14, (mw, d)
    ref = O.SMG(shape, c, *pp)
    for i in range(nrhs):
        assert _relerr(base.reshape(nrhs, n)[i], ref.apply(r[i])) <= TOL


@pytest.mark.parametrize("pp", [(1, 0), (1, 1)])
def test_workspace_prior_contents_do_not_matter(pp):
    """No kernel reads workspace memory it has not written in the same call or
    at setup: a workspace left full of NaN bytes gives bitwise the same V-cycle
    and solve as one left full of zeros."""
    shape = (45, 38, 27)
    c = (1.0, 1.0, 1.0)
    r = _dev(synth.rhs(*shape, seed=14))
    outs = []
    for fill in (0x00, 0xFF):
        G = _smg(shape, c, *pp, ws_fill=fill)
        s = G.apply(r)
        x, info = G.fpcg(r)
        outs.append((s, x, info.iters))
    assert torch.equal(outs[0][0], outs[1][0])
    assert torch.equal(outs[0][1], outs[1][1]) and outs[0][2] == outs[1][2]


@pytest.mark.parametrize("pp", [(1, 0), (1, 1)])
def test_profile_levels_partitions_the_families(pp):
    """The per-level profile stamps every launch once: its rows add up to the
    per-family profiles' launches and algorithmic bytes, each row to its
    per-family rows, the prolongation
    chain row is used only without post-smoothing, and the profiled V-cycle
    leaves the next V-cycle unchanged."""
    from paper_1212_6680_amd.smg import KERNELS
    shape = (64, 48, 40)
    c = (2.0, 1.0, 3.0)
    r = _dev(synth.rhs(*shape, seed=21))
    G = _smg(shape, c, *pp)
    rows = G.profile_levels(r, reps=2)
    nz, nlev = shape[2], 1
    while nz > 1:
        nz //= 2
        nlev += 1
    assert len(rows) == nlev + 1
    fam = [G.profile_kernel(f, r, reps=2) for f in KERNELS]
    assert sum(x[0] for x in rows) == sum(x[0] for x in fam)
    tot = sum(x[2] for x in fam)
    assert abs(sum(x[2] for x in rows) - tot) <= 1e-9 * tot
    assert all(x[0] >= 1 and x[1] > 0 for x in rows[:-1])
    split = [G.profile_levels(r, reps=1, family=f) for f in KERNELS]
    for i, row in enumerate(rows):
        assert sum(f[i][0] for f in split) == row[0]
        assert abs(sum(f[i][2] for f in split) - row[2]) <= 1e-9 * tot
    assert (rows[-1][0] == 1) == (pp[1] == 0)
    s = G.apply(r)
    G.profile_levels(r, reps=1)
    assert torch.equal(s, G.apply(r))


def test_profile_arguments_are_checked():
    """The profiling entry points take one vector of the grid's size and a
    known family; anything else fails before a launch."""
    from paper_1212_6680_amd.smg import SMGError
    shape = (16, 12, 10)
    G = _smg(shape, (1.0, 1.0, 1.0), 1, 0)
    short = torch.zeros(int(np.prod(shape)) - 1, dtype=torch.float64, device="cuda")
    ok = torch.zeros(int(np.prod(shape)), dtype=torch.float64, device="cuda")
    for call in (lambda: G.profile_levels(short), lambda: G.profile_kernel("down2", short),
                 lambda: G.profile_levels(ok, family="nonesuch"), lambda: G.profile_kernel("nonesuch", ok)):
        with pytest.raises(SMGError):
            call()
    assert len(G.profile_levels(ok, reps=1)) == 5


@pytest.mark.parametrize("prec", ["f32", "bf16"])
@pytest.mark.parametrize("shape,nrhs", [((256, 20, 12), 1), ((384, 30, 8), 1), ((128, 33, 17), 1),
                                        ((96, 17, 9), 1), ((66, 10, 7), 1), ((130, 7, 5), 1),
                                        ((33, 17, 9), 1), ((256, 12, 6), 3), ((192, 9, 10), 2)])
@pytest.mark.parametrize("pp", [(1, 0), (1, 1)])
def test_vector_streaming_kernels_match_one_point_per_thread(prec, shape, nrhs, pp):
    """The residual, restriction and prolongation-chain kernels that give each
    thread 2 or 4 consecutive points (8-byte accesses in FP32 and BF16) compute
    bitwise what the same schedule computes at one point per thread
    (kernel_mode 2), for widths that divide the row, ragged rows that fall back
    and several right-hand sides."""
    c = tuple((v + 1.0) ** 2 for v in shape)
    n = int(np.prod(shape))
    rng = np.random.default_rng(5)
    r = rng.uniform(-1, 1, size=(nrhs, n)) if nrhs > 1 else synth.rhs(*shape, seed=19)
    rd = _dev(r)
    a = _smg(shape, c, *pp, precision=prec, max_nrhs=nrhs, kernel_mode=0).apply(rd)
    b = _smg(shape, c, *pp, precision=prec, max_nrhs=nrhs, kernel_mode=2).apply(rd)
    assert torch.equal(a, b)
