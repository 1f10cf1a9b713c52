"""GPU parity of the learned post-smoother against the FP64 network oracle.

F64 check mode: every kernel (direct convolutions, input and weight
gradients, loss, Adam, correction, training pairs) is compared with the
oracle at 1e-10 relative.  BF16 mode (MFMA for the 16 -> 16 layers): the
oracle rounds to bfloat16 where the kernels store (input, weights,
activations, gradients), so what remains is FP32 accumulation and the rare
rounding-boundary flip; the bounds are stated per test.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import definitional as D
from oracle import learned as L
from oracle import oracle as O

pytestmark = pytest.mark.gpu


def _net(nvox, prec, train=True):
    from paper_1212_6680_amd.smg import Net
    return Net(nvox, prec, train=train)


def _smg(shape, c, pre, post, **kw):
    from paper_1212_6680_amd.smg import SMG
    return SMG(shape, c, pre, post, **kw)


def _dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda").to(dtype)


def _bf16_dev(a):
    """bfloat16 device tensor of a (rounded to nearest even) and the rounded values in FP64."""
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16)
    return t.to("cuda"), t.to(torch.float64).numpy()


def _layer_params(params, l):
    return params[l]


SHAPES = [(13, 11, 9), (70, 9, 6)]   # (nx, ny, nz): ragged against every tile size


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("layer", [0, 1, 2, 3])
def test_layer_forward_f64(shape, layer):
    nx, ny, nz = shape
    params = L.init_params(3)
    W, b = params[layer]
    cin = W.shape[3]
    x = np.random.default_rng(layer).standard_normal((nz, ny, nx, cin))
    ref = L.conv(x, W, b)
    if layer < 3:
        ref = np.maximum(ref, 0.0)
    net = _net(nx * ny * nz, "f64", train=False)
    net.set_params(L.flatten(params))
    out = net.layer_forward(layer, shape, _dev(x.ravel())).cpu().numpy().reshape(ref.shape)
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("shape", SHAPES + [(64, 8, 5), (130, 17, 4)])
@pytest.mark.parametrize("layer", [0, 1, 2, 3])
def test_layer_forward_bf16(shape, layer):
    """bf16 inputs and weights, FP32 accumulation: the error is at most one bf16
    rounding of the output (2^-8 relative, layers 0..2) plus FP32 accumulation
    error (<= 1e-4 of the sum of |terms| over 432 products)."""
    nx, ny, nz = shape
    params = L.init_params(4)
    W, b = params[layer]
    cin = W.shape[3]
    xd, xq = _bf16_dev(np.random.default_rng(10 + layer).standard_normal((nz, ny, nx, cin)).ravel())
    xq = xq.reshape(nz, ny, nx, cin)
    Wq = L.round_bf16(W)
    b32 = b.astype(np.float32).astype(np.float64)
    ref = L.conv(xq, Wq, b32)
    bound = L.conv(np.abs(xq), np.abs(Wq), np.abs(b32))
    net = _net(nx * ny * nz, "bf16", train=False)
    net.set_params(L.flatten(params))
    out = net.layer_forward(layer, shape, xd)
    out = out.to(torch.float64).cpu().numpy().reshape(ref.shape)
    if layer < 3:
        ref = np.maximum(ref, 0.0)
        tol = 2.0 ** -8 * np.abs(ref) + 1e-4 * bound
    else:
        tol = 1e-5 * bound
    err = np.abs(out - ref)
    assert np.all(err <= tol), (float(np.max(err / (tol + 1e-300))), float(np.max(err)))


@pytest.mark.parametrize("loss", ["mse", "energy"])
@pytest.mark.parametrize("shape", [(8, 8, 8), (13, 10, 7)])
def test_loss_and_gradient_f64(shape, loss):
    nx, ny, nz = shape
    g = np.random.default_rng(21)
    params = L.init_params(6)
    x = g.standard_normal((nz, ny, nx))
    t = 0.3 * g.standard_normal((nz, ny, nx))
    ref_loss, ref_grads = L.loss_and_grads(params, x, t, loss=loss)
    net = _net(nx * ny * nz, "f64")
    net.set_params(L.flatten(params))
    val, grad = net.loss_grad(shape, _dev(x.ravel()), _dev(t.ravel()), loss=loss)
    assert abs(val - ref_loss) <= 1e-12 * abs(ref_loss)
    ref = L.flatten(ref_grads)
    for l in range(4):
        lo, hi = _offsets(l)
        assert np.linalg.norm(grad[lo:hi] - ref[lo:hi]) <= 1e-10 * np.linalg.norm(ref[lo:hi]), l


def _offsets(l):
    off = 0
    for i, (ci, co) in enumerate(zip(L.CHANNELS[:-1], L.CHANNELS[1:])):
        n = 27 * ci * co + co
        if i == l:
            return off, off + n
        off += n


@pytest.mark.parametrize("loss", ["mse", "energy"])
@pytest.mark.parametrize("shape", [(8, 8, 8), (40, 12, 9)])
def test_loss_and_gradient_bf16(shape, loss):
    """Against the oracle rounded where the kernels store: layer gradients agree
    to 2e-3 in norm (FP32 accumulation plus occasional one-ulp flips of a stored
    bf16 value), the loss to 1e-3."""
    nx, ny, nz = shape
    g = np.random.default_rng(22)
    params = L.init_params(7)
    xd, xq = _bf16_dev(g.standard_normal(nx * ny * nz))
    t = (0.3 * g.standard_normal(nx * ny * nz)).astype(np.float32)
    pq = [(W, b.astype(np.float32).astype(np.float64)) for W, b in params]
    ref_loss, ref_grads = L.loss_and_grads(pq, xq.reshape(nz, ny, nx), t.astype(np.float64).reshape(nz, ny, nx),
                                           loss=loss, quantize=L.round_bf16)
    net = _net(nx * ny * nz, "bf16")
    net.set_params(L.flatten(params))
    val, grad = net.loss_grad(shape, xd, _dev(t, torch.float32), loss=loss)
    assert abs(val - ref_loss) <= 1e-3 * abs(ref_loss)
    ref = L.flatten(ref_grads)
    for l in range(4):
        lo, hi = _offsets(l)
        rel = np.linalg.norm(grad[lo:hi] - ref[lo:hi]) / np.linalg.norm(ref[lo:hi])
        assert rel <= 2e-3, (l, rel)


def test_adam_step_f64():
    shape = (9, 8, 7)
    nx, ny, nz = shape
    g = np.random.default_rng(23)
    params = L.init_params(8)
    x = g.standard_normal((nz, ny, nx))
    t = 0.3 * g.standard_normal((nz, ny, nx))
    net = _net(nx * ny * nz, "f64")
    net.set_params(L.flatten(params))
    state = L.zero_state(params)
    cur = params
    lr = 1e-3
    for step in range(1, 4):
        _, ref_grads = L.loss_and_grads(cur, x, t)
        net.loss_grad(shape, _dev(x.ravel()), _dev(t.ravel()))
        net.adam_step(lr)
        cur = L.adam_step(cur, ref_grads, state, lr, step)
        gflat = np.abs(L.flatten(ref_grads))
        got, ref = net.get_params(), L.flatten(cur)
        # Adam divides by |g|: elements whose gradient is at rounding level are excluded
        big = gflat > 1e-6 * gflat.max()
        assert np.max(np.abs(got - ref)[big]) <= 1e-8 * lr
        assert np.max(np.abs(got - ref)) <= 2 * step * lr


def test_correction_f64():
    shape = (20, 18, 16)
    nx, ny, nz = shape
    c = (441.0, 441.0, 441.0)
    params = L.init_params(9)
    r = synth.rhs(nx, ny, nz, 31)
    s = 1e-3 * synth.rhs(nx, ny, nz, 32)
    rp = r - O.matvec(s, shape, c)
    cbar = sum(c) / 3
    sigma = np.sqrt(np.mean((rp / cbar) ** 2))
    ref = s + sigma * L.forward(params, (rp / (cbar * sigma)).reshape(nz, ny, nx)).ravel()
    G = _smg(shape, c, 1, 0)
    net = _net(G.n, "f64", train=False)
    net.set_params(L.flatten(params))
    out, sig = net.correct(G, _dev(r), _dev(s))
    out = out.cpu().numpy()
    assert abs(sig - sigma) <= 1e-13 * sigma
    assert np.linalg.norm(out - ref) <= 1e-10 * np.linalg.norm(ref - s)


def test_correction_bf16():
    """bf16 network input and activations, as in the oracle with the same roundings:
    the correction agrees to 2e-3 relative in norm."""
    shape = (70, 24, 20)
    nx, ny, nz = shape
    c = (1.0, 1.0, 1.0)
    params = L.init_params(10)
    r = synth.rhs(nx, ny, nz, 33)
    s = 0.1 * synth.rhs(nx, ny, nz, 34)
    rp = r - O.matvec(s, shape, c)
    sigma = np.sqrt(np.mean(rp ** 2))
    pq = [(W, b.astype(np.float32).astype(np.float64)) for W, b in params]
    y = L.forward(pq, (rp / sigma).reshape(nz, ny, nx), quantize=L.round_bf16).ravel()
    G = _smg(shape, c, 1, 0)
    net = _net(G.n, "bf16", train=False)
    net.set_params(L.flatten(params))
    out, sig = net.correct(G, _dev(r), _dev(s))
    corr = (out.cpu().numpy() - s) / sig
    assert abs(sig - sigma) <= 1e-13 * sigma
    assert np.linalg.norm(corr - y) <= 2e-3 * np.linalg.norm(y)


def test_correction_bf16_full_size_sampled():
    """The bf16 correction at 256^3 (the size the learned post-smoother is applied
    at, c = 257^2) against the oracle at sampled points: corners, edges, faces
    and the interior.  An output point depends on the input within distance 4
    (four 3x3x3 layers), so the oracle runs the network on the 9^3 patch around
    each sample, cut at the domain boundary where the zero padding is the same
    as on the whole grid.  sigma is a global mean, compared in full."""
    n = 256
    shape = (n, n, n)
    c = ((n + 1.0) ** 2,) * 3
    params = L.init_params(11)
    r = synth.rhs(n, n, n, 35)
    s = 0.1 * synth.rhs(n, n, n, 36) / c[0]
    rp = r - O.matvec(s, shape, c)
    cbar = sum(c) / 3
    sigma = np.sqrt(np.mean((rp / cbar) ** 2))
    G = _smg(shape, c, 1, 0)
    net = _net(G.n, "bf16", train=False)
    net.set_params(L.flatten(params))
    out, sig = net.correct(G, _dev(r), _dev(s))
    corr = ((out.cpu().numpy() - s) / sig).reshape(n, n, n)
    assert abs(sig - sigma) <= 1e-12 * sigma
    x = (rp / (cbar * sigma)).reshape(n, n, n)
    pq = [(W, b.astype(np.float32).astype(np.float64)) for W, b in params]
    g = np.random.default_rng(5)
    ends = [0, 1, 4, n - 5, n - 2, n - 1]
    pts = [(k, j, i) for k in (0, n - 1) for j in (0, n - 1) for i in (0, n - 1)]
    pts += [tuple(int(v) for v in g.choice(ends, 3)) for _ in range(16)]
    pts += [tuple(int(v) for v in g.integers(0, n, 3)) for _ in range(24)]
    got, want = [], []
    for k, j, i in pts:
        lo = [max(0, v - 4) for v in (k, j, i)]
        hi = [min(n, v + 5) for v in (k, j, i)]
        patch = x[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        y = L.forward(pq, patch, quantize=L.round_bf16)
        want.append(y[k - lo[0], j - lo[1], i - lo[2]])
        got.append(corr[k, j, i])
    got, want = np.array(got), np.array(want)
    assert np.linalg.norm(got - want) <= 5e-3 * np.linalg.norm(want)
    assert np.max(np.abs(got - want)) <= 2e-2 * np.sqrt(np.mean(want ** 2))


def test_pairs_match_oracle_f64():
    shape = (20, 18, 16)
    nx, ny, nz = shape
    c = (441.0, 441.0, 441.0)
    Gp, Ge = _smg(shape, c, 1, 0), _smg(shape, c, 1, 1)
    net = _net(Gp.n, "f64")
    inputs, targets, sig = net.make_pairs(Gp, Ge, 2, 500, exact_rtol=1e-13, exact_max_iter=100)
    inputs = inputs.cpu().numpy().reshape(2, -1)
    targets = targets.cpu().numpy().reshape(2, -1)
    S = O.SMG(shape, c, 1, 0)
    cbar = sum(c) / 3
    for i in range(2):
        b = synth.rhs(nx, ny, nz, 500 + i)
        xp = S.apply(b)
        rp = b - O.matvec(xp, shape, c)
        sigma = np.sqrt(np.mean((rp / cbar) ** 2))
        xs = D.dst_solve(b, shape, c)
        assert abs(sig[i] - sigma) <= 1e-11 * sigma
        assert np.linalg.norm(inputs[i] - rp / (cbar * sigma)) <= 1e-10 * np.linalg.norm(rp / (cbar * sigma))
        e = (xs - xp) / sigma
        assert np.linalg.norm(targets[i] - e) <= 1e-8 * np.linalg.norm(e)


def test_training_reduces_loss_bf16():
    shape = (24, 24, 24)
    n = 24 ** 3
    c = ((25.0) ** 2,) * 3
    Gp, Ge = _smg(shape, c, 1, 0), _smg(shape, c, 1, 1)
    net = _net(n, "bf16")
    inputs, targets, _ = net.make_pairs(Gp, Ge, 8, 900, exact_rtol=1e-10)
    net.set_params(L.flatten(L.init_params(0)))
    order = np.random.default_rng(0).integers(0, 8, 150)
    hist = net.train(shape, inputs, targets, order, np.full(150, 2e-3))
    assert np.all(np.isfinite(hist))
    assert hist[-20:].mean() < 0.8 * hist[:5].mean(), (hist[:5], hist[-20:])


def _corrupt(kind, prec):
    p = L.flatten(L.init_params(0))
    if kind == "huge":
        # overflows the storage format within the four layers
        return np.full_like(p, 1e30 if prec == "bf16" else 1e150)
    q = np.zeros_like(p)
    q[-1] = 1e4                 # output bias: a constant correction
    return q


@pytest.mark.parametrize("kind", ["huge", "constant"])
@pytest.mark.parametrize("prec", ["bf16", "f64"])
def test_fallback_on_corrupted_network(kind, prec):
    n = 32
    shape, c = (n, n, n), ((n + 1.0) ** 2,) * 3
    G = _smg(shape, c, 1, 0)
    b = _dev(synth.rhs(n, n, n, 1))
    _, plain = G.fpcg(b)
    net = _net(G.n, prec, train=False)
    net.set_params(_corrupt(kind, prec))
    x, info = G.fpcg_learned(net, b)
    assert info.status == 0 and info.rel_res <= 1e-8 and info.true_rel_res <= 1.5e-8
    assert info.fallback_reason != "none"
    if kind == "huge":
        assert info.fallback_reason == "nonfinite" and info.fallback_iter == 0
    assert info.fallback_iter <= 3
    assert info.iters <= plain.iters + info.fallback_iter + 2


def test_zero_network_is_plain_fpcg():
    """All-zero parameters give a zero correction: the solve is plain FPCG-SMG(1,0)."""
    n = 32
    shape, c = (n, n, n), ((n + 1.0) ** 2,) * 3
    G = _smg(shape, c, 1, 0)
    b = _dev(synth.rhs(n, n, n, 1))
    x0, plain = G.fpcg(b, history=True)
    net = _net(G.n, "bf16", train=False)
    net.set_params(np.zeros(L.NPARAMS))
    x1, info = G.fpcg_learned(net, b, history=True)
    assert info.fallback_reason == "none" and info.iters == plain.iters
    assert np.allclose(info.history, plain.history, rtol=1e-12, atol=0)


def _loop_nets():
    """Networks for the flexible-PCG loop parity: no correction, a mild one,
    one that stagnates, one that overflows, one with a huge constant output."""
    zero = [(W * 0, b * 0) for W, b in L.init_params(0)]
    mild = [(W * (0.1 if i == 3 else 1.0), b * 0) for i, (W, b) in enumerate(L.init_params(1))]
    he = L.init_params(0)
    huge = L.unflatten(np.full(L.NPARAMS, 1e150))
    const = L.unflatten(_corrupt("constant", "f64"))
    return {"zero": zero, "mild": mild, "he": he, "huge": huge, "constant": const}


@pytest.mark.parametrize("name", ["zero", "mild", "he", "huge", "constant"])
def test_learned_fpcg_loop_matches_oracle_f64(name):
    """The learned flexible PCG (V-cycle without post-smoothing, network
    correction, the three fallback rules) against the oracle's composition of
    the same steps, with the network in FP64: the same fallback decision (reason,
    and iteration within one), iteration counts within one, solutions to 1e-6."""
    n = 24
    shape, c = (n, n, n), ((n + 1.0) ** 2,) * 3
    b = synth.rhs(n, n, n, 1)
    params = _loop_nets()[name]
    xr, kr, rels, fb_iter, fb_reason = L.fpcg_learned(b, shape, c, O.SMG(shape, c, 1, 0), params)
    G = _smg(shape, c, 1, 0)
    net = _net(G.n, "f64", train=False)
    net.set_params(L.flatten(params))
    x, info = G.fpcg_learned(net, _dev(b), history=True)
    print(name, "gpu", info.iters, info.fallback_reason, info.fallback_iter, "oracle", kr, fb_reason, fb_iter)
    assert info.status == 0 and rels[-1] <= 1e-8
    assert info.fallback_reason == fb_reason
    assert abs(info.fallback_iter - fb_iter) <= 1
    assert abs(info.iters - kr) <= 1
    assert info.true_rel_res <= 1.5e-8
    assert np.linalg.norm(x.cpu().numpy() - xr) <= 1e-6 * np.linalg.norm(xr)
    k = min(len(info.history), len(rels), 6)
    assert np.allclose(info.history[:k], rels[:k], rtol=1e-6, atol=1e-14)


def test_learned_fpcg_loop_matches_oracle_bf16():
    """The same loop with the network in BF16 storage and FP32 accumulation,
    against the oracle rounding where the kernels store: iterations within one,
    the same fallback decision, solutions to 1e-6."""
    n = 24
    shape, c = (n, n, n), ((n + 1.0) ** 2,) * 3
    b = synth.rhs(n, n, n, 3)
    params = _loop_nets()["mild"]
    pq = [(W, bb.astype(np.float32).astype(np.float64)) for W, bb in params]
    xr, kr, rels, fb_iter, fb_reason = L.fpcg_learned(b, shape, c, O.SMG(shape, c, 1, 0), pq,
                                                      quantize=L.round_bf16)
    G = _smg(shape, c, 1, 0)
    net = _net(G.n, "bf16", train=False)
    net.set_params(L.flatten(params))
    x, info = G.fpcg_learned(net, _dev(b))
    assert info.status == 0 and info.fallback_reason == fb_reason
    assert abs(info.iters - kr) <= 1
    assert np.linalg.norm(x.cpu().numpy() - xr) <= 1e-6 * np.linalg.norm(xr)


def test_trained_network_gains_over_plain_smg10():
    """What the trained network buys: trained on the GPU (pairs from SMG(1,0),
    exact solves by FPCG-SMG(1,1), Adam on the energy loss) at 32^3, then used
    in flexible PCG on right-hand sides it never saw.  It must take fewer
    iterations than FPCG-SMG(1,0) on average and never more, reach the same
    true residual, and need no fallback.  The time ratio is printed."""
    import time
    n = 32
    shape, c = (n, n, n), ((n + 1.0) ** 2,) * 3
    Gp, Ge = _smg(shape, c, 1, 0), _smg(shape, c, 1, 1)
    net = _net(Gp.n, "bf16")
    npairs, steps = 256, 1500
    inputs, targets, _ = net.make_pairs(Gp, Ge, npairs, 20000, exact_rtol=1e-10)
    net.set_params(synth.he_init(0))
    order = np.resize(np.random.default_rng(0).permutation(npairs), steps)
    lr = 2e-3 * (0.05 + 0.95 * 0.5 * (1 + np.cos(np.pi * np.arange(steps) / steps)))
    hist = net.train(shape, inputs, targets, order, lr, loss="energy")
    assert np.all(np.isfinite(hist))
    ev = _net(Gp.n, "bf16", train=False)
    ev.set_params(net.get_params())
    gains, ratios = [], []
    for seed in (7, 8, 9, 10):
        b = _dev(synth.rhs(n, n, n, seed))
        for _ in range(2):          # the second of each pair is timed
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, plain = Gp.fpcg(b)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, lrn = Gp.fpcg_learned(ev, b)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
        print(f"seed {seed}: SMG(1,0) {plain.iters} it {1e3 * (t1 - t0):.2f} ms, "
              f"learned {lrn.iters} it {1e3 * (t2 - t1):.2f} ms, fallback {lrn.fallback_reason}")
        assert lrn.status == 0 and lrn.fallback_reason == "none" and lrn.true_rel_res <= 1.5e-8
        assert lrn.iters <= plain.iters
        gains.append(plain.iters - lrn.iters)
        ratios.append((t2 - t1) / (t1 - t0))
    print(f"mean iteration gain {np.mean(gains):.2f}, mean time ratio learned/plain {np.mean(ratios):.2f}")
    assert np.mean(gains) >= 1.0
