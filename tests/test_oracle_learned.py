"""Pins of the learned-smoother network oracle (FP64 NumPy):
the convolution against torch's CPU conv3d (an independent implementation),
the hand-derived backward pass against central finite differences, and the
Adam step against torch.optim.Adam."""
import numpy as np
import pytest
import torch

from oracle import learned as L


def test_parameter_count():
    assert L.NPARAMS == 14737
    p = L.init_params(0)
    assert L.flatten(p).size == L.NPARAMS
    q = L.unflatten(L.flatten(p))
    for (W, b), (W2, b2) in zip(p, q):
        assert np.array_equal(W, W2) and np.array_equal(b, b2)


@pytest.mark.parametrize("ci,co,shape", [(1, 16, (5, 6, 7)), (16, 16, (4, 5, 3)), (16, 1, (6, 4, 5))])
def test_conv_equals_torch_conv3d(ci, co, shape):
    g = np.random.default_rng(ci * 100 + co)
    x = g.standard_normal(shape + (ci,))
    W = g.standard_normal((3, 3, 3, ci, co))
    b = g.standard_normal(co)
    ours = L.conv(x, W, b)
    xt = torch.from_numpy(x).permute(3, 0, 1, 2)[None]              # N C D H W
    Wt = torch.from_numpy(W).permute(4, 3, 0, 1, 2).contiguous()     # Cout Cin kD kH kW
    ref = torch.nn.functional.conv3d(xt, Wt, torch.from_numpy(b), padding=1)[0].permute(1, 2, 3, 0).numpy()
    assert np.allclose(ours, ref, rtol=1e-12, atol=1e-12)


def test_conv_backward_finite_differences():
    g = np.random.default_rng(3)
    x = g.standard_normal((4, 3, 5, 2))
    W = g.standard_normal((3, 3, 3, 2, 3))
    b = g.standard_normal(3)
    proj = g.standard_normal((4, 3, 5, 3))
    f = lambda x_, W_, b_: float(np.sum(L.conv(x_, W_, b_) * proj))
    din, dW, db = L.conv_backward(x, W, proj)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (2, 1, 4, 1), (3, 2, 2, 0)]:
        e = np.zeros_like(x)
        e[idx] = h
        assert abs((f(x + e, W, b) - f(x - e, W, b)) / (2 * h) - din[idx]) < 1e-7
    for idx in [(0, 0, 0, 0, 0), (1, 2, 0, 1, 2), (2, 2, 2, 1, 1)]:
        e = np.zeros_like(W)
        e[idx] = h
        assert abs((f(x, W + e, b) - f(x, W - e, b)) / (2 * h) - dW[idx]) < 1e-7
    e = np.zeros_like(b)
    e[1] = h
    assert abs((f(x, W, b + e) - f(x, W, b - e)) / (2 * h) - db[1]) < 1e-7


def test_loss_gradients_finite_differences():
    g = np.random.default_rng(5)
    params = L.init_params(1)
    x = g.standard_normal((5, 5, 5))
    t = g.standard_normal((5, 5, 5))
    loss, grads = L.loss_and_grads(params, x, t)
    h = 1e-6
    flat = L.flatten(params)
    gflat = L.flatten(grads)
    for k in [0, 17, 431, 440, 5000, 14000, 14300, L.NPARAMS - 1]:
        e = np.zeros_like(flat)
        e[k] = h
        lp = L.loss_and_grads(L.unflatten(flat + e), x, t)[0]
        lm = L.loss_and_grads(L.unflatten(flat - e), x, t)[0]
        assert abs((lp - lm) / (2 * h) - gflat[k]) <= 1e-6 * max(1.0, abs(gflat[k]))


def test_adam_matches_torch():
    params = L.init_params(2)
    g = np.random.default_rng(7)
    grads_seq = [[(g.standard_normal(W.shape), g.standard_normal(b.shape)) for W, b in params] for _ in range(3)]
    tp = [torch.nn.Parameter(torch.from_numpy(a.copy())) for W, b in params for a in (W, b)]
    opt = torch.optim.Adam(tp, lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    state = L.zero_state(params)
    cur = params
    for t, gs in enumerate(grads_seq, start=1):
        cur = L.adam_step(cur, gs, state, 1e-3, t)
        for p_, gr in zip(tp, [a for pair in gs for a in pair]):
            p_.grad = torch.from_numpy(gr.copy())
        opt.step()
    ours = L.flatten(cur)
    ref = np.concatenate([p_.detach().numpy().ravel() for p_ in tp])
    assert np.allclose(ours, ref, rtol=1e-12, atol=1e-14)


def test_energy_loss_gradients_finite_differences():
    g = np.random.default_rng(11)
    params = L.init_params(4)
    x = g.standard_normal((4, 5, 6))
    t = g.standard_normal((4, 5, 6))
    loss, grads = L.loss_and_grads(params, x, t, loss="energy")
    # energy norm of the unit stencil is a positive quadratic form
    d = L.forward(params, x) - t
    assert loss > 0 and np.isclose(loss, float(np.sum(d * L.unit_laplacian(d))) / d.size, rtol=1e-13)
    flat, gflat = L.flatten(params), L.flatten(grads)
    h = 1e-6
    for k in [3, 440, 7000, 14300, L.NPARAMS - 2]:
        e = np.zeros_like(flat)
        e[k] = h
        lp = L.loss_and_grads(L.unflatten(flat + e), x, t, loss="energy")[0]
        lm = L.loss_and_grads(L.unflatten(flat - e), x, t, loss="energy")[0]
        assert abs((lp - lm) / (2 * h) - gflat[k]) <= 1e-6 * max(1.0, abs(gflat[k]))


def test_unit_laplacian_is_the_dirichlet_stencil():
    # on a 1-voxel-thick slab the stencil is 6*d minus in-plane neighbours only
    d = np.zeros((3, 3, 3))
    d[1, 1, 1] = 1.0
    Ld = L.unit_laplacian(d)
    assert Ld[1, 1, 1] == 6.0 and Ld[0, 1, 1] == -1.0 and Ld[1, 1, 2] == -1.0 and Ld[0, 0, 0] == 0.0
    assert np.isclose(np.sum(Ld), 0.0)


def test_round_bf16_matches_torch():
    g = np.random.default_rng(12)
    a = np.concatenate([g.standard_normal(1000) * 10.0 ** g.integers(-20, 20, 1000), [0.0, -0.0, 1.0, 3.0]])
    ours = L.round_bf16(a)
    ref = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ours, ref)


def test_quantized_loss_without_rounding_equals_plain():
    g = np.random.default_rng(13)
    params = L.init_params(5)
    x = g.standard_normal((4, 4, 5))
    t = g.standard_normal((4, 4, 5))
    a = L.loss_and_grads(params, x, t)
    b = L.loss_and_grads(params, x, t, quantize=lambda v: v)
    assert a[0] == b[0]
    assert np.array_equal(L.flatten(a[1]), L.flatten(b[1]))


# --- the flexible-PCG loop with the learned correction ----------------------

def _loop_problem(n=12, seed=1):
    import synth
    from oracle import oracle as O
    shape, c = (n, n, n), ((n + 1.0) ** 2,) * 3
    return shape, c, synth.rhs(n, n, n, seed), O.SMG(shape, c, 1, 0)


def test_learned_loop_with_zero_network_is_the_c_oracles_fpcg():
    """A network with all-zero parameters adds nothing: the NumPy loop must be
    the C oracle's flexible PCG (an independent implementation of equation
    (2)), iteration for iteration."""
    from oracle import oracle as O
    shape, c, b, S = _loop_problem()
    zero = [(W * 0, bb * 0) for W, bb in L.init_params(0)]
    x, k, rels, fb_iter, fb_reason = L.fpcg_learned(b, shape, c, S, zero)
    ref = O.krylov(O.FPCG, b, shape, c, S)
    assert fb_reason == "none" and fb_iter == -1
    assert k == ref.iters
    assert np.allclose(rels, ref.hist, rtol=1e-9, atol=1e-15)
    assert np.linalg.norm(x - ref.x) <= 1e-10 * np.linalg.norm(ref.x)


def test_learned_loop_fallbacks():
    """Each fallback rule fires where its condition first holds, and the solve
    continues as plain flexible PCG (so it still converges)."""
    from oracle import oracle as O
    shape, c, b, S = _loop_problem()
    plain = O.krylov(O.FPCG, b, shape, c, S)
    # overflow: non-finite at once, then exactly plain FPCG
    huge = L.unflatten(np.full(L.NPARAMS, 1e150))
    x, k, rels, fi, fr = L.fpcg_learned(b, shape, c, S, huge)
    assert (fr, fi) == ("nonfinite", 0) and k == plain.iters
    assert np.allclose(rels, plain.hist, rtol=1e-9, atol=1e-15)
    # a constant output of the sign that makes (s, r) negative
    s0 = S.apply(b)
    rp = b - O.matvec(s0, shape, c)
    sigma = np.sqrt(np.mean((rp / c[0]) ** 2))
    v = -10.0 * abs(float(s0 @ b)) / (sigma * abs(b.sum())) * np.sign(b.sum())
    p = np.zeros(L.NPARAMS)
    p[-1] = v
    x, k, rels, fi, fr = L.fpcg_learned(b, shape, c, S, L.unflatten(p))
    assert (fr, fi) == ("sr", 0) and k == plain.iters
    # a constant output of the other sign keeps (s, r) > 0 but spoils the
    # preconditioner: the residual stops falling and the network is dropped
    p[-1] = -v
    x, k, rels, fi, fr = L.fpcg_learned(b, shape, c, S, L.unflatten(p))
    assert fr == "stagnation" and fi >= 2
    assert rels[fi] > 0.9 * rels[fi - 2]
    assert np.all(rels[2:fi] <= 0.9 * rels[:fi - 2])      # the first step where the rule holds
    assert rels[-1] <= 1e-8
    assert np.linalg.norm(b - O.matvec(x, shape, c)) <= 1.5e-8 * np.linalg.norm(b)


def test_learned_correction_definition():
    """correction() forms r' = r - A s, sigma = rms(r'/cbar) and adds sigma times
    the network of r'/(cbar sigma): with a network whose only nonzero parameter
    is the output bias beta, the result is s + sigma beta everywhere."""
    from oracle import oracle as O
    shape, c, b, S = _loop_problem(8)
    s = S.apply(b)
    p = np.zeros(L.NPARAMS)
    p[-1] = 0.37
    out, sigma = L.correction(L.unflatten(p), b, s, shape, c)
    rp = b - O.matvec(s, shape, c)
    assert np.isclose(sigma, np.linalg.norm(rp / c[0]) / np.sqrt(rp.size), rtol=1e-14)
    assert np.allclose(out - s, 0.37 * sigma, rtol=1e-13, atol=0)
