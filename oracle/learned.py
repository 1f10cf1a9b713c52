"""FP64 oracle of the learned post-smoother network.  TEST INFRASTRUCTURE ONLY.

The network (a form added beside the paper's method, not in the paper) maps a
residual to a correction: four 3x3x3 convolutions with zero padding,
1 -> 16 -> 16 -> 16 -> 1 channels, ReLU after the first three, a bias per
output channel.  Written from the definition of a cross-correlation
    out[z,y,x,o] = b[o] + sum_{dz,dy,dx,i} W[dz,dy,dx,i,o] in[z+dz-1, y+dy-1, x+dx-1, i]
(inputs outside the grid are zero), with the backward pass derived by hand:
    d in[z,y,x,i] = sum_{dz,dy,dx,o} W[dz,dy,dx,i,o] g[z-dz+1, y-dy+1, x-dx+1, o]
    d W[dz,dy,dx,i,o] = sum_{z,y,x} in[z+dz-1, y+dy-1, x+dx-1, i] g[z,y,x,o]
    d b[o] = sum_{z,y,x} g[z,y,x,o]
where g is the gradient at the layer's output after the ReLU mask.
Arrays are channels-last: (nz, ny, nx, C).  Weights: (3, 3, 3, Cin, Cout).
"""
from __future__ import annotations

import numpy as np

CHANNELS = (1, 16, 16, 16, 1)


def init_params(seed: int = 0):
    """He-style initial weights from a seeded NumPy generator (tests only)."""
    g = np.random.default_rng(seed)
    params = []
    for ci, co in zip(CHANNELS[:-1], CHANNELS[1:]):
        W = g.standard_normal((3, 3, 3, ci, co)) * np.sqrt(2.0 / (27 * ci))
        b = 0.01 * g.standard_normal(co)
        params.append((W, b))
    return params


def _pad(a):
    return np.pad(a, ((1, 1), (1, 1), (1, 1), (0, 0)))


def conv(inp, W, b):
    nz, ny, nx, _ = inp.shape
    p = _pad(inp)
    out = np.broadcast_to(b, (nz, ny, nx, W.shape[-1])).astype(np.float64).copy()
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                out += p[dz:dz + nz, dy:dy + ny, dx:dx + nx, :] @ W[dz, dy, dx]
    return out


def conv_backward(inp, W, g):
    """(d inp, d W, d b) for out = conv(inp, W, b) and output gradient g."""
    nz, ny, nx, _ = inp.shape
    p = _pad(inp)
    gp = _pad(g)
    din = np.zeros_like(inp)
    dW = np.zeros_like(W)
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                # input point (z,y,x) feeds output (z-dz+1, y-dy+1, x-dx+1)
                din += gp[2 - dz:2 - dz + nz, 2 - dy:2 - dy + ny, 2 - dx:2 - dx + nx, :] @ W[dz, dy, dx].T
                dW[dz, dy, dx] = np.einsum("zyxi,zyxo->io", p[dz:dz + nz, dy:dy + ny, dx:dx + nx, :], g)
    db = g.sum(axis=(0, 1, 2))
    return din, dW, db


def forward(params, x, keep=False, quantize=None):
    """x: (nz, ny, nx) -> (nz, ny, nx); with keep=True also the layer outputs.
    quantize: optional rounding of the input, the weights and every activation
    after its ReLU (where a reduced-precision implementation stores them)."""
    q = quantize if quantize is not None else (lambda v: v)
    a = q(x[..., None].astype(np.float64))
    acts = [a]
    for li, (W, b) in enumerate(params):
        a = conv(a, q(W), b)
        if li < len(params) - 1:
            a = q(np.maximum(a, 0.0))
        acts.append(a)
    return (a[..., 0], acts) if keep else a[..., 0]


def unit_laplacian(d):
    """The 7-point stencil 6 d - (sum of the six neighbours), zero outside the grid."""
    p = np.pad(d, 1)
    nz, ny, nx = d.shape
    nb = (p[:-2, 1:-1, 1:-1] + p[2:, 1:-1, 1:-1] + p[1:-1, :-2, 1:-1] + p[1:-1, 2:, 1:-1]
          + p[1:-1, 1:-1, :-2] + p[1:-1, 1:-1, 2:])
    return 6.0 * d - nb


def loss_and_grads(params, x, target, loss="mse", quantize=None):
    """Loss and its parameter gradients.

    loss="mse":    mean((N(x) - target)^2)
    loss="energy": mean(d * L d), d = N(x) - target, L the unit 7-point stencil
                   (the error in the energy norm of the unit-stencil operator)
    quantize: optional rounding applied where a reduced-precision implementation
    stores values: the input, the weights, every activation after its ReLU, and
    the gradient at each layer output after the ReLU mask (biases, the final
    output and the accumulated weight gradients stay exact).
    """
    q = quantize if quantize is not None else (lambda a: a)
    qp = [(q(W), b) for W, b in params]
    a = q(x[..., None].astype(np.float64))
    acts = [a]
    for li, (W, b) in enumerate(qp):
        a = conv(a, W, b)
        if li < len(qp) - 1:
            a = q(np.maximum(a, 0.0))
        acts.append(a)
    y = a[..., 0]
    n = y.size
    diff = y - target
    if loss == "mse":
        val = float(np.sum(diff * diff) / n)
        g = (2.0 / n) * diff
    elif loss == "energy":
        Ld = unit_laplacian(diff)
        val = float(np.sum(diff * Ld) / n)
        g = (2.0 / n) * Ld
    else:
        raise ValueError(loss)
    g = q(g[..., None])
    grads = [None] * len(qp)
    for li in range(len(qp) - 1, -1, -1):
        W, _ = qp[li]
        if li < len(qp) - 1:
            g = q(g * (acts[li + 1] > 0))        # ReLU mask from the layer's output
        din, dW, db = conv_backward(acts[li], W, g)
        grads[li] = (dW, db)
        g = din
    return val, grads


def round_bf16(a):
    """Round to bfloat16 (nearest even) through binary32, returned as float64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(a))


def adam_step(params, grads, state, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015) with bias correction; state holds (m, v) pairs."""
    new = []
    for k, ((W, b), (dW, db)) in enumerate(zip(params, grads)):
        outs = []
        for j, (p, gr) in enumerate(((W, dW), (b, db))):
            m, v = state[2 * k + j]
            m = beta1 * m + (1 - beta1) * gr
            v = beta2 * v + (1 - beta2) * gr * gr
            state[2 * k + j] = (m, v)
            mh = m / (1 - beta1 ** t)
            vh = v / (1 - beta2 ** t)
            outs.append(p - lr * mh / (np.sqrt(vh) + eps))
        new.append(tuple(outs))
    return new


def zero_state(params):
    st = []
    for W, b in params:
        st.append((np.zeros_like(W), np.zeros_like(W)))
        st.append((np.zeros_like(b), np.zeros_like(b)))
    return st


def flatten(params) -> np.ndarray:
    """Parameters in the library's flat order: per layer W (3,3,3,Cin,Cout) then b."""
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params])


def unflatten(flat: np.ndarray):
    out, off = [], 0
    for ci, co in zip(CHANNELS[:-1], CHANNELS[1:]):
        nw = 27 * ci * co
        W = flat[off:off + nw].reshape(3, 3, 3, ci, co)
        off += nw
        b = flat[off:off + co]
        off += co
        out.append((W.copy(), b.copy()))
    return out


NPARAMS = sum(27 * ci * co + co for ci, co in zip(CHANNELS[:-1], CHANNELS[1:]))


# ---------------------------------------------------------------------------
# Flexible PCG with the learned post-smoother (the form beside the paper).
# ---------------------------------------------------------------------------
FALLBACK_NONE, FALLBACK_SR, FALLBACK_NONFINITE, FALLBACK_STAGNATION = "none", "sr", "nonfinite", "stagnation"


def correction(params, r, s, shape, c, quantize=None):
    """s + sigma N(r' / (cbar sigma)) with r' = r - A s, cbar = (cx + cy + cz)/3 and
    sigma = rms(r' / cbar): the preconditioned residual after one V-cycle without
    post-smoothing, corrected by the network on the normalised remaining residual."""
    from oracle import oracle as O
    nx, ny, nz = shape
    rp = r - O.matvec(s, shape, c)
    cbar = (c[0] + c[1] + c[2]) / 3.0
    sigma = float(np.sqrt(np.mean((rp / cbar) ** 2)))
    with np.errstate(over="ignore", invalid="ignore"):      # a corrupted network may overflow
        y = forward(params, (rp / (cbar * sigma)).reshape(nz, ny, nx), quantize=quantize).ravel()
        return s + sigma * y, sigma


def fpcg_learned(b, shape, c, smg, params, rtol=1e-8, max_iter=500, x0=None, quantize=None):
    """Algorithm 1 of Section 2 with beta from equation (2), whose flexibility
    admits a nonlinear preconditioner: s_k = correction(T r_k) with T = smg (one
    V-cycle, normally without post-smoothing).  The network is dropped for the
    rest of the solve (s_k = T r_k from then on) when
      * the corrected s_k has a non-finite entry          -> "nonfinite" at iteration k,
      * (s_k, r_k) <= 0 for the corrected s_k              -> "sr" at iteration k,
      * ||r_{k+1}|| > 0.9 ||r_{k-1}|| (k >= 1)             -> "stagnation" from iteration k+1.
    beta_k = (s_k, r_k - r_{k-1}) / (s_{k-1}, r_{k-1}), with r_{k-1} stored.
    Returns (x, iterations, relative residual history, fallback iteration, reason)."""
    from oracle import oracle as O
    b = np.asarray(b, dtype=np.float64).ravel()
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64).ravel()
    r = b - O.matvec(x, shape, c)
    bden = np.linalg.norm(b) or 1.0
    rels = [np.linalg.norm(r) / bden]
    active, fb_iter, fb_reason = True, -1, FALLBACK_NONE
    p = r_prev = None
    sr_prev = 0.0
    k = 0
    while k < max_iter and rels[-1] > rtol:
        s = smg.apply(r)
        if active:
            sl, _ = correction(params, r, s, shape, c, quantize)
            if not np.all(np.isfinite(sl)):
                active, fb_iter, fb_reason = False, k, FALLBACK_NONFINITE
            elif not float(sl @ r) > 0.0:
                active, fb_iter, fb_reason = False, k, FALLBACK_SR
            else:
                s = sl
        sr = float(s @ r)
        if k == 0:
            p = s.copy()
        else:
            beta = (sr - float(s @ r_prev)) / sr_prev
            p = s + beta * p
        q = O.matvec(p, shape, c)
        alpha = sr / float(p @ q)
        r_prev = r.copy()
        x = x + alpha * p
        r = r - alpha * q
        sr_prev = sr
        rels.append(np.linalg.norm(r) / bden)
        if active and k >= 1 and rels[k + 1] > 0.9 * rels[k - 1]:
            active, fb_iter, fb_reason = False, k + 1, FALLBACK_STAGNATION
        k += 1
    return x, k, np.array(rels), fb_iter, fb_reason
