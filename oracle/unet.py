"""CPU oracle of the learned warm start's network (test infrastructure only).

A 4-level U-Net: at each level two 3x3 convolutions with ReLU (16, 32, 64,
128 channels), 2x2 average pooling down, nearest-neighbour upsampling, skip
concatenation (upsampled channels first, then the skip), and a 1x1 head to
one output channel.  Tensors are NHWC float64; convolutions are
cross-correlations with zero padding.  ``quantize=True`` rounds inputs,
weights and every stored activation to bfloat16 (round to nearest even), the
storage precision of the device network, while all arithmetic stays float64.

Residual learning (the start used by the solver): the network maps the
residual of the linearly extrapolated potential to the correction of that
start (``residual_sample`` / ``residual_guess``).

Parameter order (one flat list):  for every 3x3 convolution in network
order, its weight [Cout, 3, 3, Cin] then bias [Cout]; then the head weight
[16] and head bias [1].
"""
from __future__ import annotations

import numpy as np

CH = (16, 32, 64, 128)
IN_CH = 3


def conv_shapes(in_ch: int = IN_CH):
    """(Cin, Cout) of every 3x3 convolution in network order."""
    s = []
    c = in_ch
    for k, ch in enumerate(CH):          # encoder + bottleneck
        s.append((c, ch))
        s.append((ch, ch))
        c = ch
    for k in range(len(CH) - 2, -1, -1):  # decoder
        s.append((c + CH[k], CH[k]))
        s.append((CH[k], CH[k]))
        c = CH[k]
    return s


def bf16(x):
    """Round float64 values to bfloat16 (nearest even) and back."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(seed: int = 100, in_ch: int = IN_CH):
    """He-normal weights, zero biases (float32 values)."""
    rng = np.random.Generator(np.random.Philox(key=np.array([seed, 5], np.uint64)))
    ps = []
    for cin, cout in conv_shapes(in_ch):
        std = np.sqrt(2.0 / (9 * cin))
        ps.append((rng.standard_normal((cout, 3, 3, cin)) * std).astype(np.float32))
        ps.append(np.zeros(cout, np.float32))
    ps.append((rng.standard_normal(CH[0]) * np.sqrt(1.0 / CH[0])).astype(np.float32))
    ps.append(np.zeros(1, np.float32))
    return ps


def _pad(x, periodic_w):
    """One pixel of padding on each side: zeros along H; along W zeros, or
    the image's own far columns when it wraps (circular padding)."""
    B, H, W, C = x.shape
    xp = np.zeros((B, H + 2, W + 2, C))
    xp[:, 1:-1, 1:-1] = x
    if periodic_w:
        xp[:, 1:-1, 0] = x[:, :, -1]
        xp[:, 1:-1, -1] = x[:, :, 0]
    return xp


def conv3x3(x, w, b, periodic_w=False):
    B, H, W, C = x.shape
    xp = _pad(x, periodic_w)
    y = np.zeros((B, H, W, w.shape[0]))
    for dy in range(3):
        for dx in range(3):
            y += np.tensordot(xp[:, dy:dy + H, dx:dx + W], w[:, dy, dx, :], axes=([3], [1]))
    return y + b


def conv3x3_grads(x, w, gy, periodic_w=False):
    """Gradients of conv3x3 w.r.t. input, weight and bias."""
    B, H, W, C = x.shape
    xp = _pad(x, periodic_w)
    gw = np.zeros_like(w)
    gxp = np.zeros_like(xp)
    for dy in range(3):
        for dx in range(3):
            gw[:, dy, dx, :] = np.tensordot(gy, xp[:, dy:dy + H, dx:dx + W], axes=([0, 1, 2], [0, 1, 2]))
            gxp[:, dy:dy + H, dx:dx + W] += np.tensordot(gy, w[:, dy, dx, :], axes=([3], [0]))
    gx = gxp[:, 1:-1, 1:-1].copy()
    if periodic_w:                       # the padding columns are the far columns
        gx[:, :, -1] += gxp[:, 1:-1, 0]
        gx[:, :, 0] += gxp[:, 1:-1, -1]
    return gx, gw, gy.sum(axis=(0, 1, 2))


def pool(x):
    B, H, W, C = x.shape
    return x.reshape(B, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool_grad(gy):
    return np.repeat(np.repeat(gy, 2, axis=1), 2, axis=2) * 0.25


def up(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up_grad(gy):
    B, H, W, C = gy.shape
    return gy.reshape(B, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def forward(params, x, quantize=False, periodic_w=False):
    """Returns (output [B,H,W], cache for backward).  periodic_w: every
    convolution pads circularly along W (an image that wraps in W)."""
    q = bf16 if quantize else (lambda a: np.asarray(a, np.float64))
    P = [q(p) if i < len(params) - 2 else np.asarray(p, np.float64) for i, p in enumerate(params)]
    cache = {"P": P, "acts": [], "periodic_w": periodic_w}
    h = q(x)
    k = 0
    skips = []
    # encoder
    for lev in range(len(CH)):
        for _ in range(2):
            inp = h
            h = q(np.maximum(conv3x3(inp, P[2 * k], P[2 * k + 1], periodic_w), 0.0))
            cache["acts"].append((inp, h))
            k += 1
        if lev < len(CH) - 1:
            skips.append(h)
            h = q(pool(h))
    # decoder
    for lev in range(len(CH) - 2, -1, -1):
        h = np.concatenate([up(h), skips[lev]], axis=3)
        for _ in range(2):
            inp = h
            h = q(np.maximum(conv3x3(inp, P[2 * k], P[2 * k + 1], periodic_w), 0.0))
            cache["acts"].append((inp, h))
            k += 1
    out = h @ P[-2] + P[-1][0]
    cache["last"] = h
    return out, cache


def backward(cache, gout, quantize_grad=False):
    """Gradients (same order as the parameters) and the input gradient.
    quantize_grad: round the gradient entering each convolution (after the
    ReLU mask) to bfloat16, the storage precision of the device network's
    backward pass; the sums stay float64."""
    qg = bf16 if quantize_grad else (lambda a: a)
    P = cache["P"]
    pw = cache.get("periodic_w", False)
    grads = [None] * len(P)
    h = cache["last"]
    grads[-2] = np.tensordot(gout, h, axes=([0, 1, 2], [0, 1, 2]))
    grads[-1] = np.array([gout.sum()])
    g = gout[..., None] * P[-2]
    nconv = len(cache["acts"])
    ne = 2 * len(CH)                     # encoder + bottleneck convolutions
    skip_grads = [None] * (len(CH) - 1)
    k = nconv - 1
    for lev in range(0, len(CH) - 1):    # decoder in reverse: finest level first
        for _ in range(2):
            inp, out = cache["acts"][k]
            gy = qg(g * (out > 0))
            gx, grads[2 * k], grads[2 * k + 1] = conv3x3_grads(inp, P[2 * k], gy, pw)
            g = gx
            k -= 1
        cu = g.shape[3] - CH[lev]
        skip_grads[lev] = g[..., cu:]
        g = up_grad(g[..., :cu])
    for lev in range(len(CH) - 1, -1, -1):
        if lev < len(CH) - 1:
            g = pool_grad(g) + skip_grads[lev]
        for _ in range(2):
            inp, out = cache["acts"][k]
            gy = qg(g * (out > 0))
            gx, grads[2 * k], grads[2 * k + 1] = conv3x3_grads(inp, P[2 * k], gy, pw)
            g = gx
            k -= 1
    assert k == -1 and ne == 2 * len(CH)
    return grads, g


def mse(pred, target, weight):
    """Loss = sum(weight (pred - target)^2) / sum(weight) and its gradient."""
    d = pred - target
    ws = weight.sum()
    return float((weight * d * d).sum() / ws), 2.0 * weight * d / ws


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba, bias-corrected moments); t counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def features(b, node_cond, H, W, s_rho, s_v):
    """Network input [H, W, 3] of a Poisson problem: source on free nodes
    times s_rho, free-node indicator, Dirichlet value times s_v (bfloat16)."""
    bb = b[:H, :W]
    free = node_cond[:H, :W] == 0
    x = np.zeros((H, W, 3))
    x[..., 0] = np.where(free, bf16(bb * s_rho), 0.0)
    x[..., 1] = free
    x[..., 2] = np.where(free, 0.0, bf16(bb * s_v))
    return x


def guess(out, b, node_cond, s_phi):
    """Start potential: out * s_phi on free nodes of the network window, 0 on
    other free nodes, b (the Dirichlet value) on conductor nodes."""
    H, W = out.shape
    g = np.zeros(b.shape)
    g[:H, :W] = out * s_phi
    return np.where(node_cond != 0, b, g)


# ---------------------------------------------------------------------------
# residual learning: the network corrects the linear extrapolation in time of
# the potential (the warm start of the plain solver) from the residual of
# that start
# ---------------------------------------------------------------------------

def extrapolated(phi_1, phi_2):
    """Start potential 2 phi_1 - phi_2 from the two previous solutions (phi_1
    alone when phi_2 is None)."""
    return np.asarray(phi_1, np.float64).copy() if phi_2 is None else 2.0 * phi_1 - phi_2


def lagrange_extrapolation_weights(K):
    """Weights w_1 .. w_K with sum_k w_k p(-k) = p(0) for every polynomial p
    of degree below K: the Lagrange basis at the nodes t = -1 .. -K
    evaluated at t = 0, w_k = prod_{m != k} (0 - (-m)) / ((-k) - (-m))."""
    w = []
    for k in range(1, K + 1):
        num, den = 1.0, 1.0
        for m in range(1, K + 1):
            if m != k:
                num *= m
                den *= (m - k)
        w.append(num / den)
    return w


def extrapolated_k(phis, weights):
    """Time extrapolation sum_k weights[k] phis[k] (phis[0] the latest
    solution), added in this order in float64."""
    s = weights[0] * np.asarray(phis[0], np.float64)
    for w_k, p in zip(weights[1:], phis[1:]):
        s = s + w_k * np.asarray(p, np.float64)
    return s


def masked_residual(b, phi, node_cond, periodic):
    """r = b - A phi on the free nodes (0 elsewhere) of the 5-point system of
    eq. (5): A phi = 4 phi minus the free neighbours, the Dirichlet
    neighbours' potentials being part of b; neighbours wrap on a periodic
    axis (periodic = (x, y)); a free node never lies on a bounded edge."""
    NX, NY = b.shape
    free = node_cond == 0
    r = np.zeros((NX, NY))
    for i in range(NX):
        for j in range(NY):
            if not free[i, j]:
                continue
            s = 4.0 * phi[i, j]
            for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
                a, c = i + di, j + dj
                if periodic[0]:
                    a %= NX
                if periodic[1]:
                    c %= NY
                if 0 <= a < NX and 0 <= c < NY and free[a, c]:
                    s -= phi[a, c]
            r[i, j] = b[i, j] - s
    return r


def residual_sample(b, phi_1, phi_2, phi_t, node_cond, H, W, periodic, s_r, s_v, s_d):
    """Training sample of the residual-learning start on the H x W window:
    input [H, W, 3] = (r s_r on free nodes, free-node indicator, Dirichlet
    value s_v on conductor nodes) with r the residual of the extrapolated
    start, and target [H, W] = (phi_t - start) s_d on free nodes (None
    without phi_t); both rounded to bfloat16, the stored precision."""
    start = extrapolated(phi_1, phi_2)
    r = masked_residual(b, start, node_cond, periodic)
    free = node_cond[:H, :W] == 0
    x = np.zeros((H, W, 3))
    x[..., 0] = np.where(free, bf16(r[:H, :W] * s_r), 0.0)
    x[..., 1] = free
    x[..., 2] = np.where(free, 0.0, bf16(b[:H, :W] * s_v))
    t = None
    if phi_t is not None:
        t = np.where(free, bf16((phi_t[:H, :W] - start[:H, :W]) * s_d), 0.0)
    return x, t


def residual_guess(out, phi_1, phi_2, node_cond, s_d, use_output=True):
    """Start potential: the extrapolated start plus out / s_d on the free
    nodes of the network window (use_output False: the extrapolation
    alone)."""
    g = extrapolated(phi_1, phi_2)
    if use_output:
        H, W = out.shape
        free = node_cond[:H, :W] == 0
        g[:H, :W] = np.where(free, g[:H, :W] + out / s_d, g[:H, :W])
    return g


# ---------------------------------------------------------------------------
# coarse residual learning: the network works on f x f blocks of nodes, so
# that its receptive field spans the whole grid.  The smooth part of the
# start's error is what the solver spends its iterations on; the prolonged
# coarse correction supplies it.
# ---------------------------------------------------------------------------

def _block_sum(a, f, H, W):
    """Sum over the f x f block of nodes (h f + p, w f + q), p, q < f, of every
    pixel (h, w), added in the order p outer, q inner (row-major)."""
    s = np.zeros((H, W))
    for p in range(f):
        for q in range(f):
            s = s + a[p:H * f:f, q:W * f:f]
    return s


def coarse_residual_sample(b, phi_1, phi_2, phi_t, node_cond, f, H, W, periodic, s_r, s_v, s_d):
    """Training sample of the coarse residual-learning start: pixel (h, w)
    stands for the f x f block of nodes (h f .. h f + f - 1, w f .. w f + f - 1)
    (H f <= NX, W f <= NY).  Input [H, W, 3] = (block mean of r, zero on
    Dirichlet nodes, times s_r; fraction of free nodes; block mean of the
    Dirichlet values, zero on free nodes, times s_v); target [H, W] = block
    mean of (phi_t - start) on free nodes times s_d (None without phi_t).
    Sums in the order of _block_sum, one multiply by 1/f^2, then the scale,
    rounded to bfloat16 (the stored precision).  f = 1 gives
    residual_sample."""
    start = extrapolated(phi_1, phi_2)
    r = masked_residual(b, start, node_cond, periodic)
    free = node_cond == 0
    inv = 1.0 / (f * f)
    x = np.zeros((H, W, 3))
    x[..., 0] = bf16(_block_sum(np.where(free, r, 0.0), f, H, W) * inv * s_r)
    x[..., 1] = bf16(_block_sum(free.astype(np.float64), f, H, W) * inv)
    x[..., 2] = bf16(_block_sum(np.where(free, 0.0, b), f, H, W) * inv * s_v)
    t = None
    if phi_t is not None:
        t = bf16(_block_sum(np.where(free, phi_t - start, 0.0), f, H, W) * inv * s_d)
    return x, t


def _axis_weights(i, f, n, wrap):
    """Lower pixel, upper pixel and the upper weight of node index i on an
    axis of n pixels of f nodes: the node lies at pixel coordinate
    (i + 1/2)/f - 1/2 (pixel centres at integers); outside [0, n - 1] the
    pixel index wraps (wrap) or is clamped to the edge."""
    u = (i + 0.5) / f - 0.5
    lo = int(np.floor(u))
    a = u - lo
    hi = lo + 1
    if wrap:
        lo, hi = lo % n, hi % n
    else:
        lo, hi = min(max(lo, 0), n - 1), min(max(hi, 0), n - 1)
    return lo, hi, a


def coarse_residual_guess(out, phi_1, phi_2, node_cond, f, periodic, s_d, use_output=True):
    """Start potential: the extrapolated start plus c / s_d on the free nodes
    of the covered region (H f x W f nodes), c the bilinear interpolation of
    the coarse output at the node, weights (1-a)(1-b), a(1-b), (1-a)b, ab on
    pixels (lo_x, lo_y), (hi_x, lo_y), (lo_x, hi_y), (hi_x, hi_y) added in that
    order; an axis wraps when it is periodic and covered exactly (n f nodes),
    else is clamped.  Elsewhere the extrapolation alone."""
    g = extrapolated(phi_1, phi_2)
    if not use_output:
        return g
    H, W = out.shape
    NX, NY = g.shape
    wx = bool(periodic[0]) and H * f == NX
    wy = bool(periodic[1]) and W * f == NY
    o = np.asarray(out, np.float64)
    for i in range(H * f):
        h0, h1, a = _axis_weights(i, f, H, wx)
        for j in range(W * f):
            if node_cond[i, j] != 0:
                continue
            v0, v1, bq = _axis_weights(j, f, W, wy)
            c = (1 - a) * (1 - bq) * o[h0, v0]
            c = c + a * (1 - bq) * o[h1, v0]
            c = c + (1 - a) * bq * o[h0, v1]
            c = c + a * bq * o[h1, v1]
            g[i, j] = g[i, j] + c / s_d
    return g
