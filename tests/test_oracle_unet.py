"""Pins of the oracle U-Net (CPU only).

The network is this project's learned warm start, not something the paper
defines, so its oracle is pinned against independent definitions: the
convolution against SciPy's 2D correlation, bfloat16 rounding against
torch's conversion, pooling / upsampling against their adjoint identities,
the wiring (skip levels, concatenation order, pooling before upsampling)
against a closed form on a pass-through network, and the backward pass
against central finite differences of the forward pass.
"""
import math

import numpy as np
import pytest
import scipy.signal

from oracle import unet


def _rng(seed=0):
    return np.random.default_rng(seed)


def test_bf16_rounding_matches_torch():
    import torch
    r = _rng(1)
    x = np.concatenate([r.standard_normal(4000) * 10.0 ** r.integers(-6, 6, 4000),
                        np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -1.0 - 2.0 ** -8, 0.0, -0.0])])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(unet.bf16(x32), ref)


def test_conv_matches_scipy_correlate2d():
    r = _rng(2)
    B, H, W, C, Co = 2, 8, 12, 3, 5
    x = r.standard_normal((B, H, W, C))
    w = r.standard_normal((Co, 3, 3, C))
    b = r.standard_normal(Co)
    y = unet.conv3x3(x, w, b)
    for bi in range(B):
        for co in range(Co):
            ref = b[co] + sum(scipy.signal.correlate2d(x[bi, :, :, ci], w[co, :, :, ci], mode="same")
                              for ci in range(C))
            assert np.allclose(y[bi, :, :, co], ref, rtol=1e-12, atol=1e-12)


def test_pool_and_upsample_adjoints():
    r = _rng(3)
    x = r.standard_normal((2, 8, 6, 4))
    y = r.standard_normal((2, 4, 3, 4))
    assert np.isclose((unet.pool(x) * y).sum(), (x * unet.pool_grad(y)).sum())
    assert np.isclose((unet.up(y) * x).sum(), (y * unet.up_grad(x)).sum())
    assert np.allclose(unet.pool(unet.up(y)), y)
    # block mean written out
    assert np.isclose(unet.pool(x)[1, 2, 1, 3], x[1, 4:6, 2:4, 3].mean())


def test_shapes_of_the_network():
    s = unet.conv_shapes()
    assert s[:8] == [(3, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (64, 128), (128, 128)]
    assert s[8:] == [(192, 64), (64, 64), (96, 32), (32, 32), (48, 16), (16, 16)]
    ps = unet.init_params()
    assert len(ps) == 2 * len(s) + 2
    out, _ = unet.forward(ps, _rng(4).standard_normal((1, 16, 24, 3)))
    assert out.shape == (1, 16, 24)


def _block_mean(x, k):
    B, H, W = x.shape
    return x.reshape(B, H // k, k, W // k, k).mean(axis=(2, 4))


def _block_repeat(x, k):
    return np.kron(x, np.ones((1, k, k)))


def test_pass_through_network_closed_form():
    """Every convolution copies channel 0 (centre tap 1); the first decoder
    convolution of each level adds channel 0 of the upsampled input and
    channel 0 of the skip.  With a non-negative input the output is then
    x + U(P x) + U^2(P^2 x) + U^3(P^3 x) with P a 2x2 block mean and U a 2x2
    block copy; a wrong skip level, concatenation order or pool/upsample
    placement changes this sum."""
    shapes = unet.conv_shapes()
    ps = []
    for k, (cin, cout) in enumerate(shapes):
        w = np.zeros((cout, 3, 3, cin))
        w[0, 1, 1, 0] = 1.0
        if k in (8, 10, 12):          # first decoder conv: up channels first, then the skip
            w[0, 1, 1, cin - unet.CH[(12 - k) // 2]] = 1.0
        ps += [w, np.zeros(cout)]
    hw = np.zeros(unet.CH[0])
    hw[0] = 1.0
    ps += [hw, np.zeros(1)]
    x = np.zeros((2, 16, 24, 3))
    x[..., 0] = _rng(5).random((2, 16, 24))
    x[..., 1:] = _rng(6).random((2, 16, 24, 2))      # ignored channels
    out, _ = unet.forward(ps, x)
    x0 = x[..., 0]
    ref = x0 + sum(_block_repeat(_block_mean(x0, 2 ** k), 2 ** k) for k in (1, 2, 3))
    assert np.allclose(out, ref, rtol=1e-13, atol=1e-13)


def _loss(ps, x, c):
    out, cache = unet.forward(ps, x)
    return (out * c).sum(), cache


def test_backward_matches_finite_differences():
    r = _rng(7)
    ps = [p.astype(np.float64) for p in unet.init_params(seed=3)]
    for k in range(1, len(ps), 2):                   # non-zero biases
        ps[k] = r.standard_normal(ps[k].shape) * 0.1
    x = r.standard_normal((1, 16, 16, 3))
    c = r.standard_normal((1, 16, 16))
    _, cache = _loss(ps, x, c)
    grads, gx = unet.backward(cache, c)
    h = 1e-6
    checked = 0
    for pi, p in enumerate(ps):
        assert grads[pi].shape == p.shape
        flat = p.reshape(-1)
        for idx in r.choice(flat.size, size=min(4, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = _loss(ps, x, c)
            flat[idx] = old - h
            lm, _ = _loss(ps, x, c)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            g = grads[pi].reshape(-1)[idx]
            assert abs(fd - g) <= 1e-6 * max(1.0, abs(g)), (pi, idx, fd, g)
            checked += 1
    for idx in r.choice(x.size, size=6, replace=False):
        xf = x.reshape(-1)
        old = xf[idx]
        xf[idx] = old + h
        lp, _ = _loss(ps, x, c)
        xf[idx] = old - h
        lm, _ = _loss(ps, x, c)
        xf[idx] = old
        assert abs((lp - lm) / (2 * h) - gx.reshape(-1)[idx]) <= 1e-6
    assert checked >= 100


def test_backward_with_bfloat16_gradients():
    """quantize_grad rounds the gradient entering every one of the 14
    convolutions (after the ReLU mask) to bfloat16 and nothing else: the
    convolution gradients see bfloat16 values only, the unrounded pass does
    not, and the parameter gradients stay within the rounding's size (2^-9
    per value, relative L2 below 2^-7) of the float64 ones."""
    r = _rng(17)
    ps = [p.astype(np.float64) for p in unet.init_params(seed=5)]
    x = unet.bf16(r.standard_normal((1, 16, 24, 3)))
    c = r.standard_normal((1, 16, 24))
    _, cache = unet.forward(ps, x, quantize=True)
    seen = []
    orig = unet.conv3x3_grads

    def spy(xx, w, gy, periodic_w=False):
        seen.append(np.array_equal(gy, unet.bf16(gy)))
        return orig(xx, w, gy, periodic_w)

    unet.conv3x3_grads = spy
    try:
        gq, _ = unet.backward(cache, c, quantize_grad=True)
        assert len(seen) == 14 and all(seen)
        seen.clear()
        g, _ = unet.backward(cache, c)
        assert len(seen) == 14 and not all(seen)
    finally:
        unet.conv3x3_grads = orig
    for a, b in zip(gq, g):
        assert np.linalg.norm(a - b) <= 2.0 ** -7 * np.linalg.norm(b)
    assert any(not np.array_equal(a, b) for a, b in zip(gq, g))


def test_mse_gradient():
    r = _rng(8)
    p, t = r.standard_normal((2, 8, 8)), r.standard_normal((2, 8, 8))
    m = (r.random((2, 8, 8)) < 0.7).astype(float)
    L, g = unet.mse(p, t, m)
    assert np.isclose(L, ((p - t) ** 2 * m).sum() / m.sum())
    h = 1e-6
    for idx in [(0, 1, 2), (1, 7, 7), (1, 0, 3)]:
        q = p.copy()
        q[idx] += h
        Lp, _ = unet.mse(q, t, m)
        q[idx] -= 2 * h
        Lm, _ = unet.mse(q, t, m)
        assert abs((Lp - Lm) / (2 * h) - g[idx]) < 1e-7


def test_forward_sensitivity_to_float32_sums():
    """Bound used by the device forward test: rounding every convolution sum
    to float32 (with float32-sized relative noise) before the bfloat16
    rounding of the activations moves the network output by less than
    5e-3 (relative L2) at the tested shapes."""
    r = np.random.default_rng(9)
    ps = []
    for cin, cout in unet.conv_shapes():
        ps.append(r.standard_normal((cout, 3, 3, cin)) * np.sqrt(2.0 / (9 * cin)))
        ps.append(r.standard_normal(cout) * 0.05)
    ps += [r.standard_normal(16) * 0.25, np.array([0.1])]
    orig = unet.conv3x3
    noise = np.random.default_rng(1)

    def conv32(x, w, b, periodic_w=False):
        y = orig(x, w, b, periodic_w).astype(np.float32)
        return (y * (1 + noise.standard_normal(y.shape).astype(np.float32) * 3e-7)).astype(np.float64)

    for shape in [(2, 16, 24, 3), (1, 64, 48, 3)]:
        x = unet.bf16(r.standard_normal(shape))
        ref, _ = unet.forward(ps, x, quantize=True)
        unet.conv3x3 = conv32
        try:
            alt, _ = unet.forward(ps, x, quantize=True)
        finally:
            unet.conv3x3 = orig
        rel = np.linalg.norm(alt - ref) / np.linalg.norm(ref)
        assert 1e-5 < rel < 5e-3, rel


def test_float32_sized_sum_errors_stay_within_the_device_bar():
    """Calibration of the per-element bar of the device network's forward
    test, on the very networks and inputs that test uses: with every
    convolution sum carrying a uniform random error of up to 2^-20 of the sum
    of its terms' magnitudes (float32 accumulation over up to 54 partial sums,
    with margin), which flips the bfloat16 rounding of activations that lie
    next to a rounding boundary, no output element moves by more than
    UNET_STEPS bfloat16 steps of its magnitude plus the output's RMS,
    2^-8 (|ref| + rms), over six draws; and the errors do reach the
    rounding (some element moves)."""
    from gpu_util import UNET_FORWARD_CASES, UNET_STEPS, unet_params
    oc = unet.conv3x3
    noise = np.random.default_rng(2)

    def conv(x, w, b, periodic_w=False):
        mag = oc(np.abs(x), np.abs(w), np.zeros_like(b), periodic_w)
        return oc(x, w, b, periodic_w) + 2.0 ** -20 * mag * noise.uniform(-1.0, 1.0, mag.shape)

    full = np.random.default_rng(4).standard_normal((1, 1024, 512, 3))
    crops = [(12, unet.bf16(full[:, h0:h0 + 192, w0:w0 + 192]), False) for h0, w0 in [(0, 0), (448, 192), (832, 320)]]
    cases = [(ps, unet.bf16(np.random.default_rng(xs).standard_normal(shape)), per)
             for ps, xs, shape, per in UNET_FORWARD_CASES] + crops
    for seed, x, periodic in cases:
        ps = unet_params(seed, unet.conv_shapes())
        ref, _ = unet.forward(ps, x, quantize=True, periodic_w=periodic)
        rms = np.sqrt(np.mean(ref * ref))
        worst = 0.0
        for _ in range(6):
            unet.conv3x3 = conv
            try:
                alt, _ = unet.forward(ps, x, quantize=True, periodic_w=periodic)
            finally:
                unet.conv3x3 = oc
            worst = max(worst, float(np.max(np.abs(alt - ref) / (2.0 ** -8 * (np.abs(ref) + rms)))))
        assert 0.0 < worst < UNET_STEPS, (seed, x.shape, worst)


def test_time_extrapolation_weights_reproduce_polynomials():
    """The K-point time extrapolation (the start the device network corrects)
    is the Lagrange extrapolation from t = -1 .. -K to t = 0: its weights sum
    to 1, it reproduces every polynomial of degree below K exactly and misses
    t^K (by K! in magnitude: the nodal polynomial prod (t + m) at t = 0);
    K = 2 is the linear extrapolation 2 phi_1 - phi_2 bit for bit."""
    r = np.random.default_rng(23)
    for K in range(1, 7):
        w = unet.lagrange_extrapolation_weights(K)
        assert abs(sum(w) - 1.0) < 1e-12
        coef = r.standard_normal(K)
        phis = [np.full((3, 4), sum(c * (-k) ** j for j, c in enumerate(coef))) for k in range(1, K + 1)]
        got = unet.extrapolated_k(phis, w)
        assert np.allclose(got, coef[0], rtol=0, atol=1e-9 * (1 + np.abs(coef).sum() * K ** K)), K
        lead = unet.extrapolated_k([np.full(2, float((-k) ** K)) for k in range(1, K + 1)], w)
        assert abs(abs(lead[0]) - math.factorial(K)) < 1e-6 * math.factorial(K), (K, lead)
    p1, p2 = r.standard_normal((2, 5, 6))
    assert np.array_equal(unet.extrapolated_k([p1, p2], unet.lagrange_extrapolation_weights(2)),
                          unet.extrapolated(p1, p2))
    assert unet.lagrange_extrapolation_weights(4) == [4.0, -6.0, 4.0, -1.0]


def test_adam_two_steps_closed_form():
    """Two Adam steps (Kingma & Ba 2015, Algorithm 1) written out by hand.
    After step 1 the bias-corrected moments are exactly g1 and g1^2, so each
    weight moves by lr * g1 / (|g1| + eps); after step 2 they are
    (b1 g1 + g2) / (1 + b1) and (b2 g1^2 + g2^2) / (1 + b2).  A wrong
    bias-correction power, a swapped beta or a missing square fails here."""
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-8
    p0 = np.array([0.5, -1.25, 2.0, 0.0])
    g1 = np.array([0.2, -0.4, 3.0, -1e-3])
    g2 = np.array([-0.1, 0.3, 1.0, 5e-3])
    m = np.zeros(4)
    v = np.zeros(4)
    p1, m, v = unet.adam(p0, g1, m, v, 1, lr, b1, b2, eps)
    want1 = p0 - lr * g1 / (np.abs(g1) + eps)
    assert np.allclose(p1, want1, rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g1, rtol=1e-15) and np.allclose(v, 0.001 * g1 * g1, rtol=1e-12)
    p2, m, v = unet.adam(p1, g2, m, v, 2, lr, b1, b2, eps)
    mh = (0.9 * g1 + g2) / 1.9
    vh = (0.999 * g1 * g1 + g2 * g2) / 1.999
    want2 = p1 - lr * mh / (np.sqrt(vh) + eps)
    assert np.allclose(p2, want2, rtol=1e-13, atol=1e-15)
    # the first weight, by hand: step 1 moves it by 0.01 * 0.2 / (0.2 + 1e-8); then
    # m^ = (0.18 - 0.1) / 1.9 and v^ = (0.03996 + 0.01) / 1.999
    w0 = 0.5 - 0.002 / 0.20000001 - 0.01 * (0.08 / 1.9) / (np.sqrt(0.04996 / 1.999) + 1e-8)
    assert abs(p2[0] - w0) < 1e-15


# a 4 x 4 node grid: row 0 grounded (conductor 1), a 2-node RF conductor
# (conductor 2) at (3, 2) and (3, 3), the other nodes free
_NC = np.array([[1, 1, 1, 1],
                [0, 0, 0, 0],
                [0, 0, 0, 0],
                [0, 0, 2, 2]], np.uint8)
_B = np.array([[0.0, 0.0, 0.0, 0.0],        # Dirichlet values (ground)
               [1.5, -2.0, 0.25, 3.0],      # source terms on free nodes
               [-0.5, 0.125, 4.0, -1.0],
               [2.0, -3.0, 7.5, 7.5]])      # 2 free, then the RF potential 7.5


def test_features_on_a_hand_built_grid():
    """Input channels of a 4 x 4 problem written out by hand: 0 the source
    times s_rho on free nodes, 1 the free-node indicator, 2 the Dirichlet
    value times s_v on conductor nodes; a swapped channel or a value written
    on the wrong kind of node fails."""
    x = unet.features(_B, _NC, 4, 4, s_rho=0.5, s_v=0.2)
    want0 = np.array([[0, 0, 0, 0],
                      [0.75, -1.0, 0.125, 1.5],
                      [-0.25, 0.0625, 2.0, -0.5],
                      [1.0, -1.5, 0, 0]])
    want1 = np.array([[0, 0, 0, 0], [1, 1, 1, 1], [1, 1, 1, 1], [1, 1, 0, 0]], float)
    want2 = np.zeros((4, 4))
    want2[3, 2] = want2[3, 3] = unet.bf16(1.5)      # 7.5 * 0.2 rounded to bfloat16
    assert np.array_equal(x[..., 0], want0)
    assert np.array_equal(x[..., 1], want1)
    assert np.array_equal(x[..., 2], want2)
    # bfloat16 rounding of the scaled source: 1/3 is not representable
    y = unet.features(_B / 3.0, _NC, 4, 4, s_rho=1.0, s_v=1.0)
    assert y[1, 0, 0] == unet.bf16(0.5) and y[1, 1, 0] != -2.0 / 3.0
    # a window smaller than the grid cuts rows and columns
    assert unet.features(_B, _NC, 2, 2, 1.0, 1.0).shape == (2, 2, 3)


def test_guess_on_a_hand_built_grid():
    """Start potential from a network output on a 2 x 4 window of the 4 x 4
    grid: output times s_phi on free window nodes, 0 on free nodes outside
    the window, the Dirichlet value (b) on conductor nodes everywhere."""
    out = np.array([[9.0, 9.0, 9.0, 9.0],
                    [0.5, -1.0, 2.0, 0.25]])
    g = unet.guess(out, _B, _NC, s_phi=4.0)
    want = np.array([[0.0, 0.0, 0.0, 0.0],     # grounded row keeps b = 0, not 36
                     [2.0, -4.0, 8.0, 1.0],
                     [0.0, 0.0, 0.0, 0.0],     # free, outside the window
                     [0.0, 0.0, 7.5, 7.5]])    # free outside the window; RF nodes keep b
    assert np.array_equal(g, want)


def test_periodic_convolution_matches_scipy_wrap():
    """Circular padding along W: SciPy's correlate2d with wrapped boundaries
    on an image given one zero row above and below (zero padding along H),
    cropped back; and a shift of the input along W shifts the output."""
    r = _rng(11)
    B, H, W, C, Co = 1, 6, 10, 3, 4
    x = r.standard_normal((B, H, W, C))
    w = r.standard_normal((Co, 3, 3, C))
    b = r.standard_normal(Co)
    y = unet.conv3x3(x, w, b, periodic_w=True)
    for co in range(Co):
        ref = b[co]
        for ci in range(C):
            xz = np.zeros((H + 2, W))
            xz[1:-1] = x[0, :, :, ci]
            ref = ref + scipy.signal.correlate2d(xz, w[co, :, :, ci], mode="same", boundary="wrap")[1:-1]
        assert np.allclose(y[0, :, :, co], ref, rtol=1e-12, atol=1e-12)
    ys = unet.conv3x3(np.roll(x, 3, axis=2), w, b, periodic_w=True)
    assert np.allclose(ys, np.roll(y, 3, axis=2), rtol=1e-12, atol=1e-12)
    # zero padding differs from it at the first and last columns only
    y0 = unet.conv3x3(x, w, b)
    assert np.allclose(y0[:, :, 1:-1], y[:, :, 1:-1]) and not np.allclose(y0[:, :, 0], y[:, :, 0])


def test_periodic_network_is_shift_equivariant_and_its_backward_matches_differences():
    """The whole network with circular padding along W commutes with shifts
    of the image by multiples of 8 pixels (the pooling blocks of three
    levels); its backward pass matches central differences."""
    r = _rng(12)
    ps = [p.astype(np.float64) for p in unet.init_params(seed=4)]
    for k in range(1, len(ps), 2):
        ps[k] = r.standard_normal(ps[k].shape) * 0.1
    x = r.standard_normal((1, 16, 32, 3))
    out, _ = unet.forward(ps, x, periodic_w=True)
    outs, _ = unet.forward(ps, np.roll(x, 8, axis=2), periodic_w=True)
    assert np.allclose(outs, np.roll(out, 8, axis=2), rtol=1e-11, atol=1e-11)
    out0, _ = unet.forward(ps, x)
    assert not np.allclose(out0, out)
    c = r.standard_normal((1, 16, 32))
    out, cache = unet.forward(ps, x, periodic_w=True)
    grads, gx = unet.backward(cache, c)
    h = 1e-6
    for pi in (0, 7, 16, 26, 28):
        flat = ps[pi].reshape(-1)
        for idx in r.choice(flat.size, size=3, replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = (unet.forward(ps, x, periodic_w=True)[0] * c).sum()
            flat[idx] = old - h
            lm = (unet.forward(ps, x, periodic_w=True)[0] * c).sum()
            flat[idx] = old
            g = grads[pi].reshape(-1)[idx]
            assert abs((lp - lm) / (2 * h) - g) <= 1e-6 * max(1.0, abs(g)), (pi, idx)
    # input gradient at the wrapped columns
    for (hh, ww) in ((3, 0), (9, 31), (5, 16)):
        xp = x.copy()
        xp[0, hh, ww, 0] += h
        lp = (unet.forward(ps, xp, periodic_w=True)[0] * c).sum()
        xp[0, hh, ww, 0] -= 2 * h
        lm = (unet.forward(ps, xp, periodic_w=True)[0] * c).sum()
        assert abs((lp - lm) / (2 * h) - gx[0, hh, ww, 0]) <= 1e-6


def _trench_problem():
    """A small y-periodic trench potential problem: its node map, a random
    charge, and two earlier potentials."""
    import oracle
    import synth
    w = synth.trench(nx=16, ny=8, width=2, depth=4, ppc=1)
    nc = oracle.node_cond(w)
    r = _rng(13)
    ri = r.integers(0, 9 << 32, (w.NX, w.NY), dtype=np.int64)
    re = r.integers(0, 9 << 32, (w.NX, w.NY), dtype=np.int64)
    b = oracle.assemble(w, nc, re, ri, 3.0)
    return w, nc, b


def test_residual_of_the_exact_solution_is_zero_and_of_zero_is_the_source():
    """The residual of the masked 5-point system: zero for the exact
    solution of eq. (5) (direct solver), b on free nodes for a zero start,
    and by hand for a start that is 1 on one free node (4 there, -1 on each
    free neighbour, across the periodic seam too)."""
    import oracle
    w, nc, b = _trench_problem()
    phi = oracle.solve_direct(w, nc, b)
    per = (bool(w.periodic_x), bool(w.periodic_y))
    r = unet.masked_residual(b, phi, nc, per)
    assert np.max(np.abs(r)) < 1e-10 * np.max(np.abs(b))
    r0 = unet.masked_residual(b, np.zeros_like(b), nc, per)
    assert np.array_equal(r0, np.where(nc == 0, b, 0.0))
    e = np.zeros_like(b)
    e[5, 0] = 1.0                                     # free node on the periodic seam
    assert nc[5, 0] == 0 and nc[4, 0] == 0 and nc[6, 0] == 0 and nc[5, w.NY - 1] == 0
    re_ = unet.masked_residual(np.zeros_like(b), e, nc, per)
    want = np.zeros_like(b)
    want[5, 0] = -4.0
    want[4, 0] = want[6, 0] = want[5, 1] = want[5, w.NY - 1] = 1.0
    assert np.array_equal(re_, want)


def test_residual_sample_and_guess_by_hand():
    """Sample of the residual-learning start: the input holds the scaled
    residual of 2 phi_1 - phi_2 (bfloat16), the free-node indicator and the
    scaled Dirichlet values; the target is the scaled gap to phi_t; the
    guess adds out / s_d to the extrapolation on free window nodes only."""
    import oracle
    w, nc, b = _trench_problem()
    per = (False, True)
    exact = oracle.solve_direct(w, nc, b)
    r = _rng(14)
    phi_1 = exact + 0.01 * r.standard_normal(exact.shape)
    phi_2 = exact + 0.02 * r.standard_normal(exact.shape)
    H, W = 16, 8
    x, t = unet.residual_sample(b, phi_1, phi_2, exact, nc, H, W, per, 2.0, 0.5, 8.0)
    start = 2.0 * phi_1 - phi_2
    res = unet.masked_residual(b, start, nc, per)
    free = nc[:H, :W] == 0
    assert np.array_equal(x[..., 0], np.where(free, unet.bf16(2.0 * res[:H, :W]), 0.0))
    assert np.array_equal(x[..., 1], free.astype(float))
    assert np.array_equal(x[..., 2], np.where(free, 0.0, unet.bf16(0.5 * b[:H, :W])))
    assert np.array_equal(t, np.where(free, unet.bf16(8.0 * (exact - start)[:H, :W]), 0.0))
    # the target that reaches the exact solution, fed back through the guess
    g = unet.residual_guess(8.0 * (exact - start)[:H, :W], phi_1, phi_2, nc, 8.0)
    assert np.allclose(g[:H][free], exact[:H][free], rtol=0, atol=1e-12)
    assert np.array_equal(g[H:], start[H:])                       # outside the window: the extrapolation
    assert np.array_equal(g[:H][~free], start[:H][~free])         # Dirichlet nodes untouched
    g0 = unet.residual_guess(np.ones((H, W)), phi_1, phi_2, nc, 8.0, use_output=False)
    assert np.array_equal(g0, start)
    # no earlier pair: the start is phi_1
    x1, _ = unet.residual_sample(b, exact, None, None, nc, H, W, per, 1.0, 1.0, 1.0)
    assert np.max(np.abs(x1[..., 0])) < 1e-9 * np.max(np.abs(b))


def test_coarse_sample_and_guess_reduce_to_the_full_resolution_ones_at_f1():
    """f = 1 (one node per pixel) gives the residual-learning sample and
    start of the full-resolution network, bit for bit."""
    import oracle
    w, nc, b = _trench_problem()
    per = (False, True)
    exact = oracle.solve_direct(w, nc, b)
    r = _rng(21)
    phi_1 = exact + 0.01 * r.standard_normal(exact.shape)
    phi_2 = exact + 0.02 * r.standard_normal(exact.shape)
    H, W = 16, 8
    x, t = unet.residual_sample(b, phi_1, phi_2, exact, nc, H, W, per, 2.0, 0.5, 8.0)
    xc, tc = unet.coarse_residual_sample(b, phi_1, phi_2, exact, nc, 1, H, W, per, 2.0, 0.5, 8.0)
    assert np.array_equal(x, xc) and np.array_equal(t, tc)
    out = r.standard_normal((H, W)).astype(np.float32)
    assert np.array_equal(unet.residual_guess(out, phi_1, phi_2, nc, 8.0),
                          unet.coarse_residual_guess(out, phi_1, phi_2, nc, 1, per, 8.0))


def test_coarse_sample_by_brute_force():
    """Block means against a per-pixel loop over the block's nodes, on values
    that are small dyadic numbers (every sum exact, so the order of addition
    cannot matter): a 9 x 8 grid with a Dirichlet edge row and a conductor
    notch, 2 x 2 blocks, start zero (so r = b on free nodes)."""
    NX, NY, f, H, W = 9, 8, 2, 4, 3
    nc = np.zeros((NX, NY), np.uint8)
    nc[0, :] = 1
    nc[5:7, 2:4] = 2
    r = _rng(22)
    b = r.integers(-64, 64, (NX, NY)) / 8.0
    phi_t = r.integers(-64, 64, (NX, NY)) / 16.0
    zero = np.zeros((NX, NY))
    x, t = unet.coarse_residual_sample(b, zero, None, phi_t, nc, f, H, W, (False, False), 0.5, 2.0, 4.0)
    for h in range(H):
        for q in range(W):
            blk = (slice(h * f, h * f + f), slice(q * f, q * f + f))
            free = nc[blk] == 0
            assert x[h, q, 0] == unet.bf16(0.5 * np.sum(np.where(free, b[blk], 0)) / 4)
            assert x[h, q, 1] == np.count_nonzero(free) / 4
            assert x[h, q, 2] == unet.bf16(2.0 * np.sum(np.where(free, 0, b[blk])) / 4)
            assert t[h, q] == unet.bf16(4.0 * np.sum(np.where(free, phi_t[blk], 0)) / 4)
    # the pixel of rows 0-1, columns 0-1 holds two Dirichlet nodes (row 0)
    assert x[0, 0, 1] == 0.5
    # the notch: nodes (5..6, 2..3) are all Dirichlet, spread over pixels (2, 1) and (3, 1)
    assert x[2, 1, 1] == 0.5 and x[3, 1, 1] == 0.5


def test_coarse_guess_reproduces_linear_functions_and_wraps_by_shifts():
    """Bilinear prolongation with pixel centres at node (h + 1/2) f - 1/2:
    a coarse output linear in (h, w) gives the same linear function of the
    node's pixel coordinate, held at the edge pixel beyond the first and
    last centres (clamped axis); a constant gives that constant on every
    free node; on an axis that is periodic and covered exactly, rolling the
    coarse output by one pixel rolls the start by f nodes."""
    NX, NY, f, H, W = 33, 24, 4, 8, 6
    nc = np.zeros((NX, NY), np.uint8)
    nc[0, :] = 1
    nc[NX - 1, :] = 2
    nc[20:, 10:13] = 2
    zero = np.zeros((NX, NY))
    hh, ww = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    lin = (3.0 * hh - 2.0 * ww + 1.0).astype(np.float32)
    g = unet.coarse_residual_guess(lin, zero, None, nc, f, (False, False), 1.0)
    u = np.clip((np.arange(NX) + 0.5) / f - 0.5, 0, H - 1)
    v = np.clip((np.arange(NY) + 0.5) / f - 0.5, 0, W - 1)
    want = 3.0 * u[:, None] - 2.0 * v[None, :] + 1.0
    cover = np.zeros((NX, NY), bool)
    cover[:H * f, :W * f] = True
    m = cover & (nc == 0)
    assert np.array_equal(g[m], want[m])
    assert np.array_equal(g[~m], zero[~m])                 # Dirichlet and uncovered nodes: the start
    # partition of unity, also at clamped and wrapped edges
    phi_1 = _rng(23).standard_normal((NX, NY))
    gc = unet.coarse_residual_guess(np.full((H, W), 0.75, np.float32), phi_1, None, nc, f, (False, True), 2.0)
    assert np.array_equal(gc[m], phi_1[m] + 0.375)
    # periodic y (W f == NY): shift equivariance on a problem without y structure
    nc2 = np.zeros((NX, NY), np.uint8)
    nc2[0, :] = 1
    nc2[NX - 1, :] = 2
    out = _rng(24).standard_normal((H, W)).astype(np.float32)
    g1 = unet.coarse_residual_guess(out, zero, None, nc2, f, (False, True), 1.0)
    g2 = unet.coarse_residual_guess(np.roll(out, 1, axis=1), zero, None, nc2, f, (False, True), 1.0)
    assert np.array_equal(np.roll(g1, f, axis=1), g2)
    # node 0 of the periodic axis lies between the last pixel and the first:
    # pixel coordinate 1/(2f) - 1/2 in y (weight 1/2 + 1/(2f) on pixel 0), and
    # node 8 at 8.5/f - 1/2 in x
    o = out.astype(np.float64)
    a = 0.5 + 0.5 / f
    ax = (8.5 / f - 0.5) % 1
    row = lambda h: (1 - a) * o[h, W - 1] + a * o[h, 0]
    h0 = int(8.5 / f - 0.5)
    assert np.isclose(g1[8, 0], (1 - ax) * row(h0) + ax * row(h0 + 1), rtol=0, atol=1e-12)
