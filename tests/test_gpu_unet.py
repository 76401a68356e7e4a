"""GPU tests of the learned warm start's network against the oracle U-Net.

Forward: the device network (bfloat16 weights and activations, float32
accumulation on the matrix cores) against the float64 oracle with the same
bfloat16 rounding of inputs, weights and stored activations.  The two differ
only by float32 versus float64 accumulation, which moves an activation by
one bfloat16 step (2^-8 relative) where it lies next to a rounding boundary,
and the layers carry such flips to the output.  The bar is per element:
every output lies within UNET_STEPS = 8 bfloat16 steps of its own magnitude
plus the output's RMS, |got - ref| <= 8 * 2^-8 * (|ref| + rms(ref)).  On the
CPU (test_oracle_unet) the same networks and inputs, with every convolution
sum given a random error of up to 2^-20 of the sum of its terms'
magnitudes, move by at most 1.7 - 3.7 such steps; the device's largest
element deviation is about one step.  The relative L2 error is held to 1e-2
as well.

Backward: parameter gradients against the oracle's float64 backward pass
with the device's rounding of the gradient entering each convolution to
bfloat16, on the oracle's own forward activations; each gradient tensor is
held to a relative L2 error of 2e-2.  The bar is not per element: a weight
gradient element sums over every pixel with heavy cancellation, and one
flipped ReLU mask in the forward pass adds or removes a whole term of it, so
single elements move by many bfloat16 steps of their size while the tensor
moves by well under one percent.
"""
import ctypes as C

import numpy as np
import pytest

import oracle
import synth
from oracle import unet as ou
from gpu_util import UNET_STEPS, unet_params

pytestmark = pytest.mark.gpu


def _params(seed):
    return unet_params(seed, ou.conv_shapes())


def _flat(ps):
    return np.concatenate([p.reshape(-1) for p in ps]).astype(np.float32)


def _unflat(flat, like):
    out, off = [], 0
    for p in like:
        out.append(np.asarray(flat[off:off + p.size], np.float64).reshape(p.shape))
        off += p.size
    return out


def _net(B, H, W, ps):
    import torch
    from paper_1610_03918_amd.unet import UNet
    return UNet(B, H, W, params=_flat(ps)), torch


def _set_input(u, torch, x):
    u.input().copy_(torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(u.dev))


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


BF16_STEP = 2.0 ** -8


def _within(got, ref, what):
    """Per-element bar: |got - ref| <= UNET_STEPS * 2^-8 * (|ref| + rms(ref))."""
    rms = float(np.sqrt(np.mean(ref * ref)))
    ratio = np.abs(got - ref) / (UNET_STEPS * BF16_STEP * (np.abs(ref) + rms))
    print(f"{what}: rel L2 {_rel(got, ref):.2e}, largest ratio to the bar {ratio.max():.3f}, "
          f"99.9 % {np.quantile(ratio, 0.999):.3f}")
    assert np.all(np.isfinite(got)), what
    assert ratio.max() <= 1.0, (what, float(ratio.max()), np.unravel_index(int(np.argmax(ratio)), ratio.shape))


@pytest.mark.parametrize("B,H,W", [(2, 16, 24), (1, 64, 48)])
def test_forward_matches_oracle(B, H, W):
    ps = _params(11)
    u, torch = _net(B, H, W, ps)
    r = np.random.default_rng(3)
    x = ou.bf16(r.standard_normal((B, H, W, 3)))
    _set_input(u, torch, x)
    u.pic_unet_forward()
    got = u.output().cpu().numpy().astype(np.float64)
    ref, _ = ou.forward(ps, x, quantize=True)
    assert got.shape == ref.shape
    _within(got, ref, f"forward {B}x{H}x{W}")
    assert _rel(got, ref) < 1e-2, _rel(got, ref)
    u.close()


def test_forward_full_size_on_crops():
    """1024 x 512 (the trench grid's node rows): the oracle evaluates
    aligned crops; outputs farther than the receptive radius (< 64 pixels)
    from a crop edge that is not an image edge equal the full-image output."""
    H, W, M = 1024, 512, 64
    ps = _params(12)
    u, torch = _net(1, H, W, ps)
    r = np.random.default_rng(4)
    x = ou.bf16(r.standard_normal((1, H, W, 3)))
    _set_input(u, torch, x)
    u.pic_unet_forward()
    got = u.output().cpu().numpy().astype(np.float64)
    for h0, w0 in [(0, 0), (448, 192), (1024 - 192, 512 - 192)]:
        ref, _ = ou.forward(ps, x[:, h0:h0 + 192, w0:w0 + 192], quantize=True)
        hs = slice(0 if h0 == 0 else M, 192 if h0 + 192 == H else 192 - M)
        ws = slice(0 if w0 == 0 else M, 192 if w0 + 192 == W else 192 - M)
        g = got[:, h0:h0 + 192, w0:w0 + 192][:, hs, ws]
        _within(g, ref[:, hs, ws], f"forward 1024x512 crop at {h0},{w0}")
        assert _rel(g, ref[:, hs, ws]) < 1e-2, (h0, w0, _rel(g, ref[:, hs, ws]))
    u.close()


@pytest.mark.parametrize("B,H,W", [(2, 16, 24), (1, 32, 64)])
def test_backward_matches_oracle(B, H, W):
    ps = _params(13)
    u, torch = _net(B, H, W, ps)
    r = np.random.default_rng(5)
    x = ou.bf16(r.standard_normal((B, H, W, 3)))
    gout = r.standard_normal((B, H, W)).astype(np.float32)
    _set_input(u, torch, x)
    u.pic_unet_forward()
    u.grad_output().copy_(torch.from_numpy(gout).to(u.dev))
    u.pic_unet_backward()
    grads = _unflat(u.grads.cpu().numpy(), ps)
    _, cache = ou.forward(ps, x, quantize=True)
    ref, _ = ou.backward(cache, gout.astype(np.float64), quantize_grad=True)
    rels = [_rel(g, rf) for g, rf in zip(grads, ref)]
    print(f"gradients {B}x{H}x{W}: largest relative L2 {max(rels):.2e}")
    for k, (g, rf) in enumerate(zip(grads, ref)):
        assert np.all(np.isfinite(g)), k
        assert rels[k] < 2e-2, (k, rels[k])
    u.close()


def test_loss_and_adam_step():
    ps = _params(14)
    B, H, W = 2, 16, 16
    u, torch = _net(B, H, W, ps)
    r = np.random.default_rng(6)
    _set_input(u, torch, ou.bf16(r.standard_normal((B, H, W, 3))))
    t = r.standard_normal((B, H, W)).astype(np.float32)
    m = (r.random((B, H, W)) < 0.6).astype(np.float32)
    u.target().copy_(torch.from_numpy(t).to(u.dev))
    u.mask().copy_(torch.from_numpy(m).to(u.dev))
    u.pic_unet_forward()
    out = u.output().cpu().numpy().astype(np.float64)
    loss = u.pic_unet_loss()
    L, g = ou.mse(out, t.astype(np.float64), m.astype(np.float64))
    assert abs(loss - L) <= 1e-9 * max(1.0, L)
    assert np.allclose(u.grad_output().cpu().numpy(), g, rtol=1e-6, atol=1e-9)
    u.pic_unet_backward()
    p0 = u.params.cpu().numpy().astype(np.float64)
    g0 = u.grads.cpu().numpy().astype(np.float64)
    u.pic_unet_adam(1e-3)
    # the device takes the hyper-parameters as float32
    hp = dict(lr=float(np.float32(1e-3)), b1=float(np.float32(0.9)), b2=float(np.float32(0.999)),
              eps=float(np.float32(1e-8)))
    p1, m1, v1 = ou.adam(p0, g0, np.zeros_like(p0), np.zeros_like(p0), 1, **hp)
    assert np.allclose(u.params.cpu().numpy(), p1, rtol=1e-6, atol=1e-7)
    assert np.allclose(u.m.cpu().numpy(), m1, rtol=1e-6, atol=1e-12)
    assert np.allclose(u.v.cpu().numpy(), v1, rtol=1e-5, atol=1e-15)
    # a second step counts t = 2 and starts from the stored moments
    u.pic_unet_forward()
    u.pic_unet_loss()
    u.pic_unet_backward()
    g1 = u.grads.cpu().numpy().astype(np.float64)
    u.pic_unet_adam(1e-3)
    p2, _, _ = ou.adam(p1, g1, m1, v1, 2, **hp)
    assert np.allclose(u.params.cpu().numpy(), p2, rtol=1e-5, atol=1e-6), np.max(np.abs(u.params.cpu().numpy() - p2))
    u.close()


def test_snapshot_and_guess_maps():
    import torch
    from paper_1610_03918_amd import Pic
    from paper_1610_03918_amd.unet import UNet
    w = synth.workload_for_tests("trench")
    parts = synth.load(w)
    pic = Pic(w, parts)
    pic.start()
    pic.pic_step(2)
    nm = pic.pic_node_map()
    nc = oracle.node_cond(w)
    H, W = (w.NX // 8) * 8, (w.NY // 8) * 8
    u = UNet(2, H, W)
    scales = (np.float32(0.37), np.float32(1 / 50), np.float32(50.0))
    u.pic_unet_snapshot(1, pic.b, pic.phi, nm, scales)
    b = pic.b.cpu().numpy().reshape(w.NX, w.NY)
    phi = pic.phi.cpu().numpy().reshape(w.NX, w.NY)
    x = u.input()[1].float().cpu().numpy()
    assert np.array_equal(x, ou.features(b, nc.reshape(w.NX, w.NY), H, W, float(scales[0]), float(scales[1])))
    assert np.array_equal(u.target()[1].cpu().numpy(), (phi[:H, :W] / float(scales[2])).astype(np.float32))
    assert np.array_equal(u.mask()[1].cpu().numpy(), (nc.reshape(w.NX, w.NY)[:H, :W] == 0).astype(np.float32))
    u.pic_unet_forward()
    guess = torch.empty(w.NX * w.NY, dtype=torch.float64, device="cuda:0")
    u.pic_unet_guess(1, pic.b, nm, float(scales[2]), guess)
    out = u.output()[1].cpu().numpy().astype(np.float64)
    ref = ou.guess(out * np.float32(1.0), b, nc.reshape(w.NX, w.NY), float(scales[2]))
    assert np.array_equal(guess.cpu().numpy().reshape(w.NX, w.NY), ref)
    u.close()
    pic.close()


@pytest.mark.parametrize("B,H,W", [(2, 16, 24), (1, 32, 64)])
def test_periodic_forward_and_backward_match_oracle(B, H, W):
    """Circular padding along W (a y-periodic grid): forward and parameter
    gradients against the oracle network with the same padding, at the bars
    of the zero-padded network."""
    import torch
    from paper_1610_03918_amd.unet import UNet
    ps = _params(15)
    u = UNet(B, H, W, params=_flat(ps), periodic_w=True)
    r = np.random.default_rng(8)
    x = ou.bf16(r.standard_normal((B, H, W, 3)))
    gout = r.standard_normal((B, H, W)).astype(np.float32)
    _set_input(u, torch, x)
    u.pic_unet_forward()
    got = u.output().cpu().numpy().astype(np.float64)
    ref, cache = ou.forward(ps, x, quantize=True, periodic_w=True)
    _within(got, ref, f"periodic forward {B}x{H}x{W}")
    assert _rel(got, ref) < 1e-2, _rel(got, ref)
    ref0, _ = ou.forward(ps, x, quantize=True)
    assert _rel(got, ref0) > 5e-2                     # the padding matters at this size
    u.grad_output().copy_(torch.from_numpy(gout).to(u.dev))
    u.pic_unet_backward()
    grads = _unflat(u.grads.cpu().numpy(), ps)
    gref, _ = ou.backward(cache, gout.astype(np.float64), quantize_grad=True)
    rels = [_rel(g, rf) for g, rf in zip(grads, gref)]
    print(f"periodic gradients {B}x{H}x{W}: largest relative L2 {max(rels):.2e}")
    for k, (g, rf) in enumerate(zip(grads, gref)):
        assert np.all(np.isfinite(g)), k
        assert rels[k] < 2e-2, (k, rels[k])
    u.close()


def _trench_state(seed=43):
    """A small y-periodic trench with two earlier potentials and a target
    potential drawn as smooth-plus-noise fields (equal on both sides)."""
    w = synth.trench(nx=64, ny=40, width=6, depth=16, ppc=4, seed=seed)
    nc = oracle.node_cond(w)
    parts = synth.load(w)
    rho = [oracle.deposit(w, parts[s]) for s in range(2)]
    b = oracle.assemble(w, nc, rho[0], rho[1], 1.7)
    p1 = synth.random_potential(w, seed + 1, scale=3.0)
    p2 = synth.random_potential(w, seed + 2, scale=3.0)
    pt = synth.random_potential(w, seed + 3, scale=3.0)
    return w, nc, b, p1, p2, pt


def test_residual_sample_load_and_guess_are_bit_exact():
    """The residual-learning maps against the oracle on identical float64
    inputs: the sample's bfloat16 input and target, its statistics, the load
    into a batch slot (target as float32, mask from the free channel) and the
    corrected start, with and without a second earlier potential."""
    import torch
    from paper_1610_03918_amd import Pic
    from paper_1610_03918_amd.unet import UNet, residual_sample
    w, nc, b, p1, p2, pt = _trench_state()
    pic = Pic(w, synth.load(w))                       # for its node map
    nm = pic.pic_node_map()
    assert np.array_equal(pic.node_map_host(), nc)
    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    H, W = (w.NX // 8) * 8, w.NY
    sc = (float(np.float32(0.75)), float(np.float32(0.02)), float(np.float32(6.0)))
    per = (False, True)
    for second in (True, False):
        x = torch.empty((H, W, 3), dtype=torch.bfloat16, device=dev)
        t = torch.empty((H, W), dtype=torch.bfloat16, device=dev)
        stats = torch.zeros(3, dtype=torch.float64, device=dev)
        residual_sample(T(b), T(p1), T(p2) if second else None, T(pt), nm, per, H, W, sc, x, t, stats)
        xr, tr = ou.residual_sample(b, p1, p2 if second else None, pt, nc, H, W, per, *sc)
        assert np.array_equal(x.float().cpu().numpy(), xr)
        assert np.array_equal(t.float().cpu().numpy(), tr)
        start = ou.extrapolated(p1, p2 if second else None)
        res = ou.masked_residual(b, start, nc, per)[:H, :W]
        free = nc[:H, :W] == 0
        st = stats.cpu().numpy()
        assert st[2] == free.sum()
        assert abs(st[0] - np.sum(res[free] ** 2)) <= 1e-9 * st[0]
        assert abs(st[1] - np.sum((pt - start)[:H, :W][free] ** 2)) <= 1e-9 * st[1]
        u = UNet(2, H, W, periodic_w=True)
        u.pic_unet_load(1, x, t)
        assert np.array_equal(u.input()[1].float().cpu().numpy(), xr)
        assert np.array_equal(u.target()[1].cpu().numpy(), tr.astype(np.float32))
        assert np.array_equal(u.mask()[1].cpu().numpy(), free.astype(np.float32))
        u.pic_unet_forward()
        out = u.output()[1].cpu().numpy().astype(np.float64)
        g = torch.empty(w.NX * w.NY, dtype=torch.float64, device=dev)
        for use in (True, False):
            u.pic_unet_residual_guess(1, T(p1), T(p2) if second else None, nm, sc[2], g, use_output=use)
            ref = ou.residual_guess(out, p1, p2 if second else None, nc, sc[2], use_output=use)
            assert np.array_equal(g.cpu().numpy().reshape(w.NX, w.NY), ref)
        u.close()
    pic.close()


def test_time_extrapolation_is_bit_exact():
    """pic_unet_extrapolate (the K-point polynomial extrapolation in time of
    the potential, the start the network corrects) against the oracle's
    Lagrange extrapolation on the same float64 arrays, K = 1 .. 5: the
    coefficients (binomial on the device side, Lagrange weights in the
    oracle) and the sums in the same order, so bit for bit; and a potential
    that is a cubic in time is extrapolated to its next value."""
    import torch
    from paper_1610_03918_amd.unet import extrapolate, extrapolation_coefficients
    dev = torch.device("cuda:0")
    r = np.random.default_rng(61)
    phis = [r.standard_normal((97, 65)) * 10 ** k for k in range(5)]
    for K in range(1, 6):
        out = torch.empty((97, 65), dtype=torch.float64, device=dev)
        extrapolate([torch.from_numpy(p).to(dev) for p in phis[:K]], extrapolation_coefficients(K), out)
        want = ou.extrapolated_k(phis[:K], ou.lagrange_extrapolation_weights(K))
        assert np.array_equal(out.cpu().numpy(), want), K
    a, b, c, d = r.standard_normal((4, 40))
    hist = [a + b * (-k) + c * k * k - d * k ** 3 for k in range(1, 5)]
    out = torch.empty(40, dtype=torch.float64, device=dev)
    extrapolate([torch.from_numpy(h).to(dev) for h in hist], extrapolation_coefficients(4), out)
    assert np.allclose(out.cpu().numpy(), a, rtol=0, atol=1e-12)


@pytest.mark.parametrize("f,nx,ny", [(4, 64, 40), (8, 64, 64), (2, 64, 64), (16, 128, 128)])
def test_coarse_sample_and_guess_are_bit_exact(f, nx, ny):
    """The coarse residual-learning maps (network pixel = f x f block of
    nodes) against the oracle on identical float64 inputs: the sample's
    bfloat16 input and target and its statistics, and the prolonged start
    from the network's output, on grids whose periodic axis is covered
    exactly (wrapped prolongation) or not (held at the edge pixels)."""
    import torch
    from paper_1610_03918_amd import Pic
    from paper_1610_03918_amd.unet import UNet, coarse_sample
    w = synth.trench(nx=nx, ny=ny, width=6, depth=16, ppc=2, seed=44)
    nc = oracle.node_cond(w)
    parts = synth.load(w)
    rho = [oracle.deposit(w, parts[s]) for s in range(2)]
    b = oracle.assemble(w, nc, rho[0], rho[1], 1.7)
    p1, p2, pt = (synth.random_potential(w, 45 + k, scale=3.0) for k in range(3))
    pic = Pic(w, parts)                               # for its node map
    nm = pic.pic_node_map()
    dev = torch.device("cuda:0")
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    H, W = (w.NX // f // 8) * 8, (w.NY // f // 8) * 8
    sc = (float(np.float32(0.75)), float(np.float32(0.02)), float(np.float32(6.0)))
    per = (False, True)
    for second in (True, False):
        q2 = p2 if second else None
        x = torch.empty((H, W, 3), dtype=torch.bfloat16, device=dev)
        t = torch.empty((H, W), dtype=torch.bfloat16, device=dev)
        stats = torch.zeros(3, dtype=torch.float64, device=dev)
        coarse_sample(T(b), T(p1), T(q2) if second else None, T(pt), nm, per, f, H, W, sc, x, t, stats)
        xr, tr = ou.coarse_residual_sample(b, p1, q2, pt, nc, f, H, W, per, *sc)
        assert np.array_equal(x.float().cpu().numpy(), xr)
        assert np.array_equal(t.float().cpu().numpy(), tr)
        start = ou.extrapolated(p1, q2)
        res = np.where(nc == 0, ou.masked_residual(b, start, nc, per), 0.0)
        bs = lambda a: a[:H * f, :W * f].reshape(H, f, W, f).sum(axis=(1, 3)) / (f * f)
        rm, dm = bs(res), bs(np.where(nc == 0, pt - start, 0.0))
        has = bs((nc == 0).astype(float)) > 0
        st = stats.cpu().numpy()
        assert st[2] == has.sum()
        assert abs(st[0] - np.sum(rm ** 2)) <= 1e-9 * st[0]
        assert abs(st[1] - np.sum(dm ** 2)) <= 1e-9 * st[1]
        u = UNet(1, H, W, periodic_w=(W * f == w.NY))
        u.pic_unet_load(0, x, t)
        u.pic_unet_forward()
        out = u.output()[0].cpu().numpy().astype(np.float64)
        g = torch.empty(w.NX * w.NY, dtype=torch.float64, device=dev)
        for use in (True, False):
            u.pic_unet_coarse_guess(0, T(p1), T(q2) if second else None, nm, per, f, sc[2], g, use_output=use)
            ref = ou.coarse_residual_guess(out, p1, q2, nc, f, per, sc[2], use_output=use)
            assert np.array_equal(g.cpu().numpy().reshape(w.NX, w.NY), ref)
        u.close()
    pic.close()
