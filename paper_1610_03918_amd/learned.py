"""Learned warm start of the field solve: training samples from solver runs,
training with the library's own forward / backward / Adam kernels, and the
iteration counts of the plain solver from several starts.

The network corrects the solver's own start, a K-point polynomial
extrapolation in time of the last K potentials (K = 2: phi_s = 2 phi_{n-1} -
phi_{n-2}; K = 4: 4 phi_{n-1} - 6 phi_{n-2} + 4 phi_{n-3} - phi_{n-4})
(residual learning): its input is the residual b - A phi_s (with the
free-node mask and the Dirichlet potentials), its target the gap phi_n -
phi_s to the converged potential.  With a coarsening factor f > 1 a network
pixel stands for an f x f block of nodes (block means in, a block-mean
correction out, prolonged bilinearly onto the nodes), so that the network
sees the whole grid.

Orchestration only: every tensor operation on the method's data runs in the
library (see unet.py); this module decides which sample goes into which batch
slot, keeps the stored samples and the potentials' time history in device
tensors that torch allocates, and records the solver's counters.
"""
from __future__ import annotations

import math
import time

import numpy as np

from .unet import UNet, coarse_sample, extrapolate, extrapolation_coefficients, residual_sample


def window(w, f=1):
    """Network window (pixels) over the node grid at coarsening factor f:
    the largest multiples of 8 of the node counts over f."""
    return (w.NX // f // 8) * 8, (w.NY // f // 8) * 8


def points_of(K):
    """Past potentials a start stencil reads: K, or the first entry of a
    (points, degree) pair."""
    return K[0] if isinstance(K, tuple) else K


def start_of(hist, K, out):
    """The extrapolation of the history (hist[0] the latest potential) into
    out, computed by the library.  K: the points of the polynomial through
    the last K potentials, or (points, degree) for the least-squares
    polynomial of that degree through more points.  With fewer potentials
    than the stencil reads, the interpolation through those there are."""
    n = points_of(K)
    if len(hist) < n or not isinstance(K, tuple):
        k = min(n, len(hist))
        extrapolate(hist[:k], extrapolation_coefficients(k), out)
    else:
        extrapolate(hist[:n], extrapolation_coefficients(n, K[1]), out)
    return out


def sample(f, b, phi_1, phi_2, phi_t, node_map, periodic, H, W, scales, x, t=None, stats=None):
    """One training sample (or network input) at coarsening factor f, from
    the start 2 phi_1 - phi_2 (phi_1 = phi_2 = s: the start s itself)."""
    if f == 1:
        residual_sample(b, phi_1, phi_2, phi_t, node_map, periodic, H, W, scales, x, t, stats)
    else:
        coarse_sample(b, phi_1, phi_2, phi_t, node_map, periodic, f, H, W, scales, x, t, stats)


def start_guess(f, net, slot, phi_1, phi_2, node_map, periodic, s_d, guess, use_output=True):
    """The corrected start (use_output) or the extrapolation alone into guess."""
    if f == 1:
        net.pic_unet_residual_guess(slot, phi_1, phi_2, node_map, s_d, guess, use_output=use_output)
    else:
        net.pic_unet_coarse_guess(slot, phi_1, phi_2, node_map, periodic, f, s_d, guess, use_output=use_output)


def pow2_scale(rms):
    """A power of two near 1 / rms (exact rescaling in bfloat16)."""
    return float(2.0 ** round(-math.log2(rms))) if rms > 0 else 1.0


class SampleStore:
    """Stored training samples of one window size, in device memory:
    inputs bfloat16 [N, H, W, 3] and targets bfloat16 [N, H, W]."""

    def __init__(self, torch, dev, H, W, capacity):
        self.H, self.W = H, W
        self.x = torch.empty((capacity, H, W, 3), dtype=torch.bfloat16, device=dev)
        self.t = torch.empty((capacity, H, W), dtype=torch.bfloat16, device=dev)
        self.n = 0

    def full(self):
        return self.n >= self.x.shape[0]


def run_and_sample(pic, steps, stores, scales, keep=None, every=1, f=1, K=2):
    """Advances a single-instance Pic `steps` steps (solve from its
    extrapolated start, push) and writes a sample (factor f, K-point start)
    of each `every`-th step's solve into stores[(H, W)] until it is full.
    keep: a list that receives the float64 (b, [phi_{n-1} .. phi_{n-K}],
    phi_n) of every `every`-th step instead (held-out problems).  Returns the
    solver infos."""
    w = pic.w
    H, W = window(w, f)
    nm = pic.pic_node_map()
    per = (int(w.periodic_x), int(w.periodic_y))
    hist = getattr(pic, "_phi_hist", [])
    s = pic.torch.empty_like(pic.phi)
    infos = []
    for k in range(steps):
        info = pic.pic_solve(3)
        infos.append(info)
        phi = pic.phi.clone()
        if len(hist) >= points_of(K) and k % every == 0:
            if keep is not None:
                keep.append((pic.b.clone(), list(hist[:points_of(K)]), phi))
            else:
                st = stores.get((H, W))
                if st is not None and not st.full():
                    start_of(hist, K, s)
                    sample(f, pic.b, s, s, phi, nm, per, H, W, scales, st.x[st.n], st.t[st.n])
                    st.n += 1
        hist = ([phi] + hist)[:max(points_of(K), 2)]
        pic.pic_push()
    pic._phi_hist = hist
    return infos


def run_and_sample_batch(batch, steps, stores, scales, f=1, K=2):
    """As run_and_sample for every instance of a PicBatch (eager solves of
    all instances, one sample per instance and step)."""
    n = batch.n
    hist = getattr(batch, "_phi_hist", [[] for _ in range(n)])
    nms = [batch.pic_node_map(i) for i in range(n)]
    for _ in range(steps):
        batch.pic_solve(3)
        for i, w in enumerate(batch.ws):
            phi = batch.phi(i).clone()
            if len(hist[i]) >= points_of(K):
                H, W = window(w, f)
                st = stores.get((H, W))
                if st is not None and not st.full():
                    s = start_of(hist[i], K, batch.torch.empty_like(phi))
                    sample(f, batch.b(i), s, s, phi, nms[i],
                           (int(w.periodic_x), int(w.periodic_y)), H, W, scales, st.x[st.n], st.t[st.n])
                    st.n += 1
            hist[i] = ([phi] + hist[i])[:max(points_of(K), 2)]
        batch.pic_push()
    batch._phi_hist = hist


def make_nets(stores, batch_pixels, seed, periodic_w=True):
    """One network per window size over shared parameters, gradients and
    Adam moments; the batch of each holds about batch_pixels pixels."""
    nets = {}
    main = None
    for (H, W) in sorted(stores, key=lambda k: -k[0] * k[1]):
        B = max(1, min(64, batch_pixels // (H * W)))
        nets[(H, W)] = UNet(B, H, W, seed=seed, share=main, periodic_w=periodic_w)
        main = main or nets[(H, W)]
    return nets, main


def train(nets, main, stores, steps, lr=2e-3, seed=0, log=None, log_every=0):
    """Adam on the masked mean-square error of the target over random batches
    of stored samples: each step draws a window size with probability
    proportional to its stored pixels, then fills that network's batch.
    Cosine-decayed learning rate.  Returns the losses."""
    rng = np.random.default_rng(seed)
    keys = [k for k in nets if stores[k].n > 0]
    wts = np.array([stores[k].n * k[0] * k[1] for k in keys], float)
    wts /= wts.sum()
    losses = []
    for it in range(steps):
        key = keys[rng.choice(len(keys), p=wts)]
        net, st = nets[key], stores[key]
        idx = rng.choice(st.n, size=net.B, replace=st.n < net.B)
        for slot, k in enumerate(idx):
            net.pic_unet_load(slot, st.x[k], st.t[k])
        rate = lr * 0.5 * (1.0 + math.cos(math.pi * it / max(steps, 1)))
        net.pic_unet_forward()
        losses.append(net.pic_unet_loss())
        net.pic_unet_backward()
        main.pic_unet_adam(max(rate, 1e-3 * lr))
        for other in nets.values():
            other.pic_unet_params_changed()
        if log and log_every and (it % log_every == 0 or it == steps - 1):
            log(f"train step {it} ({key[0]}x{key[1]}): loss {losses[-1]:.4e}")
    return losses


def evaluate(pic_cg, net, problems, scales, torch, f=1, K=2):
    """Iterations and wall time (ms) of the solver of pic_cg on each held-out
    problem (b, [phi_{n-1} .. phi_{n-K}], phi_n) from the starts: zero on the
    free nodes (cold), the previous potential, the linear extrapolation
    (ext), the K-point extrapolation the network corrects (base, when K > 2)
    and that start corrected by the network (learned; its extrapolation,
    sample and inference included in the time).  Also the largest
    difference between the cold and learned solutions on the free nodes."""
    w = pic_cg.w
    H, W = window(w, f)
    nm = pic_cg.pic_node_map()
    per = (int(w.periodic_x), int(w.periodic_y))
    guess = torch.empty(pic_cg.nodes, dtype=torch.float64, device=pic_cg.dev)
    s = torch.empty_like(problems[0][2]) if problems else None
    free = torch.as_tensor(pic_cg.node_map_host() == 0, device=pic_cg.dev)
    s_r, s_v, s_d = scales

    def timed(fn):
        torch.cuda.synchronize(pic_cg.dev)
        t0 = time.perf_counter()
        info = fn()
        torch.cuda.synchronize(pic_cg.dev)
        info["ms"] = 1e3 * (time.perf_counter() - t0)
        return info

    def learned_start():
        start_of(hist, K, s)
        sample(f, pic_cg.b, s, s, None, nm, per, H, W, scales, net.input()[0])
        net.pic_unet_forward()
        start_guess(f, net, 0, s, s, nm, per, s_d, guess, use_output=True)
        return pic_cg.pic_solve(2, guess)

    def ext_start(k):
        start_of(hist, k, s)
        start_guess(f, net, 0, s, s, nm, per, s_d, guess, use_output=False)
        return pic_cg.pic_solve(2, guess)

    rows = []
    for (b, hist, pn) in problems:
        pic_cg.b.copy_(b)
        cold = timed(lambda: pic_cg.pic_solve(0))
        phi_cold = pic_cg.phi.clone()
        pic_cg.phi.copy_(hist[0])
        prev = timed(lambda: pic_cg.pic_solve(1))
        ext = timed(lambda: ext_start(2))
        row = {"cold": cold, "prev": prev, "ext": ext}
        if K != 2:
            row["base"] = timed(lambda: ext_start(K))
        row["learned"] = timed(learned_start)
        row["max_diff"] = float(((pic_cg.phi - phi_cold) * free).abs().max())
        row["scale"] = float(pn.abs().max())
        rows.append(row)
    return rows


def coarse_bound(pic_cg, problems, factors, torch, scale_errors=(0.99,), K=2):
    """What a perfect coarse network would give: plain-solver iterations from
    the K-point extrapolated start corrected by the exact block means (f x f)
    of the true correction phi_n - phi_s (the training target itself,
    bfloat16), prolonged as the network's output would be; and from the same
    correction with a uniform relative error (times each of scale_errors).
    Mean iterations per factor over the problems."""
    w = pic_cg.w
    nm = pic_cg.pic_node_map()
    per = (int(w.periodic_x), int(w.periodic_y))
    guess = torch.empty(pic_cg.nodes, dtype=torch.float64, device=pic_cg.dev)
    s = torch.empty_like(problems[0][2])
    out = {}
    for f in factors:
        H, W = window(w, f)
        net = UNet(1, H, W, device=pic_cg.dev, periodic_w=bool(per[1]) and W * f == w.NY)
        x = torch.empty((H, W, 3), dtype=torch.bfloat16, device=pic_cg.dev)
        t = torch.empty((H, W), dtype=torch.bfloat16, device=pic_cg.dev)
        its = {"exact": []}
        its.update({f"scaled_{e:g}": [] for e in scale_errors})
        for (b, hist, pn) in problems:
            pic_cg.b.copy_(b)
            start_of(hist, K, s)
            sample(f, b, s, s, pn, nm, per, H, W, (1.0, 1.0, 1.0), x, t)
            net.output()[0].copy_(t)
            start_guess(f, net, 0, s, s, nm, per, 1.0, guess)
            its["exact"].append(pic_cg.pic_solve(2, guess)["iterations"])
            for e in scale_errors:
                start_guess(f, net, 0, s, s, nm, per, 1.0 / e, guess)
                its[f"scaled_{e:g}"].append(pic_cg.pic_solve(2, guess)["iterations"])
        net.close()
        out[f] = {k: float(np.mean(v)) for k, v in its.items()}
    return out
