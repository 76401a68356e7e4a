"""Learned warm start of the field solve: snapshot collection from solver
runs, training with the library's own forward / backward / Adam kernels,
and the iteration counts of cold, previous-step and learned starts.

Orchestration only: every tensor operation runs in the library (see
unet.py); this module decides which snapshot goes into which batch slot and
records the solver's counters.
"""
from __future__ import annotations

import math

import numpy as np

from .unet import UNet


def window(w):
    """Network window over the node grid: the largest multiples of 8."""
    return (w.NX // 8) * 8, (w.NY // 8) * 8


def collect(pic, n, guess_kind=3):
    """n (b, phi) pairs from a running simulation: solve, record, push."""
    snaps = []
    for _ in range(n):
        pic.pic_solve(guess_kind)
        snaps.append((pic.b.clone(), pic.phi.clone()))
        pic.pic_push()
    return snaps


def scales(w, snaps, node_cond):
    """(s_rho, s_v, s_phi): the source term on free nodes scaled to unit RMS
    over the snapshots, potentials by the largest conductor amplitude.
    node_cond: host copy of the node map (NX*NY)."""
    amp = float(np.max(np.abs(np.asarray(w.v_amp, dtype=np.float64))))
    amp = amp if amp > 0 else 1.0
    free = np.asarray(node_cond).reshape(-1) == 0
    ss = 0.0
    cnt = 0
    for b, _ in snaps:
        v = b.reshape(-1).cpu().numpy()[free]
        ss += float(np.dot(v, v))
        cnt += v.size
    rms = math.sqrt(ss / max(cnt, 1)) or 1.0
    return (float(np.float32(1.0 / rms)), float(np.float32(1.0 / amp)), float(np.float32(amp)))


def train(net: UNet, snaps, node_map, sc, steps, lr=2e-3, seed=0, log_every=0, log=None):
    """Adam on the masked mean-square error of phi / s_phi over random
    batches of snapshots, cosine-decayed learning rate.  Returns the losses."""
    rng = np.random.default_rng(seed)
    losses = []
    for it in range(steps):
        idx = rng.choice(len(snaps), size=net.B, replace=len(snaps) < net.B)
        for slot, k in enumerate(idx):
            b, phi = snaps[k]
            net.pic_unet_snapshot(slot, b, phi, node_map, sc)
        rate = lr * 0.5 * (1.0 + math.cos(math.pi * it / max(steps, 1)))
        losses.append(net.train_step(max(rate, 1e-3 * lr)))
        if log and log_every and (it % log_every == 0 or it == steps - 1):
            log(f"train step {it}: loss {losses[-1]:.4e}")
    return losses


def evaluate(pic_cg, net: UNet, snaps, sc, torch):
    """Iterations and wall time (ms) of the solver of pic_cg on each
    snapshot's right-hand side from three starts: zero on the free nodes
    (cold), the previous snapshot's potential, and the network's prediction
    (its inference included).  Also the largest difference between the cold
    and learned solutions on the free nodes."""
    import time
    guess = torch.empty(pic_cg.nodes, dtype=torch.float64, device=pic_cg.dev)
    free = torch.as_tensor(pic_cg.node_map_host() == 0, device=pic_cg.dev)

    def timed(fn):
        torch.cuda.synchronize(pic_cg.dev)
        t0 = time.perf_counter()
        info = fn()
        torch.cuda.synchronize(pic_cg.dev)
        info["ms"] = 1e3 * (time.perf_counter() - t0)
        return info

    rows = []
    for k, (b, phi) in enumerate(snaps):
        pic_cg.b.copy_(b)
        cold = timed(lambda: pic_cg.pic_solve(0))
        phi_cold = pic_cg.phi.clone()
        prev = None
        if k > 0:
            pic_cg.phi.copy_(snaps[k - 1][1])
            prev = timed(lambda: pic_cg.pic_solve(1))
        learned = timed(lambda: net.pic_solve_learned(pic_cg, sc, guess))
        diff = float(((pic_cg.phi - phi_cold) * free).abs().max())
        rows.append({"cold": cold, "prev": prev, "learned": learned, "max_diff": diff,
                     "scale": float(phi.abs().max())})
    return rows
