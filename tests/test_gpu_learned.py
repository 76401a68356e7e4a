"""GPU test of the learned warm start end to end (residual learning): samples
from one run of a small y-periodic trench, training with the library's own
forward / backward / Adam kernels, and plain masked CG to 1e-8 on held-out
problems of a second run (another particle load) from these starts: zero on
the free nodes (cold), the previous potential, the linear extrapolation in
time (ext), the K-point extrapolation the network corrects (base, K = 4), and
that start corrected by the network.

Asserted, for the network on the linear start: the training loss falls, every
solve converges to the same potential, the network cuts the residual of the
extrapolated start, and it saves iterations against both the cold start and
the extrapolation alone.  For the network on the 4-point start: every solve
converges to the same potential and the corrected start beats both the
4-point start and the linear one.  The target of a >= 3x cut against the
cold start is kept as a strict expected failure at this size, with the
measured factor.  The measured factors are printed."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _trench(seed):
    return synth.trench(nx=96, ny=56, width=6, depth=24, ppc=12, seed=seed, rtol=1e-8)


def _train(seed=41, steps=1500, K=2):
    import torch
    from paper_1610_03918_amd import Pic, learned
    w = _trench(seed)
    a = Pic(w, synth.load(w))
    a.start()
    a.pic_step(40)                                   # the sheath forms
    H, W = learned.window(w)
    dev = torch.device("cuda:0")
    # probe the scales on a few steps
    probe = []
    learned.run_and_sample(a, 12 + K, {}, (1.0, 1.0, 1.0), keep=probe, K=K)
    from paper_1610_03918_amd.unet import residual_sample
    stats = torch.zeros(3, dtype=torch.float64, device=dev)
    x = torch.empty((H, W, 3), dtype=torch.bfloat16, device=dev)
    t = torch.empty((H, W), dtype=torch.bfloat16, device=dev)
    for b, hist, pn in probe:
        s0 = learned.start_of(hist, K, torch.empty_like(pn))
        residual_sample(b, s0, s0, pn, a.pic_node_map(), (0, 1), H, W, (1.0, 1.0, 1.0), x, t, stats)
    s = stats.cpu().numpy()
    sc = (learned.pow2_scale(np.sqrt(s[0] / s[2])), float(np.float32(1 / 50)),
          learned.pow2_scale(np.sqrt(s[1] / s[2])))
    stores = {(H, W): learned.SampleStore(torch, dev, H, W, 400)}
    learned.run_and_sample(a, 400 + K, stores, sc, K=K)
    a.close()
    assert stores[(H, W)].n == 400
    nets, main = learned.make_nets(stores, 8 * H * W, seed=3)
    losses = learned.train(nets, main, stores, steps, lr=2e-3, seed=1)
    return w, nets[(H, W)], sc, losses


def _evaluate(K):
    """Train on run A, evaluate on 12 held-out problems of run B."""
    import torch
    from paper_1610_03918_amd import Pic, learned
    from paper_1610_03918_amd.unet import UNet
    wa, net, sc, losses = _train(K=K)
    wb = _trench(42)
    b = Pic(wb, synth.load(wb))
    b.start()
    b.pic_step(40)
    learned.run_and_sample(b, 60, {}, sc, K=K)
    problems = []
    learned.run_and_sample(b, 24, {}, sc, keep=problems, every=2, K=K)
    b.close()
    u1 = UNet(1, net.H, net.W, params=net.params, periodic_w=True)
    cg = Pic(wb, synth.load(wb), solver=1, max_iter=20000)
    rows = learned.evaluate(cg, u1, problems, sc, torch, K=K)
    cg.close()
    u1.close()
    kinds = [k for k in ("cold", "prev", "ext", "base", "learned") if k in rows[0]]
    its = {k: np.array([r[k]["iterations"] for r in rows], float) for k in kinds}
    r0 = {k: np.median([r[k]["relres0"] for r in rows]) for k in kinds}
    print(f"K = {K}: loss", np.mean(losses[:5]), "->", np.mean(losses[-20:]))
    print({k: float(v.mean()) for k, v in its.items()}, r0,
          "cold/learned", its["cold"].mean() / its["learned"].mean(),
          "ext/learned", its["ext"].mean() / its["learned"].mean())
    return losses, rows, its, r0


@pytest.fixture(scope="module")
def evaluated():
    """The network correcting the linear extrapolation."""
    return _evaluate(2)


@pytest.fixture(scope="module")
def evaluated4():
    """The network correcting the 4-point extrapolation."""
    return _evaluate(4)


def test_learned_start_cuts_cg_iterations(evaluated):
    losses, rows, its, r0 = evaluated
    assert np.all(np.isfinite(losses))
    assert np.mean(losses[-20:]) < 0.5 * np.mean(losses[:5]), (losses[:5], losses[-20:])
    for r in rows:
        for k in ("cold", "prev", "ext", "learned"):
            assert r[k]["converged"], (k, r)
        assert r["max_diff"] <= 1e-4 * r["scale"], r
    # the network cuts the residual of the extrapolated start several times over
    assert r0["learned"] < 0.5 * r0["ext"], r0
    # and the iterations against the cold start and against the extrapolation alone
    # (measured: 275 / 182 / 176 for cold / extrapolation / learned)
    assert its["learned"].mean() < its["ext"].mean() < its["cold"].mean(), its
    assert its["cold"].mean() / its["learned"].mean() > 1.4, its


def test_network_corrects_the_four_point_start(evaluated4):
    """The network trained on the 4-point start: every solve reaches the same
    potential, and the corrected start beats both the 4-point start it
    corrects and the linear extrapolation.  On this small, noisy problem
    (12 particles per cell) the 4-point start alone is worse than the linear
    one, since its weights amplify the particle noise of the potentials
    (sum of squared weights 69 against 5); measured: cold 275, ext 182,
    base 216, learned 163 iterations, start residual 0.018 -> 0.001."""
    losses, rows, its, r0 = evaluated4
    assert np.all(np.isfinite(losses))
    assert np.mean(losses[-20:]) < 0.5 * np.mean(losses[:5]), (losses[:5], losses[-20:])
    for r in rows:
        for k in ("cold", "prev", "ext", "base", "learned"):
            assert r[k]["converged"], (k, r)
        assert r["max_diff"] <= 1e-4 * r["scale"], r
    assert r0["learned"] < 0.25 * r0["base"], r0
    assert its["learned"].mean() < its["base"].mean(), its
    assert its["learned"].mean() < its["ext"].mean(), its


@pytest.mark.xfail(strict=True, reason="at 96x56 with 12 particles per cell the corrected "
                   "4-point start needs 1.68x fewer iterations than the cold start; the "
                   "3x cut holds on the 1024x512 trench (3.66x, measured by the benchmark)")
def test_threefold_target_on_the_small_trench(evaluated4):
    losses, rows, its, r0 = evaluated4
    assert its["cold"].mean() / its["learned"].mean() >= 3.0, its


def test_learned_start_inside_a_running_simulation():
    """pic_solve_learned_residual on the live context: the corrected start of
    the context's own b and potentials, finished by the solver to rtol; the
    time history carries on (the next extrapolated, kind-3, solve converges
    in a few multigrid iterations), and the potential equals the one a cold
    solve of the same b reaches."""
    import torch
    from paper_1610_03918_amd import Pic
    from paper_1610_03918_amd.unet import UNet
    wa, net, sc, _ = _train(steps=300)
    u1 = UNet(1, net.H, net.W, params=net.params, periodic_w=True)
    p = Pic(wa, synth.load(wa))
    p.start()
    p.pic_step(30)
    guess = torch.empty(p.nodes, dtype=torch.float64, device=p.dev)
    free = torch.as_tensor(p.node_map_host() == 0, device=p.dev)
    for k in range(3):
        info = u1.pic_solve_learned_residual(p, sc, guess)
        assert info["converged"] and info["relres"] <= wa.rtol, info
        p.pic_push()
        info3 = p.pic_solve(3)
        assert info3["converged"] and info3["iterations"] <= 12, info3
        p.pic_push()
    info = u1.pic_solve_learned_residual(p, sc, guess)
    phi_l = p.phi.clone()
    cold = p.pic_solve(0)
    assert cold["converged"] and cold["iterations"] > info["iterations"], (cold, info)
    assert float(((p.phi - phi_l) * free).abs().max()) <= 1e-4 * float(phi_l.abs().max())
    u1.close()
    p.close()
