"""Throughput of the PIC hot path on one MI355X.

One step = solve (from the previous potential) + field + gather/push/wall
test + deposit of the new positions + assembly (+ re-binning when due),
over both species of the trench workload.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                  [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0         # dense bf16 MFMA
BYTES_PER_PARTICLE_STEP = 40      # 20 B read + 20 B written per particle (cell, ox, oy, vx, vy)
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "push_trench1024x512_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1610_03918_amd", "csrc", "pic_kernels.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    import synth
    if name == "trench1024x512":
        return synth.trench()
    if name == "bounded256":
        return synth.bounded_square()
    if name == "periodic64":
        return synth.periodic_square()
    if name.startswith("trench_small"):
        return synth.trench(nx=256, ny=128, width=8, depth=32, ppc=64)
    if name in synth.PRESETS:
        return synth.PRESETS[name]()
    raise SystemExit(f"unknown workload {name}")


def push_source_hash():
    """sha256 of what the push kernel is built from: the header constants it
    uses, the structs it reads (Geom, Tab, HitLog, PushArgs, the LDS size
    formula) and the particle section of the kernel source (gather, push,
    wall test, deposit), so that edits elsewhere keep its counters valid."""
    import hashlib
    import re
    hdr = open(os.path.join(os.path.dirname(KERNEL_SOURCE), "pic_internal.h"), "rb").read()
    names = (b"kNClass", b"kIadBins", b"kDiagBlocks", b"kMaxInst", b"kMaxUnits", b"kPushThreads", b"kFieldFrame")
    parts = [re.search(rb"^constexpr int " + k + rb" = [^\n]*", hdr, re.M).group(0) for k in names]
    for name in (b"struct Geom {", b"struct Tab {", b"struct HitLog {", b"struct PushArgs {",
                 b"inline size_t push_lds_bytes("):
        a = hdr.index(name)
        parts.append(hdr[a:hdr.index(b"\n}", a) + 2])
    src = open(KERNEL_SOURCE, "rb").read()
    a = src.index(b"// particles: gather, leapfrog push")
    b = src.index(b"// re-binning: counting sort")
    return hashlib.sha256(b"\n".join(parts) + src[a:b]).hexdigest()


def measured_traffic(workload_name, particles_per_launch):
    """HBM bytes per push launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE passes (scaled by the plain-copy calibration), rescaled to the
    live particle count.  None when the push kernel's source changed since
    the counters were taken, or for another workload."""
    if not workload_name.startswith("trench1024x512") or not os.path.exists(TRAFFIC_PROFILE):
        return None
    kv = {}
    for line in open(TRAFFIC_PROFILE):
        if ":" in line and not line.startswith(("|", "#", "`")):
            k, _, v = line.partition(":")
            kv[k.strip()] = v.strip()
    try:
        if kv.get("push_source_sha256") != push_source_hash():
            return None
        return float(kv["traffic_bytes_per_launch"]) * particles_per_launch / float(kv["particles_per_launch"])
    except (KeyError, ValueError, OSError):
        return None


def cpu_baseline(w, parts):
    """The oracle as it stands, full steps of the same workload on the host
    (single thread; the sparse LU factorisation happens in start()), repeated
    until about 10 s of stepping have been timed."""
    import oracle
    t0 = time.perf_counter()
    sim = oracle.Sim(w, parts)
    sim.start()
    t1 = time.perf_counter()
    done, n_steps, t_steps = 0, 0, 0.0
    while t_steps < 10.0 and n_steps < 16:
        n = sum(sim.alive(s) for s in range(2))
        t2 = time.perf_counter()
        sim.step()
        t_steps += time.perf_counter() - t2
        done += n
        n_steps += 1
    rate = done / t_steps
    log(f"oracle: start {t1 - t0:.1f}s, {n_steps} steps in {t_steps:.2f}s ({done / n_steps:.0f} particles per step)")
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": rate, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "host_cpu": model, "host_cores_available": len(os.sched_getaffinity(0)),
            "sample": f"{n_steps} full steps of {w.name} ({done // n_steps} particles, {w.nx}x{w.ny} cells) "
                      f"after the oracle's start (sparse LU factorisation excluded), "
                      f"{t_steps:.1f} s of CPU time on one thread"}


def flops_per_inference(H, W):
    """Algorithmic multiply-add flops of one U-Net inference on H x W pixels
    (2 per multiply-add over every 3x3 convolution and the 1x1 head)."""
    from paper_1610_03918_amd.unet import layers
    fl = 0
    ys = layers()
    for y in ys[:-1]:
        P = (H >> y["level"]) * (W >> y["level"])
        fl += 2 * P * y["cout"] * 9 * y["cin"]
    return fl + 2 * H * W * 16


def learned_start(w, pic, parts, args):
    """The learned warm start (residual learning): the network corrects the
    K-point polynomial extrapolation in time of the last K potentials (K =
    args.learn_stencil; K = 4: 4 phi_1 - 6 phi_2 + 4 phi_3 - phi_4; with
    args.learn_fit = D the least-squares polynomial of degree D through
    them), at full
    resolution (f = 1) or on f x f blocks of nodes (block means of the
    residual in, a block-mean correction out, prolonged bilinearly onto the
    nodes).  Training samples come from this trench run (after the timed
    steps) and from the 16-width sweep (its 1024 x 512, 512 x 256 and
    256 x 128 instances, one network per window size over shared
    parameters); training uses the library's forward / backward / Adam
    kernels.  Then plain masked CG to the workload's tolerance on held-out
    problems of the trench run from the starts: cold, previous potential,
    linear extrapolation, the K-point extrapolation alone (base) and with the
    network's correction (extrapolation, sample, inference and guess
    included in the time)."""
    import numpy as np
    import torch

    import synth
    from paper_1610_03918_amd import Pic, PicBatch, learned
    from paper_1610_03918_amd.unet import UNet
    dev = torch.device("cuda:0")
    f = args.learn_factor
    K = args.learn_stencil if args.learn_fit is None else (args.learn_stencil, args.learn_fit)
    H, W = learned.window(w, f)
    per = (int(w.periodic_x), int(w.periodic_y))
    t0 = time.perf_counter()
    # scales: powers of two near the inverse RMS of the residual and of the gap
    probe = []
    learned.run_and_sample(pic, 12 + learned.points_of(K), {}, (1.0, 1.0, 1.0), keep=probe, f=f, K=K)
    stats = torch.zeros(3, dtype=torch.float64, device=dev)
    x = torch.empty((H, W, 3), dtype=torch.bfloat16, device=dev)
    tt = torch.empty((H, W), dtype=torch.bfloat16, device=dev)
    for b, hist, pn in probe:
        s0 = learned.start_of(hist, K, torch.empty_like(pn))
        learned.sample(f, b, s0, s0, pn, pic.pic_node_map(), per, H, W, (1.0, 1.0, 1.0), x, tt, stats)
    st = stats.cpu().numpy()
    amp = float(np.max(np.abs(np.asarray(w.v_amp, np.float64)))) or 1.0
    sc = (learned.pow2_scale(np.sqrt(st[0] / st[2])), float(np.float32(1.0 / amp)),
          learned.pow2_scale(np.sqrt(st[1] / st[2])))
    del probe
    stores = {(H, W): learned.SampleStore(torch, dev, H, W, args.learn_trench_samples)}
    learned.run_and_sample(pic, args.learn_every * (args.learn_trench_samples + 2), stores, sc,
                           every=args.learn_every, f=f, K=K)
    learned.run_and_sample(pic, 50, {}, sc, f=f, K=K)           # a gap before the held-out problems
    problems = []
    learned.run_and_sample(pic, 5 * args.learn_evals, {}, sc, keep=problems, every=5, f=f, K=K)
    n_trench = stores[(H, W)].n
    t1 = time.perf_counter()
    # the 16-width sweep (batched form), eager steps after a short spin-up
    n_sweep = 0
    if args.learn_sweep_steps > 0:
        ws = synth.sweep()
        sw = PicBatch(ws, [synth.load(q) for q in ws], sort_interval=(16, 128))
        sw.start()
        sw.pic_step(args.learn_sweep_spinup)
        caps = {}
        for q in ws:
            caps[learned.window(q, f)] = caps.get(learned.window(q, f), 0) + args.learn_sweep_steps
        for k, c in caps.items():
            if k in stores:
                old = stores[k]
                new = learned.SampleStore(torch, dev, k[0], k[1], old.n + c)
                new.x[:old.n].copy_(old.x[:old.n])
                new.t[:old.n].copy_(old.t[:old.n])
                new.n = old.n
                stores[k] = new
                del old
            else:
                stores[k] = learned.SampleStore(torch, dev, k[0], k[1], c)
        before = sum(s_.n for s_ in stores.values())
        learned.run_and_sample_batch(sw, args.learn_sweep_steps + learned.points_of(K), stores, sc, f=f, K=K)
        n_sweep = sum(s_.n for s_ in stores.values()) - before
        sw.close()
        del sw
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    nets, main = learned.make_nets(stores, args.learn_batch * H * W, seed=5)
    losses = learned.train(nets, main, stores, args.learn_steps, lr=args.learn_rate, seed=2)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    log(f"learned start (f = {f}): {n_trench} trench + {n_sweep} sweep samples in {t2 - t0:.1f}s "
        f"({', '.join(f'{k[0]}x{k[1]}: {v.n}' for k, v in stores.items())}), {args.learn_steps} training steps "
        f"in {t3 - t2:.1f}s, loss {np.mean(losses[:5]):.3e} -> {np.mean(losses[-10:]):.3e}")
    u1 = UNet(1, H, W, params=main.params, periodic_w=True)
    for n_ in nets.values():
        n_.close()
    del stores
    torch.cuda.empty_cache()
    u1.input().zero_()
    u1.pic_unet_forward()
    u1.pic_unet_set_timing(True)
    for _ in range(20):
        u1.pic_unet_forward()
    fwd_ms, _ = u1.pic_unet_forward_timing()
    u1.pic_unet_set_timing(False)
    few = [{k: p[k][:4096] for k in p} for p in parts]
    cg = Pic(w, few, solver=1, max_iter=50000)
    rows = learned.evaluate(cg, u1, problems, sc, torch, f=f, K=K)
    u1.close()
    bound = learned.coarse_bound(cg, problems[:args.learn_bound_problems], (4, 8, 16), torch, K=K)
    cg.close()
    log(f"  exact coarse targets (mean iterations): {bound}")
    kinds = ("cold", "prev", "ext", "base", "learned") if K != 2 else ("cold", "prev", "ext", "learned")
    for r in rows:
        log("  " + " | ".join(f"{k} {r[k]['iterations']} it {r[k]['ms']:.1f} ms (relres0 {r[k]['relres0']:.2g})"
                              for k in kinds) + f" | max diff {r['max_diff']:.2e}")

    def mean(kind, key):
        return float(np.mean([r[kind][key] for r in rows]))

    fl = flops_per_inference(H, W)
    tf = fl / (fwd_ms * 1e-3) / 1e12
    if isinstance(K, tuple):
        stencil = f"the least-squares polynomial of degree {K[1]} through the last {K[0]} potentials"
    else:
        stencil = {2: "2 phi_(n-1) - phi_(n-2)", 3: "3 phi_(n-1) - 3 phi_(n-2) + phi_(n-3)",
                   4: "4 phi_(n-1) - 6 phi_(n-2) + 4 phi_(n-3) - phi_(n-4)"}.get(K, f"the {K}-point extrapolation")
    return {
        "solver": f"plain masked CG (float64 refinement of float32 CG), rtol {w.rtol:g}",
        "start": (f"coarse residual learning: the network maps block means ({f}x{f} nodes) of the residual of "
                  f"the start {stencil} to a block-mean correction, prolonged bilinearly onto the free nodes"
                  if f > 1 else f"residual learning: network(residual of the start {stencil}) corrects that start"),
        "factor": f,
        "stencil_points": learned.points_of(K),
        "stencil_degree": K[1] if isinstance(K, tuple) else K - 1,
        "problems_evaluated": len(rows),
        **{k: {"iterations": mean(k, "iterations"), "ms": mean(k, "ms"),
               "relres0": float(np.median([r[k]["relres0"] for r in rows]))} for k in kinds},
        "iterations_cold_over_learned": mean("cold", "iterations") / mean("learned", "iterations"),
        "iterations_ext_over_learned": mean("ext", "iterations") / mean("learned", "iterations"),
        "iterations_cold_over_ext": mean("cold", "iterations") / mean("ext", "iterations"),
        **({"iterations_cold_over_base": mean("cold", "iterations") / mean("base", "iterations"),
            "iterations_base_over_learned": mean("base", "iterations") / mean("learned", "iterations")}
           if K != 2 else {}),
        "ms_cold_over_learned": mean("cold", "ms") / mean("learned", "ms"),
        "target_cold_over_learned": 3.0,
        "coarse_exact_target_iterations": {
            "what": "extrapolation + the exact f x f block means of the true correction (a perfect coarse network), "
                    "and the same with a 1 % uniform error",
            "problems": min(len(problems), args.learn_bound_problems),
            **{f"f{k}": v for k, v in bound.items()}},
        "all_converged": all(r[k]["converged"] for r in rows for k in kinds),
        "max_solution_diff_over_scale": max(r["max_diff"] / r["scale"] for r in rows),
        "training": {"samples_trench1024x512": n_trench, "samples_sweep16": n_sweep,
                     "trench_sample_every": args.learn_every,
                     "sample_windows": sorted({f"{k[0]}x{k[1]}" for k in nets}), "steps": args.learn_steps,
                     "batch_pixels": args.learn_batch * H * W, "scales": list(sc),
                     "loss_first": float(np.mean(losses[:5])), "loss_last": float(np.mean(losses[-10:])),
                     "seconds_sampling": t2 - t0, "seconds_training": t3 - t2},
        "unet": {"pixels": [H, W], "periodic_w": True, "forward_ms": fwd_ms, "gflop_per_inference": fl / 1e9,
                 "roofline": {"bound": "mfma", "achieved": tf, "peak": BF16_PEAK_TFLOPS,
                              "unit": "TFLOP/s", "frac": tf / BF16_PEAK_TFLOPS}},
    }


def run_unet(args):
    """The learned start's network alone on the trench's 1024 x 512 node
    window: forward passes at batch 1 (inference) and training steps at
    batch 4, random bfloat16 inputs."""
    import torch

    from paper_1610_03918_amd.unet import UNet
    H, W = 1024, 512
    fl = flops_per_inference(H, W)
    out = {"metric": "U-Net inference (1024 x 512, batch 1)", "unit": "ms", "n_gpus": 1,
           "higher_is_better": False, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": "learned-start network, 4 levels 16/32/64/128", "pixels": [H, W]}}
    u = UNet(1, H, W, seed=3)
    g = torch.Generator(device="cpu").manual_seed(5)
    u.input().copy_(torch.randn(1, H, W, 3, generator=g).to(torch.bfloat16))
    for _ in range(3):
        u.pic_unet_forward()
    torch.cuda.synchronize()
    u.pic_unet_set_timing(True)
    for _ in range(20):
        u.pic_unet_forward()
    ms, n = u.pic_unet_forward_timing()
    u.close()
    tf = fl / (ms * 1e-3) / 1e12
    out.update(value=ms, roofline={"bound": "mfma", "achieved": tf, "peak": BF16_PEAK_TFLOPS,
                                   "unit": "TFLOP/s", "frac": tf / BF16_PEAK_TFLOPS, "traffic": None},
               gflop_per_inference=fl / 1e9)
    t4 = UNet(4, H, W, seed=3)
    t4.input().copy_(torch.randn(4, H, W, 3, generator=g).to(torch.bfloat16))
    t4.target().normal_(generator=None)
    t4.mask().fill_(1.0)
    t4.train_step(1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        t4.train_step(1e-4)
    torch.cuda.synchronize()
    out["train_step_ms_batch4"] = 1e3 * (time.perf_counter() - t0) / 5
    t4.close()
    print(json.dumps(out), flush=True)


def run_solvers(args):
    """The solvers side by side from a cold start (phi = 0 on free nodes) on the
    periodic 64 x 64 and the grounded 256 x 256 squares: multigrid-
    preconditioned CG, plain CG, and the paper's own Jacobi and Gauss-Seidel
    sweeps (Sec. II), each to the workload's tolerance."""
    import torch

    import synth
    from paper_1610_03918_amd import Pic
    rows = []
    for w in (synth.periodic_square(n=64, ppc=4), synth.bounded_square(n=256, ppc=4)):
        parts = synth.load(w)
        for solver, name in ((0, "multigrid CG"), (1, "CG"), (2, "Jacobi"), (3, "Gauss-Seidel")):
            pic = Pic(w, parts, solver=solver, max_iter=2_000_000, sort_interval=(0, 0))
            pic.pic_solve(0)                      # graphs captured, caches warm
            torch.cuda.synchronize()
            reps = 3
            t0 = time.perf_counter()
            for _ in range(reps):
                info = pic.pic_solve(0)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / reps
            pic.close()
            rows.append({"workload": w.name, "solver": name, "rtol": w.rtol, "iterations": info["iterations"],
                         "ms_per_solve": ms, "relres": info["relres"], "converged": bool(info["converged"])})
            log(f"{w.name:12s} {name:14s} {info['iterations']:8d} it {ms:10.3f} ms relres {info['relres']:.2e}")
    print(json.dumps({"metric": "Poisson solve from a cold start: ms and iterations (sweeps for Jacobi and "
                                "Gauss-Seidel)", "n_gpus": 1, "data": "synthetic", "results": rows}), flush=True)


PAPER_TRENCH_COUNTS = {   # Sec. III.C-D: ions reaching the bottom / the two sidewalls
    "paper_trench_w15": (2137, 4920),
    "paper_trench_w4": (831, 1558),
    "paper_trench_w15_charged": (1094, 3820),
}


def run_trench_study(args):
    """The trench runs of Sec. III.C-D at the paper's parameters (80 x 30
    cells, 100 particles per cell, dt = 0.1 to t = 1000, ions recycled into
    the bulk): ions reaching the trench bottom (class 4, +x inside the trench
    box) and the two sidewalls (classes 6 and 7) over 600 <= t <= 1000
    (700 <= t <= 1000 with the charged bottom, as the paper counts), their
    ratio, the same with only the sidewall hits at least 5 cells below the
    trench mouth (the paper draws its sidewalls from x = 65 to 80), the
    cumulative counts every 50 time units, and the mean impact angle of the
    bottom and sidewall hits.  With --see GI,GE the trench surfaces emit
    secondary electrons (Sec. IV; constant yields per ion / electron impact,
    emission speed --see-vth): the same counts, the electrons emitted, and the
    potential at the trench's mid-depth centre averaged over the window."""
    import numpy as np
    import torch

    import synth
    from paper_1610_03918_amd import Pic
    see = tuple(float(x) for x in args.see.split(",")) if args.see else None
    rows = []
    for width, charged, t_from in ((15, False, 600), (4, False, 600), (15, True, 700)):
        w = synth.paper_trench(width, charged, seed=args.study_seed)
        if see:
            w.see_yield = (see[1], see[0])            # species 0 electrons, 1 ions
            w.see_vth = args.see_vth
        cap = 1 << (22 if see else 21)
        pic = Pic(w, synth.load(w), hitlog_capacity=cap, hitlog_species_mask=2,
                  capacity=None if not see else (2 * w.n_particles(0), w.n_particles(1)))
        pic.start()
        k_from = int(round(t_from / w.dt))
        every = int(round(50 / w.dt))
        curve = []
        base = None
        im = (w.box_i_top + w.nx) // 2
        jc = (w.box_j_lo + w.box_j_hi) // 2
        phi_mid = []
        t0 = time.perf_counter()
        for k in range(0, w.steps, every):
            pic.pic_step(every)
            tal = pic.pic_diagnostics()["tally"][1]
            curve.append([round((k + every) * w.dt, 3), tal[4], tal[6] + tal[7]])
            if k + every == k_from:
                base = (tal[4], tal[6] + tal[7])
            if k + every > k_from:
                phi_mid.append(float(pic.phi[im, jc]))
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        d = pic.pic_diagnostics()
        tal = d["tally"][1]
        nb, ns = tal[4] - base[0], tal[6] + tal[7] - base[1]
        hits = pic.pic_read_hits()
        h = hits[(hits["step"] >= k_from) & ((hits["species_class"] >> 8) == 1)]
        cls = h["species_class"] & 0xFF
        ang = np.degrees(np.arctan2(np.abs(h["vy"]), np.abs(h["vx"])))
        pic.close()
        assert d["hits_logged"] <= cap, "hit log wrapped"
        side = (cls == 6) | (cls == 7)
        deep = side & ((h["cell"] >> 16) >= w.extra["electrode_top"] + 5)
        pb, ps = PAPER_TRENCH_COUNTS[w.name]
        row = {"workload": w.name, "t_from": t_from, "t_to": w.steps * w.dt,
               "n_bottom": int(nb), "n_sidewalls": int(ns), "ratio": ns / max(nb, 1),
               "paper_n_bottom": pb, "paper_n_sidewalls": ps, "paper_ratio": round(ps / pb, 2),
               "n_sidewalls_below_mouth_5": int(deep.sum()),
               "ratio_below_mouth_5": int(deep.sum()) / max(int((cls == 4).sum()), 1),
               "hits_logged_in_window": int(h.size), "hits_total": int(d["hits_logged"]),
               "mean_angle_bottom_deg": float(ang[cls == 4].mean()) if np.any(cls == 4) else None,
               "mean_angle_sidewall_deg": float(ang[side].mean()) if np.any(side) else None,
               # impact angle from the surface normal in 10-degree bins (Fig. 5-7(b)): bottom hits
               # against |atan(v_y / v_x)|, sidewall hits against |atan(v_x / v_y)|
               "angle_hist_bottom_10deg": np.histogram(ang[cls == 4], bins=9, range=(0, 90))[0].tolist(),
               "angle_hist_sidewall_10deg": np.histogram(90.0 - ang[side], bins=9, range=(0, 90))[0].tolist(),
               "electrons_alive": d["alive"][0], "ions_alive": d["alive"][1],
               "phi_trench_mid_depth_mean": float(np.mean(phi_mid)),
               "secondary_emission": ({"yield_ion": see[0], "yield_electron": see[1], "vth": args.see_vth,
                                       "emitted": d["see_emitted"], "dropped": d["see_dropped"]} if see else None),
               "ms_per_step": 1e3 * secs / w.steps, "cumulative_t_bottom_side": curve}
        rows.append(row)
        log(f"{w.name:26s} bottom {nb:6d} sidewalls {ns:6d} ratio {row['ratio']:.2f} "
            f"(x >= {w.extra['electrode_top'] + 5}: {int(deep.sum())}, {row['ratio_below_mouth_5']:.2f}) "
            f"(paper {pb}/{ps} = {ps / pb:.2f}) {row['ms_per_step']:.3f} ms/step")
    print(json.dumps({"metric": "ions reaching the trench bottom and sidewalls (Sec. III.C-D)",
                      "n_gpus": 1, "data": "synthetic", "seed": args.study_seed, "results": rows}),
          flush=True)


def run_trench_study_batched(args):
    """The three trench runs of Sec. III.C-D advanced together as one batch:
    every launch covers the three instances and the steps replay as captured
    graphs with a fixed solver schedule (per-instance early exit).  Bottom and
    sidewall counts from the tallies over the same windows as the one-run-at-
    a-time study, and the time per step of the three together."""
    import torch

    import synth
    from paper_1610_03918_amd import PicBatch, autotune
    cases = ((15, False, 600), (4, False, 600), (15, True, 700))
    ws = [synth.paper_trench(wd, ch, seed=args.study_seed) for wd, ch, _ in cases]
    b = PicBatch(ws, [synth.load(w) for w in ws])
    b.start()
    warm = 200
    passes, iters, later = autotune.solver_schedule(b, warm)      # eager steps 0 .. warm-1
    tallies = {}
    step = warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    unconv0 = [b.pic_batch_solve_info(i)["unconverged_pushes"] for i in range(b.n)]
    for target in (6000, 7000, ws[0].steps):
        infos = b.pic_batch_step(target - step, passes, iters, later, allow_unconverged=True)
        step = target
        tallies[target] = [b.pic_batch_diagnostics(i)["tally"][1] for i in range(b.n)]
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / (step - warm)
    unconverged = sum(x["unconverged_pushes"] - u for x, u in zip(infos, unconv0))
    converged = unconverged == 0
    b.close()
    rows = []
    for i, (w, (_, _, t_from)) in enumerate(zip(ws, cases)):
        k_from = int(round(t_from / w.dt))
        a, z = tallies[k_from][i], tallies[w.steps][i]
        nb, ns = z[4] - a[4], (z[6] + z[7]) - (a[6] + a[7])
        pb, ps = PAPER_TRENCH_COUNTS[w.name]
        rows.append({"workload": w.name, "t_from": t_from, "n_bottom": int(nb), "n_sidewalls": int(ns),
                     "ratio": ns / max(nb, 1), "paper_ratio": round(ps / pb, 2)})
        log(f"{w.name:26s} bottom {nb:6d} sidewalls {ns:6d} ratio {ns / max(nb, 1):.2f} (paper {ps / pb:.2f})")
    log(f"batched: {ms:.3f} ms per step of the three instances")
    print(json.dumps({"metric": "ions reaching the trench bottom and sidewalls (Sec. III.C-D), batched",
                      "n_gpus": 1, "data": "synthetic", "seed": args.study_seed,
                      "ms_per_step_three_instances": ms, "all_converged": converged,
                      "unconverged_pushes": unconverged,
                      "solver_schedule": {"passes": passes, "iters_first": iters, "iters_later": later},
                      "results": rows}), flush=True)


def run_sweep(args):
    """The 16-width trench sweep advanced as one batch with captured graphs."""
    import torch

    import synth
    from paper_1610_03918_amd import PicBatch
    ws = synth.sweep()
    t = time.perf_counter()
    parts = [synth.load(w) for w in ws]
    n0 = sum(p["cell"].size for q in parts for p in q)
    log(f"loaded {len(ws)} instances, {n0} particles in {time.perf_counter() - t:.1f}s")
    from paper_1610_03918_amd import autotune
    entry = autotune.lookup(ws, parts)
    if entry is None and args.autotune:
        log("no cached schedule for this batch: running the autotuner")
        entry = autotune.tune(ws, parts, log=log)
    if entry is not None:
        sch = entry["schedule"]
        source = f"autotuned (cache key {autotune.signature(ws, parts)})"
    else:
        sch = dict(autotune.DEFAULT)
        sch.update(sort_interval=[int(x) for x in args.sort.split(",")], chunk=args.chunk,
                   push_unroll=args.unroll)
        source = "command line (no cached autotune result)"
    sort = tuple(sch["sort_interval"])
    b = PicBatch(ws, parts, sort_interval=sort, chunk=sch["chunk"], push_unroll=sch["push_unroll"],
                 push_merge=sch["push_merge"], tile=tuple(sch["tile"]), halo=sch["halo"])
    b.start()
    # eager steps tell how many passes and iterations the captured schedule needs
    # (after the spin-up steps, which bring the instances to their long-run state)
    passes, iters, iters_later = autotune.solver_schedule(b, args.spinup + args.warmup)
    infos = b.pic_batch_step(sort[0] if sort[0] > 0 else 8, passes, iters, iters_later, allow_unconverged=True)
    unconv0 = [x["unconverged_pushes"] for x in infos]
    torch.cuda.synchronize()
    a0 = sum(sum(b.pic_batch_diagnostics(i)["alive"]) for i in range(b.n))
    start_step = b.pic_batch_diagnostics(0)["step"]
    t0 = time.perf_counter()
    infos = b.pic_batch_step(args.steps, passes, iters, iters_later, allow_unconverged=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    a1 = sum(sum(b.pic_batch_diagnostics(i)["alive"]) for i in range(b.n))
    unconverged = sum(x["unconverged_pushes"] - u for x, u in zip(infos, unconv0))
    conv = unconverged == 0
    value = 0.5 * (a0 + a1) * args.steps / (t1 - t0)
    out = {"metric": "particle-steps/s (push+deposit+solve)", "value": value,
           "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * (t1 - t0) / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "trench-width sweep x16 (batched, graph-captured)",
                      "widths": list(synth.SWEEP_WIDTHS), "ppc": ws[0].species[0].ppc,
                      "particles": int(n0), "solver_schedule": {"passes": passes, "iters_first": iters, "iters_later": iters_later},
                      "all_converged": conv, "unconverged_pushes": unconverged,
                      "timed_from_step": start_step, "schedule": sch, "schedule_source": source}}
    b.close()
    print(json.dumps(out), flush=True)


def measured_copy_rate():
    """HBM bytes per second of a plain 1 GiB device-to-device copy (read +
    written), timed with events: what a streaming kernel reaches on this GPU,
    beside the published peak."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * 4 * n / (ms * 1e-3) / 1e9


def copy_calibration():
    """A plain device copy of known size (1 GiB read + 1 GiB written), the
    reference for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE to HBM bytes."""
    import torch
    n = 1 << 28                                     # 2^28 float32 = 1 GiB
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20, help="untimed steps before the timed ones")
    ap.add_argument("--spinup", type=int, default=400,
                    help="steps that bring the trench workload to its long-run state (the sheath forms, the "
                         "electrons heat and the push settles to its long-run rate) before the warm-up steps")
    ap.add_argument("--workload", default="trench1024x512")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--unet-only", action="store_true",
                    help="only time the learned start's network (1024 x 512)")
    ap.add_argument("--solvers", action="store_true",
                    help="only compare the solvers (MG-CG, CG, Jacobi, Gauss-Seidel) from a cold start")
    ap.add_argument("--trench-study", action="store_true",
                    help="the paper's trench runs: bottom and sidewall ion counts")
    ap.add_argument("--study-seed", type=int, default=5)
    ap.add_argument("--batched", action="store_true", help="with --trench-study: the three runs as one batch")
    ap.add_argument("--see", default="", help="with --trench-study: secondary emission yields per ion and per "
                    "electron impact on the trench surfaces, e.g. 0.2,0.2")
    ap.add_argument("--see-vth", type=float, default=0.4472,
                    help="thermal speed of the emitted electrons (sqrt(T_se / T_e); 0.4472: 2 eV at T_e = 10 eV)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--sort", default="8,64")
    ap.add_argument("--unroll", type=int, default=4)
    ap.add_argument("--merge", type=int, default=0)
    ap.add_argument("--tile", default="16,16")
    ap.add_argument("--chunk", type=int, default=4096)
    ap.add_argument("--halo", type=int, default=4)
    ap.add_argument("--warm", type=int, default=1, help="0 previous phi, 1 extrapolated")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-start measurement")
    ap.add_argument("--no-autotuned", action="store_true",
                    help="ignore a cached autotuned schedule for the workload")
    ap.add_argument("--autotune", action="store_true",
                    help="sweep: tune the schedule when the cache has no entry for the batch")
    ap.add_argument("--learn-bound-problems", type=int, default=5,
                    help="held-out problems of the exact-coarse-target bound")
    ap.add_argument("--learn-factor", type=int, default=1,
                    help="nodes per network pixel along each axis (1, 2, 4, 8 or 16)")
    ap.add_argument("--learn-trench-samples", type=int, default=4000,
                    help="training samples from the trench run")
    ap.add_argument("--learn-every", type=int, default=1, help="steps of the trench run per sample")
    ap.add_argument("--learn-sweep-steps", type=int, default=250,
                    help="eager steps of the 16-width sweep sampled (16 samples per step)")
    ap.add_argument("--learn-sweep-spinup", type=int, default=100)
    ap.add_argument("--learn-steps", type=int, default=4000, help="training steps")
    ap.add_argument("--learn-batch", type=int, default=4, help="batch, in trench-window images")
    ap.add_argument("--learn-rate", type=float, default=2e-3, help="Adam's initial learning rate")
    ap.add_argument("--learn-evals", type=int, default=20, help="held-out problems")
    ap.add_argument("--learn-fit", type=int, default=None,
                    help="degree of a least-squares polynomial through the --learn-stencil points "
                         "(default: the polynomial through all of them)")
    ap.add_argument("--learn-stencil", type=int, default=4,
                    help="points of the polynomial extrapolation in time the network corrects (2: linear)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "multi-GPU runs are not implemented: this benchmark measures one GPU",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.copy_calibration:
        return copy_calibration()
    if args.unet_only:
        return run_unet(args)
    if args.workload == "sweep":
        return run_sweep(args)
    if args.solvers:
        return run_solvers(args)
    if args.trench_study:
        return run_trench_study_batched(args) if args.batched else run_trench_study(args)

    import numpy as np
    import torch

    import synth
    from paper_1610_03918_amd import Pic

    w = workload(args.workload)
    t = time.perf_counter()
    parts = synth.load(w)
    n0 = [p["cell"].size for p in parts]
    log(f"loaded {n0} particles in {time.perf_counter() - t:.1f}s")
    from paper_1610_03918_amd import autotune
    entry = None if args.no_autotuned else autotune.lookup([w], [parts])
    if entry is not None:
        sch = entry["schedule"]
        args.sort = ",".join(str(x) for x in sch["sort_interval"])
        args.tile = ",".join(str(x) for x in sch["tile"])
        args.unroll, args.merge, args.chunk, args.halo = (sch["push_unroll"], sch["push_merge"],
                                                          sch["chunk"], sch["halo"])
        schedule_source = f"autotuned (cache key {autotune.signature([w], [parts])})"
    else:
        schedule_source = "command line"
    sort = tuple(int(x) for x in args.sort.split(","))
    tile = tuple(int(x) for x in args.tile.split(","))
    opts = dict(sort_interval=sort, push_unroll=args.unroll, push_merge=args.merge, tile=tile,
                chunk=args.chunk, halo=args.halo, warm_start=args.warm)
    pic = Pic(w, parts, device="cuda:0", **opts)
    info0 = pic.start()
    log(f"start solve: {info0}")
    spinup = args.spinup if w.name.startswith("trench") else 0
    t_spin = time.perf_counter()
    pic.pic_step(spinup)
    torch.cuda.synchronize()
    if spinup:
        log(f"spin-up: {spinup} steps in {time.perf_counter() - t_spin:.1f}s")
    pic.pic_step(args.warmup)
    torch.cuda.synchronize()
    d0 = pic.pic_diagnostics()
    start_step = int(d0["step"])
    # timed region: the library's own step loop (solve, field, push, deposit,
    # assembly, re-binning when due), no host work between steps
    pic.pic_set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pic.pic_step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    d1 = pic.pic_diagnostics()
    push_ms, _, launches = pic.pic_push_timing()
    pic.pic_set_timing(False)
    elapsed = t1 - t0
    # Poisson figures: further steps one call at a time, the solve timed on the host
    nps = min(args.steps, 50)
    solve_t = 0.0
    iters = 0
    r0 = []
    gk = 3 if args.warm == 1 else 1
    for _ in range(nps):
        a = time.perf_counter()
        info = pic.pic_solve(gk)
        solve_t += time.perf_counter() - a
        iters += info["iterations"]
        r0.append(info["relres0"])
        pic.pic_push()
        torch.cuda.synchronize()
    alive0, alive1 = sum(d0["alive"]), sum(d1["alive"])
    particle_steps = 0.5 * (alive0 + alive1) * args.steps
    value = particle_steps / elapsed
    per_launch = 0.5 * (alive0 + alive1)           # one push launch covers both species
    achieved = per_launch * BYTES_PER_PARTICLE_STEP / (push_ms * 1e-3) / 1e9
    traffic = measured_traffic(w.name, per_launch)
    copy_gbs = measured_copy_rate()
    out = {
        "metric": "particle-steps/s (push+deposit+solve); Poisson ms/step, plain vs learned start",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "cells": [w.nx, w.ny], "ppc": w.species[0].ppc,
                   "particles": n0, "dt": w.dt, "rtol": w.rtol, "sort_interval": list(sort),
                   "tile": list(tile), "chunk": args.chunk, "halo": args.halo,
                   "push_unroll": args.unroll, "push_merge": args.merge, "warm_start": args.warm,
                   "schedule_source": schedule_source, "spinup_steps": spinup,
                   "timed_from_step": start_step},
        "poisson_ms_per_step": 1e3 * solve_t / nps,
        "poisson_iters_per_step": iters / nps,
        "poisson_steps": nps,
        "poisson_start_relres_median": float(np.median(r0)),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0)",
                     "kernel": f"k_push<true,{args.unroll},{args.merge}>", "avg_launch_ms": push_ms, "launches": launches,
                     "steps_measured": [start_step, start_step + args.steps],
                     "bytes_per_launch": per_launch * BYTES_PER_PARTICLE_STEP,
                     "plain_copy_GBs": copy_gbs, "frac_of_plain_copy": achieved / copy_gbs},
    }
    if not args.no_learned and w.name.startswith("trench"):
        out["learned_start"] = learned_start(w, pic, parts, args)
    pic.close()
    del pic
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, parts)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
