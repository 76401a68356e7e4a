"""Long-run statistical parity of the GPU path with the oracle (Sec. III.C-D:
the angular distribution of the ions reaching the trench bottom, the split of
ion hits between bottom and sidewalls, and the potential inside the trench).

Workloads: the 256 x 128 trench instances of the width sweep at widths 4 and
16 (64 particles per cell, RF bias 50 sin(0.05 t), bottom charge build-up),
four seeded loads per width on each side.  The GPU runs other seeds than the
oracle (tests/golden/longrun_trench256x128.json, written by
tests/golden/make_longrun.py from the oracle alone), so the two ensembles are
independent and the comparison is statistical, not a replay of one
trajectory.  After a burn-in of 500 steps both sides record over two whole
RF periods (2513 steps): every ion absorbed by the trench bottom with its
impact angle theta = atan2(|v_y|, v_x) from the plate normal, the sidewall
hits, and the potential averaged over the window along the trench's
mid-depth node row and centre node column.

Bars, pooled over the four runs of a width: the mean and RMS of theta and
the ratio of sidewall to bottom hits within 2 % of the oracle's value, or
within three standard errors of the difference where shot noise exceeds
that (the standard errors come from the samples: theta's spread, Poisson
counts); the 10-degree histogram of theta within 0.02 per bin (or three
standard errors); the window-averaged potential at free nodes within 2 % of
the oracle profile's scale (its range or mean magnitude, whichever is
larger), or three standard errors of the difference (from the spread of the
four runs' profiles on each side)."""
import json
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "longrun_trench256x128.json")
GPU_SEED_OFFSET = 100


def _rows(w):
    return (w.box_i_top + w.nx) // 2, (w.box_j_lo + w.box_j_hi) // 2


def _gpu_run(width, seed, burn, window, bottom, sides, nbins):
    import torch
    from paper_1610_03918_amd import Pic
    w = synth.sweep_instance(width, seed=seed)
    pic = Pic(w, synth.load(w), hitlog_capacity=1 << 21, hitlog_species_mask=2)
    pic.start()
    pic.pic_step(burn)
    d0 = pic.pic_diagnostics()
    acc = torch.zeros_like(pic.phi)
    for _ in range(window):
        pic.pic_step(1)
        acc += pic.phi
    d1 = pic.pic_diagnostics()
    rec = pic.pic_read_hits()
    assert d1["hits_logged"] == rec.size < (1 << 21)
    rec = rec[d0["hits_logged"]:]
    sel = (rec["species_class"] >> 8 == 1) & (rec["species_class"] & 0xFF == bottom)
    th = np.arctan2(np.abs(rec["vy"][sel].astype(np.float64)), rec["vx"][sel].astype(np.float64))
    tally = np.array(d1["tally"][1]) - np.array(d0["tally"][1])
    assert tally[bottom] == th.size
    phi = (acc / window).cpu().numpy().reshape(w.NX, w.NY)
    pic.close()
    im, jc = _rows(w)
    return {"bottom": int(th.size), "theta_sum": float(th.sum()), "theta_sq_sum": float((th * th).sum()),
            "theta_4_sum": float((th ** 4).sum()),
            "theta_hist_10deg": np.histogram(np.degrees(th), bins=nbins, range=(0.0, 90.0))[0].tolist(),
            "tally_ions_window": tally.tolist(),
            "across_mid_depth": phi[im, w.box_j_lo:w.box_j_hi + 1].tolist(),
            "down_centre": phi[w.box_i_top - 16:, jc].tolist()}


def _pooled(runs, sides):
    n = sum(r["bottom"] for r in runs)
    m1 = sum(r["theta_sum"] for r in runs) / n
    m2 = sum(r["theta_sq_sum"] for r in runs) / n
    m4 = sum(r["theta_4_sum"] for r in runs) / n
    ns = sum(r["tally_ions_window"][c] for r in runs for c in sides)
    h = np.sum([r["theta_hist_10deg"] for r in runs], axis=0) / n
    rms = np.sqrt(m2)
    return {"n": n, "mean": m1, "se_mean": np.sqrt(max(m2 - m1 * m1, 0.0) / n),
            "rms": rms, "se_rms": np.sqrt(max(m4 - m2 * m2, 0.0) / n) / (2 * rms),
            "ratio": ns / n, "se_ratio": ns / n * np.sqrt(1.0 / max(ns, 1) + 1.0 / n), "hist": h,
            "across": np.mean([r["across_mid_depth"] for r in runs], axis=0),
            "se_across": np.std([r["across_mid_depth"] for r in runs], axis=0, ddof=1) / np.sqrt(len(runs)),
            "down": np.mean([r["down_centre"] for r in runs], axis=0),
            "se_down": np.std([r["down_centre"] for r in runs], axis=0, ddof=1) / np.sqrt(len(runs))}


@pytest.mark.parametrize("width", [4, 16])
def test_long_run_statistics_match_oracle_ensemble(width):
    gold = json.load(open(GOLD))
    burn, window = gold["burn_steps"], gold["window_steps"]
    bottom, sides = gold["bottom_class"], gold["side_classes"]
    nbins = len(gold["hist_bins_deg"]) - 1
    orc = [r for r in gold["runs"] if r["width"] == width]
    assert len(orc) >= 4
    gpu = [_gpu_run(width, r["seed"] + GPU_SEED_OFFSET, burn, window, bottom, sides, nbins) for r in orc]
    g, o = _pooled(gpu, sides), _pooled(orc, sides)
    print(f"width {width}: bottom hits gpu {g['n']} oracle {o['n']}")
    for k in ("mean", "rms", "ratio"):
        se = np.hypot(g["se_" + k], o["se_" + k])
        tol = max(0.02 * abs(o[k]), 3 * se)
        print(f"  {k}: gpu {g[k]:.5f} oracle {o[k]:.5f} diff {g[k] - o[k]:+.5f} "
              f"(2 % = {0.02 * abs(o[k]):.5f}, 3 se = {3 * se:.5f})")
        assert abs(g[k] - o[k]) <= tol, k
    se_h = np.sqrt(o["hist"] * (1 - o["hist"]) * (1.0 / g["n"] + 1.0 / o["n"]))
    print("  hist gpu", np.round(g["hist"], 4), "\n  hist orc", np.round(o["hist"], 4))
    assert np.all(np.abs(g["hist"] - o["hist"]) <= np.maximum(0.02, 3 * se_h))
    w = synth.sweep_instance(width)
    nc = oracle.node_cond(w)
    im, jc = _rows(w)
    free_a = nc[im, w.box_j_lo:w.box_j_hi + 1] == 0
    free_d = nc[w.box_i_top - 16:, jc] == 0
    for name, free in (("across", free_a), ("down", free_d)):
        ref, got = o[name][free], g[name][free]
        scale = max(np.ptp(ref), np.mean(np.abs(ref)))
        se = np.hypot(o["se_" + name][free], g["se_" + name][free])
        print(f"  {name}: max diff {np.max(np.abs(got - ref)):.4f}, 2 % of scale {0.02 * scale:.4f}, "
              f"largest 3 se {np.max(3 * se):.4f}")
        assert np.all(np.abs(got - ref) <= np.maximum(0.02 * scale, 3 * se)), name
    # the wide trench gathers >= 10^4 bottom hits per side (three standard
    # errors of the mean angle's difference about 3 %); the narrow one about
    # 800 (its ions mostly reach the sidewalls: three standard errors about
    # 10 %)
    least = {4: 500, 16: 10000}[width]
    assert o["n"] >= least and g["n"] >= least
