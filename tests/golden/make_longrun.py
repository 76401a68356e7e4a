"""Writes longrun_trench256x128.json: the oracle's side of the long-run
statistical parity test (tests/test_gpu_longrun_stats.py).  Calls only the
oracle and the seeded input generator.

Workloads: the 256 x 128 trench instances of the width sweep (64 particles
per cell, RF bias 50 sin(0.05 t), trench bottom charge build-up) at widths 4
and 16, several seeds each.  Each run takes BURN steps to let the sheath
form, then records over WINDOW steps (two whole RF periods, 2 x 1256.6
steps at dt = 0.1) the ions absorbed by the trench bottom (count, sums of
their impact angle theta = atan2(|v_y|, v_x), of theta^2 and theta^4, a
histogram),
the sidewall hits, and the potential averaged over the window along the
trench's mid-depth node row and its centre node column.

  python tests/golden/make_longrun.py [--procs 8]
"""
import argparse
import json
import os
import sys
import time
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

BURN, WINDOW = 500, 2513
WIDTHS = (4, 16)
SEEDS = (4, 5, 6, 7)
BOTTOM, SIDE_M, SIDE_P = 4, 7, 6      # hit classes: +x, -y, +y inside the trench box
HIST_BINS = 9                         # theta over [0, 90) degrees in 10-degree bins


def rows(w):
    """Node rows/columns of the profiles: mid-depth row across the trench
    (columns j_lo .. j_hi), centre column from 16 rows above the mouth to
    the bottom."""
    im = (w.box_i_top + w.nx) // 2
    jc = (w.box_j_lo + w.box_j_hi) // 2
    return im, jc


def run(args):
    import numpy as np

    import oracle
    import synth
    width, seed = args
    w = synth.sweep_instance(width, seed=seed)
    parts = synth.load(w)
    sim = oracle.Sim(w, parts)
    sim.start()
    im, jc = rows(w)
    across = np.zeros(w.box_j_hi - w.box_j_lo + 1)
    down = np.zeros(w.NX - (w.box_i_top - 16))
    n = 0
    s1 = s2 = s4 = 0.0
    hist = np.zeros(HIST_BINS, np.int64)
    t0 = time.time()
    tally0 = None
    for k in range(BURN + WINDOW):
        if k == BURN:
            tally0 = sim.tally[1].copy()
        prev = sim.p[1]["cell"].copy()
        sim.step()
        if k < BURN:
            continue
        cur = sim.p[1]["cell"]
        h = (prev >= 0) & (cur == -1 - BOTTOM)
        if h.any():
            th = np.arctan2(np.abs(sim.p[1]["vy"][h].astype(np.float64)), sim.p[1]["vx"][h].astype(np.float64))
            n += int(th.size)
            s1 += float(th.sum())
            s2 += float((th * th).sum())
            s4 += float((th ** 4).sum())
            hist += np.histogram(np.degrees(th), bins=HIST_BINS, range=(0.0, 90.0))[0]
        phi = sim.phi.reshape(w.NX, w.NY)
        across += phi[im, w.box_j_lo:w.box_j_hi + 1]
        down += phi[w.box_i_top - 16:, jc]
    return {"width": width, "seed": seed, "nx": w.nx, "ny": w.ny, "particles": [int(p["cell"].size) for p in parts],
            "bottom": n, "theta_sum": s1, "theta_sq_sum": s2, "theta_4_sum": s4, "theta_hist_10deg": hist.tolist(),
            "tally_ions_window": (sim.tally[1] - tally0).tolist(),
            "across_mid_depth": (across / WINDOW).tolist(), "down_centre": (down / WINDOW).tolist(),
            "seconds": time.time() - t0}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=8)
    ap.add_argument("--out", default=os.path.join(HERE, "longrun_trench256x128.json"))
    a = ap.parse_args()
    jobs = [(wd, s) for wd in WIDTHS for s in SEEDS]
    with Pool(min(a.procs, len(jobs))) as pool:
        res = pool.map(run, jobs)
    out = {"what": "oracle side of the long-run statistical parity test", "burn_steps": BURN,
           "window_steps": WINDOW, "bottom_class": BOTTOM, "side_classes": [SIDE_P, SIDE_M],
           "hist_bins_deg": [10 * k for k in range(HIST_BINS + 1)], "runs": res}
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
    for r in res:
        print(r["width"], r["seed"], r["bottom"], r["tally_ions_window"], round(r["seconds"]))


if __name__ == "__main__":
    main()
