"""Schedule autotuner of the batched form.

The particle kernels have free choices that change only the time per step,
never a result (the deposit is integer and order-free, particles are
independent): the tile of cells a block owns (its LDS charge window), the
particles per block (chunk), the push variant (particles per thread per pass,
wavefront-level merging of equal cells before the LDS atomics) and the
re-binning intervals of electrons and ions.  The tuner times candidates on
the GPU with the captured batched step and keeps the fastest:

  1. layout (tile, chunk): each candidate needs its own context;
  2. push variant (unroll, merge) on the best layout, via pic_tune;
  3. re-binning intervals, via pic_tune.

Results are cached in ``tuning/schedules.json`` under a key derived from the
instances' grids, geometry and particle counts.

  python -m paper_1610_03918_amd.autotune [--sweep] [--out PATH]
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning", "schedules.json")

DEFAULT = {"tile": [16, 16], "chunk": 4096, "halo": 4, "push_unroll": 4, "push_merge": 0,
           "sort_interval": [8, 64]}
# (tile, chunk, halo): the halo bounds how far particles may drift between re-binnings before their
# charge goes to global memory directly, so it trades against the re-binning interval
LAYOUTS = [((16, 16), 4096, 4), ((16, 16), 8192, 4), ((16, 16), 8192, 6), ((32, 16), 4096, 4),
           ((16, 32), 4096, 4), ((32, 32), 8192, 4)]
VARIANTS = [(1, 0), (2, 0), (4, 0), (2, 2), (4, 2)]
SORTS = [(4, 32), (8, 64), (12, 128), (16, 64), (16, 128), (24, 128), (32, 128)]


def signature(workloads, parts):
    """Key of a batch: grids, geometry, species and particle counts."""
    desc = []
    for w, p in zip(workloads, parts):
        desc.append([w.nx, w.ny, int(w.periodic_x), int(w.periodic_y), w.box_i_top, w.box_j_lo,
                     w.box_j_hi, [int(q["cell"].size) for q in p], [s.alpha for s in w.species]])
    return hashlib.sha1(json.dumps(desc, sort_keys=True).encode()).hexdigest()[:16]


def load_cache(path=CACHE):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def lookup(workloads, parts, path=CACHE):
    """The cached schedule of this batch, or None."""
    return load_cache(path).get(signature(workloads, parts))


def _measure(b, period, steps, passes, iters, iters_later=0, repeats=2):
    """Best of `repeats` timings of `steps` captured steps (ms/step)."""
    import torch
    infos = b.pic_batch_step(period or 8, passes, iters, iters_later, allow_unconverged=True)  # capture + warm
    before = [x["unconverged_pushes"] for x in infos]
    best = None
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = b.pic_batch_step(steps, passes, iters, iters_later, allow_unconverged=True)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        best = ms if best is None else min(best, ms)
    # every timed step of every instance pushed a converged potential
    ok = all(x["unconverged_pushes"] == n for x, n in zip(infos, before))
    return best, ok


def solver_schedule(b, warm, window=100):
    """Fixed solver schedule for captured steps, (passes, first-pass
    iterations, later-pass iterations), from `warm` eager steps: the most
    any instance needed over the last `window` of them, with margins."""
    first = later = 0
    passes = 1
    n = max(2, warm)
    for k in range(n):
        b.pic_step(1)
        if k < n - window:
            continue
        for i in range(b.n):
            info = b.pic_batch_solve_info(i)
            first = max(first, info["iterations_first"])
            later = max(later, info["iterations"] - info["iterations_first"])
            passes = max(passes, info["outer"])
    # a second, short pass always: a step that the window did not show may
    # need it, and an instance that converged skips it
    return max(passes, 2), min(128, first + 2), min(128, max(2, later + 1))


def _solver_schedule(b, warm):
    return solver_schedule(b, warm)


def tune(workloads, parts, steps=32, log=None, path=CACHE):
    """Times the candidates, stores and returns the best schedule."""
    from .pic import PicBatch
    say = log or (lambda *a: None)
    trials = []
    best = None
    schedule = None
    for tile, chunk, halo in LAYOUTS:
        opts = dict(DEFAULT)
        opts.update(tile=list(tile), chunk=chunk, halo=halo)
        b = PicBatch(workloads, parts, tile=tuple(tile), chunk=chunk, halo=opts["halo"],
                     push_unroll=opts["push_unroll"], push_merge=opts["push_merge"],
                     sort_interval=tuple(opts["sort_interval"]))
        b.start()
        if schedule is None:
            schedule = _solver_schedule(b, 3)
        ms, ok = _measure(b, opts["sort_interval"][0], steps, *schedule)
        b.close()
        trials.append({"stage": "layout", "tile": list(tile), "chunk": chunk, "halo": halo, "ms": ms,
                       "converged": ok})
        say(f"layout tile {tile} chunk {chunk} halo {halo}: {ms:.3f} ms/step")
        if ok and (best is None or ms < best[0]):
            best = (ms, opts)
    opts = dict(best[1])
    b = PicBatch(workloads, parts, tile=tuple(opts["tile"]), chunk=opts["chunk"], halo=opts["halo"],
                 push_unroll=opts["push_unroll"], push_merge=opts["push_merge"],
                 sort_interval=tuple(opts["sort_interval"]))
    b.start()
    _solver_schedule(b, 2)
    cur = None
    for unroll, merge in VARIANTS:
        b.pic_tune(unroll, merge, opts["sort_interval"])
        ms, ok = _measure(b, opts["sort_interval"][0], steps, *schedule)
        trials.append({"stage": "push", "push_unroll": unroll, "push_merge": merge, "ms": ms, "converged": ok})
        say(f"push unroll {unroll} merge {merge}: {ms:.3f} ms/step")
        if ok and (cur is None or ms < cur[0]):
            cur = (ms, unroll, merge)
    opts["push_unroll"], opts["push_merge"] = cur[1], cur[2]
    cur = None
    for sort in SORTS:
        b.pic_tune(opts["push_unroll"], opts["push_merge"], sort)
        n = max(steps, 2 * sort[0])
        ms, ok = _measure(b, sort[0], n, *schedule)
        trials.append({"stage": "sort", "sort_interval": list(sort), "ms": ms, "converged": ok})
        say(f"sort {sort}: {ms:.3f} ms/step")
        if ok and (cur is None or ms < cur[0]):
            cur = (ms, sort)
    opts["sort_interval"] = list(cur[1])
    b.close()
    entry = {"schedule": opts, "ms_per_step": cur[0], "solver_schedule": list(schedule),
             "instances": len(workloads), "trials": trials}
    cache = load_cache(path)
    cache[signature(workloads, parts)] = entry
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path + ".tmp", "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(path + ".tmp", path)
    return entry


def main():
    import argparse
    sys.path.insert(0, os.path.dirname(HERE))
    import synth
    ap = argparse.ArgumentParser()
    ap.add_argument("--sweep", action="store_true", help="the 16-width trench sweep (default)")
    ap.add_argument("--trench", action="store_true", help="the single 1024 x 512 trench instead")
    ap.add_argument("--steps", type=int, default=32)
    ap.add_argument("--out", default=CACHE)
    args = ap.parse_args()
    ws = [synth.trench()] if args.trench else synth.sweep()
    parts = [synth.load(w) for w in ws]
    entry = tune(ws, parts, steps=args.steps, log=lambda m: print(m, flush=True), path=args.out)
    print(json.dumps({k: v for k, v in entry.items() if k != "trials"}), flush=True)


if __name__ == "__main__":
    main()
