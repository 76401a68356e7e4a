"""GPU tests of the schedule knobs the autotuner turns: particle tile, block
chunk, push variant and re-binning intervals change only the time per step.
Runs with different layouts, and a run whose schedule is switched midway
with pic_tune, end bit-identical (integer charge, potential, particles,
counters) to the default run."""
import numpy as np
import pytest

import synth
from gpu_util import canonical, live

pytestmark = pytest.mark.gpu


def _batch():
    return [synth.trench(nx=64, ny=32, width=4, depth=8, ppc=8, seed=31, rtol=1e-9),
            synth.trench(nx=128, ny=64, width=12, depth=16, ppc=6, seed=32, rtol=1e-9)]


def _state(b, i):
    return ([b.rho(i, s).cpu().numpy() for s in range(2)], b.phi(i).cpu().numpy(),
            [canonical(live(b.particles_numpy(i, s))) for s in range(2)], b.pic_batch_diagnostics(i))


def _same(x, y):
    for s in range(2):
        assert np.array_equal(x[0][s], y[0][s])
        assert np.array_equal(x[2][s], y[2][s])
    assert np.array_equal(x[1], y[1])
    assert x[3]["tally"] == y[3]["tally"] and x[3]["alive"] == y[3]["alive"]
    assert x[3]["surf_hits"] == y[3]["surf_hits"]


def _run(ws, parts, steps, switch=None, **opts):
    from paper_1610_03918_amd import PicBatch
    b = PicBatch(ws, parts, **opts)
    b.start()
    if switch:
        b.pic_batch_step(steps // 2, passes=3, iters=32)
        b.pic_tune(*switch)
        b.pic_batch_step(steps - steps // 2, passes=3, iters=32)
    else:
        b.pic_batch_step(steps, passes=3, iters=32)
    out = [_state(b, i) for i in range(len(ws))]
    b.close()
    return out


def test_schedules_do_not_change_results():
    ws = _batch()
    parts = [synth.load(w) for w in ws]
    ref = _run(ws, parts, 12, sort_interval=(4, 8))
    variants = [
        dict(tile=(32, 16), chunk=8192, push_unroll=4, push_merge=2, sort_interval=(4, 8)),
        dict(tile=(16, 32), chunk=2048, push_unroll=1, push_merge=0, sort_interval=(4, 8)),
        dict(sort_interval=(4, 8), switch=(4, 2, (2, 4))),
    ]
    for v in variants:
        got = _run(ws, parts, 12, **v)
        for i in range(len(ws)):
            _same(ref[i], got[i])
