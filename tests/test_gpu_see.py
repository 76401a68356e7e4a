"""GPU parity of the secondary electron emission at the trench surfaces
(Sec. IV; constant yield per impact of an electron or an ion on the trench
bottom or a sidewall).

Bars: on identical particle states and an identical potential, one push
with emission gives bit-identical tallies, the same number of emitted
electrons, and bit-identical cells and offsets for every electron, the
emitted ones included (their cell and offsets come from the removal record
and integer Philox words); the velocities of emitted electrons come from a
float64 transform whose log/cos may round differently on the two sides by
an ulp before the cast to float32, so they are held to 1e-6 relative of the
emission speed; every other velocity is bit-identical.  The new electrons'
charge joins the deposit exactly.  Over a run with re-binning: electrons
alive = loaded - removed + emitted, and the deposited electron charge is
alive x 2^32.  A batch mixing an emitting and a plain instance, advanced by
captured steps, equals each instance alone."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import canonical, live

pytestmark = pytest.mark.gpu


def _workload(seed=51, ge=0.5, gi=1.0):
    w = synth.workload_for_tests("trench")
    w.seed = seed
    w.see_yield = (ge, gi)
    w.see_vth = 0.3
    return w


def test_one_push_with_emission_matches_oracle():
    from paper_1610_03918_amd import Pic
    w = _workload()
    parts = synth.load(w)
    # fast ions, so that many reach the trench surfaces in this one push
    for f in ("vx", "vy"):
        parts[1][f] = (3.0 * parts[0][f]).astype(np.float32)
    n0 = parts[0]["cell"].size
    pic = Pic(w, parts, rtol=1e-12, sort_interval=(0, 0), capacity=(n0 + 20000, parts[1]["cell"].size))
    nc = oracle.node_cond(w)
    phi = synth.random_potential(w, 52, scale=4.0)
    phi[nc != 0] = oracle.voltages(w, 0.0)[nc[nc != 0]]
    pic.phi.copy_(pic.torch.from_numpy(phi))
    pic.pic_push()
    Ex, Ey = oracle.field(w, nc, phi)
    ref = [{k: v.copy() for k, v in parts[s].items()} for s in range(2)]
    tally = np.zeros((2, 9), np.int64)
    removals = []
    for s in range(2):
        hits = oracle.HitRecords(ref[s]["cell"].size)
        oracle.push(w, s, ref[s], Ex, Ey, "f32", tally[s], None, step=0, hits=hits)
        removals.append((s, hits.rows()))
    new = oracle.emit(w, removals, 0)
    d = pic.pic_diagnostics()
    assert np.array_equal(np.array(d["tally"]), tally)
    trench = tally[:, [4, 6, 7]].sum(axis=1)
    assert trench[0] > 20 and trench[1] > 20, trench
    assert d["see_emitted"] == new["cell"].size > 0 and d["see_dropped"] == 0
    # ions: the plain push, bit for bit
    assert np.array_equal(canonical(live(pic.particles_numpy(1))), canonical(live(ref[1])))
    # electrons: pushed ones and emitted ones together
    want = {k: np.concatenate([ref[0][k], new[k]]) for k in ref[0]}
    got = pic.particles_numpy(0)
    assert int((got["cell"] >= 0).sum()) == int((want["cell"] >= 0).sum()) == d["alive"][0]
    A, B = canonical(live(got)), canonical(live(want))
    assert np.array_equal(A[:, :3], B[:, :3]), "cells or offsets differ"
    va = A[:, 3:].view(np.float32).astype(np.float64)
    vb = B[:, 3:].view(np.float32).astype(np.float64)
    assert np.all(np.abs(va - vb) <= 1e-6 * np.maximum(np.abs(vb), w.see_vth))
    assert np.array_equal(pic.rho(0).cpu().numpy(), oracle.deposit(w, want))
    assert np.array_equal(pic.rho(1).cpu().numpy(), oracle.deposit(w, ref[1]))
    pic.close()


def test_run_with_emission_and_rebinning_conserves_charge():
    from paper_1610_03918_amd import Pic
    w = _workload(seed=53)
    parts = synth.load(w)
    n0 = parts[0]["cell"].size
    pic = Pic(w, parts, sort_interval=(4, 8), capacity=(2 * n0, parts[1]["cell"].size))
    pic.start()
    emitted = 0
    for k in range(12):
        pic.pic_step(5)
        d = pic.pic_diagnostics()
        lost = sum(d["tally"][0])
        assert d["alive"][0] == n0 - lost + d["see_emitted"]
        assert d["charge"][0] == d["alive"][0] << 32
        p = pic.particles_numpy(0)
        assert int((p["cell"] >= 0).sum()) == d["alive"][0]
        assert d["see_emitted"] >= emitted
        emitted = d["see_emitted"]
    assert emitted > 0 and d["see_dropped"] == 0
    pic.close()


def test_batched_steps_with_emission_equal_each_instance_alone():
    from paper_1610_03918_amd import PicBatch
    ws = [_workload(seed=54), synth.trench(nx=64, ny=32, width=4, depth=8, ppc=8, seed=55, rtol=1e-9)]
    parts = [synth.load(w) for w in ws]
    steps = 13

    def run(idx):
        caps = [(2 * parts[i][0]["cell"].size, parts[i][1]["cell"].size) for i in idx]
        b = PicBatch([ws[i] for i in idx], [parts[i] for i in idx], capacities=caps, sort_interval=(4, 8))
        b.start()
        b.pic_batch_step(steps, passes=3, iters=32)
        out = []
        for q in range(len(idx)):
            d = b.pic_batch_diagnostics(q)
            out.append({"parts": [canonical(live(b.particles_numpy(q, s))) for s in range(2)],
                        "rho": [b.rho(q, s).cpu().numpy() for s in range(2)],
                        "tally": d["tally"], "alive": d["alive"], "emitted": d["see_emitted"]})
        b.close()
        return out

    both = run([0, 1])
    for i in range(2):
        one = run([i])[0]
        for s in range(2):
            assert np.array_equal(both[i]["parts"][s], one["parts"][s])
            assert np.array_equal(both[i]["rho"][s], one["rho"][s])
        assert both[i]["tally"] == one["tally"] and both[i]["alive"] == one["alive"]
        assert both[i]["emitted"] == one["emitted"]
    assert both[0]["emitted"] > 0 and both[1]["emitted"] == 0
