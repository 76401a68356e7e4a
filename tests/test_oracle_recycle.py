"""Pins of the oracle's ion recycling (Sec. III.A, III.C: a lost ion is
replaced by a thermal ion in the bulk plasma) and of its generator.

* Philox4x32-10 reproduces the published known-answer vectors of the
  generator (Salmon, Moraes, Dror, Shaw, SC 2011; the kat_vectors of their
  Random123 distribution): zero counter and key, all-ones counter and key,
  and the pi-digit counter and key.
* A recycled ion lies in the bulk rows with offsets in [0, 1); over many
  draws its cells are uniform over the bulk and its velocity components
  have mean 0 and standard deviation vth (Box-Muller).
* In a run the number of ions stays constant, every removal is tallied, and
  the state after a step does not depend on the order the ions are stored
  in (the draw is keyed by the lost ion's own state)."""
import numpy as np

import oracle
import synth


def test_philox_known_answers():
    kat = [
        ([0, 0, 0, 0], [0, 0], [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]),
        ([0xffffffff] * 4, [0xffffffff] * 2, [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]),
        ([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344], [0xa4093822, 0x299f31d0],
         [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]),
    ]
    for ctr, key, out in kat:
        assert list(oracle.philox4x32_10(ctr, key)) == out


def _workload():
    w = synth.trench(nx=48, ny=24, width=6, depth=12, ppc=8, seed=23, amp=5.0, omega=0.01)
    w.recycle_rows = 36
    return w


def test_recycled_ion_distribution():
    w = _workload()
    rng = np.random.default_rng(3)
    n = 20000
    ux = rng.standard_normal(n).astype(np.float32)
    ox = rng.random(n, np.float32)
    rows = np.zeros(n, np.int64)
    v = np.zeros((n, 2))
    for k in range(n):
        c, x, y, vx, vy = oracle.recycled_ion(w, 7, float(ux[k]), float(ox[k]), 0.5)
        i, j = c >> 16, c & 0xFFFF
        assert 0 <= i < w.recycle_rows and 0 <= j < w.ny and 0.0 <= x < 1.0 and 0.0 <= y < 1.0
        rows[k] = i
        v[k] = (vx, vy)
    vth = w.species[1].vth
    assert np.all(np.abs(v.mean(axis=0)) < 4 * vth / np.sqrt(n))
    assert np.all(np.abs(v.std(axis=0) / vth - 1.0) < 0.03)
    counts = np.bincount(rows, minlength=w.recycle_rows)
    expect = n / w.recycle_rows
    chi2 = float(np.sum((counts - expect) ** 2 / expect))
    assert chi2 < w.recycle_rows + 5 * np.sqrt(2 * w.recycle_rows)


def test_run_keeps_ion_count_and_is_order_free():
    w = _workload()
    parts = synth.load(w)
    sim = oracle.Sim(w, parts)
    sim.start()
    n_ions = sim.alive(1)
    for _ in range(60):
        sim.step()
    assert sim.alive(1) == n_ions
    assert sim.tally[1].sum() > 0
    # the same state pushed once more, ions stored in another order
    perm = np.random.default_rng(4).permutation(sim.p[1]["cell"].size)
    other = oracle.Sim(w, [sim.p[0], {k: v[perm] for k, v in sim.p[1].items()}])
    other.step_index = sim.step_index
    other.surf[:] = sim.surf
    sim.step()
    other.step()
    key = lambda p: np.lexsort((p["vy"], p["vx"], p["oy"], p["ox"], p["cell"]))
    a, b = sim.p[1], other.p[1]
    ka, kb = key(a), key(b)
    for f in ("cell", "ox", "oy", "vx", "vy"):
        assert np.array_equal(a[f][ka], b[f][kb])
