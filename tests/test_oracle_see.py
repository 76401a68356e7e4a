"""Pins of the oracle's secondary electron emission at the trench surfaces
(Sec. IV; the paper gives no yield model, the reading is a constant yield
per impact).  Pinned by: the count of emitted electrons at yield 1 and 0
(exactly one per trench-surface impact, none elsewhere), their start on the
struck face of the struck cell and their direction away from the wall,
the Bernoulli fraction at an intermediate yield, the moments of the
flux-weighted half-Maxwellian (Rayleigh normal speed: mean v sqrt(pi/2),
second moment 2 v^2; Gaussian tangential velocity: mean 0, second moment
v^2), uniform positions along the face, and charge conservation over a run
(electrons alive = loaded - removed + emitted, the deposited electron
charge = alive x 2^32 exactly)."""
import numpy as np
import pytest

import oracle
import synth

BELOW1 = np.nextafter(np.float32(1), np.float32(0))


def _trench(ppc=1, seed=71, gi=1.0, ge=0.0):
    w = synth.trench(nx=48, ny=40, width=6, depth=12, ppc=ppc, seed=seed)
    w.see_yield = (ge, gi)
    w.see_vth = 0.3
    return w


def _hand_placed(w):
    top, jl, jh, nx = w.box_i_top, w.box_j_lo, w.box_j_hi, w.nx
    c = [(nx - 1, jl + 1, 0.8, 0.5, 5.0, 0.0),       # bottom (class 4)
         (nx - 1, jh - 2, 0.9, 0.3, 3.0, 0.0),       # bottom
         (top + 2, jl, 0.5, 0.1, 0.0, -2.0),         # -y sidewall (class 7)
         (top + 3, jh - 1, 0.5, 0.9, 0.0, 2.0),      # +y sidewall (class 6)
         (top - 3, 2, 0.5, 0.5, 35.0, 0.0),          # electrode top outside the trench (class 0)
         (0, 3, 0.05, 0.5, -1.0, 0.0),               # grounded plate (class 1)
         (5, 5, 0.5, 0.5, 0.1, 0.1)]                 # stays
    cell = np.array([(i << 16) | j for i, j, *_ in c], np.int32)
    f = lambda k: np.array([x[k] for x in c], np.float32)
    return {"cell": cell, "ox": f(2), "oy": f(3), "vx": f(4), "vy": f(5)}


def _push_with_hits(w, s, p, step=3):
    nc = oracle.node_cond(w)
    phi = np.zeros((w.NX, w.NY))
    phi[nc != 0] = oracle.voltages(w, 0.0)[nc[nc != 0]]
    Ex, Ey = oracle.field(w, nc, np.zeros((w.NX, w.NY)))
    hits = oracle.HitRecords(p["cell"].size)
    tally = np.zeros(9, np.int64)
    oracle.push(w, s, p, Ex, Ey, "f32", tally, None, step=step, hits=hits)
    return hits.rows(), tally


def test_one_electron_per_trench_impact_at_yield_one_none_at_zero():
    w = _trench(gi=1.0)
    p = _hand_placed(w)
    rows, tally = _push_with_hits(w, 1, p)
    assert tally[4] == 2 and tally[7] == 1 and tally[6] == 1 and tally[0] == 1 and tally[1] == 1
    assert rows.shape[0] == 6
    new = oracle.emit(w, [(1, rows)], 3)
    assert new["cell"].size == 4                              # classes 4, 4, 7, 6
    w0 = _trench(gi=0.0)
    assert oracle.emit(w0, [(1, rows)], 3)["cell"].size == 0
    # electrons hitting the same faces emit with the electron yield only
    assert oracle.emit(_trench(gi=0.0, ge=1.0), [(0, rows)], 3)["cell"].size == 4


def test_emitted_electrons_start_on_the_struck_face_moving_away():
    w = _trench(gi=1.0)
    p = _hand_placed(w)
    rows, _ = _push_with_hits(w, 1, p)
    new = oracle.emit(w, [(1, rows)], 3)
    trench = rows[np.isin(rows[:, 0], (4, 6, 7))]
    assert np.array_equal(np.sort(new["cell"]), np.sort(trench[:, 1]))
    for k in range(new["cell"].size):
        cls = trench[trench[:, 1] == new["cell"][k]][0, 0]
        ox, oy, vx, vy = (new[f][k] for f in ("ox", "oy", "vx", "vy"))
        assert 0.0 <= ox < 1.0 and 0.0 <= oy < 1.0
        if cls == 4:
            assert ox == BELOW1 and vx < 0
        elif cls == 6:
            assert oy == BELOW1 and vy < 0
        else:
            assert oy == 0.0 and vy > 0
        i, j = new["cell"][k] >> 16, new["cell"][k] & 0xFFFF
        assert w.cell_cond[i, j] == 0 and i >= w.box_i_top and w.box_j_lo <= j < w.box_j_hi


def test_emission_statistics():
    """200,000 synthetic bottom impacts at yield 0.3: the emitted fraction,
    the half-Maxwellian's moments and uniform positions along the face."""
    w = _trench(gi=0.3)
    rng = np.random.default_rng(5)
    n = 200_000
    rows = np.zeros((n, 4), np.int32)
    rows[:, 0] = 4
    rows[:, 1] = ((w.nx - 1) << 16) | (w.box_j_lo + 1)
    rows[:, 2] = rng.standard_normal(n).astype(np.float32).view(np.int32)
    rows[:, 3] = rng.standard_normal(n).astype(np.float32).view(np.int32)
    new = oracle.emit(w, [(1, rows)], 11)
    m = new["cell"].size
    assert abs(m / n - 0.3) < 4 * np.sqrt(0.3 * 0.7 / n)
    v = w.see_vth
    vn, vt = -new["vx"].astype(np.float64), new["vy"].astype(np.float64)
    assert np.all(vn > 0)
    se = lambda x: np.std(x) / np.sqrt(m)
    assert abs(vn.mean() - v * np.sqrt(np.pi / 2)) < 4 * se(vn)
    assert abs((vn ** 2).mean() - 2 * v * v) < 4 * se(vn ** 2)
    assert abs(vt.mean()) < 4 * se(vt)
    assert abs((vt ** 2).mean() - v * v) < 4 * se(vt ** 2)
    h, _ = np.histogram(new["oy"], bins=10, range=(0.0, 1.0))
    chi2 = np.sum((h - m / 10) ** 2 / (m / 10))
    assert chi2 < 30.0                                  # 9 degrees of freedom
    # another step draws other numbers
    assert not np.array_equal(oracle.emit(w, [(1, rows)], 12)["oy"][:100], new["oy"][:100])


def test_charge_conservation_over_a_run_with_emission():
    w = _trench(ppc=4, gi=1.0, ge=0.5)
    parts = synth.load(w)
    n0 = parts[0]["cell"].size
    sim = oracle.Sim(w, parts)
    sim.start()
    ion_trench = 0
    for _ in range(120):
        before = sim.tally[1][[4, 6, 7]].sum()
        sim.step()
        ion_trench += sim.tally[1][[4, 6, 7]].sum() - before
        alive_e = sim.alive(0)
        assert alive_e == n0 - sim.tally[0].sum() + sim.emitted
        rho = oracle.deposit(w, sim.p[0])
        assert int(rho.sum()) == alive_e << 32
    e_trench = sim.tally[0][[4, 6, 7]].sum()
    print("trench impacts: ions", ion_trench, "electrons", e_trench, "emitted", sim.emitted)
    assert ion_trench >= 1 and e_trench > 50
    # ions emit one electron each, electrons one with probability 1/2
    extra = sim.emitted - ion_trench
    assert 0 <= extra <= e_trench
    assert abs(extra - 0.5 * e_trench) < 4 * np.sqrt(0.25 * e_trench)
