"""GPU tests of the diagnostics (a9): kinetic energy of the live particles,
field energy of the node field, and the angular histogram of ions absorbed
by the trench bottom, against host computations from the same state."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def test_energies_and_bottom_angle_histogram():
    from paper_1610_03918_amd import Pic
    w = synth.trench(nx=64, ny=64, width=16, depth=16, ppc=32, seed=9, rtol=1e-10)
    pic = Pic(w, synth.load(w), hitlog_capacity=1 << 16, hitlog_species_mask=2)
    pic.start()
    pic.pic_step(600)
    d = pic.pic_diagnostics()
    # kinetic: 0.5 (m_s/m_e) w sum v^2 over live particles
    for s in range(2):
        p = pic.particles_numpy(s)
        live = p["cell"] >= 0
        v2 = (p["vx"][live].astype(np.float64) ** 2 + p["vy"][live].astype(np.float64) ** 2).sum()
        ref = 0.5 * w.weight * v2 / abs(w.species[s].alpha)
        assert abs(d["kinetic"][s] - ref) <= 1e-12 * ref, (s, d["kinetic"][s], ref)
    # field energy: 0.5 sum |E|^2 of the oracle's node field of the same phi
    nc = oracle.node_cond(w)
    Ex, Ey = oracle.field(w, nc, pic.phi.cpu().numpy())
    ref = 0.5 * float((Ex.astype(np.float64) ** 2 + Ey.astype(np.float64) ** 2).sum())
    assert abs(d["field_energy"] - ref) <= 1e-6 * ref, (d["field_energy"], ref)
    # angle histogram against the hit records of the same absorptions
    rec = pic.pic_read_hits()
    sel = (rec["species_class"] >> 8 == 1) & (rec["species_class"] & 0xFF == 4)
    ang = np.arctan2(rec["vy"][sel], rec["vx"][sel])
    h = np.floor((ang + np.float32(np.pi / 2)) * np.float32(90 / np.pi)).astype(int).clip(0, 89)
    ref = np.bincount(h, minlength=90)
    got = np.array(d["iad"])
    assert got.sum() == sel.sum() == d["tally"][1][4] > 100
    assert np.abs(got - ref).sum() <= 4             # float32 atan2 differences at bin edges
    prof_across, prof_down = pic.trench_profiles()
    assert prof_across.shape == (w.box_j_hi - w.box_j_lo + 9,)
    assert prof_down.shape == (w.NX - (w.box_i_top - 16),)
    pic.close()
