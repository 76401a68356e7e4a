"""Pins of the oracle's full cycle and of the synthetic loader (CPU only).

The cold-plasma oscillation checks the whole loop at once: the sign of the
Poisson source, the electron charge/mass factor alpha_e = -1, the particle
weight normalisation (n_0 = 1) and the leapfrog timing.  With immobile ions
a small sinusoidal electron displacement oscillates at omega_e = 1, which the
leapfrog with dt = 0.1 turns into the period 2 pi / ((2/dt) asin(dt/2)).
"""
import math

import numpy as np
import pytest

import oracle
import synth


def _quiet_plasma(nx, ny, sub, amp, k_mode):
    """sub x sub particles per cell at regular offsets; electrons displaced
    along x by amp*sin(k x0); ions undisplaced (and immobile)."""
    offs = (np.arange(sub) + 0.5) / sub
    I, J, A, B = np.meshgrid(np.arange(nx), np.arange(ny), offs, offs, indexing="ij")
    x0 = (I + A).ravel()
    y0 = (J + B).ravel()
    k = 2 * math.pi * k_mode / nx
    out = []
    for disp in (amp * np.sin(k * x0), np.zeros_like(x0)):
        x = (x0 + disp) % nx
        ci = np.floor(x).astype(np.int64)
        cj = np.floor(y0).astype(np.int64)
        out.append({"cell": ((ci << 16) | cj).astype(np.int32),
                    "ox": (x - ci), "oy": (y0 - cj),
                    "vx": np.zeros_like(x), "vy": np.zeros_like(x)})
    return out, x0, k


def test_cold_plasma_oscillation_period():
    nx, ny, sub = 64, 4, 4
    w = synth.periodic_square(n=nx, ppc=sub * sub)
    w.ny = ny
    w.cell_cond = np.zeros((nx, ny), np.uint8)
    w.species[1].alpha = 0.0
    parts, x0, k = _quiet_plasma(nx, ny, sub, 0.02, 1)
    sim = oracle.Sim(w, parts, precision="f64")
    sim.start()
    X = []
    for n in range(260):
        p = sim.p[0]
        x = (p["cell"].astype(np.int64) >> 16) + p["ox"]
        d = (x - x0 + nx / 2) % nx - nx / 2
        X.append(np.dot(d, np.sin(k * x0)) / np.dot(np.sin(k * x0), np.sin(k * x0)))
        sim.step()
    X = np.array(X)
    assert abs(X[0] - 0.02) < 1e-6
    t = np.arange(X.size) * w.dt
    zc = []
    for n in range(X.size - 1):
        if X[n] == 0 or X[n] * X[n + 1] < 0:
            zc.append(t[n] + w.dt * X[n] / (X[n] - X[n + 1]))
    assert len(zc) >= 5
    period = (zc[4] - zc[0]) / 2
    expect = 2 * math.pi / ((2 / w.dt) * math.asin(w.dt / 2))
    assert abs(period / expect - 1) < 5e-3, (period, expect)
    # the wrong sign of the source or of alpha_e gives growth, not oscillation
    assert np.max(np.abs(X)) < 0.0201


def test_loader_places_ppc_particles_in_every_plasma_cell():
    w = synth.workload_for_tests("trench")
    for s in range(2):
        p = synth.load_species(w, s)
        i = p["cell"] >> 16
        j = p["cell"] & 0xFFFF
        assert np.all(w.cell_cond[i, j] == 0)
        counts = np.zeros((w.nx, w.ny), np.int64)
        np.add.at(counts, (i, j), 1)
        assert np.all(counts[w.cell_cond == 0] == w.species[s].ppc)
        assert p["ox"].dtype == np.float32 and p["ox"].min() >= 0 and p["ox"].max() < 1
        sig = w.species[s].vth
        assert abs(p["vx"].std() / sig - 1) < 0.05


def test_loader_is_seeded():
    w = synth.workload_for_tests("bounded")
    a = synth.load_species(w, 0)
    b = synth.load_species(w, 0)
    c = synth.load_species(w, 1)
    assert all(np.array_equal(a[k], b[k]) for k in a)
    assert not np.array_equal(a["ox"], c["ox"])


def test_trench_preset_sizes():
    w = synth.trench()
    assert (w.NX, w.NY) == (1025, 512)
    assert w.plasma_cells() == 459776
    assert w.n_particles(0) == 91955200
    nc = oracle.node_cond(w)
    assert int((nc == 0).sum()) == 459136
    assert w.species[1].vth == pytest.approx(0.00522, abs=1e-5)


def test_sweep_sizes():
    ws = synth.sweep()
    shapes = sorted({(w.nx, w.ny) for w in ws})
    assert shapes == [(256, 128), (512, 256), (1024, 512)]
    assert sum(1 for w in ws if w.ny == 128) == 11
    assert all(w.box_j_hi - w.box_j_lo == w.extra["width"] for w in ws)


def test_short_run_conserves_particles_and_counts_hits():
    """Bounded square: every particle is either alive or counted in exactly
    one wall class; the accumulated charge equals the alive count."""
    w = synth.workload_for_tests("bounded")
    sim = oracle.Sim(w, synth.load(w))
    n0 = [q["cell"].size for q in sim.p]
    sim.start()
    for _ in range(8):
        sim.step()
    for s in range(2):
        assert sim.alive(s) + int(sim.tally[s].sum()) == n0[s]
        rho = oracle.deposit(w, sim.p[s])
        assert int(rho.sum()) == sim.alive(s) * (1 << 32)
    assert sim.tally[0].sum() > 0
