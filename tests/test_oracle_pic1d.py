"""Pins of the one-dimensional PIC oracle (the comparison model of Sec. III.B).

* The three-point solve reproduces the exact parabola x(L - x)/2 plus the
  linear lift V x / L of a uniform ion density between a grounded and a
  biased plate (the discrete second difference of a quadratic is exact).
* The deposit's zeroth and first moments equal the particle count and the
  sum of positions times the weight; a particle on a node lands there alone.
* Field and gather of a linear potential give its constant field.
* Free streaming with no field: positions advance by v dt and particles
  past a plate are counted at that plate.
* Recycling: every ion lost comes back inside the recycling length with a
  Gaussian velocity of the given deviation; electrons are not recycled.
* A 2D oracle run on a load that repeats one 1D load in every column (v_y = 0)
  keeps a y-independent potential and moves every copy as the 1D oracle
  moves the original: the equivalence the paper states for the slab.  The
  two differ only by the 2D deposit's 16-bit weights (2^-17 per weight), which
  after 40 steps moves positions and velocities by about 1e-5: the bars are
  1e-4, while a wrong sign, factor or index anywhere in either step moves
  them by 1e-2 or more."""
import math

import numpy as np

import oracle
from oracle import pic1d
import synth


def test_solve_uniform_density_parabola():
    L, V = 24, 3.0
    phi = pic1d.solve(L, np.ones(L + 1), 0.0, V)
    x = np.arange(L + 1, dtype=np.float64)
    assert np.max(np.abs(phi - (x * (L - x) / 2 + V * x / L))) < 1e-11


def test_deposit_moments_and_node_particle():
    L, w = 20, 0.37
    rng = np.random.default_rng(1)
    x = rng.random(5000) * L
    n = pic1d.deposit(L, x, w)
    assert abs(n.sum() - w * x.size) < 1e-9
    assert abs((n * np.arange(L + 1)).sum() - w * x.sum()) < 1e-8
    n1 = pic1d.deposit(L, np.array([7.0]), w)
    assert n1[7] == w and np.count_nonzero(n1) == 1


def test_field_of_linear_potential():
    L = 16
    phi = 0.25 - 1.5 * np.arange(L + 1)
    E = pic1d.field(phi)
    assert np.allclose(E, 1.5, atol=1e-14)
    x = np.random.default_rng(2).random(100) * L
    assert np.allclose(pic1d.gather(E, x), 1.5, atol=1e-14)


def test_free_streaming_and_plate_counts():
    L = 10
    x = np.array([0.05, 5.0, 9.97, 4.0])
    v = np.array([-1.0, 0.5, 1.0, 0.0])
    sim = pic1d.Slab1D(L, 0.1, 0.0, [(-1.0, -1, x, v)], amp=0.0, omega=0.0, recycle_species=-1)
    sim.step()
    assert sim.lost[0].tolist() == [1, 1]
    assert np.allclose(sim.x[0], [5.05, 4.0])


def _replicated_pair(ny=4, ppc=20, seed=9):
    w = synth.paper_slab(ppc=ppc, ny=ny, recycle=False, seed=seed)
    rng = np.random.default_rng(seed)
    loads = []
    for s in range(2):
        n = w.nx * ppc
        x = (np.repeat(np.arange(w.nx), ppc) + rng.random(n)).astype(np.float64)
        ox = (x - np.floor(x)).astype(np.float32)
        x = np.floor(x) + ox.astype(np.float64)          # the position the 2D side stores
        v = (rng.standard_normal(n) * w.species[s].vth).astype(np.float32).astype(np.float64)
        loads.append((x, v))
    parts = [synth.replicate_columns(w, x, v) for x, v in loads]
    sp = [(w.species[s].alpha, w.species[s].sign, loads[s][0], loads[s][1]) for s in range(2)]
    one = pic1d.Slab1D(w.nx, w.dt, w.weight, sp, amp=w.v_amp[2], omega=w.v_omega[2])
    return w, parts, one


def test_2d_oracle_on_replicated_load_equals_1d():
    w, parts, one = _replicated_pair()
    two = oracle.Sim(w, parts, precision="f64")
    two.start()
    one.start()
    scale = 1.0
    for k in range(40):
        two.step()
        one.step()
        phi2 = two.phi.reshape(w.NX, w.NY)
        assert np.max(np.abs(phi2 - phi2.mean(axis=1, keepdims=True))) < 1e-9
        scale = max(scale, np.max(np.abs(one.phi)))
        assert np.max(np.abs(phi2.mean(axis=1) - one.phi)) < 1e-4 * scale, k
    for s in range(2):
        q = two.p[s]
        live = q["cell"] >= 0
        x2 = (q["cell"][live] >> 16).astype(np.float64) + q["ox"][live]
        assert x2.size == w.ny * one.x[s].size
        a = np.sort(x2)[:: w.ny]
        b = np.sort(one.x[s])
        assert np.max(np.abs(a - b)) < 1e-4
        vb = np.sort(one.v[s])
        va = np.sort(q["vx"][live])[:: w.ny]
        assert np.max(np.abs(va - vb)) < 1e-4 * max(1.0, np.max(np.abs(vb)))
        assert np.max(np.abs(q["vy"][live])) < 1e-12      # E_y is rounding noise only
    # the comparison is not vacuous: particles were lost at both plates
    assert one.lost[0].min() > 0
    assert two.tally[0][:2].tolist() == [w.ny * one.lost[0][1], w.ny * one.lost[0][0]]
    assert math.isfinite(scale)


def test_recycling_keeps_ion_count_and_draws_thermal_ions():
    """Ions lost at a plate come back at uniform positions in [0, recycle_len)
    with Gaussian velocities of the given deviation; electrons are not
    recycled."""
    L, n = 20, 4000
    rng = np.random.default_rng(5)
    xe, xi = rng.random(n) * L, rng.random(n) * L
    ve = rng.standard_normal(n)
    vi = np.where(rng.random(n) < 0.5, -1.0, 1.0) * 50.0       # 25 cells in one step: every ion leaves
    sim = pic1d.Slab1D(L, 0.5, 0.0, [(-1.0, -1, xe, ve), (0.0, 1, xi, vi)], amp=0.0, omega=0.0,
                       recycle_len=8.0, recycle_vth=0.25, recycle_species=1, seed=3)
    sim.step()
    assert sim.x[1].size == n and sim.x[0].size < n
    lost = int(sim.lost[1].sum())
    assert lost == n
    assert np.all((sim.x[1] >= 0) & (sim.x[1] < 8.0))
    assert abs(sim.x[1].mean() - 4.0) < 0.2
    assert abs(sim.v[1].std() / 0.25 - 1.0) < 0.05 and abs(sim.v[1].mean()) < 0.02
