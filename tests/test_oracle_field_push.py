"""Pins of the oracle's field, gather and leapfrog push (CPU only).

Closed forms: a linear potential has a constant gradient at every node;
bilinear interpolation reproduces constant and linear fields; a particle in
a uniform field follows x0 + v0 t + alpha E t^2 / 2 exactly under leapfrog
with the half-step start; hand-placed particles hit the face, corner and
trench surfaces they must.
"""
import numpy as np
import pytest

import oracle
import synth


def test_linear_potential_gives_constant_field_everywhere():
    w = synth.workload_for_tests("bounded")
    nc = oracle.node_cond(w)
    I, J = np.meshgrid(np.arange(w.NX), np.arange(w.NY), indexing="ij")
    phi = 0.7 * I - 1.3 * J + 2.0
    Ex, Ey = oracle.field(w, nc, phi)
    assert np.allclose(Ex, -0.7, atol=1e-13) and np.allclose(Ey, 1.3, atol=1e-13)


def test_conductor_surface_rules_in_trench():
    """Tangential E vanishes along an equipotential conductor, the normal
    component uses the two-point difference toward the plasma (Sec. II,
    Sec. III.A)."""
    w = synth.workload_for_tests("trench")
    nc = oracle.node_cond(w)
    rng = np.random.default_rng(2)
    phi = rng.standard_normal((w.NX, w.NY))
    V = 3.0
    phi[nc != 0] = np.where(nc[nc != 0] == 2, V, 0.0)
    Ex, Ey = oracle.field(w, nc, phi)
    top = w.box_i_top
    j = 2                                  # on the electrode top, away from the trench
    assert nc[top, j] == 2 and nc[top - 1, j] == 0
    assert Ey[top, j] == 0.0
    assert Ex[top, j] == -(phi[top, j] - phi[top - 1, j])
    # sidewall node: y one-sided toward the trench interior, x tangential = 0
    jl = w.box_j_lo
    i = top + 3
    assert nc[i, jl] == 2 and nc[i, jl + 1] == 0
    assert Ey[i, jl] == -(phi[i, jl + 1] - phi[i, jl])
    assert Ex[i, jl] == 0.0
    # grounded plate x = 0: only one x neighbour exists
    assert Ex[0, 5] == -(phi[1, 5] - phi[0, 5])
    # free node: central
    assert Ex[10, 7] == -(phi[11, 7] - phi[9, 7]) * 0.5
    assert Ey[10, 7] == -(phi[10, 8] - phi[10, 6]) * 0.5


def _one(i, j, ox, oy, vx, vy, dt=np.float64):
    return {"cell": np.array([(i << 16) | j], np.int32),
            "ox": np.array([ox], dt), "oy": np.array([oy], dt),
            "vx": np.array([vx], dt), "vy": np.array([vy], dt)}


def test_uniform_field_leapfrog_closed_form():
    w = synth.periodic_square(n=32, ppc=1)
    sp = w.species[0]
    E0, E1 = 0.37, -0.21
    Ex = np.full((w.NX, w.NY), E0)
    Ey = np.full((w.NX, w.NY), E1)
    x0, y0, v0x, v0y = 3.25, 17.5, 0.8, -0.45
    p = _one(3, 17, 0.25, 0.5, v0x, v0y)
    oracle.rewind(w, 0, p, Ex, Ey, "f64")
    L = 32
    for n in range(1, 301):
        oracle.push(w, 0, p, Ex, Ey, "f64")
        t = n * w.dt
        ex = x0 + v0x * t + 0.5 * sp.alpha * E0 * t * t
        ey = y0 + v0y * t + 0.5 * sp.alpha * E1 * t * t
        c = int(p["cell"][0])
        gx = (c >> 16) + p["ox"][0]
        gy = (c & 0xFFFF) + p["oy"][0]
        dx = (gx - ex + L / 2) % L - L / 2
        dy = (gy - ey + L / 2) % L - L / 2
        assert abs(dx) < 1e-9 and abs(dy) < 1e-9, (n, dx, dy)
        vx = v0x + (n - 0.5) * sp.alpha * E0 * w.dt   # after push n: v^{n-1/2}
        assert abs(p["vx"][0] - vx) < 1e-12


def test_bilinear_gather_reproduces_linear_field():
    """A field linear in x and y is reproduced exactly at the particle: one
    step from rest (dt=1, alpha=1) gives v = E(x_p)."""
    w = synth.bounded_square(n=10, ppc=1)
    w.dt = 1.0
    w.species[0].alpha = 1.0
    I, J = np.meshgrid(np.arange(w.NX), np.arange(w.NY), indexing="ij")
    Ex = 0.01 * I + 0.02 * J
    Ey = -0.03 * I + 0.005 * J
    rng = np.random.default_rng(0)
    for _ in range(50):
        i, j = rng.integers(1, 8, 2)
        ox, oy = rng.random(2)
        p = _one(int(i), int(j), ox, oy, 0.0, 0.0)
        oracle.push(w, 0, p, Ex, Ey, "f64")
        assert abs(p["vx"][0] - (0.01 * (i + ox) + 0.02 * (j + oy))) < 1e-12
        assert abs(p["vy"][0] - (-0.03 * (i + ox) + 0.005 * (j + oy))) < 1e-12


def _push_one(w, s, p, prec="f32"):
    Ex = np.zeros((w.NX, w.NY))
    Ey = np.zeros((w.NX, w.NY))
    tally = np.zeros(9, np.int64)
    surf = np.zeros(w.ny, np.int64)
    oracle.push(w, s, p, Ex, Ey, prec, tally, surf)
    return tally, surf


def test_wall_hits_bounded_square():
    w = synth.bounded_square(n=8, ppc=1)
    f = np.float32
    cases = [  # (i, j, ox, oy, vx, vy, class)
        (7, 3, 0.9, 0.5, 2.0, 0.0, 0),     # +x wall
        (0, 3, 0.05, 0.5, -1.0, 0.0, 1),   # -x wall
        (4, 7, 0.5, 0.95, 0.0, 1.0, 2),    # +y wall
        (4, 0, 0.5, 0.02, 0.0, -1.0, 3),   # -y wall
    ]
    for i, j, ox, oy, vx, vy, cls in cases:
        p = _one(i, j, ox, oy, vx, vy, f)
        tally, _ = _push_one(w, 0, p)
        assert p["cell"][0] == -1 - cls
        assert tally[cls] == 1 and tally.sum() == 1


def test_corner_crossing_order_and_tie():
    """Diagonal move out of the corner cell: the earlier face decides the
    class; an exact tie crosses x first."""
    w = synth.bounded_square(n=8, ppc=1)
    f = np.float32
    # x face reached first: 0.1 to go in x at speed 10, 0.5 in y at speed 10
    p = _one(7, 7, 0.9, 0.5, 10.0, 10.0, f)
    _push_one(w, 0, p)
    assert p["cell"][0] == -1 - 0
    # y face first
    p = _one(7, 7, 0.5, 0.9, 10.0, 10.0, f)
    _push_one(w, 0, p)
    assert p["cell"][0] == -1 - 2
    # exact tie: both faces at 0.5, equal speeds -> x
    p = _one(7, 7, 0.5, 0.5, 10.0, 10.0, f)
    _push_one(w, 0, p)
    assert p["cell"][0] == -1 - 0


def test_multi_cell_move_stops_at_first_solid():
    w = synth.trench(nx=32, ny=16, width=4, depth=8, ppc=1)
    top = w.box_i_top                      # first electrode row (24)
    f = np.float32
    # fast ion going +x over the electrode top lands on it after 2 cells
    p = _one(top - 3, 2, 0.5, 0.5, 35.0, 0.0, f)
    tally, surf = _push_one(w, 1, p)
    assert p["cell"][0] == -1 - 0 and tally[0] == 1 and surf.sum() == 0
    # ion in the trench bottom row moving +x -> trench bottom, surface charge
    jl = w.box_j_lo
    p = _one(w.nx - 1, jl + 1, 0.8, 0.5, 5.0, 0.0, f)
    tally, surf = _push_one(w, 1, p)
    assert p["cell"][0] == -1 - 4 and tally[4] == 1 and surf[jl + 1] == 1
    # ion in the trench moving -y into the sidewall
    p = _one(top + 2, jl, 0.5, 0.1, 0.0, -2.0, f)
    tally, _ = _push_one(w, 1, p)
    assert p["cell"][0] == -1 - (4 + 3)
    # ion entering the trench mouth straight down stays alive
    p = _one(top - 1, jl + 2, 0.9, 0.5, 3.0, 0.0, f)
    _push_one(w, 1, p)
    c = int(p["cell"][0])
    assert c >= 0 and (c >> 16) == top and (c & 0xFFFF) == jl + 2
    assert abs(p["ox"][0] - 0.2) < 1e-6
    # periodic y wrap
    p = _one(3, w.ny - 1, 0.5, 0.9, 0.0, 2.0, f)
    _push_one(w, 0, p)
    c = int(p["cell"][0])
    assert c >= 0 and (c & 0xFFFF) == 0 and (c >> 16) == 3


def test_offset_stays_below_one():
    """o' - floor(o') can round to 1 for a tiny negative o'; the offset is
    kept in [0, 1) and the cell is the lower one."""
    w = synth.periodic_square(n=8, ppc=1)
    f = np.float32
    p = _one(4, 4, 1e-9, 0.5, -2e-7, 0.0, f)   # moves just below the face
    _push_one(w, 0, p)
    c = int(p["cell"][0])
    assert (c >> 16) == 3 and 0 <= p["ox"][0] < 1


def test_rewind_half_step():
    w = synth.periodic_square(n=8, ppc=1)
    Ex = np.full((w.NX, w.NY), 0.5)
    Ey = np.full((w.NX, w.NY), -0.25)
    p = _one(2, 2, 0.3, 0.3, 1.0, 1.0)
    oracle.rewind(w, 0, p, Ex, Ey, "f64")
    a = w.species[0].alpha
    assert abs(p["vx"][0] - (1.0 - 0.5 * a * 0.5 * w.dt)) < 1e-15
    assert abs(p["vy"][0] - (1.0 + 0.5 * a * 0.25 * w.dt)) < 1e-15


def test_float32_and_float64_push_agree_closely():
    w = synth.workload_for_tests("trench")
    nc = oracle.node_cond(w)
    phi = synth.random_potential(w, 3, scale=5.0)
    Ex, Ey = oracle.field(w, nc, phi)
    p = synth.load_species(w, 0)
    q32 = {k: v.copy() for k, v in p.items()}
    q64 = {"cell": p["cell"].copy(), **{k: p[k].astype(np.float64) for k in ("ox", "oy", "vx", "vy")}}
    oracle.push(w, 0, q32, Ex, Ey, "f32")
    oracle.push(w, 0, q64, Ex, Ey, "f64")
    alive = (q32["cell"] >= 0) & (q64["cell"] >= 0)
    assert alive.mean() > 0.9
    assert np.mean(q32["cell"] == q64["cell"]) > 0.999
    same = alive & (q32["cell"] == q64["cell"])
    assert np.max(np.abs(q32["vx"][same] - q64["vx"][same])) < 1e-5
    assert np.max(np.abs(q32["ox"][same] - q64["ox"][same])) < 1e-5
