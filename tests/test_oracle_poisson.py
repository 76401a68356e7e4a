"""Pins of the oracle's Poisson assembly and solve, eq. (5) (CPU only).

eq. (5): lap(phi) = n_e - n_i, i.e. -lap_h(phi) = n_i - n_e with the 5-point
Laplacian at unit spacing.  The pins are independent of the oracle's sparse
matrix: closed forms (a quadratic slab, Fourier and sine-series solutions),
the full-grid stencil applied to the solution with numpy slicing, and a
second solver (CG in C).
"""
import math

import numpy as np
import pytest
import scipy.fft as sfft

import oracle
import synth

TWO32 = float(1 << 32)


def full_stencil(phi, px, py):
    """4 phi - (sum of the 4 neighbours) on the whole node grid; entries whose
    stencil leaves a bounded axis are returned as NaN."""
    p = phi
    out = 4 * p
    out = out.copy()
    for ax, per in ((0, px), (1, py)):
        for sh in (1, -1):
            if per:
                out -= np.roll(p, sh, axis=ax)
            else:
                q = np.full_like(p, np.nan)
                if ax == 0:
                    if sh == 1:
                        q[1:] = p[:-1]
                    else:
                        q[:-1] = p[1:]
                else:
                    if sh == 1:
                        q[:, 1:] = p[:, :-1]
                    else:
                        q[:, :-1] = p[:, 1:]
                out -= q
    return out


def test_uniform_ion_slab_is_exact_parabola():
    """Grounded plates at x=0 and x=L, y periodic, uniform n_i = 1, no
    electrons: -phi'' = 1 gives phi = x (L - x) / 2, which the 3-point second
    difference reproduces exactly.  Positive charge -> positive potential."""
    L, ny = 20, 6
    w = synth.trench(nx=L, ny=ny, width=0, depth=0, ppc=1)
    w.cell_cond[:] = 0
    w.v_amp = (0.0,) * 8
    w.charge_mode = 0
    nc = oracle.node_cond(w)
    rho_i = np.full((w.NX, w.NY), 1 << 32, np.int64)   # weight 1 -> n_i = 1
    rho_e = np.zeros_like(rho_i)
    w.weight = 1.0
    b = oracle.assemble(w, nc, rho_e, rho_i, 0.0)
    phi = oracle.solve_direct(w, nc, b)
    x = np.arange(w.NX, dtype=np.float64)
    expect = x * (L - x) / 2
    assert np.allclose(phi, expect[:, None], atol=1e-11, rtol=0)
    assert phi[L // 2, 0] > 0


def test_periodic_matches_fourier_series():
    w = synth.periodic_square(n=24, ppc=1)
    nc = oracle.node_cond(w)
    assert not nc.any()
    rng = np.random.default_rng(3)
    b = rng.standard_normal((w.NX, w.NY))
    b -= b.mean()
    phi = oracle.solve_direct(w, nc, b)
    k = np.arange(w.NX)[:, None]
    l = np.arange(w.NY)[None, :]
    lam = 4 - 2 * np.cos(2 * np.pi * k / w.NX) - 2 * np.cos(2 * np.pi * l / w.NY)
    B = sfft.fft2(b)
    lam[0, 0] = 1.0
    P = B / lam
    P[0, 0] = 0.0
    ref = np.real(sfft.ifft2(P))
    assert np.max(np.abs(phi - ref)) < 1e-12 * max(1, np.max(np.abs(ref)))
    assert abs(phi.mean()) < 1e-13


def test_grounded_square_matches_sine_series():
    n = 18
    w = synth.bounded_square(n=n, ppc=1)
    nc = oracle.node_cond(w)
    assert nc[0].all() and nc[-1].all() and nc[:, 0].all() and nc[:, -1].all()
    assert not nc[1:-1, 1:-1].any()
    rng = np.random.default_rng(4)
    b = np.zeros((w.NX, w.NY))
    b[1:-1, 1:-1] = rng.standard_normal((n - 1, n - 1))
    phi = oracle.solve_direct(w, nc, b)
    k = np.arange(1, n)[:, None]
    l = np.arange(1, n)[None, :]
    lam = 4 - 2 * np.cos(np.pi * k / n) - 2 * np.cos(np.pi * l / n)
    B = sfft.dstn(b[1:-1, 1:-1], type=1)
    ref = sfft.idstn(B / lam, type=1)
    assert np.max(np.abs(phi[1:-1, 1:-1] - ref)) < 1e-12 * max(1, np.max(np.abs(ref)))
    assert not phi[0].any() and not phi[-1].any()


@pytest.mark.parametrize("kind", ["bounded", "trench"])
def test_assemble_and_solve_satisfy_full_stencil(kind):
    """Random integer charges and the RF potential at t = 7: the solution must
    satisfy 4 phi - sum(nb) = (N_i - N_e) w 2^-32 at every free node, with
    Dirichlet neighbours at their conductor potential, and phi = V on them."""
    w = synth.workload_for_tests(kind)
    nc = oracle.node_cond(w)
    rng = np.random.default_rng(8)
    ri = rng.integers(0, 50 << 32, (w.NX, w.NY), dtype=np.int64)
    re = rng.integers(0, 50 << 32, (w.NX, w.NY), dtype=np.int64)
    t = 7.0
    b = oracle.assemble(w, nc, re, ri, t)
    phi = oracle.solve_direct(w, nc, b)
    V = oracle.voltages(w, t)
    fixed = nc != 0
    assert np.array_equal(phi[fixed], V[nc[fixed]])
    rho_bar = (ri - re).astype(np.float64) * w.weight / TWO32
    st = full_stencil(phi, w.periodic_x, w.periodic_y)
    err = np.abs(st - rho_bar)[~fixed]
    assert np.max(err) < 1e-9 * max(1.0, np.max(np.abs(phi)))
    if kind == "trench":
        assert V[2] != 0 and np.any(nc == 2)


def test_cg_agrees_with_direct_solve():
    w = synth.workload_for_tests("trench")
    nc = oracle.node_cond(w)
    rng = np.random.default_rng(9)
    ri = rng.integers(0, 20 << 32, (w.NX, w.NY), dtype=np.int64)
    b = oracle.assemble(w, nc, np.zeros_like(ri), ri, 3.3)
    d = oracle.solve_direct(w, nc, b)
    c, it, rr = oracle.cg(w, nc, b, rtol=1e-13)
    assert it > 0 and rr <= 1e-13
    assert np.max(np.abs(c - d)) < 1e-9 * np.max(np.abs(d))
    assert oracle.residual(w, nc, b, d) < 1e-12


def test_charge_buildup_modes():
    """Mode 2: one ion on the bottom face of trench column j adds half a
    particle to nodes (row, j) and (row, j+1).  Mode 1: a fixed extra ion
    density on one row over an inclusive y range."""
    w = synth.trench(nx=16, ny=8, width=4, depth=4, ppc=4)
    nc = oracle.node_cond(w)
    z = np.zeros((w.NX, w.NY), np.int64)
    surf = np.zeros(w.ny, np.int64)
    j = w.box_j_lo + 1
    surf[j] = 3
    b0 = oracle.assemble(w, nc, z, z, 0.0, np.zeros(w.ny, np.int64))
    b1 = oracle.assemble(w, nc, z, z, 0.0, surf)
    d = b1 - b0
    row = w.charge_row
    assert d[row, j] == pytest.approx(1.5 * w.weight)
    assert d[row, j + 1] == pytest.approx(1.5 * w.weight)
    d[row, j] = d[row, j + 1] = 0
    assert not d.any()
    w.charge_mode = 1
    w.static_density = 5.0
    w.static_j_lo, w.static_j_hi = w.box_j_lo, w.box_j_hi
    b2 = oracle.assemble(w, nc, z, z, 0.0)
    d2 = b2 - b0
    cols = [jj for jj in range(w.static_j_lo, w.static_j_hi + 1) if nc[row, jj] == 0]
    assert cols and all(d2[row, jj] == 5.0 for jj in cols)
    d2[row, cols] = 0
    assert not d2.any()


def test_second_order_convergence_to_continuum():
    """Manufactured continuum solution phi = sin(pi x / L) sin(2 pi y / H) on a
    grounded-x, periodic-y slab: error falls ~4x per grid doubling."""
    errs = []
    for L in (16, 32, 64):
        H = L // 2
        w = synth.trench(nx=L, ny=H, width=0, depth=0, ppc=1)
        w.cell_cond[:] = 0
        w.v_amp = (0.0,) * 8
        nc = oracle.node_cond(w)
        x = np.arange(w.NX)[:, None]
        y = np.arange(w.NY)[None, :]
        ex = np.sin(np.pi * x / L) * np.sin(2 * np.pi * y / H)
        src = ((np.pi / L) ** 2 + (2 * np.pi / H) ** 2) * ex
        b = np.where(nc == 0, src, 0.0)
        phi = oracle.solve_direct(w, nc, b)
        errs.append(np.max(np.abs(phi - ex)))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


def test_conductor_potentials_follow_the_rf_bias():
    """V(t) of the trench workload: the grounded plate stays at 0 and the RF
    electrode (bottom plate and trench walls) follows 50 sin(0.05 t); the
    paper-parameter trench runs use 5 sin(0.01 t) (Sec. III.B)."""
    w = synth.trench(nx=32, ny=16, width=4, depth=8, ppc=1)
    for t in (0.0, 0.1, 7.3, 31.4159, 1000.0):
        V = oracle.voltages(w, t)
        assert V.shape == (8,) and V[0] == 0.0 and V[1] == 0.0 and not V[3:].any()
        assert abs(V[2] - 50.0 * np.sin(0.05 * t)) <= 1e-12 * 50.0
    assert abs(oracle.voltages(w, 10 * np.pi)[2] - 50.0) < 1e-12    # quarter period: the crest
    p = synth.paper_trench(15)
    assert abs(oracle.voltages(p, 50 * np.pi)[2] - 5.0) < 1e-12
    assert not oracle.voltages(synth.bounded_square(n=8, ppc=1), 3.0).any()
