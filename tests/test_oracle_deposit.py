"""Pins of the oracle's area-weighting deposit (CPU only).

Area weighting distributes each particle over the four corners of its cell
with bilinear weights.  Those weights are fixed uniquely by four moments:
the total (1), the x and y first moments and the xy cross moment of the
deposited charge equal the particle's own (quantised) 1, x, y, xy.  Checking
all four on single particles and on ensembles pins every corner weight,
including which corner receives which weight.
"""
import numpy as np
import pytest

import oracle
import synth

S = 1 << 16


def _single(w, i, j, ox, oy):
    p = {"cell": np.array([(i << 16) | j], np.int32),
         "ox": np.array([ox], np.float32), "oy": np.array([oy], np.float32)}
    return oracle.deposit(w, p)


def _quantised(p):
    ux = np.floor(p["ox"].astype(np.float64) * S).astype(np.int64)
    uy = np.floor(p["oy"].astype(np.float64) * S).astype(np.int64)
    i = (p["cell"].astype(np.int64) >> 16)
    j = (p["cell"].astype(np.int64) & 0xFFFF)
    return S * i + ux, S * j + uy


@pytest.mark.parametrize("kind", ["periodic", "bounded", "trench"])
def test_total_charge_is_exact(kind):
    w = synth.workload_for_tests(kind)
    for s in range(2):
        p = synth.load_species(w, s)
        rho = oracle.deposit(w, p)
        assert int(rho.sum()) == p["cell"].size * (1 << 32)


def test_corner_particle_lands_on_one_node():
    w = synth.bounded_square(n=6, ppc=1)
    rho = _single(w, 2, 3, 0.0, 0.0)
    assert rho[2, 3] == 1 << 32
    assert np.count_nonzero(rho) == 1


def test_single_particle_moments_fix_all_four_weights():
    """For one particle, the 4 corner values are the unique solution of the
    four moment equations; the xy moment distinguishes the two diagonals."""
    w = synth.bounded_square(n=8, ppc=1)
    rng = np.random.default_rng(5)
    for _ in range(200):
        i, j = rng.integers(0, 8, 2)
        ox, oy = rng.random(2, dtype=np.float32)
        rho = _single(w, int(i), int(j), ox, oy)
        p = {"cell": np.array([(i << 16) | j], np.int32), "ox": np.array([ox]), "oy": np.array([oy])}
        X, Y = _quantised(p)
        I, J = np.meshgrid(np.arange(w.NX), np.arange(w.NY), indexing="ij")
        r = rho.astype(object)
        assert int((r).sum()) == S * S
        assert int((r * I).sum()) == S * int(X[0])
        assert int((r * J).sum()) == S * int(Y[0])
        assert int((r * I * J).sum()) == int(X[0]) * int(Y[0])
        assert np.count_nonzero(rho) <= 4
        nz = np.argwhere(rho)
        assert nz[:, 0].min() >= i and nz[:, 0].max() <= i + 1
        assert nz[:, 1].min() >= j and nz[:, 1].max() <= j + 1


def test_ensemble_moments_bounded():
    w = synth.workload_for_tests("bounded")
    p = synth.load_species(w, 0)
    rho = oracle.deposit(w, p).astype(object)
    X, Y = _quantised(p)
    I, J = np.meshgrid(np.arange(w.NX), np.arange(w.NY), indexing="ij")
    assert int((rho * I).sum()) == S * int(sum(int(x) for x in X))
    assert int((rho * J).sum()) == S * int(sum(int(y) for y in Y))
    assert int((rho * I * J).sum()) == int(sum(int(x) * int(y) for x, y in zip(X, Y)))


def test_periodic_wrap_and_order_independence():
    w = synth.periodic_square(n=5, ppc=3)
    p = synth.load_species(w, 0)
    rho = oracle.deposit(w, p)
    perm = np.random.default_rng(1).permutation(p["cell"].size)
    q = {k: v[perm] for k, v in p.items()}
    assert np.array_equal(rho, oracle.deposit(w, q))
    # a particle in the last cell wraps onto row/column 0
    r = _single(w, 4, 4, 0.5, 0.5)
    assert r[0, 0] == r[4, 4] == r[0, 4] == r[4, 0] == 1 << 30


def test_removed_particles_deposit_nothing():
    w = synth.bounded_square(n=6, ppc=2)
    p = synth.load_species(w, 1)
    p["cell"][::3] = -5
    rho = oracle.deposit(w, p)
    assert int(rho.sum()) == int((p["cell"] >= 0).sum()) * (1 << 32)
