"""Fine multigrid levels 1 and 2 in one launch per half-cycle, on the
1024 x 512 trench (the grid here deep enough to pair two levels below
level 0): the potential equals the one-level-per-launch path bit for bit
(the paired kernels repeat the same operations in the same order on a wider
window), and matches the exact sparse-direct solution of the same
right-hand side (Sec. II)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def test_paired_levels_equal_single_levels_and_direct_solution():
    """Two contexts on the same input, one with paired levels and one
    without, each solving twice: the solve's pass lengths adapt to the
    previous solve, so each comparison is between solves with the same
    history."""
    from paper_1610_03918_amd import Pic
    w = synth.trench(ppc=2)
    parts = synth.load(w)
    nc = oracle.node_cond(w)
    rho = [oracle.deposit(w, parts[s]) for s in range(2)]
    ref = oracle.solve_direct(w, nc, oracle.assemble(w, nc, rho[0], rho[1], 0.0))
    runs = {}
    for paired in (True, False):
        pic = Pic(w, parts, rtol=1e-11, sort_interval=(0, 0))
        pic.pic_set_level_pairs(paired)
        out = []
        for _ in range(2):
            info = pic.pic_solve(0)
            out.append((info, pic.phi.cpu().numpy().copy()))
        pic.close()
        runs[paired] = out
    for k in range(2):
        (ip, pp), (is_, ps) = runs[True][k], runs[False][k]
        print("solve", k, "iterations paired", ip["iterations"], "single", is_["iterations"])
        assert ip["converged"] and is_["converged"]
        assert ip["iterations"] == is_["iterations"]
        assert np.array_equal(pp, ps)
    phi_p = runs[True][0][1]
    err = float(np.max(np.abs(phi_p - ref)))
    assert err <= 1e-6 * max(1.0, float(np.max(np.abs(ref)))), err
    # a correct V-cycle keeps the cold solve to 1e-11 short
    assert runs[True][0][0]["iterations"] <= 40
