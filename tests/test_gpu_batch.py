"""GPU tests of the batched form: several instances of uneven size advanced
together (every kernel launch covers all of them, steps replayed as captured
HIP graphs) give, instance by instance, bit-identical integer charge,
particles, counters and potential to the same instance run alone."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import canonical, live

pytestmark = pytest.mark.gpu


def mixed_batch():
    return [
        synth.trench(nx=64, ny=32, width=4, depth=8, ppc=8, seed=31, rtol=1e-9),
        synth.workload_for_tests("trench"),
        synth.workload_for_tests("bounded"),
        synth.trench(nx=128, ny=64, width=12, depth=16, ppc=6, seed=32, rtol=1e-9),
    ]


def state(b, i):
    return {
        "rho": [b.rho(i, s).cpu().numpy() for s in range(2)],
        "phi": b.phi(i).cpu().numpy(),
        "parts": [canonical(live(b.particles_numpy(i, s))) for s in range(2)],
        "diag": b.pic_batch_diagnostics(i),
    }


def assert_same(a, c):
    for s in range(2):
        assert np.array_equal(a["rho"][s], c["rho"][s])
        assert np.array_equal(a["parts"][s], c["parts"][s])
    assert np.array_equal(a["phi"], c["phi"])
    assert a["diag"]["tally"] == c["diag"]["tally"]
    assert a["diag"]["alive"] == c["diag"]["alive"]
    assert a["diag"]["surf_hits"] == c["diag"]["surf_hits"]


def test_batch_init_deposit_matches_oracle():
    from paper_1610_03918_amd import PicBatch
    ws = mixed_batch()
    parts = [synth.load(w) for w in ws]
    b = PicBatch(ws, parts, sort_interval=(4, 8))
    for i, w in enumerate(ws):
        nc = oracle.node_cond(w)
        rho = [oracle.deposit(w, parts[i][s]) for s in range(2)]
        for s in range(2):
            assert np.array_equal(b.rho(i, s).cpu().numpy(), rho[s])
        assert np.array_equal(b.b(i).cpu().numpy(), oracle.assemble(w, nc, rho[0], rho[1], 0.0))
    info = b.start()
    assert all(x["converged"] for x in info)
    # after a push the Dirichlet nodes carry the conductor potentials at t = dt
    for _ in range(3):
        b.pic_push()
    for i, w in enumerate(ws):
        nc = oracle.node_cond(w)
        V = oracle.voltages(w, 3 * w.dt)
        got = b.b(i).cpu().numpy()
        assert np.array_equal(got[nc != 0], V[nc[nc != 0]])
        if w.v_amp[2]:
            assert np.any(got[nc == 2] != 0.0)
    b.close()


def test_batched_graph_steps_equal_each_instance_alone():
    from paper_1610_03918_amd import PicBatch
    ws = mixed_batch()
    parts = [synth.load(w) for w in ws]
    steps = 13
    b = PicBatch(ws, parts, sort_interval=(4, 8))
    b.start()
    infos = b.pic_batch_step(steps, passes=3, iters=32)
    assert all(x["converged"] for x in infos), infos
    got = [state(b, i) for i in range(len(ws))]
    b.close()
    for i, w in enumerate(ws):
        one = PicBatch([w], [parts[i]], sort_interval=(4, 8))
        one.start()
        inf = one.pic_batch_step(steps, passes=3, iters=32)
        assert inf[0]["converged"]
        assert_same(got[i], state(one, 0))
        one.close()


def test_graph_steps_track_eager_steps():
    """The captured schedule (fixed passes, per-instance early exit) and the
    host-driven solve reach the same tolerance: same counters up to
    round-off-driven differences, potential within the solver tolerance."""
    from paper_1610_03918_amd import PicBatch
    ws = mixed_batch()[:2]
    parts = [synth.load(w) for w in ws]
    g = PicBatch(ws, parts, sort_interval=(4, 8))
    e = PicBatch(ws, parts, sort_interval=(4, 8))
    for x in (g, e):
        x.start()
    g.pic_batch_step(8, passes=3, iters=32)
    e.pic_step(8)
    for i in range(len(ws)):
        dg, de = g.pic_batch_diagnostics(i), e.pic_batch_diagnostics(i)
        for s in range(2):
            assert abs(dg["alive"][s] - de["alive"][s]) <= 2
        pg, pe = g.phi(i).cpu().numpy(), e.phi(i).cpu().numpy()
        assert np.max(np.abs(pg - pe)) <= 1e-4 * max(1.0, np.max(np.abs(pe)))
    g.close()
    e.close()


def test_batched_push_matches_oracle_on_identical_potential():
    """One batched push (the launch a batched step makes after its solve) on
    a potential given to both sides: every instance's particles, charge,
    wall tallies and trench-bottom counts equal the oracle's float32 push
    bit for bit (Sec. II eqs. 1-4, the wall test of Sec. III.A)."""
    from paper_1610_03918_amd import PicBatch
    ws = mixed_batch()
    parts = [synth.load(w) for w in ws]
    b = PicBatch(ws, parts, sort_interval=(4, 8))
    fields = []
    for i, w in enumerate(ws):
        nc = oracle.node_cond(w)
        phi = synth.random_potential(w, 60 + i, scale=2.0)
        phi[nc != 0] = oracle.voltages(w, 0.0)[nc[nc != 0]]
        b.phi(i).copy_(b.torch.from_numpy(phi))
        fields.append(oracle.field(w, nc, phi))
    b.pic_push()
    for i, w in enumerate(ws):
        Ex, Ey = fields[i]
        tally = np.zeros((2, 9), np.int64)
        surf = np.zeros(w.ny, np.int64)
        d = b.pic_batch_diagnostics(i)
        for s in range(2):
            q = {k: v.copy() for k, v in parts[i][s].items()}
            oracle.push(w, s, q, Ex, Ey, "f32", tally[s], surf if (w.charge_mode == 2 and s == 1) else None)
            got = b.particles_numpy(i, s)
            assert np.array_equal(canonical(live(got)), canonical(live(q))), f"instance {i} species {s}"
            assert np.array_equal(b.rho(i, s).cpu().numpy(), oracle.deposit(w, q)), f"instance {i} species {s}"
            assert d["alive"][s] == int(np.count_nonzero(q["cell"] >= 0))
        assert np.array_equal(np.array(d["tally"]), tally), (i, d["tally"], tally)
        assert d["surf_hits"] == int(surf.sum())
    assert sum(sum(map(sum, b.pic_batch_diagnostics(i)["tally"])) for i in range(len(ws))) > 0
    b.close()
