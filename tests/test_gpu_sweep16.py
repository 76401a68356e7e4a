"""Parity of the batched form at its full size: the 16-width trench sweep
(widths 1 .. 96, 64 particles per cell, 161.6M particles over 16 grids of
256 x 128 to 1024 x 512 cells; the width comparison of Sec. III.C), in the
launch configuration the sweep benchmark uses (the cached autotuned
schedule).

Per instance, bit for bit against the oracle: the charge of both species at
load and the assembled right-hand side; then, after one batched push of
every particle on the oracle's exact potential of each instance, the charge
of both species, the alive counts, the wall tallies per class and the
trench-bottom counts."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def test_sixteen_width_sweep_load_and_push_match_oracle():
    from paper_1610_03918_amd import PicBatch, autotune
    ws = synth.sweep()
    assert len(ws) == 16
    parts = [synth.load(w) for w in ws]
    total = sum(p["cell"].size for q in parts for p in q)
    assert total > 160_000_000, total
    entry = autotune.lookup(ws, parts)
    sch = dict(autotune.DEFAULT) if entry is None else entry["schedule"]
    b = PicBatch(ws, parts, sort_interval=tuple(sch["sort_interval"]), chunk=sch["chunk"],
                 push_unroll=sch["push_unroll"], push_merge=sch["push_merge"],
                 tile=tuple(sch["tile"]), halo=sch["halo"])
    fields = []
    for i, w in enumerate(ws):
        nc = oracle.node_cond(w)
        rho = [oracle.deposit(w, parts[i][s]) for s in range(2)]
        for s in range(2):
            assert np.array_equal(b.rho(i, s).cpu().numpy(), rho[s]), f"width {w.box_j_hi - w.box_j_lo} species {s}"
        rhs = oracle.assemble(w, nc, rho[0], rho[1], 0.0)
        assert np.array_equal(b.b(i).cpu().numpy(), rhs), f"instance {i} right-hand side"
        phi = oracle.solve_direct(w, nc, rhs)
        b.phi(i).copy_(b.torch.from_numpy(phi))
        fields.append(oracle.field(w, nc, phi))
        del rho, rhs, phi
    b.pic_push()
    hits = 0
    for i, w in enumerate(ws):
        Ex, Ey = fields[i]
        fields[i] = None
        tally = np.zeros((2, 9), np.int64)
        surf = np.zeros(w.ny, np.int64)
        d = b.pic_batch_diagnostics(i)
        for s in range(2):
            q = parts[i][s]
            parts[i][s] = None
            oracle.push(w, s, q, Ex, Ey, "f32", tally[s], surf if s == 1 else None)
            assert np.array_equal(b.rho(i, s).cpu().numpy(), oracle.deposit(w, q)), f"instance {i} species {s}"
            assert d["alive"][s] == int(np.count_nonzero(q["cell"] >= 0))
            del q
        assert np.array_equal(np.array(d["tally"]), tally), (i, d["tally"], tally)
        assert d["surf_hits"] == int(surf.sum())
        hits += int(tally.sum())
    assert hits > 0
    b.close()
