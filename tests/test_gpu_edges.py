"""GPU parity on hand-placed particles: the boundary cases of the wall test
(Sec. II boundaries, Sec. III.A particle loss) that random loads almost
never produce, pushed through pic_push and compared bit for bit with the
oracle's float32 push on the same potential: exact ties between an x and a
y face, corner crossings, multi-cell moves that stop at the first solid
cell, trench-bottom hits with their surface charge, sidewall hits, a walk
into the trench mouth, periodic wraps over one and many cells, an offset
that rounds up to 1, landings exactly on a face, zero velocities, and
non-finite or runaway displacements (class 8).  Once with a zero field
(every tie exact) and once with a random potential."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import FIELDS

def _case_list(w):
    """(i, j, ox, oy, vx, vy) of the hand-placed particles of workload w."""
    c = []
    nx, ny = w.nx, w.ny
    # walls of a bounded axis or wraps of a periodic one, in all four directions
    c += [(nx - 1, 3, 0.9, 0.5, 2.0, 0.0), (0, 3, 0.05, 0.5, -1.0, 0.0),
          (4, ny - 1, 0.5, 0.95, 0.0, 1.0), (4, 0, 0.5, 0.02, 0.0, -1.0)]
    # corner crossings: x face first, y face first, an exact tie (x first), all four diagonals
    c += [(nx - 1, ny - 1, 0.9, 0.5, 10.0, 10.0), (nx - 1, ny - 1, 0.5, 0.9, 10.0, 10.0),
          (nx - 1, ny - 1, 0.5, 0.5, 10.0, 10.0), (0, 0, 0.5, 0.5, -10.0, -10.0),
          (0, ny - 1, 0.5, 0.5, -10.0, 10.0), (nx - 1, 0, 0.5, 0.5, 10.0, -10.0)]
    # interior ties and exact face landings: D = 0.5 from 0.5 lands on the face (offset 0 of the next cell)
    c += [(3, 3, 0.5, 0.5, 5.0, 5.0), (3, 4, 0.5, 0.25, 5.0, 0.0), (3, 5, 0.25, 0.5, 0.0, -2.5),
          (2, 2, 0.5, 0.5, -5.0, 5.0), (2, 3, 0.75, 0.75, -7.5, -7.5)]
    # multi-cell moves along both axes and diagonally
    c += [(1, 2, 0.3, 0.6, 25.0, 0.0), (1, 2, 0.3, 0.6, 0.0, 35.0), (2, 1, 0.1, 0.2, 33.0, 27.0),
          (5, 5, 0.4, 0.7, -43.0, 19.0)]
    # an offset just above 0 moving by a tiny negative amount: o' - floor(o') rounds to 1
    c += [(4, 4, 1e-9, 0.5, -2e-7, 0.0), (4, 4, 0.5, 1e-9, 0.0, -2e-7)]
    # zero velocity, non-finite and runaway velocities
    c += [(3, 2, 0.3, 0.3, 0.0, 0.0), (3, 2, 0.3, 0.3, np.nan, 0.0), (3, 2, 0.3, 0.3, 0.0, np.inf),
          (3, 2, 0.3, 0.3, -np.inf, 1.0), (3, 2, 0.3, 0.3, 1e8, 0.0), (3, 2, 0.3, 0.3, 0.0, -3e7)]
    if w.box_i_top < nx:                       # trench cases
        top, jl, jh = w.box_i_top, w.box_j_lo, w.box_j_hi
        c += [(top - 3, 2, 0.5, 0.5, 35.0, 0.0),           # multi-cell onto the electrode top
              (nx - 1, jl + 1, 0.8, 0.5, 5.0, 0.0),        # trench bottom
              (nx - 1, jh - 1, 0.5, 0.5, 5.0, 5.0),        # bottom/sidewall corner: exact tie -> bottom
              (nx - 2, jh - 1, 0.5, 0.5, 15.0, 5.0),       # two cells down, then the corner
              (top + 2, jl, 0.5, 0.1, 0.0, -2.0),          # sidewall -y
              (top + 2, jh - 1, 0.5, 0.9, 0.0, 2.0),       # sidewall +y
              (top - 1, jl + 1, 0.9, 0.5, 3.0, 0.0),       # into the mouth, alive
              (top - 1, jl, 0.5, 0.5, 5.0, -5.0),          # mouth corner, exact tie: x face first -> inside
              (top - 1, jh - 1, 0.5, 0.5, 5.0, 5.0),       # the other mouth corner
              (top - 1, jl - 1, 0.5, 0.5, 5.0, 5.0),       # diagonal into the electrode corner
              (top + 1, jl + 1, 0.5, 0.5, 120.0, 0.0),     # deep drop to the bottom from inside
              (nx - 1, jl, 0.5, 0.5, 0.0, 0.0)]            # resting in the bottom corner cell
    # the generic cases that would start inside a solid cell (the electrode) are left out
    return [x for x in c if w.cell_cond[x[0], x[1]] == 0]


def _particles(w, cases):
    cell = np.array([(i << 16) | j for i, j, *_ in cases], np.int32)
    f = lambda k: np.array([x[k] for x in cases], np.float64).astype(np.float32)
    return {"cell": cell, "ox": f(2), "oy": f(3), "vx": f(4), "vy": f(5)}


def _keys(p):
    """Rows of the five state arrays as int32 bits, every NaN replaced by one
    canonical quiet NaN (payloads are not results), sorted."""
    out = []
    for f in FIELDS:
        a = np.ascontiguousarray(p[f])
        if a.dtype != np.int32:
            a = np.where(np.isnan(a), np.float32(np.nan), a).astype(np.float32).view(np.int32)
        out.append(a)
    order = np.lexsort(out[::-1])
    return np.stack([x[order] for x in out], axis=1)


WORKLOADS = {
    "bounded": lambda: synth.bounded_square(n=40, ppc=1, seed=91),
    "periodic": lambda: synth.periodic_square(n=40, ppc=1, seed=92),
    "trench": lambda: synth.trench(nx=48, ny=40, width=6, depth=12, ppc=1, seed=93),
}


def _oracle_push(w, parts, phi):
    nc = oracle.node_cond(w)
    Ex, Ey = oracle.field(w, nc, phi)
    tally = np.zeros((2, 9), np.int64)
    surf = np.zeros(w.ny, np.int64)
    ref = []
    for s in range(2):
        q = {k: v.copy() for k, v in parts[s].items()}
        oracle.push(w, s, q, Ex, Ey, "f32", tally[s], surf if (w.charge_mode == 2 and s == 1) else None)
        ref.append(q)
    return ref, tally, surf


def _potential(w, field):
    nc = oracle.node_cond(w)
    phi = np.zeros((w.NX, w.NY)) if field == "zero" else synth.random_potential(w, 94, scale=3.0)
    phi[nc != 0] = oracle.voltages(w, 0.0)[nc[nc != 0]]
    return phi


@pytest.mark.parametrize("kind", list(WORKLOADS))
def test_cases_reach_the_classes_they_were_placed_for(kind):
    """CPU check of the case list on the oracle with a zero field (every tie
    exact): the classes the cases were written to produce occur."""
    w = WORKLOADS[kind]()
    cases = _case_list(w)
    assert len(cases) >= 25
    p = _particles(w, cases)
    _, tally, surf = _oracle_push(w, [p, {k: v.copy() for k, v in p.items()}], _potential(w, "zero"))
    assert tally[0][8] == 5 and tally[1][8] == 5            # nan, +-inf, two runaways
    if kind == "trench":
        assert tally[1][4] >= 4 and surf.sum() == tally[1][4]
        assert tally[1][6] >= 1 and tally[1][7] >= 1
    if kind == "bounded":
        assert all(tally[0][k] >= 1 for k in range(4))
    if kind == "periodic":
        assert tally.sum() == 10                            # only class 8: nothing leaves a torus


@pytest.mark.gpu
@pytest.mark.parametrize("field", ["zero", "random"])
@pytest.mark.parametrize("kind", list(WORKLOADS))
def test_hand_placed_particles_bit_exact(kind, field):
    from paper_1610_03918_amd import Pic
    w = WORKLOADS[kind]()
    cases = _case_list(w)
    p = _particles(w, cases)
    parts = [p, {k: v.copy() for k, v in p.items()}]
    pic = Pic(w, parts, sort_interval=(0, 0))
    phi = _potential(w, field)
    pic.phi.copy_(pic.torch.from_numpy(phi))
    pic.pic_push()
    ref, tally, surf = _oracle_push(w, parts, phi)
    d = pic.pic_diagnostics()
    assert np.array_equal(np.array(d["tally"]), tally), (d["tally"], tally)
    assert d["surf_hits"] == int(surf.sum())
    for s in range(2):
        got = pic.particles_numpy(s)
        assert np.array_equal(_keys(got), _keys(ref[s])), f"species {s}"
        assert np.array_equal(pic.rho(s).cpu().numpy(), oracle.deposit(w, ref[s])), f"species {s} charge"
    pic.close()
