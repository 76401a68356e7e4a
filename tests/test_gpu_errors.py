"""GPU tests of the library's error reporting through the C ABI: the
device error bit (forced from the host), the count of pushes made with an
unconverged potential in batched steps, the leapfrog stability check at
init, batched steps longer than the device window of conductor potentials,
and the zero-step call."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _small(seed=61, **kw):
    return synth.trench(nx=64, ny=32, width=4, depth=16, ppc=4, seed=seed, **kw)


def test_device_error_bit_is_reported_and_sticks():
    from paper_1610_03918_amd import Pic
    from paper_1610_03918_amd.pic import PicError
    w = _small()
    p = Pic(w, synth.load(w))
    p.start()
    p.pic_step(2)
    p.pic_inject_fault(1)
    p.pic_push()                                     # the assembly finds the counter outside the window
    with pytest.raises(PicError) as e:
        p.pic_diagnostics()
    assert e.value.status == -7 and "window of conductor potentials" in str(e.value)
    for call in (lambda: p.pic_step(1), lambda: p.pic_solve(1), lambda: p.pic_push()):
        with pytest.raises(PicError) as e:
            call()
        assert e.value.status == -7
    p.close()


def test_batched_steps_count_unconverged_pushes():
    """A schedule far too short (one pass of one iteration) leaves every step
    above rtol: pic_batch_step still runs all steps, then reports
    PIC_ERR_NOT_CONVERGED with the count of such pushes per instance; an
    adequate schedule adds none."""
    from paper_1610_03918_amd import PicBatch
    from paper_1610_03918_amd.pic import PicError
    ws = [_small(62), _small(63)]
    b = PicBatch(ws, [synth.load(w) for w in ws], sort_interval=(4, 8))
    b.start()
    infos = b.pic_batch_step(6, 3, 20, 10)
    base = [x["unconverged_pushes"] for x in infos]
    assert all(x["converged"] for x in infos)
    with pytest.raises(PicError) as e:
        b.pic_batch_step(5, 1, 1, 1)
    assert e.value.status == -4
    infos = [b.pic_batch_solve_info(i) for i in range(b.n)]
    for i, x in enumerate(infos):
        assert x["unconverged_pushes"] - base[i] == 5, x
        assert x["worst_relres"] > ws[i].rtol, x
    d = b.pic_batch_diagnostics(0)
    assert d["step"] == 6 + 5
    b.close()


def test_unstable_time_step_is_refused_at_init():
    """omega_pe dt >= 2 at the loaded mean density: PIC_ERR_CFL."""
    from paper_1610_03918_amd import Pic
    from paper_1610_03918_amd.pic import PicError
    w = _small(64)
    w.dt = 2.5
    with pytest.raises(PicError) as e:
        Pic(w, synth.load(w))
    assert e.value.status == -5
    w.dt = 1.5
    Pic(w, synth.load(w)).close()


def test_batched_steps_longer_than_the_potential_window():
    """A re-binning period of 600 steps (longer than the 512-step device
    window of conductor potentials): the graphs split the period, the
    Dirichlet nodes hold V(t) of the right step after 700 steps and no
    device error is raised; nsteps = 0 changes nothing."""
    from paper_1610_03918_amd import PicBatch
    w = synth.trench(nx=32, ny=16, width=4, depth=8, ppc=2, seed=65)
    b = PicBatch([w], [synth.load(w)], sort_interval=(600, 0))
    b.start()
    b.pic_batch_step(0, 2, 12, 6)
    assert b.pic_batch_diagnostics(0)["step"] == 0
    b.pic_batch_step(700, 2, 12, 6, allow_unconverged=True)
    d = b.pic_batch_diagnostics(0)
    assert d["step"] == 700
    nc = oracle.node_cond(w)
    V = oracle.voltages(w, 700 * w.dt)
    bb = b.b(0).cpu().numpy().reshape(w.NX, w.NY)
    fixed = nc != 0
    assert np.array_equal(bb[fixed], V[nc[fixed]])
    b.close()
