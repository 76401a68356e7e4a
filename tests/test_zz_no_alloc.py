"""GPU test of the entry point that allocates nothing
(pic_unet_residual_sample_noalloc): through the C ABI, two calls in a row,
the second on a smaller window, each equal bit for bit to the
work-array entry point (pic_unet_residual_sample) on the same inputs -
sample, target and statistics - and a window beyond the static scratch is
refused before anything is launched."""
import ctypes as C

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _problem(w, seed):
    import torch
    dev = torch.device("cuda:0")
    nc = oracle.node_cond(w)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    b = synth.random_potential(w, seed, scale=2.0)
    p1 = synth.random_potential(w, seed + 1, scale=5.0)
    p2 = synth.random_potential(w, seed + 2, scale=5.0)
    pt = synth.random_potential(w, seed + 3, scale=5.0)
    return T(nc), T(b), T(p1), T(p2), T(pt)


def _call(noalloc, w, arrays, H, W, sc):
    import torch
    from paper_1610_03918_amd import unet
    L = unet.lib()
    nc, b, p1, p2, pt = arrays
    dev = b.device
    x = torch.full((H, W, 3), 7.0, dtype=torch.bfloat16, device=dev)
    t = torch.full((H, W), 7.0, dtype=torch.bfloat16, device=dev)
    stats = torch.zeros(3, dtype=torch.float64, device=dev)
    vp = lambda a: C.c_void_p(a.data_ptr())
    stream = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    common = (vp(b), vp(p1), vp(p2), vp(pt), vp(nc), w.NX, w.NY, int(w.periodic_x), int(w.periodic_y), H, W,
              *sc, vp(x), vp(t), vp(stats))
    if noalloc:
        st = L.pic_unet_residual_sample_noalloc(*common, stream)
    else:
        nb = C.c_size_t(0)
        assert L.pic_unet_residual_sample_work_bytes(H, W, C.byref(nb)) == 0
        work = torch.empty(nb.value, dtype=torch.uint8, device=dev)
        st = L.pic_unet_residual_sample(*common, vp(work), nb.value, stream)
    assert st == 0, st
    torch.cuda.synchronize(dev)
    return x.view(torch.int16).cpu().numpy(), t.view(torch.int16).cpu().numpy(), stats.cpu().numpy()


def test_noalloc_sample_equals_work_array_sample_on_two_calls():
    sc = (float(np.float32(0.5)), float(np.float32(0.02)), float(np.float32(4.0)))
    big = synth.trench(nx=1024, ny=512, width=8, depth=128, ppc=1)
    small = synth.trench(nx=96, ny=56, width=6, depth=24, ppc=1)
    for w, seed in ((big, 71), (small, 81)):
        arrays = _problem(w, seed)
        H, W = (w.NX // 8) * 8, w.NY
        ref = _call(False, w, arrays, H, W, sc)
        got = _call(True, w, arrays, H, W, sc)
        for a, r in zip(got, ref):
            assert np.array_equal(a, r)
        assert ref[2][2] == np.count_nonzero(oracle.node_cond(w)[:H, :W] == 0)
        assert ref[2][0] > 0 and ref[2][1] > 0


def test_noalloc_refuses_a_window_beyond_its_scratch():
    import torch
    from paper_1610_03918_amd import unet
    L = unet.lib()
    dev = torch.device("cuda:0")
    NX, NY = 2056, 2048                              # 4,210,688 pixels > 4,194,304
    f = torch.zeros(NX * NY, dtype=torch.float64, device=dev)
    nc = torch.zeros(NX * NY, dtype=torch.uint8, device=dev)
    x = torch.empty((NX, NY, 3), dtype=torch.bfloat16, device=dev)
    stats = torch.zeros(3, dtype=torch.float64, device=dev)
    vp = lambda a: C.c_void_p(a.data_ptr())
    st = L.pic_unet_residual_sample_noalloc(vp(f), vp(f), None, None, vp(nc), NX, NY, 0, 1, NX, NY, 1.0, 1.0,
                                            1.0, vp(x), None, vp(stats), None)
    assert st == -8
    assert float(stats.abs().sum()) == 0.0
