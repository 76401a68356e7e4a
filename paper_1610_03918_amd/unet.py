"""Python binding of the learned warm start (include/pic_unet.h).

Argument marshalling only: torch allocates the parameters, gradients, Adam
moments and the workspace on the device; the forward and backward passes,
the loss, the Adam step and the maps between the Poisson problem and the
network's tensors run in the library's HIP kernels.  The random initial
parameters are drawn here (He-normal, seeded), which is set-up, not part of
the method.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import pic as _pic
from .pic import PIC_OK, PicError, pic_solve_info

NCONV = 14
UNET_ENTRY_POINTS = ["pic_unet_param_count", "pic_unet_layer_info", "pic_unet_workspace_size",
                     "pic_unet_create", "pic_unet_io_buffers", "pic_unet_params_changed",
                     "pic_unet_forward", "pic_unet_loss", "pic_unet_backward", "pic_unet_adam",
                     "pic_unet_snapshot", "pic_unet_guess", "pic_solve_learned",
                     "pic_unet_set_periodic", "pic_unet_residual_sample_work_bytes",
                     "pic_unet_residual_sample", "pic_unet_residual_sample_noalloc", "pic_unet_load",
                     "pic_unet_residual_guess", "pic_solve_learned_residual",
                     "pic_unet_coarse_sample_work_bytes", "pic_unet_coarse_sample", "pic_unet_coarse_guess",
                     "pic_solve_learned_coarse", "pic_unet_extrapolate",
                     "pic_unet_set_timing", "pic_unet_forward_timing", "pic_unet_destroy",
                     "pic_unet_last_error"]


class pic_unet_layer(C.Structure):
    _fields_ = [("cin", C.c_int32), ("cout", C.c_int32), ("level", C.c_int32), ("pad", C.c_int32),
                ("w_offset", C.c_int64), ("b_offset", C.c_int64)]


class pic_unet_io(C.Structure):
    _fields_ = [("input", C.c_void_p), ("output", C.c_void_p), ("target", C.c_void_p),
                ("mask", C.c_void_p), ("grad_output", C.c_void_p)]


_bound = False


def lib():
    global _bound
    L = _pic.lib()
    if _bound:
        return L
    P, i32, i64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_float
    L.pic_unet_param_count.restype = i64
    L.pic_unet_param_count.argtypes = []
    L.pic_unet_layer_info.argtypes = [i32, C.POINTER(pic_unet_layer)]
    L.pic_unet_workspace_size.argtypes = [i32, i32, i32, C.POINTER(C.c_size_t)]
    L.pic_unet_create.argtypes = [i32, i32, i32, P, P, P, P, P, C.c_size_t, P, C.POINTER(P)]
    L.pic_unet_io_buffers.argtypes = [P, C.POINTER(pic_unet_io)]
    L.pic_unet_params_changed.argtypes = [P]
    L.pic_unet_forward.argtypes = [P]
    L.pic_unet_loss.argtypes = [P, C.POINTER(C.c_double)]
    L.pic_unet_backward.argtypes = [P]
    L.pic_unet_adam.argtypes = [P, f32, f32, f32, f32]
    L.pic_unet_snapshot.argtypes = [P, i32, P, P, P, i32, i32, f32, f32, f32]
    L.pic_unet_guess.argtypes = [P, i32, P, P, i32, i32, f32, P]
    L.pic_solve_learned.argtypes = [P, P, P, f32, f32, f32, P, C.POINTER(pic_solve_info)]
    L.pic_unet_set_periodic.argtypes = [P, i32]
    L.pic_unet_residual_sample_work_bytes.argtypes = [i32, i32, C.POINTER(C.c_size_t)]
    L.pic_unet_residual_sample.argtypes = [P, P, P, P, P, i32, i32, i32, i32, i32, i32, f32, f32, f32, P, P,
                                           P, P, C.c_size_t, P]
    L.pic_unet_residual_sample_noalloc.argtypes = [P, P, P, P, P, i32, i32, i32, i32, i32, i32, f32, f32, f32,
                                                   P, P, P, P]
    L.pic_unet_load.argtypes = [P, i32, P, P]
    L.pic_unet_residual_guess.argtypes = [P, i32, P, P, P, i32, i32, f32, i32, P]
    L.pic_solve_learned_residual.argtypes = [P, P, f32, f32, f32, P, C.POINTER(pic_solve_info)]
    L.pic_unet_coarse_sample_work_bytes.argtypes = [i32, i32, i32, C.POINTER(C.c_size_t)]
    L.pic_unet_coarse_sample.argtypes = [P, P, P, P, P, i32, i32, i32, i32, i32, i32, i32, f32, f32, f32, P, P,
                                         P, P, C.c_size_t, P]
    L.pic_unet_coarse_guess.argtypes = [P, i32, P, P, P, i32, i32, i32, i32, i32, f32, i32, P]
    L.pic_solve_learned_coarse.argtypes = [P, P, i32, f32, f32, f32, P, C.POINTER(pic_solve_info)]
    L.pic_unet_extrapolate.argtypes = [C.POINTER(P), C.POINTER(C.c_double), i32, i64, P, P]
    L.pic_unet_set_timing.argtypes = [P, i32]
    L.pic_unet_forward_timing.argtypes = [P, C.POINTER(C.c_double), C.POINTER(i32)]
    L.pic_unet_destroy.argtypes = [P]
    L.pic_unet_destroy.restype = None
    L.pic_unet_last_error.argtypes = [P]
    L.pic_unet_last_error.restype = C.c_char_p
    for nm in UNET_ENTRY_POINTS:
        if nm not in ("pic_unet_param_count", "pic_unet_destroy", "pic_unet_last_error"):
            getattr(L, nm).restype = i32
    _bound = True
    return L


def layers():
    """Shapes and parameter offsets of the 14 convolutions and the head."""
    out = []
    for k in range(NCONV + 1):
        y = pic_unet_layer()
        st = lib().pic_unet_layer_info(k, C.byref(y))
        if st != PIC_OK:
            raise PicError(st, f"layer {k}")
        out.append({"cin": y.cin, "cout": y.cout, "level": y.level, "w": y.w_offset, "b": y.b_offset})
    return out


def param_count():
    return int(lib().pic_unet_param_count())


def init_params(seed=100):
    """He-normal weights (std sqrt(2 / (9 Cin))), zero biases, head std
    sqrt(1/16); float32, flat in the library's layout."""
    rng = np.random.Generator(np.random.Philox(key=np.array([seed, 7], np.uint64)))
    p = np.zeros(param_count(), np.float32)
    for k, y in enumerate(layers()):
        n = y["cout"] * (9 if k < NCONV else 1) * y["cin"]
        std = np.sqrt(2.0 / (9 * y["cin"])) if k < NCONV else np.sqrt(1.0 / 16)
        p[y["w"]:y["w"] + n] = rng.standard_normal(n) * std
    return p


class UNet:
    """The network over caller-owned torch buffers; method names follow the C ABI."""

    def __init__(self, batch, H, W, device="cuda:0", params=None, seed=100, share=None, periodic_w=False):
        """share: another UNet whose parameter, gradient and Adam moment
        arrays this one uses too (networks of other image sizes trained
        together); periodic_w: circular padding along W."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the U-Net kernels need a GPU (no CPU fallback)")
        L = lib()
        self.torch = torch
        self.dev = torch.device(device)
        self.B, self.H, self.W = int(batch), int(H), int(W)
        n = param_count()
        if share is not None:
            self.params, self.grads, self.m, self.v = share.params, share.grads, share.m, share.v
        else:
            if params is None:
                params = init_params(seed)
            if isinstance(params, torch.Tensor):
                self.params = params.detach().to(self.dev, torch.float32).clone().contiguous()
            else:
                self.params = torch.as_tensor(np.asarray(params, np.float32)).to(self.dev).contiguous()
            self.grads = torch.zeros(n, dtype=torch.float32, device=self.dev)
            self.m = torch.zeros(n, dtype=torch.float32, device=self.dev)
            self.v = torch.zeros(n, dtype=torch.float32, device=self.dev)
        assert self.params.numel() == n
        nb = C.c_size_t(0)
        st = L.pic_unet_workspace_size(self.B, self.H, self.W, C.byref(nb))
        if st != PIC_OK:
            raise PicError(st, f"network shape {batch}x{H}x{W} (H, W multiples of 8)")
        self.ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.dev)
        base = self.ws.data_ptr()
        base += (-base) % 256
        self.stream = torch.cuda.current_stream(self.dev)
        torch.cuda.synchronize(self.dev)
        h = C.c_void_p()
        st = L.pic_unet_create(self.B, self.H, self.W, C.c_void_p(self.params.data_ptr()),
                               C.c_void_p(self.grads.data_ptr()), C.c_void_p(self.m.data_ptr()),
                               C.c_void_p(self.v.data_ptr()), C.c_void_p(base), nb.value,
                               C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != PIC_OK:
            raise PicError(st, "pic_unet_create")
        self.h = h
        io = pic_unet_io()
        self._chk(L.pic_unet_io_buffers(self.h, C.byref(io)))
        self.io = io
        if periodic_w:
            self._chk(L.pic_unet_set_periodic(self.h, 1))

    def _chk(self, st):
        if st != PIC_OK:
            raise PicError(st, lib().pic_unet_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().pic_unet_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- views of the library's tensors (for tests and data handling) ----------
    def _view(self, ptr, dtype, shape):
        t = self.torch
        n = int(np.prod(shape))
        esize = t.empty((), dtype=dtype).element_size()
        # wrap the device memory by slicing the workspace tensor
        off = ptr - self.ws.data_ptr()
        return self.ws[off:off + n * esize].view(dtype).view(*shape)

    def input(self):
        """bfloat16 [B, H, W, 3]."""
        return self._view(self.io.input, self.torch.bfloat16, (self.B, self.H, self.W, 3))

    def output(self):
        return self._view(self.io.output, self.torch.float32, (self.B, self.H, self.W))

    def target(self):
        return self._view(self.io.target, self.torch.float32, (self.B, self.H, self.W))

    def mask(self):
        return self._view(self.io.mask, self.torch.float32, (self.B, self.H, self.W))

    def grad_output(self):
        return self._view(self.io.grad_output, self.torch.float32, (self.B, self.H, self.W))

    # -- ABI calls ------------------------------------------------------------
    def pic_unet_params_changed(self):
        self._chk(lib().pic_unet_params_changed(self.h))

    def pic_unet_forward(self):
        self._chk(lib().pic_unet_forward(self.h))

    def pic_unet_loss(self):
        x = C.c_double(0.0)
        self._chk(lib().pic_unet_loss(self.h, C.byref(x)))
        return x.value

    def pic_unet_backward(self):
        self._chk(lib().pic_unet_backward(self.h))

    def pic_unet_adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self._chk(lib().pic_unet_adam(self.h, lr, beta1, beta2, eps))

    def pic_unet_snapshot(self, slot, b, phi, node_map, scales):
        ptr, NX, NY = node_map
        s_rho, s_v, s_phi = scales
        self._chk(lib().pic_unet_snapshot(self.h, int(slot), C.c_void_p(b.data_ptr()),
                                          C.c_void_p(phi.data_ptr()) if phi is not None else None,
                                          C.c_void_p(ptr), NX, NY, s_rho, s_v, s_phi))

    def pic_unet_guess(self, slot, b, node_map, s_phi, guess):
        ptr, NX, NY = node_map
        self._chk(lib().pic_unet_guess(self.h, int(slot), C.c_void_p(b.data_ptr()), C.c_void_p(ptr),
                                       NX, NY, s_phi, C.c_void_p(guess.data_ptr())))

    def pic_solve_learned(self, pic, scales, guess):
        """Learned start for instance 0 of a Pic (guess: device float64 NX*NY scratch)."""
        s_rho, s_v, s_phi = scales
        info = pic_solve_info()
        st = lib().pic_solve_learned(pic.ctx, self.h, C.c_void_p(pic.b.data_ptr()), s_rho, s_v, s_phi,
                                     C.c_void_p(guess.data_ptr()), C.byref(info))
        if st != PIC_OK:
            msg = lib().pic_unet_last_error(self.h).decode() or _pic.lib().pic_last_error(pic.ctx).decode()
            raise PicError(st, msg)
        return info.as_dict()

    def pic_unet_load(self, slot, x, t=None):
        """Stored sample (device bfloat16 tensors x [H, W, 3], t [H, W]) into a batch slot."""
        self._chk(lib().pic_unet_load(self.h, int(slot), C.c_void_p(x.data_ptr()),
                                      C.c_void_p(t.data_ptr()) if t is not None else None))

    def pic_unet_residual_guess(self, slot, phi_1, phi_2, node_map, s_d, guess, use_output=True):
        ptr, NX, NY = node_map
        self._chk(lib().pic_unet_residual_guess(self.h, int(slot), C.c_void_p(phi_1.data_ptr()),
                                                C.c_void_p(phi_2.data_ptr()) if phi_2 is not None else None,
                                                C.c_void_p(ptr), NX, NY, float(s_d), 1 if use_output else 0,
                                                C.c_void_p(guess.data_ptr())))

    def pic_solve_learned_residual(self, pic, scales, guess):
        """Residual-learning start for instance 0 of a running Pic (scales:
        s_r, s_v, s_d; guess: device float64 NX*NY scratch)."""
        s_r, s_v, s_d = scales
        info = pic_solve_info()
        st = lib().pic_solve_learned_residual(pic.ctx, self.h, s_r, s_v, s_d, C.c_void_p(guess.data_ptr()),
                                              C.byref(info))
        if st != PIC_OK:
            msg = lib().pic_unet_last_error(self.h).decode() or _pic.lib().pic_last_error(pic.ctx).decode()
            raise PicError(st, msg)
        return info.as_dict()

    def pic_unet_coarse_guess(self, slot, phi_1, phi_2, node_map, periodic, f, s_d, guess, use_output=True):
        ptr, NX, NY = node_map
        self._chk(lib().pic_unet_coarse_guess(self.h, int(slot), C.c_void_p(phi_1.data_ptr()),
                                              C.c_void_p(phi_2.data_ptr()) if phi_2 is not None else None,
                                              C.c_void_p(ptr), NX, NY, int(periodic[0]), int(periodic[1]),
                                              int(f), float(s_d), 1 if use_output else 0,
                                              C.c_void_p(guess.data_ptr())))

    def pic_solve_learned_coarse(self, pic, f, scales, guess):
        """Coarse residual-learning start (factor f) for instance 0 of a
        running Pic (scales: s_r, s_v, s_d; guess: device float64 NX*NY scratch)."""
        s_r, s_v, s_d = scales
        info = pic_solve_info()
        st = lib().pic_solve_learned_coarse(pic.ctx, self.h, int(f), s_r, s_v, s_d, C.c_void_p(guess.data_ptr()),
                                            C.byref(info))
        if st != PIC_OK:
            msg = lib().pic_unet_last_error(self.h).decode() or _pic.lib().pic_last_error(pic.ctx).decode()
            raise PicError(st, msg)
        return info.as_dict()

    def pic_unet_set_timing(self, on=True):
        self._chk(lib().pic_unet_set_timing(self.h, 1 if on else 0))

    def pic_unet_forward_timing(self):
        ms, n = C.c_double(0.0), C.c_int32(0)
        self._chk(lib().pic_unet_forward_timing(self.h, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def train_step(self, lr=1e-3):
        """forward, loss, backward, Adam; returns the loss before the update."""
        self.pic_unet_forward()
        loss = self.pic_unet_loss()
        self.pic_unet_backward()
        self.pic_unet_adam(lr)
        return loss


def extrapolation_coefficients(K, degree=None):
    """Coefficients of the extrapolation to the next step from the last K
    solutions, latest first.  degree None (or K - 1): the polynomial through
    all K, (-1)^(k+1) binomial(K, k), k = 1 .. K.  A lower degree: the value
    at the next step of the least-squares polynomial of that degree through
    the K solutions at steps -1 .. -K, e0^T (V^T V)^-1 V^T with V the
    Vandermonde matrix of those steps."""
    if degree is None or degree == K - 1:
        return [float((-1) ** (k + 1) * math.comb(K, k)) for k in range(1, K + 1)]
    if not 0 <= degree < K:
        raise ValueError("degree must lie in 0 .. K - 1")
    import numpy as np
    t = -np.arange(1, K + 1, dtype=np.float64)
    V = np.vander(t, degree + 1, increasing=True)
    return [float(x) for x in np.linalg.solve(V.T @ V, V.T)[0]]


def extrapolate(phis, coefs, out, stream=None):
    """pic_unet_extrapolate on device tensors: out = sum_k coefs[k] phis[k]
    (float64 tensors of one shape, phis[0] the latest)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(out.device)
    K = len(phis)
    ptrs = (C.c_void_p * K)(*[C.c_void_p(p.data_ptr()) for p in phis])
    cs = (C.c_double * K)(*[float(c) for c in coefs])
    st = lib().pic_unet_extrapolate(ptrs, cs, K, int(out.numel()), C.c_void_p(out.data_ptr()),
                                    C.c_void_p(stream.cuda_stream))
    if st != PIC_OK:
        raise PicError(st, "pic_unet_extrapolate")


def residual_sample(b, phi_1, phi_2, phi_t, node_map, periodic, H, W, scales, x, t=None, stats=None,
                    stream=None):
    """pic_unet_residual_sample on device tensors: b, phi_1, phi_2 (or None),
    phi_t (or None) float64 [NX, NY]; node_map (pointer, NX, NY); periodic
    (x, y); scales (s_r, s_v, s_d); x bfloat16 [H, W, 3], t bfloat16 [H, W]
    (or None); stats float64 [3] (or None)."""
    import torch
    ptr, NX, NY = node_map
    s_r, s_v, s_d = scales
    if stream is None:
        stream = torch.cuda.current_stream(b.device)

    def vp(a):
        return C.c_void_p(a.data_ptr()) if a is not None else None

    work, nbytes = None, 0
    if stats is not None:
        nb = C.c_size_t(0)
        lib().pic_unet_residual_sample_work_bytes(int(H), int(W), C.byref(nb))
        nbytes = nb.value
        work = torch.empty(nbytes, dtype=torch.uint8, device=b.device)
    st = lib().pic_unet_residual_sample(vp(b), vp(phi_1), vp(phi_2), vp(phi_t), C.c_void_p(ptr), NX, NY,
                                        int(periodic[0]), int(periodic[1]), int(H), int(W), float(s_r),
                                        float(s_v), float(s_d), vp(x), vp(t), vp(stats), vp(work), nbytes,
                                        C.c_void_p(stream.cuda_stream))
    if st != PIC_OK:
        raise PicError(st, "pic_unet_residual_sample: bad window, pointer or launch")


def coarse_sample(b, phi_1, phi_2, phi_t, node_map, periodic, f, H, W, scales, x, t=None, stats=None,
                  stream=None):
    """pic_unet_coarse_sample on device tensors: as residual_sample, with the
    network pixel standing for an f x f block of nodes."""
    import torch
    ptr, NX, NY = node_map
    s_r, s_v, s_d = scales
    if stream is None:
        stream = torch.cuda.current_stream(b.device)

    def vp(a):
        return C.c_void_p(a.data_ptr()) if a is not None else None

    work, nbytes = None, 0
    if stats is not None:
        nb = C.c_size_t(0)
        st = lib().pic_unet_coarse_sample_work_bytes(int(f), int(H), int(W), C.byref(nb))
        if st != PIC_OK:
            raise PicError(st, "pic_unet_coarse_sample_work_bytes: bad factor or window")
        nbytes = nb.value
        work = torch.empty(nbytes, dtype=torch.uint8, device=b.device)
    st = lib().pic_unet_coarse_sample(vp(b), vp(phi_1), vp(phi_2), vp(phi_t), C.c_void_p(ptr), NX, NY,
                                      int(periodic[0]), int(periodic[1]), int(f), int(H), int(W), float(s_r),
                                      float(s_v), float(s_d), vp(x), vp(t), vp(stats), vp(work), nbytes,
                                      C.c_void_p(stream.cuda_stream))
    if st != PIC_OK:
        raise PicError(st, "pic_unet_coarse_sample: bad factor, window, pointer or launch")
