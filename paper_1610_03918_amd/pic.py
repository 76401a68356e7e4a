"""Python binding of the gfx950 PIC library (include/pic.h).

Argument marshalling only: torch allocates the device buffers and supplies
the stream; every step of the method runs in the library's HIP kernels.
There is no CPU fallback: without ``lib/libpic.so`` (built by ``build.py``)
or without a GPU, constructing :class:`Pic` raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libpic.so")

MAX_COND = 8
NCLASS = 9
IAD_BINS = 90

PIC_OK = 0
STATUS = {0: "PIC_OK", -1: "PIC_ERR_ARG", -3: "PIC_ERR_HIP", -4: "PIC_ERR_NOT_CONVERGED",
          -5: "PIC_ERR_CFL", -6: "PIC_ERR_OVERFLOW", -7: "PIC_ERR_STATE", -8: "PIC_ERR_CAPACITY"}


class pic_config(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("periodic_x", C.c_int32), ("periodic_y", C.c_int32),
        ("dt", C.c_double), ("cell_cond", C.c_void_p), ("edge_cond", C.c_int32 * 4),
        ("v_amp", C.c_double * MAX_COND), ("v_omega", C.c_double * MAX_COND),
        ("weight", C.c_double), ("alpha", C.c_double * 2),
        ("box_i_top", C.c_int32), ("box_j_lo", C.c_int32), ("box_j_hi", C.c_int32),
        ("charge_mode", C.c_int32), ("charge_row", C.c_int32), ("static_density", C.c_double),
        ("static_j_lo", C.c_int32), ("static_j_hi", C.c_int32), ("rtol", C.c_double),
        ("max_iter", C.c_int32), ("solver", C.c_int32), ("sort_interval", C.c_int32 * 2),
        ("tile_x", C.c_int32), ("tile_y", C.c_int32), ("halo", C.c_int32), ("chunk", C.c_int32),
        ("push_unroll", C.c_int32), ("push_merge", C.c_int32),
        ("hitlog_capacity", C.c_int64), ("hitlog_species_mask", C.c_int32),
        ("warm_start", C.c_int32), ("recycle_rows", C.c_int32), ("recycle_key", C.c_uint32 * 2),
        ("recycle_vth", C.c_double), ("see_yield", C.c_double * 2), ("see_vth", C.c_double),
        ("see_key", C.c_uint32 * 2),
    ]


class pic_species_buffers(C.Structure):
    _fields_ = [("capacity", C.c_int64), ("count", C.c_int64), ("cell", C.c_void_p * 2),
                ("ox", C.c_void_p * 2), ("oy", C.c_void_p * 2), ("vx", C.c_void_p * 2),
                ("vy", C.c_void_p * 2)]


class pic_buffers(C.Structure):
    _fields_ = [("sp", pic_species_buffers * 2), ("rho", C.c_void_p * 2), ("phi", C.c_void_p),
                ("b", C.c_void_p), ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t)]


class pic_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("outer", C.c_int32), ("converged", C.c_int32),
                ("iterations_first", C.c_int32), ("relres0", C.c_double), ("relres", C.c_double),
                ("unconverged_pushes", C.c_int32), ("pad", C.c_int32), ("worst_relres", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k in ("iterations", "iterations_first", "outer", "converged", "relres0",
                                              "relres", "unconverged_pushes", "worst_relres")}


class pic_diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("t", C.c_double), ("alive", C.c_int64 * 2),
                ("loaded", C.c_int64 * 2), ("charge", C.c_int64 * 2),
                ("tally", (C.c_int64 * NCLASS) * 2), ("surf_hits", C.c_int64),
                ("hits_logged", C.c_int64), ("deposit_fallbacks", C.c_int64),
                ("last_solve", pic_solve_info), ("kinetic", C.c_double * 2),
                ("field_energy", C.c_double), ("iad", C.c_int64 * IAD_BINS),
                ("see_emitted", C.c_int64), ("see_dropped", C.c_int64)]


class pic_hit(C.Structure):
    _fields_ = [("species_class", C.c_int32), ("cell", C.c_int32), ("vx", C.c_float),
                ("vy", C.c_float), ("step", C.c_int32), ("pad", C.c_int32)]


_lib = None

ENTRY_POINTS = ["pic_workspace_size", "pic_init", "pic_deposit", "pic_solve", "pic_rewind",
                "pic_push", "pic_step", "pic_diagnostics", "pic_particles", "pic_read_hits",
                "pic_sort", "pic_push_timing", "pic_set_timing", "pic_batch_workspace_size",
                "pic_batch_init", "pic_batch_step", "pic_batch_diagnostics", "pic_batch_particles",
                "pic_batch_solve_info", "pic_node_map", "pic_tune", "pic_set_level_pairs", "pic_inject_fault",
                "pic_destroy", "pic_last_error", "pic_version"]


def lib():
    """Loads lib/libpic.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_1610_03918_amd.build` "
                           "(the PIC path has no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    P, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.pic_workspace_size.argtypes = [C.POINTER(pic_config), C.POINTER(C.c_int64), C.POINTER(C.c_size_t)]
    L.pic_init.argtypes = [C.POINTER(pic_config), C.POINTER(pic_buffers), P, C.POINTER(P)]
    L.pic_deposit.argtypes = [P]
    L.pic_solve.argtypes = [P, i32, P, C.POINTER(pic_solve_info)]
    L.pic_rewind.argtypes = [P]
    L.pic_push.argtypes = [P]
    L.pic_step.argtypes = [P, i32]
    L.pic_diagnostics.argtypes = [P, C.POINTER(pic_diag)]
    L.pic_particles.argtypes = [P, i32, C.POINTER(i32), C.POINTER(i64)]
    L.pic_read_hits.argtypes = [P, C.POINTER(pic_hit), i64, C.POINTER(i64)]
    L.pic_sort.argtypes = [P, i32]
    L.pic_push_timing.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(i32)]
    L.pic_set_timing.argtypes = [P, i32]
    L.pic_batch_workspace_size.argtypes = [i32, C.POINTER(pic_config), C.POINTER(C.c_int64),
                                           C.POINTER(C.c_size_t)]
    L.pic_batch_init.argtypes = [i32, C.POINTER(pic_config), C.POINTER(pic_buffers), P, C.c_size_t, P,
                                 C.POINTER(P)]
    L.pic_batch_step.argtypes = [P, i32, i32, i32, i32]
    L.pic_batch_diagnostics.argtypes = [P, i32, C.POINTER(pic_diag)]
    L.pic_batch_particles.argtypes = [P, i32, i32, C.POINTER(i32), C.POINTER(i64)]
    L.pic_batch_solve_info.argtypes = [P, i32, C.POINTER(pic_solve_info)]
    L.pic_node_map.argtypes = [P, i32, C.POINTER(P), P, C.POINTER(i32), C.POINTER(i32)]
    L.pic_tune.argtypes = [P, i32, i32, i32, i32]
    L.pic_set_level_pairs.argtypes = [P, i32]
    L.pic_inject_fault.argtypes = [P, i32]
    L.pic_destroy.argtypes = [P]
    L.pic_destroy.restype = None
    L.pic_last_error.argtypes = [P]
    L.pic_last_error.restype = C.c_char_p
    L.pic_version.restype = C.c_char_p
    for nm in ENTRY_POINTS:
        f = getattr(L, nm)
        if nm not in ("pic_destroy", "pic_last_error", "pic_version"):
            f.restype = i32
    _lib = L
    return L


class PicError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def make_config(w, *, solver=0, max_iter=2000, sort_interval=(8, 64), tile=(16, 16), halo=4,
                chunk=4096, push_unroll=4, push_merge=0, hitlog_capacity=0,
                hitlog_species_mask=2, rtol=None, warm_start=1):
    """pic_config from a workload description (see synth.Workload)."""
    cc = np.ascontiguousarray(w.cell_cond, dtype=np.uint8)
    cfg = pic_config()
    cfg.nx, cfg.ny = w.nx, w.ny
    cfg.periodic_x, cfg.periodic_y = int(w.periodic_x), int(w.periodic_y)
    cfg.dt = w.dt
    cfg.cell_cond = cc.ctypes.data
    for k in range(4):
        cfg.edge_cond[k] = int(w.edge_cond[k])
    for k in range(MAX_COND):
        cfg.v_amp[k] = float(w.v_amp[k])
        cfg.v_omega[k] = float(w.v_omega[k])
    cfg.weight = float(w.weight)
    cfg.alpha[0] = float(w.species[0].alpha)
    cfg.alpha[1] = float(w.species[1].alpha)
    cfg.box_i_top, cfg.box_j_lo, cfg.box_j_hi = w.box_i_top, w.box_j_lo, w.box_j_hi
    cfg.charge_mode, cfg.charge_row = w.charge_mode, w.charge_row
    cfg.static_density = w.static_density
    cfg.static_j_lo, cfg.static_j_hi = w.static_j_lo, w.static_j_hi
    cfg.rtol = float(w.rtol if rtol is None else rtol)
    cfg.max_iter = max_iter
    cfg.solver = solver
    cfg.sort_interval[0], cfg.sort_interval[1] = sort_interval
    cfg.tile_x, cfg.tile_y = tile
    cfg.halo = halo
    cfg.chunk = chunk
    cfg.push_unroll = push_unroll
    cfg.push_merge = push_merge
    cfg.hitlog_capacity = hitlog_capacity
    cfg.hitlog_species_mask = hitlog_species_mask
    cfg.warm_start = warm_start
    cfg.recycle_rows = int(getattr(w, "recycle_rows", 0))
    if cfg.recycle_rows:
        k0, k1 = w.recycle_key()
        cfg.recycle_key[0], cfg.recycle_key[1] = k0, k1
        cfg.recycle_vth = float(w.species[1].vth)
    see = tuple(float(y) for y in getattr(w, "see_yield", (0.0, 0.0)))
    if any(y > 0.0 for y in see):
        cfg.see_yield[0], cfg.see_yield[1] = see
        cfg.see_vth = float(w.see_vth)
        cfg.see_key[0], cfg.see_key[1] = w.see_key()
        # the emission reads every removal of the emitting species from the hit ring
        cfg.hitlog_capacity = max(int(cfg.hitlog_capacity), 1 << 20)
        cfg.hitlog_species_mask |= (1 if see[0] > 0.0 else 0) | (2 if see[1] > 0.0 else 0)
    return cfg, cc


class _Instance:
    """Device buffers of one instance, allocated with torch."""

    def __init__(self, torch, dev, w, particles, capacity, opts):
        t = torch
        self.w = w
        self.cfg, self._cc = make_config(w, **opts)
        counts = [int(p["cell"].size) for p in particles]
        cap = [int(capacity[s]) if capacity else max(counts[s], 1) for s in range(2)]
        self.capacity = cap
        self.sets = []
        bufs = pic_buffers()
        for s in range(2):
            sets = []
            for k in range(2):
                d = {"cell": t.full((cap[s],), -1, dtype=t.int32, device=dev)}
                for f in ("ox", "oy", "vx", "vy"):
                    d[f] = t.zeros((cap[s],), dtype=t.float32, device=dev)
                sets.append(d)
            p = particles[s]
            n = counts[s]
            for f in ("cell", "ox", "oy", "vx", "vy"):
                sets[0][f][:n].copy_(t.from_numpy(np.ascontiguousarray(p[f])))
            self.sets.append(sets)
            sb = bufs.sp[s]
            sb.capacity = cap[s]
            sb.count = n
            for k in range(2):
                sb.cell[k] = sets[k]["cell"].data_ptr()
                sb.ox[k] = sets[k]["ox"].data_ptr()
                sb.oy[k] = sets[k]["oy"].data_ptr()
                sb.vx[k] = sets[k]["vx"].data_ptr()
                sb.vy[k] = sets[k]["vy"].data_ptr()
        self.rho_t = [t.zeros((w.NX, w.NY), dtype=t.int64, device=dev) for _ in range(2)]
        self.phi_t = t.zeros((w.NX, w.NY), dtype=t.float64, device=dev)
        self.b_t = t.zeros((w.NX, w.NY), dtype=t.float64, device=dev)
        bufs.rho[0] = self.rho_t[0].data_ptr()
        bufs.rho[1] = self.rho_t[1].data_ptr()
        bufs.phi = self.phi_t.data_ptr()
        bufs.b = self.b_t.data_ptr()
        self.bufs = bufs


class _Context:
    """Shared parts of Pic and PicBatch: the context handle and error checks."""

    ctx = None

    def _chk(self, st, allow=()):
        if st != PIC_OK and st not in allow:
            raise PicError(st, lib().pic_last_error(self.ctx).decode())
        return st

    def _workspace(self, nbytes):
        self.ws_t = self.torch.empty((nbytes + 256,), dtype=self.torch.uint8, device=self.dev)
        base = self.ws_t.data_ptr()
        return base + (-base) % 256

    def pic_node_map(self, i=0):
        """(device pointer, NX, NY) of the library's node map of instance i."""
        p, nx, ny = C.c_void_p(), C.c_int32(), C.c_int32()
        self._chk(lib().pic_node_map(self.ctx, int(i), C.byref(p), None, C.byref(nx), C.byref(ny)))
        return p.value, nx.value, ny.value

    def node_map_host(self, i=0):
        """Host copy (numpy uint8 [NX, NY]) of the node map of instance i."""
        _, nx, ny = self.pic_node_map(i)
        out = np.zeros((nx, ny), np.uint8)
        self._chk(lib().pic_node_map(self.ctx, int(i), None, out.ctypes.data_as(C.c_void_p), None, None))
        return out

    def pic_tune(self, push_unroll, push_merge, sort_interval):
        self._chk(lib().pic_tune(self.ctx, int(push_unroll), int(push_merge), int(sort_interval[0]),
                                 int(sort_interval[1])))

    def pic_set_level_pairs(self, on):
        self._chk(lib().pic_set_level_pairs(self.ctx, int(bool(on))))

    def pic_inject_fault(self, what=1):
        """Test hook of the device error path (see pic.h)."""
        self._chk(lib().pic_inject_fault(self.ctx, int(what)))

    def close(self):
        if getattr(self, "ctx", None):
            lib().pic_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _fail_init(self, st, ctx):
        L = lib()
        msg = L.pic_last_error(ctx).decode() if ctx.value else "init failed"
        L.pic_destroy(ctx)
        self.ctx = None
        raise PicError(st, msg)


class Pic(_Context):
    """One simulation context on one GPU.  Method names follow the C ABI."""

    def __init__(self, w, particles, device="cuda:0", capacity=None, **opts):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the PIC library needs a GPU (no CPU fallback)")
        L = lib()
        self.torch = torch
        self.w = w
        self.dev = torch.device(device)
        inst = _Instance(torch, self.dev, w, particles, capacity, opts)
        self.inst = inst
        self.cfg = inst.cfg
        self.capacity = inst.capacity
        self.sets = inst.sets
        self.rho_t, self.phi_t, self.b_t = inst.rho_t, inst.phi_t, inst.b_t
        ws = C.c_size_t(0)
        capa = (C.c_int64 * 2)(*inst.capacity)
        st = L.pic_workspace_size(C.byref(inst.cfg), capa, C.byref(ws))
        if st != PIC_OK:
            raise PicError(st, "invalid configuration")
        bufs = inst.bufs
        bufs.workspace = self._workspace(ws.value)
        bufs.workspace_bytes = ws.value
        self.bufs = bufs
        self.stream = torch.cuda.current_stream(self.dev)
        torch.cuda.synchronize(self.dev)
        ctx = C.c_void_p()
        st = L.pic_init(C.byref(inst.cfg), C.byref(bufs), C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        self.ctx = ctx
        if st != PIC_OK:
            self._fail_init(st, ctx)
        self.nodes = w.NX * w.NY

    # -- ABI calls ------------------------------------------------------
    def pic_deposit(self):
        self._chk(lib().pic_deposit(self.ctx))

    def pic_solve(self, guess_kind=1, guess=None, allow_unconverged=False):
        info = pic_solve_info()
        ptr = C.c_void_p(guess.data_ptr()) if guess is not None else None
        allow = (-4,) if allow_unconverged else ()
        self._chk(lib().pic_solve(self.ctx, int(guess_kind), ptr, C.byref(info)), allow)
        return info.as_dict()

    def pic_rewind(self):
        self._chk(lib().pic_rewind(self.ctx))

    def pic_push(self):
        self._chk(lib().pic_push(self.ctx))

    def pic_step(self, n=1):
        self._chk(lib().pic_step(self.ctx, int(n)))

    def pic_sort(self, s):
        self._chk(lib().pic_sort(self.ctx, int(s)))

    def pic_diagnostics(self):
        d = pic_diag()
        self._chk(lib().pic_diagnostics(self.ctx, C.byref(d)))
        return {
            "step": d.step, "t": d.t, "alive": list(d.alive), "loaded": list(d.loaded),
            "charge": list(d.charge),
            "tally": [list(d.tally[s]) for s in range(2)], "surf_hits": d.surf_hits,
            "hits_logged": d.hits_logged, "deposit_fallbacks": d.deposit_fallbacks,
            "kinetic": list(d.kinetic), "field_energy": d.field_energy, "iad": list(d.iad),
            "last_solve": d.last_solve.as_dict(), "see_emitted": d.see_emitted, "see_dropped": d.see_dropped,
        }

    def pic_particles(self, s):
        sset = C.c_int32(0)
        slots = C.c_int64(0)
        self._chk(lib().pic_particles(self.ctx, int(s), C.byref(sset), C.byref(slots)))
        return sset.value, slots.value

    def pic_read_hits(self, max_n=None):
        cap = int(self.cfg.hitlog_capacity)
        if cap <= 0:
            return np.zeros(0, dtype=[("species_class", "i4"), ("cell", "i4"), ("vx", "f4"),
                                      ("vy", "f4"), ("step", "i4"), ("pad", "i4")])
        m = cap if max_n is None else int(max_n)
        arr = (pic_hit * m)()
        n = C.c_int64(0)
        self._chk(lib().pic_read_hits(self.ctx, arr, m, C.byref(n)))
        dt = np.dtype([("species_class", "i4"), ("cell", "i4"), ("vx", "f4"), ("vy", "f4"),
                       ("step", "i4"), ("pad", "i4")])
        return np.frombuffer(bytes(arr), dtype=dt)[: n.value].copy()

    def pic_set_timing(self, on=True):
        self._chk(lib().pic_set_timing(self.ctx, int(bool(on))))

    def pic_push_timing(self):
        ms, npart, k = C.c_double(0), C.c_double(0), C.c_int32(0)
        self._chk(lib().pic_push_timing(self.ctx, C.byref(ms), C.byref(npart), C.byref(k)))
        return ms.value, npart.value, k.value

    # -- views ------------------------------------------------------------
    def particles(self, s):
        """Current particle arrays of species s (torch views of the live slots)."""
        k, n = self.pic_particles(s)
        return {f: v[:n] for f, v in self.sets[s][k].items()}

    def particles_numpy(self, s):
        self.torch.cuda.synchronize(self.dev)
        return {f: v.cpu().numpy() for f, v in self.particles(s).items()}

    def rho(self, s):
        return self.rho_t[s]

    @property
    def phi(self):
        return self.phi_t

    @property
    def b(self):
        return self.b_t

    def start(self):
        """Solve at t = 0 and move the velocities back half a step (leapfrog start)."""
        info = self.pic_solve(0)
        self.pic_rewind()
        return info

    def trench_profiles(self):
        """Potential across the trench at mid-depth (node row, columns
        box_j_lo - 4 .. box_j_hi + 4) and down its centre line (node column,
        rows box_i_top - 16 .. NX - 1); a copy of the caller's phi."""
        w = self.w
        phi = self.phi.cpu().numpy().reshape(w.NX, w.NY)
        jc = (w.box_j_lo + w.box_j_hi) // 2
        im = (w.box_i_top + w.nx) // 2
        return phi[im, w.box_j_lo - 4:w.box_j_hi + 5].copy(), phi[w.box_i_top - 16:, jc].copy()


class PicBatch(_Context):
    """Several independent instances (e.g. a trench-width sweep) in one
    context; every kernel launch covers all of them (pic_batch_* calls)."""

    def __init__(self, workloads, particles, device="cuda:0", capacities=None, **opts):
        """capacities: per instance (electron, ion) slot counts, or None for
        the loaded counts."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the PIC library needs a GPU (no CPU fallback)")
        L = lib()
        self.torch = torch
        self.dev = torch.device(device)
        self.ws = list(workloads)
        self.n = len(self.ws)
        caps = capacities if capacities is not None else [None] * self.n
        self.insts = [_Instance(torch, self.dev, w, p, c, opts) for w, p, c in zip(self.ws, particles, caps)]
        cfgs = (pic_config * self.n)(*[x.cfg for x in self.insts])
        bufs = (pic_buffers * self.n)(*[x.bufs for x in self.insts])
        caps = (C.c_int64 * (2 * self.n))(*[c for x in self.insts for c in x.capacity])
        nb = C.c_size_t(0)
        st = L.pic_batch_workspace_size(self.n, cfgs, caps, C.byref(nb))
        if st != PIC_OK:
            raise PicError(st, "invalid configuration")
        wsp = self._workspace(nb.value)
        self._cfgs, self._bufs = cfgs, bufs
        self.stream = torch.cuda.current_stream(self.dev)
        torch.cuda.synchronize(self.dev)
        ctx = C.c_void_p()
        st = L.pic_batch_init(self.n, cfgs, bufs, C.c_void_p(wsp), nb.value,
                              C.c_void_p(self.stream.cuda_stream), C.byref(ctx))
        self.ctx = ctx
        if st != PIC_OK:
            self._fail_init(st, ctx)

    def pic_solve(self, guess_kind=1):
        self._chk(lib().pic_solve(self.ctx, int(guess_kind), None, None))
        return [self.pic_batch_solve_info(i) for i in range(self.n)]

    def pic_rewind(self):
        self._chk(lib().pic_rewind(self.ctx))

    def pic_push(self):
        self._chk(lib().pic_push(self.ctx))

    def pic_step(self, n=1):
        self._chk(lib().pic_step(self.ctx, int(n)))

    def pic_batch_step(self, n, passes=2, iters=12, iters_later=0, allow_unconverged=False):
        """Steps as captured graphs; raises PicError(PIC_ERR_NOT_CONVERGED) when a
        step of some instance pushed a potential above rtol, unless
        allow_unconverged (then the per-instance infos carry the counts)."""
        allow = (-4,) if allow_unconverged else ()
        self._chk(lib().pic_batch_step(self.ctx, int(n), int(passes), int(iters), int(iters_later)), allow)
        return [self.pic_batch_solve_info(i) for i in range(self.n)]

    def pic_batch_solve_info(self, i):
        info = pic_solve_info()
        self._chk(lib().pic_batch_solve_info(self.ctx, int(i), C.byref(info)))
        return info.as_dict()

    def pic_batch_diagnostics(self, i):
        d = pic_diag()
        self._chk(lib().pic_batch_diagnostics(self.ctx, int(i), C.byref(d)))
        return {
            "step": d.step, "t": d.t, "alive": list(d.alive), "loaded": list(d.loaded),
            "charge": list(d.charge), "tally": [list(d.tally[s]) for s in range(2)],
            "surf_hits": d.surf_hits, "hits_logged": d.hits_logged,
            "deposit_fallbacks": d.deposit_fallbacks,
            "kinetic": list(d.kinetic), "field_energy": d.field_energy, "iad": list(d.iad), "last_solve": d.last_solve.as_dict(),
            "see_emitted": d.see_emitted, "see_dropped": d.see_dropped,
        }

    def pic_batch_particles(self, i, s):
        sset, slots = C.c_int32(0), C.c_int64(0)
        self._chk(lib().pic_batch_particles(self.ctx, int(i), int(s), C.byref(sset), C.byref(slots)))
        return sset.value, slots.value

    def particles_numpy(self, i, s):
        k, n = self.pic_batch_particles(i, s)
        self.torch.cuda.synchronize(self.dev)
        return {f: v[:n].cpu().numpy() for f, v in self.insts[i].sets[s][k].items()}

    def rho(self, i, s):
        return self.insts[i].rho_t[s]

    def phi(self, i):
        return self.insts[i].phi_t

    def b(self, i):
        return self.insts[i].b_t

    def start(self):
        info = self.pic_solve(0)
        self.pic_rewind()
        return info
