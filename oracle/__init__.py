"""CPU oracle for the 2D electrostatic PIC cycle (arXiv:1610.03918, Sec. II).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``, never by the GPU library.  It
shares no code with the HIP path.  Particle and grid loops are plain C
(``pic_oracle.c``, built with ``-ffp-contract=off``); the Poisson solve is a
direct sparse factorisation of the discrete operator (SciPy SuperLU), i.e.
the exact discrete solution up to rounding.

Functions and the passages they follow:
  node_cond      Dirichlet nodes from the conductor map        Sec. II, III.A, III.C
  voltages       conductor potentials V_k(t)                   Sec. III.B
  deposit        area weighting, integer fixed point            (weighting not stated; see readings)
  assemble       source of eq. (5) plus Dirichlet lifts          eq. (5), Sec. III.D
  solve_direct   exact solution of the 5-point system           eq. (5)
  cg             double-precision CG (independent check)       eq. (5)
  jacobi         the paper's Jacobi iteration                   Sec. II
  gauss_seidel   the paper's Gauss-Seidel iteration (red-black)  Sec. II
  field          E = -grad(phi), central / two-point at walls   Sec. II
  push_f32/f64   gather + leapfrog + wall test                  eqs. (1)-(4), Sec. III
  rewind_f32/f64 leapfrog start (half step back)                eqs. (1)-(2)
  Sim            one step = deposit, solve, field, push          Sec. II ordering (reading Q1)

``oracle.unet`` is the float64 reference of the learned warm start's network
(forward, backward, loss, Adam, and the maps between the Poisson problem
and the network's tensors).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pic_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile the C part of the oracle (gcc, -O2 -ffp-contract=off)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        P = C.c_void_p
        i, i64, d = C.c_int, C.c_int64, C.c_double
        L.or_node_cond.argtypes = [i, i, i, i, P, P, P]
        L.or_node_cond.restype = i
        L.or_deposit.argtypes = [i, i, i, i, i64, P, P, P, P]
        L.or_deposit.restype = None
        L.or_assemble.argtypes = [i, i, i, i, P, P, P, d, P, i, i, P, d, i, i, P]
        L.or_assemble.restype = None
        L.or_cg.argtypes = [i, i, i, i, P, P, P, d, i, P]
        L.or_cg.restype = i
        L.or_field.argtypes = [i, i, i, i, P, P, P, P]
        L.or_field.restype = None
        for nm in ("or_push_f32", "or_push_f64"):
            f = getattr(L, nm)
            f.argtypes = [i, i, i, i, P, i, i, i, d, d, P, P, i64, P, P, P, P, P, P, P, P, P]
            f.restype = i64
        L.or_philox4x32_10.argtypes = [P, P, P]
        L.or_emit.restype = i64
        L.or_emit.argtypes = [i64, P, P, i64, C.c_uint32, C.c_uint32, P, d, P, P, P, P, P]
        L.or_philox4x32_10.restype = None
        L.or_recycled_ion.argtypes = [P, C.c_float, C.c_float, C.c_float, i, P, P, P, P, P]
        L.or_recycled_ion.restype = None
        for nm in ("or_rewind_f32", "or_rewind_f64"):
            f = getattr(L, nm)
            f.argtypes = [i, i, i, i, d, d, P, P, i64, P, P, P, P, P]
            f.restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags.c_contiguous
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ---------------------------------------------------------------------------
# grid
# ---------------------------------------------------------------------------

def node_cond(w) -> np.ndarray:
    """uint8 (NX, NY): 0 free, k > 0 Dirichlet node of conductor k."""
    out = np.zeros((w.NX, w.NY), np.uint8)
    cc = _c(w.cell_cond, np.uint8)
    ec = np.array(w.edge_cond, np.int32)
    rc = lib().or_node_cond(w.nx, w.ny, int(w.periodic_x), int(w.periodic_y), _p(cc), _p(ec), _p(out))
    if rc != 0:
        raise ValueError("two different conductors meet at a node")
    return out


def deposit(w, p: dict, rho: np.ndarray | None = None) -> np.ndarray:
    """int64 (NX, NY) node charge of one species in units of 2^-32 particle."""
    if rho is None:
        rho = np.zeros((w.NX, w.NY), np.int64)
    cell = _c(p["cell"], np.int32)
    ox = _c(p["ox"], np.float32)
    oy = _c(p["oy"], np.float32)
    lib().or_deposit(w.nx, w.ny, int(w.periodic_x), int(w.periodic_y), cell.size,
                     _p(cell), _p(ox), _p(oy), _p(rho))
    return rho


def voltages(w, t: float) -> np.ndarray:
    """Conductor potentials V_k(t) = amp_k sin(omega_k t) (Sec. III.B: the
    RF electrode's sinusoidal bias; amplitude 0 for grounded conductors),
    float64[8] indexed by conductor id, with the host's libm sin."""
    import math
    v = np.zeros(8, dtype=np.float64)
    for k in range(1, 8):
        a = float(w.v_amp[k])
        if a != 0.0:
            v[k] = a * math.sin(float(w.v_omega[k]) * t)
    return v


def assemble(w, nc, rho_e, rho_i, t: float, surf=None) -> np.ndarray:
    """float64 (NX, NY) right-hand side; Dirichlet nodes carry V(t).
    Fully periodic grids get the mean removed (gauge: mean(phi) = 0)."""
    b = np.zeros((w.NX, w.NY), np.float64)
    V = voltages(w, t)
    if surf is None:
        surf = np.zeros(w.ny, np.int64)
    lib().or_assemble(w.nx, w.ny, int(w.periodic_x), int(w.periodic_y), _p(_c(nc, np.uint8)),
                      _p(_c(rho_e, np.int64)), _p(_c(rho_i, np.int64)), float(w.weight), _p(V),
                      int(w.charge_mode), int(w.charge_row), _p(_c(surf, np.int64)),
                      float(w.static_density), int(w.static_j_lo), int(w.static_j_hi), _p(b))
    if w.periodic_x and w.periodic_y:
        b -= b.mean()
    return b


# ---------------------------------------------------------------------------
# Poisson (eq. 5): exact discrete solution
# ---------------------------------------------------------------------------

_fact_cache: dict = {}


def operator(w, nc):
    """Sparse matrix of the 5-point operator 4 phi - sum(neighbours) restricted
    to the free nodes (Dirichlet neighbours moved to the right-hand side).
    A fully periodic grid pins node (0, 0) to make the matrix regular."""
    import scipy.sparse as sp
    NX, NY = w.NX, w.NY
    fixed = (nc.reshape(-1) != 0).copy()
    if w.periodic_x and w.periodic_y:
        fixed[0] = True
    free = np.nonzero(~fixed)[0]
    idx = -np.ones(NX * NY, np.int64)
    idx[free] = np.arange(free.size)
    I, J = np.divmod(free, NY)
    rows = [np.arange(free.size)]
    cols = [np.arange(free.size)]
    vals = [np.full(free.size, 4.0)]
    for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        a, b = I + di, J + dj
        ok = np.ones(free.size, bool)
        if w.periodic_x:
            a = a % NX
        else:
            ok &= (a >= 0) & (a < NX)
        if w.periodic_y:
            b = b % NY
        else:
            ok &= (b >= 0) & (b < NY)
        nb = np.where(ok, a * NY + np.where(ok, b, 0), 0)
        k = np.where(ok, idx[nb], -1)
        m = k >= 0
        rows.append(np.arange(free.size)[m])
        cols.append(k[m])
        vals.append(np.full(m.sum(), -1.0))
    A = sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(free.size, free.size))
    return A, free, fixed


def solve_direct(w, nc, b) -> np.ndarray:
    """phi (NX, NY) float64 with A phi = b on free nodes, phi = b on Dirichlet
    nodes; fully periodic grids return the zero-mean solution."""
    from scipy.sparse.linalg import splu
    key = (w.nx, w.ny, w.periodic_x, w.periodic_y, nc.tobytes())
    if key not in _fact_cache:
        A, free, fixed = operator(w, nc)
        _fact_cache.clear()
        _fact_cache[key] = (splu(A, permc_spec="COLAMD"), free, fixed)
    lu, free, fixed = _fact_cache[key]
    bf = b.reshape(-1)
    phi = np.zeros(w.NX * w.NY, np.float64)
    phi[nc.reshape(-1) != 0] = bf[nc.reshape(-1) != 0]
    phi[free] = lu.solve(bf[free])
    if w.periodic_x and w.periodic_y:
        phi -= phi.mean()
    return phi.reshape(w.NX, w.NY)


def cg(w, nc, b, phi0=None, rtol=1e-13, maxit=200000):
    phi = np.zeros((w.NX, w.NY)) if phi0 is None else np.array(phi0, np.float64, copy=True)
    rr = np.zeros(1)
    it = lib().or_cg(w.NX, w.NY, int(w.periodic_x), int(w.periodic_y), _p(_c(nc, np.uint8)),
                     _p(_c(b, np.float64)), _p(phi), float(rtol), int(maxit), _p(rr))
    return phi, it, float(rr[0])


def _sweep_setup(w, nc):
    """Fixed-node mask (Dirichlet nodes, plus node (0, 0) on a fully periodic
    grid) and, per direction x-1, x+1, y-1, y+1, the neighbour index of every
    node (-1 outside a bounded axis)."""
    NX, NY = w.NX, w.NY
    fixed = nc.reshape(-1) != 0
    if w.periodic_x and w.periodic_y:
        fixed = fixed.copy()
        fixed[0] = True
    I, J = np.divmod(np.arange(NX * NY), NY)
    nbrs = []
    for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        a, c = I + di, J + dj
        ok = np.ones(NX * NY, bool)
        if w.periodic_x:
            a = a % NX
        else:
            ok &= (a >= 0) & (a < NX)
        if w.periodic_y:
            c = c % NY
        else:
            ok &= (c >= 0) & (c < NY)
        nbrs.append(np.where(ok, a * NY + np.where(ok, c, 0), -1))
    return fixed, nbrs, (I + J) % 2


def _sweep_values(phi, b, fixed, nbrs):
    """(b + sum of the free neighbours) / 4 at every node, the neighbours added
    in the order x-1, x+1, y-1, y+1 (a fixed neighbour's potential is in b)."""
    s = b.copy()
    for nb in nbrs:
        use = (nb >= 0) & ~fixed[np.maximum(nb, 0)]
        s = s + np.where(use, phi[np.maximum(nb, 0)], 0.0)
    return s * 0.25


def jacobi(w, nc, b, phi0, sweeps):
    """`sweeps` Jacobi iterations of the masked 5-point system (Sec. II: the
    paper solves eq. (5) with Jacobi or Gauss-Seidel iterations): every free
    node from the previous iterate at once.  Fixed nodes keep phi0."""
    fixed, nbrs, _ = _sweep_setup(w, nc)
    phi = np.array(phi0, np.float64).reshape(-1).copy()
    bf = np.asarray(b, np.float64).reshape(-1)
    for _ in range(sweeps):
        phi = np.where(fixed, phi, _sweep_values(phi, bf, fixed, nbrs))
    return phi.reshape(w.NX, w.NY)


def gauss_seidel(w, nc, b, phi0, sweeps):
    """`sweeps` Gauss-Seidel iterations in red-black order (Sec. II): the
    red nodes (i + j even) from the current iterate, then the black nodes from
    the updated reds.  With an even node count on every periodic axis no two
    nodes of one colour are neighbours, so each colour is one simultaneous
    update.  Fixed nodes keep phi0."""
    fixed, nbrs, colour = _sweep_setup(w, nc)
    phi = np.array(phi0, np.float64).reshape(-1).copy()
    bf = np.asarray(b, np.float64).reshape(-1)
    for _ in range(sweeps):
        for col in (0, 1):
            upd = (colour == col) & ~fixed
            phi = np.where(upd, _sweep_values(phi, bf, fixed, nbrs), phi)
    return phi.reshape(w.NX, w.NY)


def residual(w, nc, b, phi) -> float:
    """Relative residual ||b - A phi|| / ||b|| over the free nodes, double."""
    A, free, fixed = operator(w, nc)
    bf = b.reshape(-1)[free]
    r = bf - A @ phi.reshape(-1)[free]
    nb = np.linalg.norm(bf)
    return float(np.linalg.norm(r) / (nb if nb > 0 else 1.0))


def field(w, nc, phi):
    Ex = np.zeros((w.NX, w.NY))
    Ey = np.zeros((w.NX, w.NY))
    lib().or_field(w.NX, w.NY, int(w.periodic_x), int(w.periodic_y), _p(_c(nc, np.uint8)),
                   _p(_c(phi, np.float64)), _p(Ex), _p(Ey))
    return Ex, Ey


# ---------------------------------------------------------------------------
# particles
# ---------------------------------------------------------------------------

def _state(p: dict, dt):
    return {"cell": _c(p["cell"], np.int32).copy(),
            **{k: _c(p[k], dt).copy() for k in ("ox", "oy", "vx", "vy")}}


class _Recycle(C.Structure):
    _fields_ = [("rows", C.c_int32), ("k0", C.c_uint32), ("k1", C.c_uint32), ("vth", C.c_double),
                ("step", C.c_int64)]


def philox4x32_10(ctr, key):
    """Philox4x32-10 (Salmon et al., SC 2011) of one counter (4 words) and key
    (2 words), the generator of the recycled ions."""
    c = np.array(ctr, np.uint32)
    k = np.array(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def recycled_ion(w, step, ux, ox0, oy0):
    """(cell code, ox, oy, vx, vy) of the ion that replaces one lost in the
    push of ``step`` with v_x = ux after the kick and offsets ox0, oy0 before
    the move (float32 offsets, float64 velocities)."""
    k0, k1 = w.recycle_key()
    rc = _Recycle(int(w.recycle_rows), k0, k1, float(w.species[1].vth), int(step))
    code = C.c_int32()
    ox, oy = C.c_float(), C.c_float()
    vx, vy = C.c_double(), C.c_double()
    lib().or_recycled_ion(C.cast(C.pointer(rc), C.c_void_p), float(ux), float(ox0), float(oy0), w.ny,
                          C.cast(C.pointer(code), C.c_void_p), C.cast(C.pointer(ox), C.c_void_p),
                          C.cast(C.pointer(oy), C.c_void_p), C.cast(C.pointer(vx), C.c_void_p),
                          C.cast(C.pointer(vy), C.c_void_p))
    return code.value, ox.value, oy.value, vx.value, vy.value


class _Hits(C.Structure):
    _fields_ = [("cap", C.c_int64), ("n", C.c_int64), ("rec", C.c_void_p)]


class HitRecords:
    """Removals recorded by one push: rows (class, packed last cell, bits of
    the kicked float32 v_x, v_y)."""

    def __init__(self, capacity: int):
        self.rec = np.zeros((max(int(capacity), 1), 4), np.int32)
        self.h = _Hits(self.rec.shape[0], 0, self.rec.ctypes.data)

    def rows(self):
        assert self.h.n <= self.h.cap, "hit record buffer too small"
        return self.rec[:self.h.n]


def push(w, s: int, p: dict, Ex, Ey, precision="f32", tally=None, surf=None, step=None, hits=None) -> int:
    """In-place push of species s.  precision 'f32' needs float32 state,
    'f64' float64 state.  Returns the number of particles removed.  With
    w.recycle_rows > 0 and the step index given, lost ions (species 1) are
    replaced by recycled ones (Sec. III.A).  hits: a HitRecords that receives
    every removal."""
    sp = w.species[s]
    rc = None
    if s == 1 and w.recycle_rows > 0 and step is not None:
        k0, k1 = w.recycle_key()
        rc = _Recycle(int(w.recycle_rows), k0, k1, float(sp.vth), int(step))
    f = lib().or_push_f32 if precision == "f32" else lib().or_push_f64
    dt = np.float32 if precision == "f32" else np.float64
    for k in ("ox", "oy", "vx", "vy"):
        assert p[k].dtype == dt and p[k].flags.c_contiguous
    if tally is None:
        tally = np.zeros(9, np.int64)
    surf_p = _p(surf) if surf is not None else None
    return f(w.nx, w.ny, int(w.periodic_x), int(w.periodic_y), _p(_c(w.cell_cond, np.uint8)),
             int(w.box_i_top), int(w.box_j_lo), int(w.box_j_hi), float(w.dt), float(sp.alpha),
             _p(_c(Ex, np.float64)), _p(_c(Ey, np.float64)), p["cell"].size, _p(p["cell"]),
             _p(p["ox"]), _p(p["oy"]), _p(p["vx"]), _p(p["vy"]), _p(tally), surf_p,
             C.cast(C.pointer(rc), C.c_void_p) if rc is not None else None,
             C.cast(C.pointer(hits.h), C.c_void_p) if hits is not None else None)


def see_thresholds(w):
    """Integer emission thresholds floor(yield_s 2^24) of the two species."""
    return np.array([int(np.floor(float(y) * 16777216.0)) for y in w.see_yield], np.uint32)


def emit(w, removals, step):
    """Secondary electrons freed by the removals of one step (Sec. IV;
    constant-yield reading, see or_emit): removals is a list of (species,
    rows) with rows as HitRecords.rows() gives them.  Returns the new
    electrons as float32 state arrays."""
    sp = np.concatenate([np.full(len(r), s, np.int32) for s, r in removals]) if removals else np.zeros(0, np.int32)
    rec = np.ascontiguousarray(np.concatenate([r for _, r in removals]) if removals else np.zeros((0, 4), np.int32),
                               dtype=np.int32)
    n = sp.size
    out = {"cell": np.zeros(max(n, 1), np.int32),
           **{k: np.zeros(max(n, 1), np.float32) for k in ("ox", "oy", "vx", "vy")}}
    k0, k1 = w.see_key()
    th = see_thresholds(w)
    m = lib().or_emit(n, _p(sp), _p(rec), int(step), k0, k1, _p(th), float(w.see_vth), _p(out["cell"]),
                      _p(out["ox"]), _p(out["oy"]), _p(out["vx"]), _p(out["vy"]))
    return {k: v[:m].copy() for k, v in out.items()}


def rewind(w, s: int, p: dict, Ex, Ey, precision="f32"):
    sp = w.species[s]
    f = lib().or_rewind_f32 if precision == "f32" else lib().or_rewind_f64
    f(w.nx, w.ny, int(w.periodic_x), int(w.periodic_y), float(w.dt), float(sp.alpha),
      _p(_c(Ex, np.float64)), _p(_c(Ey, np.float64)), p["cell"].size, _p(p["cell"]),
      _p(p["ox"]), _p(p["oy"]), _p(p["vx"]), _p(p["vy"]))


class Sim:
    """Full cycle, one step (reading of the ordering in Sec. II):
    deposit x^n -> assemble at t^n -> exact solve -> field -> push both
    species (v^{n-1/2} -> v^{n+1/2}, x^n -> x^{n+1}) with wall tests.
    ``start()`` performs the half step back of the velocities."""

    def __init__(self, w, particles: list, precision="f32"):
        self.w = w
        self.prec = precision
        dt = np.float32 if precision == "f32" else np.float64
        self.p = [_state(q, dt) for q in particles]
        self.nc = node_cond(w)
        self.step_index = 0
        self.emitted = 0
        self.tally = np.zeros((len(self.p), 9), np.int64)
        self.surf = np.zeros(w.ny, np.int64)
        self.phi = None
        self.b = None
        self.rho = None

    @property
    def t(self):
        return self.step_index * self.w.dt

    def deposit_assemble(self):
        w = self.w
        self.rho = [deposit(w, q) for q in self.p]
        surf = self.surf if w.charge_mode == 2 else None
        self.b = assemble(w, self.nc, self.rho[0], self.rho[1], self.t, surf)
        return self.b

    def solve(self):
        self.phi = solve_direct(self.w, self.nc, self.b)
        return self.phi

    def start(self):
        self.deposit_assemble()
        self.solve()
        Ex, Ey = field(self.w, self.nc, self.phi)
        for s, q in enumerate(self.p):
            rewind(self.w, s, q, Ex, Ey, self.prec)

    def step(self):
        w = self.w
        self.deposit_assemble()
        self.solve()
        Ex, Ey = field(w, self.nc, self.phi)
        see = any(float(y) > 0.0 for y in w.see_yield)
        removals = []
        for s, q in enumerate(self.p):
            surf = self.surf if (w.charge_mode == 2 and w.species[s].sign > 0) else None
            hits = HitRecords(min(q["cell"].size, 1 << 20)) if see else None
            push(w, s, q, Ex, Ey, self.prec, self.tally[s], surf, step=self.step_index, hits=hits)
            if see:
                removals.append((s, hits.rows()))
        if see:
            # secondary electrons of this step's trench-surface impacts join the
            # electrons after both pushes (pushed from the next step on)
            new = emit(w, removals, self.step_index)
            self.emitted += int(new["cell"].size)
            dt = self.p[0]["ox"].dtype
            self.p[0] = {k: np.concatenate([self.p[0][k], new[k].astype(self.p[0][k].dtype if k == "cell" else dt)])
                         for k in self.p[0]}
        self.step_index += 1

    def alive(self, s):
        return int(np.count_nonzero(self.p[s]["cell"] >= 0))
