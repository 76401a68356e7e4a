"""Seeded synthetic workloads for the 2D electrostatic PIC trench problem.

This module is shared by the GPU path and by the CPU oracle.  It holds only
problem *definitions* and *random draws*: grid sizes, the conductor map of the
cells, plasma parameters and the initial particle loading.  It contains none
of the method's arithmetic (no weighting, no Poisson solve, no field, no push).

Units are the paper's normalised ones (Sec. II): length in Debye lengths,
time in 1/omega_e, potential in T_e/e, velocity in v_e = lambda_e omega_e,
density in n_0.  x is the plate-normal axis, y is parallel to the plates.

Particle layout (structure of arrays, one set per species):
  cell  int32   packed cell index (i << 16) | j, i = x cell, j = y cell
  ox,oy float32 in-cell offsets in [0, 1)
  vx,vy float32 velocities

Loading follows Sec. III.A: uniform random positions, Gaussian velocities of
eq. (6) with sigma_e = 1 and sigma_i = sqrt(tau * m_e / m_i).  Each non-solid
cell receives exactly ``ppc`` particles per species.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
import math
import numpy as np

MAX_COND = 8          # conductor ids 1..7; id 0 means plasma / free
CODE_SHIFT = 16       # packed cell code: (i << 16) | j


@dataclass
class Species:
    name: str
    alpha: float      # dv/dt = alpha * E  (eqs. 1-2): -1 electrons, m_e/m_i * q_i/e ions
    sign: int         # charge sign in the Poisson source (eq. 5): -1 electrons, +1 ions
    vth: float        # Gaussian sigma of each velocity component (eq. 6)
    ppc: int          # particles per non-solid cell at load


@dataclass
class Workload:
    name: str
    nx: int                       # cells along x (plate normal)
    ny: int                       # cells along y
    periodic_x: bool
    periodic_y: bool
    dt: float
    steps: int
    cell_cond: np.ndarray         # uint8 (nx, ny): 0 plasma, k>0 solid conductor k
    edge_cond: tuple              # conductor id of (x-low, x-high, y-low, y-high) edges, bounded axes only
    v_amp: tuple                  # per conductor id (index 0 unused): V_k(t) = amp*sin(omega*t)
    v_omega: tuple
    species: list
    weight: float                 # density carried by one particle, 1/ppc (n_0 units)
    rtol: float = 1e-8
    # trench box for hit classification: cells i >= box_i_top and box_j_lo <= j < box_j_hi
    box_i_top: int = 0
    box_j_lo: int = 0
    box_j_hi: int = 0
    # surface charge: 0 off, 1 static extra ion density, 2 accumulate ion bottom hits
    charge_mode: int = 0
    charge_row: int = 0           # node row (x index) receiving the charge
    static_density: float = 0.0
    static_j_lo: int = 0
    static_j_hi: int = -1
    seed: int = 0
    # ion recycling (Sec. III.A, III.C): a lost ion is replaced by a thermal ion
    # in the bulk cell rows 0 .. recycle_rows-1 (0: off)
    recycle_rows: int = 0
    # secondary electron emission at the trench surfaces (Sec. IV): electrons
    # freed per impact of an electron / an ion (0: off), and the thermal
    # speed of the emitted electrons (electron thermal speed units)
    see_yield: tuple = (0.0, 0.0)
    see_vth: float = 0.0
    extra: dict = field(default_factory=dict)

    def recycle_key(self) -> tuple:
        """Key of the recycling generator (two 32-bit words)."""
        return (int(self.seed) & 0xFFFFFFFF, 0x1610D3F1)

    def see_key(self) -> tuple:
        """Key of the secondary-emission generator (two 32-bit words)."""
        return (int(self.seed) & 0xFFFFFFFF, 0x5EE0E1EC)

    @property
    def NX(self) -> int:
        """Nodes along x: cells on a periodic axis, cells+1 on a bounded one."""
        return self.nx if self.periodic_x else self.nx + 1

    @property
    def NY(self) -> int:
        return self.ny if self.periodic_y else self.ny + 1

    def plasma_cells(self) -> int:
        return int(np.count_nonzero(self.cell_cond == 0))

    def n_particles(self, s: int) -> int:
        return self.plasma_cells() * self.species[s].ppc


def _species(mass_ratio: float, temp_ratio: float, ppc: int, ion_alpha=None):
    ion_a = (1.0 / mass_ratio) if ion_alpha is None else ion_alpha
    return [
        Species("electron", -1.0, -1, 1.0, ppc),
        Species("ion", ion_a, +1, math.sqrt(temp_ratio / mass_ratio), ppc),
    ]


def _amps(**kw):
    amp = [0.0] * MAX_COND
    om = [0.0] * MAX_COND
    for k, (a, w) in kw.items():
        idx = int(k[1:])
        amp[idx] = a
        om[idx] = w
    return tuple(amp), tuple(om)


GROUND, RF = 1, 2


def trench_cells(nx: int, ny: int, electrode_top: int, j_lo: int, j_hi: int,
                 cond: int = RF) -> np.ndarray:
    """Cells i >= electrode_top are solid conductor ``cond`` except the trench
    columns j_lo <= j < j_hi, which stay plasma down to the x = nx edge."""
    cc = np.zeros((nx, ny), dtype=np.uint8)
    cc[electrode_top:, :] = cond
    cc[electrode_top:, j_lo:j_hi] = 0
    return cc


def periodic_square(n: int = 64, ppc: int = 16, steps: int = 200, seed: int = 1) -> Workload:
    """Periodic square, m_i/m_e = 100, T_i/T_e = 0.1, 1e-10 relative residual."""
    amp, om = _amps()
    return Workload(
        name=f"periodic{n}", nx=n, ny=n, periodic_x=True, periodic_y=True, dt=0.1,
        steps=steps, cell_cond=np.zeros((n, n), np.uint8), edge_cond=(0, 0, 0, 0),
        v_amp=amp, v_omega=om, species=_species(100.0, 0.1, ppc), weight=1.0 / ppc,
        rtol=1e-10, box_i_top=n, seed=seed)


def bounded_square(n: int = 256, ppc: int = 100, steps: int = 2000, seed: int = 2) -> Workload:
    """All four walls grounded, particles absorbed at the walls (Sec. III.A)."""
    amp, om = _amps()
    return Workload(
        name=f"bounded{n}", nx=n, ny=n, periodic_x=False, periodic_y=False, dt=0.1,
        steps=steps, cell_cond=np.zeros((n, n), np.uint8),
        edge_cond=(GROUND, GROUND, GROUND, GROUND), v_amp=amp, v_omega=om,
        species=_species(1836.0, 0.05, ppc), weight=1.0 / ppc, rtol=1e-8,
        box_i_top=n, seed=seed)


def trench(nx: int = 1024, ny: int = 512, width: int = 8, depth: int = 128,
           ppc: int = 200, steps: int = 20000, amp: float = 50.0, omega: float = 0.05,
           charge_mode: int = 2, seed: int = 3, rtol: float = 1e-8) -> Workload:
    """Trench CCP (Sec. III.C-D): grounded plate at x = 0, RF plate at x = nx,
    y periodic, an RF electrode of thickness ``depth`` with a trench of
    ``width`` cells cut through it, centred in y.  The trench bottom is the
    x = nx edge.  charge_mode 2 accumulates ion hits on the trench bottom one
    node row above it (the paper's x = 79 row above the x = 80 bottom)."""
    top = nx - depth
    j_lo = (ny - width) // 2
    j_hi = j_lo + width
    a, o = _amps(c1=(0.0, 0.0), c2=(amp, omega))
    return Workload(
        name=f"trench{nx}x{ny}w{width}", nx=nx, ny=ny, periodic_x=False, periodic_y=True,
        dt=0.1, steps=steps, cell_cond=trench_cells(nx, ny, top, j_lo, j_hi),
        edge_cond=(GROUND, RF, 0, 0), v_amp=a, v_omega=o,
        species=_species(1836.0, 0.05, ppc), weight=1.0 / ppc, rtol=rtol,
        box_i_top=top, box_j_lo=j_lo, box_j_hi=j_hi,
        charge_mode=charge_mode, charge_row=nx - 1, seed=seed,
        extra={"width": width, "depth": depth, "electrode_top": top})


PAPER_TRENCH_J_LO = {15: 5, 4: 10}


def paper_trench(width: int = 15, charged: bool = False, ppc: int = 100,
                 steps: int = 10000, seed: int = 5) -> Workload:
    """The trench runs of Sec. III.C-D at the paper's parameters: the 60-row
    periodic bulk of Sec. III.B plus a 20-row trench cut through the RF
    electrode (80 x 30 cells, y periodic), m_i/m_e = 3672, T_i = T_e, 100
    particles per cell, dt = 0.1, RF amplitude 5 at omega 0.01 on the trench
    side, ions lost at any wall recycled into the bulk rows 0..59.  Width 15
    puts the trench at 5 <= j < 20 (Fig. 5), width 4 at 10 <= j < 14
    (Fig. 6).  ``charged`` adds the static extra ion density 5 on node row 79
    over 5 <= j <= 20 (Sec. III.D, Fig. 7)."""
    nx, ny, depth = 80, 30, 20
    top = nx - depth
    j_lo = PAPER_TRENCH_J_LO.get(width, (ny - width) // 2)
    j_hi = j_lo + width
    a, o = _amps(c1=(0.0, 0.0), c2=(5.0, 0.01))
    w = Workload(
        name=f"paper_trench_w{width}" + ("_charged" if charged else ""),
        nx=nx, ny=ny, periodic_x=False, periodic_y=True, dt=0.1, steps=steps,
        cell_cond=trench_cells(nx, ny, top, j_lo, j_hi), edge_cond=(GROUND, RF, 0, 0),
        v_amp=a, v_omega=o, species=_species(3672.0, 1.0, ppc), weight=1.0 / ppc,
        rtol=1e-8, box_i_top=top, box_j_lo=j_lo, box_j_hi=j_hi, seed=seed,
        recycle_rows=top, extra={"width": width, "depth": depth, "electrode_top": top})
    if charged:
        w.charge_mode = 1
        w.charge_row = nx - 1
        w.static_density = 5.0
        w.static_j_lo, w.static_j_hi = j_lo, j_hi
    return w


def paper_slab(ppc: int = 100, steps: int = 5000, seed: int = 6, ny: int = 30,
               recycle: bool = True) -> Workload:
    """The y-periodic RF slab of Sec. III.B (Fig. 2-3): 60 x ny cells with no
    trench, grounded plate at x = 0, RF plate at x = 60 with amplitude 5 at
    omega 0.01, m_i/m_e = 3672, T_i = T_e, dt = 0.1, lost ions recycled over
    the whole slab.  Its dynamics depend on x alone (the 1D equivalence)."""
    nx = 60
    a, o = _amps(c1=(0.0, 0.0), c2=(5.0, 0.01))
    return Workload(
        name=f"paper_slab60x{ny}", nx=nx, ny=ny, periodic_x=False, periodic_y=True, dt=0.1,
        steps=steps, cell_cond=np.zeros((nx, ny), np.uint8), edge_cond=(GROUND, RF, 0, 0),
        v_amp=a, v_omega=o, species=_species(3672.0, 1.0, ppc), weight=1.0 / ppc,
        rtol=1e-8, box_i_top=nx, seed=seed, recycle_rows=nx if recycle else 0)


def replicate_columns(w: Workload, x: np.ndarray, vx: np.ndarray, oy: float = 0.5) -> dict:
    """A 2D particle load that repeats one 1D load (positions 0 <= x < nx,
    velocities vx) in every column j, at offset ``oy`` and with v_y = 0: its
    charge, potential and x dynamics do not depend on y."""
    i = np.floor(x).astype(np.int64)
    ox = (x - i).astype(np.float32)
    n, ny = x.size, w.ny
    j = np.repeat(np.arange(ny, dtype=np.int64)[None, :], n, axis=0).ravel()
    ii = np.repeat(i, ny)
    return {
        "cell": ((ii << CODE_SHIFT) | j).astype(np.int32),
        "ox": np.repeat(ox, ny), "oy": np.full(n * ny, oy, np.float32),
        "vx": np.repeat(vx.astype(np.float32), ny), "vy": np.zeros(n * ny, np.float32),
    }


SWEEP_WIDTHS = (1, 2, 3, 4, 6, 8, 12, 16, 20, 24, 32, 40, 48, 56, 64, 96)


def sweep_instance(width: int, ppc: int = 64, steps: int = 5000, seed: int = 4) -> Workload:
    """One trench-width instance of the batched sweep: ny = max(128, pow2 >= 4w),
    nx = 2 ny, electrode thickness (trench depth) nx / 8."""
    ny = 128
    while ny < 4 * width:
        ny *= 2
    nx = 2 * ny
    w = trench(nx=nx, ny=ny, width=width, depth=nx // 8, ppc=ppc, steps=steps,
               seed=seed * 1000 + width)
    w.name = f"sweep_w{width}"
    return w


def sweep(ppc: int = 64, steps: int = 5000):
    return [sweep_instance(w, ppc, steps) for w in SWEEP_WIDTHS]


PRESETS = {
    "periodic64": lambda: periodic_square(),
    "bounded256": lambda: bounded_square(),
    "trench1024x512": lambda: trench(),
    "paper_trench_w15": lambda: paper_trench(15),
    "paper_trench_w4": lambda: paper_trench(4),
    "paper_trench_w15_charged": lambda: paper_trench(15, charged=True),
    "paper_slab60x30": lambda: paper_slab(),
}


# --------------------------------------------------------------------------
# particle loading (random draws only)
# --------------------------------------------------------------------------

def cell_codes(cell_cond: np.ndarray) -> np.ndarray:
    """Packed codes (i << 16) | j of the plasma cells, row-major in (i, j)."""
    ii, jj = np.nonzero(cell_cond == 0)
    return ((ii.astype(np.int64) << CODE_SHIFT) | jj.astype(np.int64)).astype(np.int32)


def rng_for(seed: int, species: int, stream: int = 0) -> np.random.Generator:
    """Philox counter-based generator keyed by (workload seed, species, stream)."""
    key = np.array([seed & 0xFFFFFFFFFFFFFFFF, (species << 32) | stream], dtype=np.uint64)
    return np.random.Generator(np.random.Philox(key=key))


def load_species(w: Workload, s: int, ppc: int | None = None) -> dict:
    """Uniform positions in every non-solid cell and Gaussian velocities (eq. 6)."""
    sp = w.species[s]
    ppc = sp.ppc if ppc is None else ppc
    codes = cell_codes(w.cell_cond)
    n = codes.size * ppc
    rng = rng_for(w.seed, s)
    cell = np.repeat(codes, ppc)
    off = rng.random((2, n), dtype=np.float32)
    vel = rng.standard_normal((2, n))
    vel *= sp.vth
    return {
        "cell": cell,
        "ox": off[0].copy(), "oy": off[1].copy(),
        "vx": vel[0].astype(np.float32), "vy": vel[1].astype(np.float32),
    }


def load(w: Workload) -> list:
    return [load_species(w, s) for s in range(len(w.species))]


def subsample(p: dict, stride: int) -> dict:
    return {k: v[::stride].copy() for k, v in p.items()}


def random_potential(w: Workload, seed: int, scale: float = 1.0) -> np.ndarray:
    """A smooth-plus-noise float64 potential on the node grid, for tests that
    feed one potential to both sides (drawn here, never computed by either)."""
    rng = np.random.Generator(np.random.Philox(key=np.array([seed, 7], np.uint64)))
    X, Y = np.meshgrid(np.arange(w.NX), np.arange(w.NY), indexing="ij")
    kx = 2 * math.pi / max(w.NX, 2)
    ky = 2 * math.pi / max(w.NY, 2)
    phi = scale * (np.sin(kx * X + 0.3) * np.cos(2 * ky * Y + 0.1)
                   + 0.05 * rng.standard_normal((w.NX, w.NY)))
    return phi.astype(np.float64)


def workload_for_tests(kind: str) -> Workload:
    """Reduced instances that still span several 16x16 tiles with a ragged tail."""
    if kind == "periodic":
        return periodic_square(n=40, ppc=8, steps=20, seed=11)
    if kind == "bounded":
        return replace(bounded_square(n=72, ppc=10, steps=20, seed=12))
    if kind == "trench":
        return trench(nx=96, ny=56, width=6, depth=24, ppc=12, steps=20, seed=13)
    raise ValueError(kind)
