"""One-dimensional electrostatic PIC: the comparison model of Sec. III.B.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, never by the GPU library,
and sharing no code with it.

With the y axis periodic and no trench, the slab between the grounded plate
at x = 0 and the RF plate at x = L carries dynamics that depend on x alone
(Sec. III.B).  This module is that one-dimensional system written out in
float64 NumPy, in the same normalised units as the 2D model (Sec. II): the
mesh is the Debye length, time is in inverse plasma periods, each particle
carries density ``weight`` per unit length.

  deposit    linear (cloud-in-cell) weighting to the nodes 0..L
  solve      phi[k-1] - 2 phi[k] + phi[k+1] = -(n_i - n_e)[k] on the free
             nodes 1..L-1, phi(0) = 0, phi(L) = amp sin(omega t)     (eq. 5)
  field      E = -dphi/dx: central inside, two-point at the plates    (Sec. II)
  push       v += alpha E dt, x += v dt (leapfrog), removal at x < 0 or
             x >= L                                                   (eqs. 1-4)
  recycling  a removed ion is replaced by an ion at a uniform position in
             [0, recycle_len) with a Gaussian velocity of deviation
             ``recycle_vth`` (Sec. III.A); the draws come from a NumPy
             generator of the caller's seed, so runs compare statistically
             with the 2D model, not particle by particle
  Slab1D     one step = deposit x^n, solve at t^n, field, push; ``start``
             takes the velocities half a step back (leapfrog start)
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import solve_banded


def deposit(L: int, x: np.ndarray, weight: float) -> np.ndarray:
    """Density at nodes 0..L of particles at positions 0 <= x < L."""
    i = np.floor(x).astype(np.int64)
    f = x - i
    n = np.bincount(i, weights=(1.0 - f) * weight, minlength=L + 1)
    n += np.bincount(i + 1, weights=f * weight, minlength=L + 1)
    return n[: L + 1]


def solve(L: int, rho: np.ndarray, v_left: float, v_right: float) -> np.ndarray:
    """Exact solution of the three-point Poisson system on nodes 1..L-1
    with the plate potentials as Dirichlet values (eq. 5 in one dimension)."""
    m = L - 1
    rhs = -np.asarray(rho[1:L], np.float64).copy()
    rhs[0] -= v_left
    rhs[-1] -= v_right
    ab = np.zeros((3, m))
    ab[0, 1:] = 1.0
    ab[1, :] = -2.0
    ab[2, :-1] = 1.0
    phi = np.empty(L + 1)
    phi[0], phi[L] = v_left, v_right
    phi[1:L] = solve_banded((1, 1), ab, rhs)
    return phi


def field(phi: np.ndarray) -> np.ndarray:
    """E = -dphi/dx at the nodes: central difference at free nodes, the
    two-point difference toward the plasma at each plate."""
    E = np.empty_like(phi)
    E[1:-1] = 0.5 * (phi[:-2] - phi[2:])
    E[0] = phi[0] - phi[1]
    E[-1] = phi[-2] - phi[-1]
    return E


def gather(E: np.ndarray, x: np.ndarray) -> np.ndarray:
    i = np.floor(x).astype(np.int64)
    f = x - i
    return (1.0 - f) * E[i] + f * E[i + 1]


class Slab1D:
    """The 1D slab of Sec. III.B: ``species`` is a list of (alpha, sign, x, v)
    with alpha the acceleration per unit field (eqs. 1-2) and sign the charge
    sign in the source of eq. (5)."""

    def __init__(self, L: int, dt: float, weight: float, species, amp: float,
                 omega: float, recycle_len: float = 0.0, recycle_vth: float = 0.0,
                 recycle_species: int = 1, seed: int = 0):
        self.L, self.dt, self.weight = L, dt, weight
        self.alpha = [float(a) for a, _, _, _ in species]
        self.sign = [int(s) for _, s, _, _ in species]
        self.x = [np.asarray(x, np.float64).copy() for _, _, x, _ in species]
        self.v = [np.asarray(v, np.float64).copy() for _, _, _, v in species]
        self.amp, self.omega = amp, omega
        self.recycle_len, self.recycle_vth = recycle_len, recycle_vth
        self.recycle_species = recycle_species
        self.rng = np.random.default_rng(seed)
        self.step_index = 0
        self.lost = np.zeros((len(species), 2), np.int64)    # [s, 0]: x < 0, [s, 1]: x >= L
        self.phi = None

    @property
    def t(self) -> float:
        return self.step_index * self.dt

    def potential(self) -> np.ndarray:
        rho = np.zeros(self.L + 1)
        for s in range(len(self.x)):
            rho += self.sign[s] * deposit(self.L, self.x[s], self.weight)
        v_right = self.amp * math.sin(self.omega * self.t) if self.amp else 0.0
        self.phi = solve(self.L, rho, 0.0, v_right)
        return self.phi

    def start(self):
        E = field(self.potential())
        for s in range(len(self.x)):
            self.v[s] -= 0.5 * self.alpha[s] * self.dt * gather(E, self.x[s])

    def step(self):
        E = field(self.potential())
        for s in range(len(self.x)):
            x, v = self.x[s], self.v[s]
            v += self.alpha[s] * self.dt * gather(E, x)
            x += v * self.dt
            lo, hi = x < 0.0, x >= self.L
            self.lost[s, 0] += int(lo.sum())
            self.lost[s, 1] += int(hi.sum())
            out = lo | hi
            if not out.any():
                continue
            if s == self.recycle_species and self.recycle_len > 0:
                k = int(out.sum())
                x[out] = self.rng.random(k) * self.recycle_len
                v[out] = self.rng.standard_normal(k) * self.recycle_vth
            else:
                self.x[s], self.v[s] = x[~out], v[~out]
        self.step_index += 1
