"""Pins of the oracle's Jacobi and red-black Gauss-Seidel iterations (the
paper's own solvers of eq. (5), Sec. II), without any GPU:

* Jacobi maps the slowest Dirichlet eigenmode sin(pi i/nx) sin(pi j/ny) of a
  grounded square onto itself times (cos(pi/nx) + cos(pi/ny)) / 2 (closed
  form of the Jacobi iteration matrix's spectrum);
* red-black Gauss-Seidel contracts the error by the square of that number
  per sweep asymptotically;
* the exact solution (sparse direct) is a fixed point of both;
* one sweep equals the same update written with the sparse operator matrix
  (D = 4 I) on a masked trench grid."""
import math

import numpy as np

import oracle
import synth


def _square(n):
    w = synth.bounded_square(n=n, ppc=1, steps=1)
    return w, oracle.node_cond(w)


def test_jacobi_eigenmode_closed_form():
    w, nc = _square(16)
    i = np.arange(w.NX)[:, None]
    j = np.arange(w.NY)[None, :]
    mode = np.sin(math.pi * i / w.nx) * np.sin(math.pi * j / w.ny)
    mode[nc != 0] = 0.0
    rho = 0.5 * (math.cos(math.pi / w.nx) + math.cos(math.pi / w.ny))
    out = oracle.jacobi(w, nc, np.zeros_like(mode), mode, 1)
    assert np.max(np.abs(out - rho * mode)) < 1e-14


def test_gauss_seidel_asymptotic_rate():
    w, nc = _square(16)
    rng = np.random.default_rng(5)
    phi = rng.standard_normal((w.NX, w.NY))
    phi[nc != 0] = 0.0
    b = np.zeros_like(phi)
    phi = oracle.gauss_seidel(w, nc, b, phi, 300)
    n0 = np.linalg.norm(phi)
    n1 = np.linalg.norm(oracle.gauss_seidel(w, nc, b, phi, 1))
    rho = 0.5 * (math.cos(math.pi / w.nx) + math.cos(math.pi / w.ny))
    assert abs(n1 / n0 - rho * rho) < 1e-4


def _trench_problem():
    w = synth.trench(nx=32, ny=16, width=4, depth=8, ppc=4, seed=21)
    nc = oracle.node_cond(w)
    parts = synth.load(w)
    rho = [oracle.deposit(w, parts[s]) for s in range(2)]
    b = oracle.assemble(w, nc, rho[0], rho[1], 3.0)
    return w, nc, b


def test_direct_solution_is_a_fixed_point():
    w, nc, b = _trench_problem()
    ref = oracle.solve_direct(w, nc, b)
    scale = max(1.0, float(np.max(np.abs(ref))))
    for f in (oracle.jacobi, oracle.gauss_seidel):
        assert np.max(np.abs(f(w, nc, b, ref, 1) - ref)) < 1e-12 * scale


def test_one_sweep_against_the_operator_matrix():
    w, nc, b = _trench_problem()
    A, free, fixed = oracle.operator(w, nc)
    rng = np.random.default_rng(6)
    phi0 = np.where(nc != 0, b, rng.standard_normal(b.shape))
    x = phi0.reshape(-1)[free]
    bf = b.reshape(-1)[free]
    # Jacobi: x' = (b - (A - 4 I) x) / 4
    xj = (bf - (A @ x - 4.0 * x)) / 4.0
    got = oracle.jacobi(w, nc, b, phi0, 1).reshape(-1)[free]
    assert np.max(np.abs(got - xj)) < 1e-13 * max(1.0, np.max(np.abs(xj)))
    # Gauss-Seidel: reds from x, then blacks from the updated reds
    I, J = np.divmod(free, w.NY)
    red = (I + J) % 2 == 0
    y = x.copy()
    y[red] = ((bf - (A @ y - 4.0 * y)) / 4.0)[red]
    y[~red] = ((bf - (A @ y - 4.0 * y)) / 4.0)[~red]
    got = oracle.gauss_seidel(w, nc, b, phi0, 1).reshape(-1)[free]
    assert np.max(np.abs(got - y)) < 1e-13 * max(1.0, np.max(np.abs(y)))
