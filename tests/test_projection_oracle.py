"""Pins of the oracle's projection around the solve (divergence of the staggered face
velocities, jump-consistent pressure-gradient correction).  CPU only."""
import numpy as np

import oracle as O
from paper_2312_11740_amd import problems as G


def random_faces(n, seed):
    rng = np.random.default_rng(seed)
    u = [rng.standard_normal((n, n, n)) for _ in range(3)]
    u[0][:, :, 0] = 0.0   # wall faces (x = 0, y = 0, z = 0 of the low-face layout)
    u[1][:, 0, :] = 0.0
    u[2][0, :, :] = 0.0
    return u


def test_divergence_sums_to_zero():
    """Discrete Gauss theorem: with zero normal velocity on the walls, the cell
    divergences add up to zero."""
    n = 12
    f = O.divergence(random_faces(n, 1), dt=0.5)
    assert abs(f.sum()) <= 1e-12 * np.abs(f).sum()


def test_divergence_of_a_discrete_gradient_is_the_laplacian():
    """u = face differences of q (zero through the walls): div u equals the
    constant-coefficient operator applied to q, computed by the oracle's apply."""
    n = 10
    q = np.random.default_rng(2).standard_normal((n, n, n))
    h = 1.0 / n
    ux = np.zeros_like(q)
    uy = np.zeros_like(q)
    uz = np.zeros_like(q)
    ux[:, :, 1:] = (q[:, :, 1:] - q[:, :, :-1]) / h
    uy[:, 1:, :] = (q[:, 1:, :] - q[:, :-1, :]) / h
    uz[1:, :, :] = (q[1:, :, :] - q[:-1, :, :]) / h
    ones = [np.ones_like(q) for _ in range(3)]
    ones[0][:, :, 0] = 0.0
    ones[1][:, 0, :] = 0.0
    ones[2][0, :, :] = 0.0
    lap = O.apply(ones, q)
    f = O.divergence((ux, uy, uz), dt=1.0)
    assert np.max(np.abs(f - lap)) <= 1e-11 * np.max(np.abs(lap))


def test_wall_faces_read_as_zero():
    n = 8
    u = random_faces(n, 3)
    f0 = O.divergence(u, dt=1.0)
    u[0][:, :, 0] = 7.0
    u[1][:, 0, :] = -3.0
    assert np.array_equal(O.divergence(u, dt=1.0), f0)


def test_uniform_density_reduces_to_the_plain_projection():
    """sigma = 0 and one phase: u - dt (1/rho) (p_b - p_a)/h on interior faces."""
    n = 8
    phi = -np.ones((n, n, n))              # all on the "-" side
    p = np.random.default_rng(4).standard_normal((n, n, n))
    u = random_faces(n, 5)
    kappa = np.zeros_like(p)
    ux, uy, uz = O.project(phi, kappa, p, 2.0, 5.0, 0.0, 0.25, u)
    h = 1.0 / n
    ex = u[0].copy()
    ex[:, :, 1:] -= 0.25 * 0.5 * (p[:, :, 1:] - p[:, :, :-1]) / h
    ex[:, :, 0] = 0.0
    assert np.allclose(ux, ex, rtol=0, atol=1e-13)
    assert np.all(uy[:, 0, :] == 0.0) and np.all(uz[0, :, :] == 0.0)


def test_projection_is_divergence_free_with_jumps():
    """f = div(u*)/dt, p solves the ghost-fluid system with the sigma kappa jump, and the
    corrected velocity has zero discrete divergence (to the solver's tolerance): the
    jump in the correction is the one the right-hand side took out."""
    n = 24
    rng = np.random.default_rng(6)
    phi = G.bubble_phi(n, [(0.45, 0.5, 0.55), (0.7, 0.3, 0.3)], [0.2, 0.12])
    rn, rp, sg, dt = 1e-3, 1.0, 0.01, 0.1
    u = random_faces(n, 7)
    f = O.divergence(u, dt)
    p, d, info = O.solve(phi, f, rn, rp, sg, tol=1e-13)
    assert abs(d["mean"]) <= 1e-9 * np.abs(f).max()
    un = O.project(phi, d["kappa"], p, rn, rp, sg, dt, u)
    div = O.divergence(un, dt)
    assert np.linalg.norm(div) <= 1e-9 * np.linalg.norm(f)
    # the jump matters: a correction without it leaves a divergence at the interface
    u0 = O.project(phi, d["kappa"], p, rn, rp, 0.0, dt, u)
    assert np.linalg.norm(O.divergence(u0, dt)) > 1e-3 * np.linalg.norm(f)
