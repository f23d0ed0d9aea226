"""Pins of the oracle's implicit heat-diffusion step (backward Euler on
dT/dt = div(K grad T) + f, K by phase, insulated walls): the discrete eigenmodes of the
constant-coefficient operator, the exact steady profile of conduction through two
materials in series, conservation of the total, the maximum principle and symmetry."""
import numpy as np
import pytest

import oracle as O
from paper_2312_11740_amd import problems as G


def cos_mode(n, a, b, c):
    t = (np.arange(n) + 0.5) / n
    return (np.cos(np.pi * c * t)[:, None, None] * np.cos(np.pi * b * t)[None, :, None]
            * np.cos(np.pi * a * t)[None, None, :])


def neumann_eigenvalue(n, a, b, c):
    # cos(pi a (i+1/2)/n) is an eigenvector of the 1-D second difference with zero-flux
    # ends, eigenvalue -(4/h^2) sin^2(pi a / (2 n))
    return 4.0 * n * n * sum(np.sin(np.pi * q / (2 * n)) ** 2 for q in (a, b, c))


@pytest.mark.parametrize("sign,k", [(1.0, 0.7), (-1.0, 0.3)])
@pytest.mark.parametrize("mode", [(1, 0, 0), (2, 3, 1), (0, 0, 5), (4, 4, 4)])
def test_cosine_mode_decays_by_its_eigenvalue(sign, k, mode):
    # one phase everywhere: K of that phase on every face; the step divides each
    # eigenmode by 1 + dt K lambda
    n, dt = 12, 0.004
    fc = O.heat_faces(np.full((n, n, n), sign), 0.3, 0.7)
    t0 = cos_mode(n, *mode)
    t1, it, rel = O.heat_step(fc, t0, dt)
    assert rel <= 1e-13
    expect = t0 / (1.0 + dt * k * neumann_eigenvalue(n, *mode))
    assert np.max(np.abs(t1 - expect)) <= 1e-12


def test_two_materials_in_series_steady_profile():
    # a planar interface at z = 0.37 (inside a cell), K = 0.3 below, 2.0 above; heat
    # enters the bottom layer and leaves the top layer at the rate s per volume.  In
    # the steady state every plane between two layers carries the flux s h, and the
    # temperature falls by flux x resistance between neighbouring centres: h/K in one
    # material, theta h / K_a + (1 - theta) h / K_b across the interface.  The
    # discrete operator must give div(K grad T) = -f exactly for that profile.
    n, z0, kn, kp, s = 10, 0.37, 0.3, 2.0, 5.0
    h = 1.0 / n
    zc = (np.arange(n) + 0.5) * h
    phi = np.broadcast_to((zc - z0)[:, None, None], (n, n, n)).copy()
    fc = O.heat_faces(phi, kn, kp)
    prof = np.zeros(n)
    for k in range(n - 1):
        if zc[k] < z0 < zc[k + 1]:
            theta = (z0 - zc[k]) / h
            res = theta * h / kn + (1 - theta) * h / kp
        else:
            res = h / (kn if zc[k + 1] < z0 else kp)
        prof[k + 1] = prof[k] - s * h * res
    T = np.broadcast_to(prof[:, None, None], (n, n, n)).copy()
    f = np.zeros((n, n, n))
    f[0], f[-1] = s, -s
    div = T - O.heat_apply(fc, 1.0, T)          # = div(K grad T)
    assert np.max(np.abs(div + f)) <= 1e-12 * s


def test_total_is_conserved_with_two_phases():
    n, dt = 24, 0.01
    rng = np.random.default_rng(5)
    phi = G.bubble_phi(n, [(0.4, 0.5, 0.45), (0.7, 0.3, 0.6)], [0.2, 0.12])
    fc = O.heat_faces(phi, 0.05, 1.0)
    t0 = rng.uniform(0.0, 1.0, (n, n, n))
    f = rng.standard_normal((n, n, n))
    t1, _, rel = O.heat_step(fc, t0, dt, src=f)
    assert rel <= 1e-13
    total = t0.sum() + dt * f.sum()
    assert abs(t1.sum() - total) <= 1e-11 * np.abs(t0).sum()


def test_maximum_principle():
    n, dt = 20, 0.05
    rng = np.random.default_rng(6)
    phi = G.bubble_phi(n, [(0.5, 0.5, 0.5)], [0.3])
    fc = O.heat_faces(phi, 0.02, 1.0)
    t0 = rng.uniform(-1.0, 2.0, (n, n, n))
    t1, _, _ = O.heat_step(fc, t0, dt)
    assert t1.min() >= t0.min() - 1e-12 and t1.max() <= t0.max() + 1e-12
    # and it smooths: the spread shrinks
    assert t1.max() - t1.min() < t0.max() - t0.min()


def test_heat_matrix_is_symmetric_positive():
    n = 14
    rng = np.random.default_rng(7)
    phi = G.bubble_phi(n, [(0.45, 0.55, 0.5)], [0.27]) + 0.01 * rng.standard_normal((n, n, n))
    fc = O.heat_faces(phi, 0.1, 3.0)
    x, y = rng.standard_normal((2, n, n, n))
    hx, hy = O.heat_apply(fc, 0.02, x), O.heat_apply(fc, 0.02, y)
    assert abs(np.vdot(y, hx) - np.vdot(x, hy)) <= 1e-12 * np.abs(y * hx).sum()
    assert np.vdot(x, hx) >= np.vdot(x, x)   # I - dt A with A negative semidefinite


def test_zero_dt_is_identity_and_long_steps_flatten():
    n = 10
    rng = np.random.default_rng(8)
    kmin = 0.2
    fc = O.heat_faces(G.bubble_phi(n, [(0.5, 0.5, 0.5)], [0.3]), kmin, 1.0)
    t0 = rng.standard_normal((n, n, n))
    t1, it, _ = O.heat_step(fc, t0, 0.0)
    assert np.array_equal(t1, t0) and it == 1
    # every face conducts at least kmin, so on zero-mean fields -div(K grad) >= kmin
    # times the smallest nonzero eigenvalue of the Neumann Laplacian: one step shrinks
    # the deviation from the (kept) mean by at least 1 + dt kmin lambda_1 in the 2-norm
    dt = 10.0
    t2, _, rel = O.heat_step(fc, t0, dt)
    assert rel <= 1e-13
    assert abs(t2.mean() - t0.mean()) <= 1e-13 * np.abs(t0).max()
    shrink = 1.0 + dt * kmin * neumann_eigenvalue(n, 1, 0, 0)
    assert np.linalg.norm(t2 - t2.mean()) <= np.linalg.norm(t0 - t0.mean()) / shrink * (1 + 1e-9)


def test_heat_bad_arguments():
    n = 4
    fc = O.heat_faces(np.ones((n, n, n)), 1.0, 1.0)
    t0 = np.ones((n, n, n))
    with pytest.raises(O.OracleError):
        O.heat_step(fc, t0, -1.0)
    with pytest.raises(O.OracleError):
        O.heat_step(fc, t0, float("inf"))
    with pytest.raises(O.OracleError):
        O.heat_step(fc, t0, 0.1, tol=0.0)
