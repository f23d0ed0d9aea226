"""Pins of the level-set oracle (advection by the face velocities, re-distancing) against
closed forms, exact properties and symmetries; CPU only."""
import numpy as np
import pytest

import oracle as O


def centres(n):
    return (np.arange(n) + 0.5) / n


def along(axis, v, n):
    """A field varying along one axis (0 = x, 1 = y, 2 = z) of an [z][y][x] grid."""
    shape = [1, 1, 1]
    shape[2 - axis] = n
    return np.broadcast_to(np.asarray(v).reshape(shape), (n, n, n)).copy()


def faces_along(axis, value, n):
    """Face velocities: `value` on every interior face normal to `axis`, 0 elsewhere."""
    u = [np.zeros((n, n, n)) for _ in range(3)]
    sl = [slice(None)] * 3
    sl[2 - axis] = slice(1, None)
    u[axis][tuple(sl)] = value
    return u


def interior(axis, lo, hi, n):
    sl = [slice(None)] * 3
    sl[2 - axis] = slice(lo, n - hi)
    return tuple(sl)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("direction", [1.0, -1.0])
def test_advect_at_unit_courant_number_is_an_exact_shift(axis, direction):
    # u dt / h = 1: the upwind step moves every interior value by one cell, exactly for
    # integer-valued phi (the differences are exact)
    n = 16
    phi = np.random.default_rng(1 + axis).integers(-100, 100, (n, n, n)).astype(float)
    out = O.ls_advect(phi, faces_along(axis, direction, n), dt=1.0 / n)
    shifted = np.roll(phi, int(direction), axis=2 - axis)
    assert np.array_equal(out[interior(axis, 1, 1, n)], shifted[interior(axis, 1, 1, n)])


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_advect_linear_field(axis):
    # upwind differences are exact for a linear profile: phi - dt u a away from walls
    n = 32
    a, u, dt = 0.5, -0.75, 0.01
    phi = along(axis, 0.25 + a * centres(n), n)
    out = O.ls_advect(phi, faces_along(axis, u, n), dt)
    ref = phi - dt * u * a
    sel = interior(axis, 1, 1, n)
    assert np.max(np.abs(out[sel] - ref[sel])) <= 1e-14


def test_advect_reflection_symmetry():
    # mirroring x -> 1 - x together with the velocity gives the mirrored step, exactly
    n = 20
    rng = np.random.default_rng(5)
    phi = rng.standard_normal((n, n, n))
    u = [rng.standard_normal((n, n, n)) for _ in range(3)]
    u[0][:, :, 0] = 0.0
    u[1][:, 0, :] = 0.0
    u[2][0, :, :] = 0.0
    out = O.ls_advect(phi, u, 0.003)
    # mirrored fields: the low face of mirrored cell i is the high face of cell n-1-i
    ux_m = np.zeros_like(u[0])
    ux_m[:, :, 1:] = -u[0][:, :, 1:][:, :, ::-1]
    um = [ux_m, u[1][:, :, ::-1].copy(), u[2][:, :, ::-1].copy()]
    out_m = O.ls_advect(phi[:, :, ::-1].copy(), um, 0.003)
    assert np.array_equal(out_m, out[:, :, ::-1])


def test_advect_translates_a_sphere():
    # a sphere moved by a uniform upward velocity: the centroid of the phi < 0 region
    # travels u t to within half a cell (first-order scheme)
    n = 32
    h = 1.0 / n
    x = centres(n)
    X, Y, Z = x[None, None, :], x[None, :, None], x[:, None, None]
    phi = np.sqrt((X - 0.5) ** 2 + (Y - 0.45) ** 2 + (Z - 0.4) ** 2) - 0.2
    phi0 = phi.copy()
    u = faces_along(2, 1.0, n)
    for _ in range(16):
        phi = O.ls_advect(phi, u, 0.5 * h)
    zc = lambda p: np.broadcast_to(Z, p.shape)[p < 0].mean()
    assert abs((zc(phi) - zc(phi0)) - 16 * 0.5 * h) <= 0.5 * h


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_reinit_keeps_a_planar_distance(axis, sign):
    # a planar signed distance has |grad phi| = 1 everywhere (walls included): a fixed
    # point of the re-distancing step
    n = 24
    phi = along(axis, sign * (centres(n) - 0.37), n)
    out = O.ls_reinit(phi, phi, 20, 0.5 / n)
    assert np.max(np.abs(out - phi)) <= 1e-14


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_reinit_restores_unit_slope(sign):
    # phi = 3 (x - 0.37) relaxes to slope 1 everywhere; the zero crossing moves by less
    # than a quarter cell (first-order scheme) and no cell changes side
    n = 32
    h = 1.0 / n
    x = centres(n)
    phi = along(0, sign * 3 * (x - 0.37), n)
    out = O.ls_reinit(phi, phi, 200, 0.5 * h)
    prof = out[5, 7, :]
    slope = np.diff(prof) / h * sign
    assert np.all(np.abs(slope - 1.0) <= 1e-12)
    i = int(np.nonzero(np.sign(prof[:-1]) != np.sign(prof[1:]))[0][0])
    xz = x[i] - prof[i] * (x[i + 1] - x[i]) / (prof[i + 1] - prof[i])
    assert abs(xz - 0.37) <= 0.25 * h
    assert np.array_equal(np.sign(out), np.sign(phi))


def test_reinit_of_a_sphere_distance():
    # an exact sphere distance: signs are kept and cells within two cells of the
    # interface move by less than a fifth of a cell
    n = 32
    h = 1.0 / n
    x = centres(n)
    X, Y, Z = x[None, None, :], x[None, :, None], x[:, None, None]
    phi = np.sqrt((X - 0.5) ** 2 + (Y - 0.45) ** 2 + (Z - 0.55) ** 2) - 0.25
    out = O.ls_reinit(phi, phi, 10, 0.5 * h)
    assert np.array_equal(np.sign(out), np.sign(phi))
    near = np.abs(phi) < 2 * h
    assert np.max(np.abs(out - phi)[near]) <= 0.2 * h


def test_reinit_zero_iterations_is_identity():
    n = 8
    phi = np.random.default_rng(2).standard_normal((n, n, n))
    assert np.array_equal(O.ls_reinit(phi, phi, 0, 0.01), phi)


def test_levelset_rejects_bad_arguments():
    n = 8
    phi = np.zeros((n, n, n))
    u = [np.zeros((n, n, n))] * 3
    with pytest.raises(Exception):
        O.ls_advect(phi, u, 0.0)
    with pytest.raises(Exception):
        O.ls_reinit(phi, phi, -1, 0.1)
