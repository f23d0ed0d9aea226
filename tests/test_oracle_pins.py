"""Pins of the FP64 CPU oracle against facts the mathematics fixes.

Each test checks the oracle against something other than itself: closed forms of the
discrete operator, exact discrete solutions of problems whose continuous solution is
known, invariants, symmetries, and brute-force dense solves on tiny grids.  Chosen so
that a plausible slip (a dropped term, a wrong sign, an off-by-one face, a swapped
interpolation weight, a transposed axis) fails one of them.

Grid arrays are (n, n, n) indexed [k, j, i]; cell centres at (i + 1/2)/n.
"""
import math

import numpy as np
import pytest

from paper_2312_11740_amd import problems as G


def centres(n):
    return (np.arange(n) + 0.5) / n


def mesh(n):
    x = centres(n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return X, Y, Z


def zm(a):
    return a - a.mean()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# ---------------------------------------------------------------------------------
# P1: eigenfunctions of the constant-coefficient operator with Neumann walls
# ---------------------------------------------------------------------------------
@pytest.mark.parametrize("n", [8, 13, 16])
@pytest.mark.parametrize("kv", [(1, 0, 0), (1, 1, 1), (3, 2, 1), (0, 2, 5)])
def test_p1_eigenfunctions(oracle, n, kv):
    # with rho = 2 on both sides every face carries 1/2, whatever phi is
    X, Y, Z = mesh(n)
    phi = G.bubble_phi(n, [(0.4, 0.55, 0.5)], [0.27])
    fc = oracle.faces(phi, 2.0, 2.0)
    v = np.cos(np.pi * kv[0] * X) * np.cos(np.pi * kv[1] * Y) * np.cos(np.pi * kv[2] * Z)
    h = 1.0 / n
    lam = -(4.0 / h ** 2) * sum(math.sin(math.pi * kd * h / 2) ** 2 for kd in kv) * 0.5
    Av = oracle.apply(fc, v)
    assert np.max(np.abs(Av - lam * v)) <= 1e-12 * max(abs(lam), 1.0)


# ---------------------------------------------------------------------------------
# P2: manufactured solution, constant coefficient: the exact discrete solution
# ---------------------------------------------------------------------------------
@pytest.mark.parametrize("n,err_expected", [(16, None), (32, 8.0358e-4), (64, 2.0082e-4)])
def test_p2_mms_second_order(oracle, n, err_expected):
    X, Y, Z = mesh(n)
    pstar = np.cos(np.pi * X) * np.cos(np.pi * Y) * np.cos(np.pi * Z)
    phi = G.bubble_phi(n, [(0.5, 0.5, 0.5)], [0.25])
    f = -3 * np.pi ** 2 * pstar
    p, d, info = oracle.solve(phi, f, 1.0, 1.0, 0.0, tol=1e-13)
    h = 1.0 / n
    factor = (np.pi * h / 2) ** 2 / math.sin(np.pi * h / 2) ** 2
    assert rel(p, factor * pstar) < 1e-10
    err = rel(p, pstar)
    assert abs(err - (factor - 1.0)) < 1e-10
    assert abs(err - np.pi ** 2 * h ** 2 / 12) < 0.01 * err
    if err_expected is not None:
        assert abs(err - err_expected) < 5e-4 * err_expected


# ---------------------------------------------------------------------------------
# P3: solve inverts apply with interface coefficients
# ---------------------------------------------------------------------------------
@pytest.mark.parametrize("ratio", [10.0, 1000.0])
def test_p3_discrete_exactness(oracle, ratio):
    n = 32
    X, Y, Z = mesh(n)
    phi = G.bubble_phi(n, [(0.5, 0.5, 0.5)], [0.25])
    fc = oracle.faces(phi, 1.0 / ratio, 1.0)
    pstar = zm(np.cos(np.pi * X) * np.cos(np.pi * Y) * np.cos(np.pi * Z) + X * Y)
    f = oracle.apply(fc, pstar)
    p, info = oracle.solve_mg_pcg(fc, f, tol=1e-14)
    assert rel(p, pstar) < 1e-9


# ---------------------------------------------------------------------------------
# P4: planar interface -> exact piecewise-quadratic solution of the 1D problem
# ---------------------------------------------------------------------------------
def planar_case(n, x0, rho_left, rho_right):
    """Flux F(x) continuous, piecewise linear with kinks at two cell centres; f is its
    exact cell-wise divergence.  With F constant around the interface the continuous
    solution u = int_0^x F rho is reproduced exactly at cell centres by a
    series-resistance face coefficient (and by nothing else)."""
    h = 1.0 / n
    ia, ib = n // 4, (3 * n) // 4
    xa, xb = (ia + 0.5) * h, (ib + 0.5) * h
    assert xa < x0 < xb

    def F(x):
        return np.where(x <= xa, x / xa, np.where(x <= xb, 1.0, (1.0 - x) / (1.0 - xb)))

    faces_lo = np.arange(n) * h
    f1 = (F(faces_lo + h) - F(faces_lo)) / h

    def u(x):
        # int_0^x F(s) rho(s) ds, rho = rho_left for s < x0 else rho_right (xa < x0 < xb)
        x = np.asarray(x, dtype=float)
        out = np.empty_like(x)
        ua = rho_left * xa / 2
        u0 = ua + rho_left * (x0 - xa)
        ub = u0 + rho_right * (xb - x0)
        m1 = x <= xa
        m2 = (x > xa) & (x <= x0)
        m3 = (x > x0) & (x <= xb)
        m4 = x > xb
        out[m1] = rho_left * x[m1] ** 2 / (2 * xa)
        out[m2] = ua + rho_left * (x[m2] - xa)
        out[m3] = u0 + rho_right * (x[m3] - x0)
        s = x[m4] - xb
        out[m4] = ub + rho_right * (s - s ** 2 / (2 * (1.0 - xb)) - s * xb / (1.0 - xb) + xb * s / (1.0 - xb))
        return out

    return f1, u(centres(n))


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("orient", [1, -1])
@pytest.mark.parametrize("n,ratio", [(16, 1000.0), (32, 10.0), (24, 1000.0)])
def test_p4_planar_interface_exact(oracle, axis, orient, n, ratio):
    x0 = 0.37 + 1e-3 * math.sqrt(2)
    rho_neg, rho_pos = 1.0 / ratio, 1.0
    c = centres(n)
    phi1 = orient * (c - x0)                   # "+" right of x0 when orient = 1
    rho_left = rho_neg if orient == 1 else rho_pos
    rho_right = rho_pos if orient == 1 else rho_neg
    f1, u1 = planar_case(n, x0, rho_left, rho_right)
    shape = [1, 1, 1]
    shape[2 - axis] = n                         # array axes are [k, j, i]
    phi = np.broadcast_to(phi1.reshape(shape), (n, n, n)).copy()
    f = np.broadcast_to(f1.reshape(shape), (n, n, n)).copy()
    u = np.broadcast_to(u1.reshape(shape), (n, n, n)).copy()
    p, d, info = oracle.solve(phi, f, rho_neg, rho_pos, 0.0, tol=1e-14)
    assert abs(d["mean"]) < 1e-12
    assert np.max(np.abs(p - zm(u))) < 1e-9 * np.max(np.abs(u))


def test_p4_arithmetic_mean_would_fail(oracle):
    # the planar pin is sharp: the same case with an averaged face density is off
    n, x0, ratio = 16, 0.37 + 1e-3 * math.sqrt(2), 1000.0
    c = centres(n)
    f1, u1 = planar_case(n, x0, 1.0 / ratio, 1.0)
    phi = np.broadcast_to((c - x0)[None, None, :], (n, n, n)).copy()
    f = np.broadcast_to(f1[None, None, :], (n, n, n)).copy()
    bx, by, bz = oracle.faces(phi, 1.0 / ratio, 1.0)
    i = int(np.floor(x0 * n - 0.5)) + 1        # the crossing x-face
    theta = abs(phi[0, 0, i - 1]) / (abs(phi[0, 0, i - 1]) + abs(phi[0, 0, i]))
    assert bx[0, 0, i] == pytest.approx(1.0 / (theta / ratio + (1 - theta) * 1.0), rel=1e-15)
    bx2 = bx.copy()
    bx2[:, :, i] = theta * ratio + (1 - theta) * 1.0      # arithmetic mean of 1/rho
    b, _ = oracle.rhs(f)
    p2, _ = oracle.solve_mg_pcg((bx2, by, bz), b, tol=1e-13)
    u = np.broadcast_to(u1[None, None, :], (n, n, n))
    assert np.max(np.abs(p2 - zm(u))) > 1e-3 * np.max(np.abs(u))


# ---------------------------------------------------------------------------------
# P5: Laplace jump: p = C + sigma*kappa on the "+" side, exactly
# ---------------------------------------------------------------------------------
@pytest.mark.parametrize("ratio", [1.0, 1000.0])
@pytest.mark.parametrize("orient", [1, -1])
def test_p5_laplace_jump_exact_kappa(oracle, ratio, orient):
    n, R, sigma = 32, 0.25, 0.01
    d0 = G.bubble_phi(n, [(0.5, 0.5, 0.5)], [R])     # |x-c| - R
    phi = orient * d0
    # kappa = -div(grad phi/|grad phi|) = -2/R (orient=1) or +2/R (orient=-1)
    kappa = np.full((n, n, n), -orient * 2.0 / R)
    rho_in, rho_out = 1.0 / ratio, 1.0
    rho_neg, rho_pos = (rho_in, rho_out) if orient == 1 else (rho_out, rho_in)
    f = np.zeros((n, n, n))
    p, d, info = oracle.solve(phi, f, rho_neg, rho_pos, sigma, tol=1e-14, kappa_override=kappa)
    inside = (d0 <= 0).astype(float)
    expect = zm(2 * sigma / R * inside)             # Young-Laplace: p_in - p_out = 2 sigma/R
    assert np.max(np.abs(p - expect)) < 1e-11 * (2 * sigma / R)
    assert abs(np.sum(d["jterm"])) < 1e-12 * np.sum(np.abs(d["jterm"]))


@pytest.mark.parametrize("orient", [1, -1])
def test_p5_jump_interpolates_kappa_at_interface(oracle, orient):
    # planar interface, affine kappa field: the jump must be sigma*kappa(x0) exactly
    n, sigma = 16, 1.0
    x0 = 0.43 + 1e-3 * math.sqrt(3)
    c = centres(n)
    phi = np.broadcast_to(orient * (c - x0)[None, None, :], (n, n, n)).copy()
    k0, k1 = 0.3, 2.0
    kappa = np.broadcast_to((k0 + k1 * c)[None, None, :], (n, n, n)).copy()
    p, d, info = oracle.solve(phi, np.zeros((n, n, n)), 0.01, 1.0, sigma, tol=1e-14,
                              kappa_override=kappa)
    plus = (phi > 0).astype(float)
    expect = zm(sigma * (k0 + k1 * x0) * plus)
    assert np.max(np.abs(p - expect)) < 1e-11


def test_p5_laplace_jump_converges_with_fd_kappa(oracle):
    R, sigma = 0.25, 0.01
    errs = []
    for n in (16, 32, 64):
        phi = G.bubble_phi(n, [(0.5, 0.5, 0.5)], [R])
        p, d, info = oracle.solve(phi, np.zeros((n, n, n)), 0.001, 1.0, sigma, tol=1e-13)
        inside = phi <= 0
        jump = p[inside].mean() - p[~inside].mean()
        errs.append(abs(jump - 2 * sigma / R))
    assert errs[2] < 0.02 * 2 * sigma / R
    assert errs[2] < errs[0]


# ---------------------------------------------------------------------------------
# P6: radial solution with a density jump and continuous flux (convergence)
# ---------------------------------------------------------------------------------
def radial_case(n, r0=0.25, r1=0.45, beta_in=1000.0, beta_out=1.0):
    X, Y, Z = mesh(n)
    r = np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 0.5) ** 2)
    q = np.clip(r1 ** 2 - r ** 2, 0.0, None)
    f = np.where(r < r1, 3 * q ** 2 * (r1 ** 2 - 3 * r ** 2), 0.0)
    u_in = (r1 ** 8 - q ** 4) / (8 * beta_in)
    u_r0 = (r1 ** 8 - (r1 ** 2 - r0 ** 2) ** 4) / (8 * beta_in)
    u_out = u_r0 + ((r1 ** 2 - r0 ** 2) ** 4 - q ** 4) / (8 * beta_out)
    u = np.where(r <= r0, u_in, u_out)
    phi = r - r0
    return phi, f, u


def test_p6_radial_kink_convergence(oracle):
    errs2, errsi = [], []
    for n in (32, 64, 128):
        phi, f, u = radial_case(n)
        p, d, info = oracle.solve(phi, f, 1.0 / 1000.0, 1.0, 0.0, tol=1e-12)
        e = p - zm(u)
        errs2.append(np.sqrt(np.mean(e ** 2)) / np.sqrt(np.mean(zm(u) ** 2)))
        errsi.append(np.max(np.abs(e)) / np.max(np.abs(zm(u))))
    o2 = [math.log2(errs2[i] / errs2[i + 1]) for i in range(2)]
    oi = [math.log2(errsi[i] / errsi[i + 1]) for i in range(2)]
    assert min(o2) >= 0.9, (errs2, o2)
    assert min(oi) >= 0.9, (errsi, oi)
    assert errs2[-1] < 1e-2


# ---------------------------------------------------------------------------------
# P7: operator structure
# ---------------------------------------------------------------------------------
def test_p7_symmetry_nullspace_definiteness(oracle):
    n = 12
    rng = np.random.default_rng(7)
    phi = G.bubble_phi(n, [(0.45, 0.5, 0.55), (0.2, 0.2, 0.8)], [0.2, 0.1])
    fc = oracle.faces(phi, 0.001, 1.0)
    x, y = rng.standard_normal((2, n, n, n))
    Ax, Ay = oracle.apply(fc, x), oracle.apply(fc, y)
    assert abs(np.vdot(x, Ay) - np.vdot(Ax, y)) < 1e-13 * np.linalg.norm(x) * np.linalg.norm(Ay)
    assert np.all(oracle.apply(fc, np.ones((n, n, n))) == 0.0)
    for _ in range(5):
        z = rng.standard_normal((n, n, n))
        assert np.vdot(z, oracle.apply(fc, z)) < 0.0


def test_p7_dense_spectrum(oracle):
    n = 6
    phi = G.bubble_phi(n, [(0.5, 0.5, 0.5)], [0.3])
    fc = oracle.faces(phi, 0.01, 1.0)
    m = n ** 3
    A = np.empty((m, m))
    for c in range(m):
        e = np.zeros(m)
        e[c] = 1.0
        A[:, c] = oracle.apply(fc, e.reshape(n, n, n)).reshape(-1)
    assert np.allclose(A, A.T, rtol=0, atol=1e-12 * np.abs(A).max())
    w = np.linalg.eigvalsh(A)
    assert abs(w[-1]) < 1e-10 * abs(w[0])
    assert np.all(w[:-1] < -1e-6)


# ---------------------------------------------------------------------------------
# P8: brute force on tiny grids
# ---------------------------------------------------------------------------------
TINY = [
    (4, [(0.5, 0.5, 0.5)], [0.3], 10.0, 0.02),
    (6, [(0.4, 0.5, 0.6)], [0.28], 1000.0, 0.01),
    (8, [(0.3, 0.3, 0.3), (0.7, 0.68, 0.7)], [0.16, 0.18], 1000.0, 0.05),
    (12, [(0.25, 0.3, 0.3), (0.7, 0.7, 0.3), (0.5, 0.5, 0.75)], [0.12, 0.15, 0.14], 100.0, 0.01),
]


@pytest.mark.parametrize("n,cs,rs,ratio,sigma", TINY)
def test_p8_brute_force(oracle, n, cs, rs, ratio, sigma):
    rng = np.random.default_rng(n)
    phi = G.bubble_phi(n, cs, rs)
    f = rng.uniform(-1, 1, (n, n, n))
    d = oracle.pipeline(phi, f, 1.0 / ratio, 1.0, sigma)
    fc, b = d["faces"], d["b"]
    m = n ** 3
    A = np.empty((m, m))
    for c in range(m):
        e = np.zeros(m)
        e[c] = 1.0
        A[:, c] = oracle.apply(fc, e.reshape(n, n, n)).reshape(-1)
    p_ls = np.linalg.lstsq(A, b.reshape(-1), rcond=None)[0]
    p_ls = zm(p_ls).reshape(n, n, n)
    p_ch = zm(oracle.solve_dense(fc, b))
    p_j, ij = oracle.solve_jacobi_pcg(fc, b, tol=1e-14)
    scale = np.linalg.norm(p_ls)
    assert np.linalg.norm(p_ch - p_ls) < 1e-10 * scale
    assert np.linalg.norm(p_j - p_ls) < 1e-10 * scale
    if n >= 8:
        p_m, im = oracle.solve_mg_pcg(fc, b, tol=1e-14)
        assert np.linalg.norm(p_m - p_ls) < 1e-10 * scale


# ---------------------------------------------------------------------------------
# P9: compatibility of the jump term
# ---------------------------------------------------------------------------------
def test_p9_jump_term_sums_to_zero(oracle):
    pr = G.many_bubbles_problem(n=64, count=8, seed=3)
    d = oracle.pipeline(pr.phi, pr.f, pr.rho_neg, pr.rho_pos, pr.sigma)
    jt = d["jterm"]
    assert np.count_nonzero(jt) > 0
    assert abs(np.sum(jt)) <= 1e-12 * np.sum(np.abs(jt))
    # the jump term lives only on interface-adjacent cells
    assert np.all((jt != 0) <= (d["kappa"] != 0) | (jt == 0))


# ---------------------------------------------------------------------------------
# P10: symmetries and linearity
# ---------------------------------------------------------------------------------
def test_p10_reflection_and_permutation(oracle):
    n = 16
    rng = np.random.default_rng(11)
    phi = G.bubble_phi(n, [(0.35, 0.55, 0.5), (0.7, 0.3, 0.62)], [0.17, 0.12])
    f = rng.uniform(-1, 1, (n, n, n))
    args = (0.002, 1.0, 0.03)
    p, _, _ = oracle.solve(phi, f, *args, tol=1e-14)
    # reflect x -> 1 - x  (array axis 2)
    pr_, _, _ = oracle.solve(phi[:, :, ::-1].copy(), f[:, :, ::-1].copy(), *args, tol=1e-14)
    assert np.max(np.abs(pr_ - p[:, :, ::-1])) < 1e-11 * np.max(np.abs(p))
    # swap x and z
    pt, _, _ = oracle.solve(phi.transpose(2, 1, 0).copy(), f.transpose(2, 1, 0).copy(), *args, tol=1e-14)
    assert np.max(np.abs(pt - p.transpose(2, 1, 0))) < 1e-11 * np.max(np.abs(p))
    # cycle x -> y -> z
    pc, _, _ = oracle.solve(phi.transpose(1, 2, 0).copy(), f.transpose(1, 2, 0).copy(), *args, tol=1e-14)
    assert np.max(np.abs(pc - p.transpose(1, 2, 0))) < 1e-11 * np.max(np.abs(p))


def test_p10_linearity(oracle):
    n = 16
    rng = np.random.default_rng(12)
    phi = G.bubble_phi(n, [(0.5, 0.45, 0.5)], [0.22])
    f, g = rng.uniform(-1, 1, (2, n, n, n))
    a, b = 0.7, -2.5
    s = lambda q: oracle.solve(phi, q, 0.01, 1.0, 0.0, tol=1e-14)[0]
    lhs = s(a * f + b * g)
    rhs_ = a * s(f) + b * s(g)
    assert np.max(np.abs(lhs - rhs_)) < 1e-11 * np.max(np.abs(lhs))


# ---------------------------------------------------------------------------------
# Curvature: mean curvature of spheres and cylinders, second order
# ---------------------------------------------------------------------------------
def _kappa_error(oracle, n, kind):
    X, Y, Z = mesh(n)
    c = (0.47, 0.52, 0.5)
    R = 0.23
    if kind == "sphere":
        rr = np.sqrt((X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2)
        exact = -2.0 / rr
    else:
        rr = np.sqrt((X - c[0]) ** 2 + (Z - c[2]) ** 2)   # axis along y
        exact = -1.0 / rr
    phi = rr - R
    k = oracle.curvature(phi)
    mask = k != 0
    assert mask.sum() > 0
    return np.max(np.abs(k[mask] - exact[mask]))


@pytest.mark.parametrize("kind", ["sphere", "cylinder"])
def test_curvature_second_order(oracle, kind):
    e1 = _kappa_error(oracle, 32, kind)
    e2 = _kappa_error(oracle, 64, kind)
    assert e2 < 0.35 * e1          # ratio 4 expected
    assert e2 < 0.05


def test_curvature_planar_near_walls_is_zero(oracle):
    n = 16
    X, Y, Z = mesh(n)
    phi = 0.3 * X - 0.5 * Y + 0.2 * Z - 0.02          # planar, crosses walls
    k = oracle.curvature(phi)
    assert np.count_nonzero(phi > 0) > 0
    assert np.max(np.abs(k)) < 1e-9


def test_curvature_only_on_interface_cells(oracle):
    n = 16
    phi = G.bubble_phi(n, [(0.5, 0.5, 0.5)], [0.3])
    k = oracle.curvature(phi)
    s = phi > 0
    adj = np.zeros_like(s)
    for ax in range(3):
        d = np.diff(s.astype(int), axis=ax) != 0
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[ax] = slice(0, n - 1)
        hi[ax] = slice(1, n)
        adj[tuple(lo)] |= d
        adj[tuple(hi)] |= d
    assert np.array_equal(k != 0, adj)


def test_tie_break_phi_zero_is_minus_side(oracle):
    # phi == 0 exactly at the centre of cell 5 (0.34375 is exact in binary): that cell
    # belongs to the phi <= 0 side, so the jump sits between cells 5 and 6
    n, sigma, k0 = 16, 1.0, 0.7
    c = centres(n)
    phi1 = c - c[5]
    assert phi1[5] == 0.0
    phi = np.broadcast_to(phi1[None, None, :], (n, n, n)).copy()
    kappa = np.full((n, n, n), k0)
    p, d, info = oracle.solve(phi, np.zeros((n, n, n)), 0.01, 1.0, sigma, tol=1e-14,
                              kappa_override=kappa)
    expect = zm(sigma * k0 * (phi > 0).astype(float))
    assert np.max(np.abs(p - expect)) < 1e-11
    assert np.all(d["jterm"][:, :, 4] == 0.0) and np.all(d["jterm"][:, :, 5] != 0.0)
