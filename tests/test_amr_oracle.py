"""Pins of the oracle's two-level composite grid (level-0 blocks, some covered by level-1
blocks of half the spacing; the finite-volume operator with flux matching at coarse-fine
faces, and the guard-cell fill between levels).

The operator is pinned by what holds for any conservative finite-volume Laplacian:
constants are in its null space, the volume-weighted sum of A x vanishes, diag(V) A is
symmetric and negative semi-definite; by its reductions: with nothing refined it is the
uniform operator at the coarse spacing, with everything refined the uniform operator at
the fine spacing; and by brute force on tiny grids, where the leaf cells are boxes and
faces are found from the geometry alone.  The fill is pinned by its reductions to the
uniform fill and by the leaf field's volume average over each guard cell."""
import itertools

import numpy as np
import pytest

import oracle as O
from paper_2312_11740_amd import problems as G

RN, RP = 1.0, 1e-3


def level_phis(n0, seed):
    rng = np.random.default_rng(seed)
    cs = [tuple(rng.uniform(0.3, 0.7, 3))]
    rs = [rng.uniform(0.15, 0.25)]
    return G.bubble_phi(n0, cs, rs), G.bubble_phi(2 * n0, cs, rs)


def random_flags(m, seed, frac=0.4):
    f = (np.random.default_rng(seed).random((m, m, m)) < frac).astype(np.uint8)
    return f


def leaf_mask1(flags, nb):
    """(2 n0)^3 bool: level-1 cells that are leaves."""
    return np.repeat(np.repeat(np.repeat(flags, 2 * nb, 0), 2 * nb, 1), 2 * nb, 2).astype(bool)


def leaf_mask0(flags, nb):
    return ~np.repeat(np.repeat(np.repeat(flags, nb, 0), nb, 1), nb, 2).astype(bool)


def volumes(n0):
    return 1.0 / n0 ** 3, 1.0 / (2 * n0) ** 3


def wdot(flags, nb, a0, a1, b0, b1):
    n0 = a0.shape[0]
    v0, v1 = volumes(n0)
    m0, m1 = leaf_mask0(flags, nb), leaf_mask1(flags, nb)
    return v0 * np.sum((a0 * b0)[m0]) + v1 * np.sum((a1 * b1)[m1])


@pytest.mark.parametrize("n0,nb,seed", [(8, 4, 1), (8, 2, 2), (12, 4, 3)])
def test_constants_are_annihilated(n0, nb, seed):
    p0, p1 = level_phis(n0, seed)
    flags = random_flags(n0 // nb, seed)
    y0, y1 = O.amr_apply(flags, nb, p0, p1, np.full_like(p0, 2.5), np.full_like(p1, 2.5), RN, RP)
    assert np.all(y0 == 0.0) and np.all(y1 == 0.0)


@pytest.mark.parametrize("n0,nb,seed", [(8, 4, 1), (8, 2, 2), (12, 4, 3)])
def test_conservation_symmetry_definiteness(n0, nb, seed):
    p0, p1 = level_phis(n0, seed)
    flags = random_flags(n0 // nb, seed + 10)
    assert 0 < flags.sum() < flags.size
    rng = np.random.default_rng(seed)
    x0, x1, z0, z1 = (rng.standard_normal(p.shape) for p in (p0, p1, p0, p1))
    ax0, ax1 = O.amr_apply(flags, nb, p0, p1, x0, x1, RN, RP)
    az0, az1 = O.amr_apply(flags, nb, p0, p1, z0, z1, RN, RP)
    one0, one1 = np.ones_like(p0), np.ones_like(p1)
    v0, v1 = volumes(n0)
    scale = v0 * np.abs(ax0).sum() + v1 * np.abs(ax1).sum()
    # every flux leaves one leaf cell and enters another
    assert abs(wdot(flags, nb, one0, one1, ax0, ax1)) < 1e-13 * scale
    # diag(V) A symmetric
    s1 = wdot(flags, nb, z0, z1, ax0, ax1)
    s2 = wdot(flags, nb, x0, x1, az0, az1)
    assert abs(s1 - s2) < 1e-12 * max(abs(s1), 1.0)
    # and negative semi-definite (x not constant: strictly negative)
    assert wdot(flags, nb, x0, x1, ax0, ax1) < 0.0
    # non-leaf cells are left at zero
    assert np.all(ax0[~leaf_mask0(flags, nb)] == 0.0)
    assert np.all(ax1[~leaf_mask1(flags, nb)] == 0.0)


@pytest.mark.parametrize("n0,nb", [(8, 4), (12, 3)])
def test_reduces_to_the_uniform_operator(n0, nb):
    p0, p1 = level_phis(n0, 5)
    rng = np.random.default_rng(7)
    x0, x1 = rng.standard_normal(p0.shape), rng.standard_normal(p1.shape)
    m = n0 // nb
    none = np.zeros((m, m, m), np.uint8)
    y0, y1 = O.amr_apply(none, nb, p0, p1, x0, x1, RN, RP)
    ref0 = O.apply(O.faces(p0, RN, RP), x0)
    assert np.allclose(y0, ref0, rtol=1e-13, atol=1e-13 * np.abs(ref0).max())
    assert np.all(y1 == 0.0)
    y0, y1 = O.amr_apply(np.ones_like(none), nb, p0, p1, x0, x1, RN, RP)
    ref1 = O.apply(O.faces(p1, RN, RP), x1)
    assert np.allclose(y1, ref1, rtol=1e-13, atol=1e-13 * np.abs(ref1).max())
    assert np.all(y0 == 0.0)


def brute_force_apply(flags, nb, p0, p1, x0, x1):
    """Leaf cells as boxes on the integer lattice of the fine level (a level-0 cell spans
    2 units, a level-1 cell 1); two leaves share a face when their boxes touch along one
    axis and overlap with positive area in the other two.  The flux through it is
    area * beta * (x_b - x_a) / (distance of the centres along the axis), beta the
    series-resistance coefficient of the two cells (lower cell first)."""
    n0 = p0.shape[0]
    h1 = 0.5 / n0
    leaves = []   # (lo(3), size, level, index, phi, x)
    for K, J, I in itertools.product(range(n0), repeat=3):
        if not flags[K // nb, J // nb, I // nb]:
            leaves.append(((2 * I, 2 * J, 2 * K), 2, 0, (K, J, I), p0[K, J, I], x0[K, J, I]))
    for k, j, i in itertools.product(range(2 * n0), repeat=3):
        if flags[k // (2 * nb), j // (2 * nb), i // (2 * nb)]:
            leaves.append(((i, j, k), 1, 1, (k, j, i), p1[k, j, i], x1[k, j, i]))

    def beta(pa, pb):
        ra = RP if pa > 0 else RN
        rb = RP if pb > 0 else RN
        if (pa > 0) == (pb > 0):
            return 1.0 / ra
        t = abs(pa) / (abs(pa) + abs(pb))
        return 1.0 / (t * ra + (1 - t) * rb)

    # index the leaves by the fine lattice points they cover
    owner = {}
    for li, (lo, s, *_rest) in enumerate(leaves):
        for d in itertools.product(range(s), repeat=3):
            owner[(lo[0] + d[0], lo[1] + d[1], lo[2] + d[2])] = li
    acc = np.zeros(len(leaves))
    for a, (lo, s, lev, idx, pa, xa) in enumerate(leaves):
        for ax in range(3):
            # neighbours across the upper face of a
            nbrs = set()
            for d in itertools.product(range(s), repeat=2):
                q = list(lo)
                q[ax] = lo[ax] + s
                o = [e for e in range(3) if e != ax]
                q[o[0]] += d[0]
                q[o[1]] += d[1]
                if tuple(q) in owner:
                    nbrs.add(owner[tuple(q)])
            for b in nbrs:
                lob, sb, _, _, pb, xb = leaves[b]
                o = [e for e in range(3) if e != ax]
                area = 1.0
                for e in o:
                    area *= max(0, min(lo[e] + s, lob[e] + sb) - max(lo[e], lob[e]))
                dist = (lob[ax] + sb / 2) - (lo[ax] + s / 2)
                flux = area * h1 * h1 * beta(pa, pb) * (xb - xa) / (dist * h1)
                acc[a] += flux
                acc[b] -= flux
    y0, y1 = np.zeros_like(x0), np.zeros_like(x1)
    for a, (lo, s, lev, idx, *_r) in enumerate(leaves):
        vol = (s * h1) ** 3
        (y1 if lev else y0)[idx] = acc[a] / vol
    return y0, y1


@pytest.mark.parametrize("n0,nb,seed", [(4, 2, 1), (4, 2, 2), (6, 2, 3)])
def test_brute_force_geometry(n0, nb, seed):
    p0, p1 = level_phis(n0, seed)
    flags = random_flags(n0 // nb, seed + 20, 0.5)
    if flags.sum() in (0, flags.size):
        flags.flat[0] ^= 1
    rng = np.random.default_rng(seed)
    x0, x1 = rng.standard_normal(p0.shape), rng.standard_normal(p1.shape)
    y0, y1 = O.amr_apply(flags, nb, p0, p1, x0, x1, RN, RP)
    b0, b1 = brute_force_apply(flags, nb, p0, p1, x0, x1)
    scale = max(np.abs(b0).max(), np.abs(b1).max())
    assert np.allclose(y0, b0, rtol=1e-12, atol=1e-12 * scale)
    assert np.allclose(y1, b1, rtol=1e-12, atol=1e-12 * scale)


def prolong(v0):
    return np.repeat(np.repeat(np.repeat(v0, 2, 0), 2, 1), 2, 2)


def restrict(v1):
    n = v1.shape[0] // 2
    return v1.reshape(n, 2, n, 2, n, 2).mean(axis=(1, 3, 5))


@pytest.mark.parametrize("n0,nb,g", [(8, 4, 1), (8, 2, 2), (12, 4, 2)])
def test_fill_reductions(n0, nb, g):
    rng = np.random.default_rng(n0 + nb + g)
    m = n0 // nb
    flags = random_flags(m, g, 0.5)
    v0 = rng.standard_normal((n0, n0, n0))
    # a level-1 field that is the prolongation of level 0: both levels fill as uniform grids
    b0, b1 = O.amr_fill(flags, nb, g, v0, prolong(v0))
    assert np.array_equal(b0, O.blocks_fill_guards(O.blocks_scatter(v0, nb, g), n0, nb, g))
    assert np.array_equal(b1, O.blocks_fill_guards(O.blocks_scatter(prolong(v0), nb, g),
                                                   2 * n0, nb, g))
    # nothing refined: level 0 as the uniform fill whatever level 1 holds
    v1 = rng.standard_normal((2 * n0,) * 3)
    b0, _ = O.amr_fill(np.zeros_like(flags), nb, g, v0, v1)
    assert np.array_equal(b0, O.blocks_fill_guards(O.blocks_scatter(v0, nb, g), n0, nb, g))
    # everything refined: level 1 as the uniform fill whatever level 0 holds
    _, b1 = O.amr_fill(np.ones_like(flags), nb, g, v0, v1)
    assert np.array_equal(b1, O.blocks_fill_guards(O.blocks_scatter(v1, nb, g), 2 * n0, nb, g))


@pytest.mark.parametrize("n0,nb,g", [(8, 4, 1), (8, 2, 2)])
def test_fill_is_the_leaf_average_over_the_guard_cell(n0, nb, g):
    rng = np.random.default_rng(3 * n0 + g)
    m = n0 // nb
    flags = random_flags(m, 7 + g, 0.5)
    v0, v1 = rng.standard_normal((n0,) * 3), rng.standard_normal((2 * n0,) * 3)
    b0, b1 = O.amr_fill(flags, nb, g, v0, v1)
    leaf = np.where(leaf_mask1(flags, nb), v1, prolong(v0))   # leaf field on the fine lattice
    mir = lambda a, n: -1 - a if a < 0 else (2 * n - 1 - a if a >= n else a)
    P = nb + 2 * g
    for lev, blocks, n in ((0, b0, n0), (1, b1, 2 * n0)):
        nbx = n // nb
        for blk in rng.integers(0, nbx ** 3, 12):
            bi, bj, bk = blk % nbx, (blk // nbx) % nbx, blk // nbx ** 2
            for _ in range(60):
                lk, lj, li = rng.integers(-g, nb + g, 3)
                if all(0 <= c < nb for c in (li, lj, lk)):
                    continue
                I, J, K = (mir(b * nb + c, n) for b, c in ((bi, li), (bj, lj), (bk, lk)))
                if lev == 0:
                    want = leaf[2 * K:2 * K + 2, 2 * J:2 * J + 2, 2 * I:2 * I + 2].mean()
                else:
                    want = leaf[K, J, I]
                got = blocks[blk, lk + g, lj + g, li + g]
                assert got == pytest.approx(want, rel=1e-15, abs=1e-15)
    assert b0.shape == (m ** 3, P, P, P)


def test_refinement_flags_follow_the_interface():
    p0, _ = level_phis(16, 4)
    flags = G.refine_near_interface(p0, 4, 2.0 / 16)
    assert 0 < flags.sum() < flags.size
    near = np.abs(p0) < 2.0 / 16
    assert np.array_equal(flags.astype(bool),
                          near.reshape(4, 4, 4, 4, 4, 4).any(axis=(1, 3, 5)))


def test_rejects_bad_arguments():
    p0, p1 = level_phis(8, 1)
    with pytest.raises(O.OracleError):
        O.amr_apply(np.zeros((3, 3, 3), np.uint8), 3, p0, p1, p0, p1, RN, RP)   # 8 % 3
    with pytest.raises(O.OracleError):
        O.amr_fill(np.zeros((2, 2, 2), np.uint8), 4, 5, p0, p1)                 # g > nb


def test_solve_reaches_its_residual():
    n0, nb = 8, 2
    p0, p1 = level_phis(n0, 31)
    flags = random_flags(n0 // nb, 31, 0.4)
    rng = np.random.default_rng(31)
    b0, b1 = rng.standard_normal(p0.shape), rng.standard_normal(p1.shape)
    x0, x1, it, rel = O.amr_solve(flags, nb, p0, p1, b0, b1, 1e-3, 1.0, rtol=1e-11)
    assert rel <= 1e-11 and it > 0
    # recomputed from the operator, with b's weighted mean removed
    m0, m1 = leaf_mask0(flags, nb), leaf_mask1(flags, nb)
    v0, v1 = volumes(n0)
    mean = v0 * b0[m0].sum() + v1 * b1[m1].sum()
    a0, a1 = O.amr_apply(flags, nb, p0, p1, x0, x1, 1e-3, 1.0)
    r0, r1 = np.where(m0, b0 - mean - a0, 0.0), np.where(m1, b1 - mean - a1, 0.0)
    bb0, bb1 = np.where(m0, b0 - mean, 0.0), np.where(m1, b1 - mean, 0.0)
    assert np.sqrt(wdot(flags, nb, r0, r1, r0, r1)) <= 1.01e-11 * np.sqrt(wdot(flags, nb, bb0, bb1, bb0, bb1))
    assert abs(wdot(flags, nb, x0, x1, np.ones_like(x0), np.ones_like(x1))) < 1e-14
    assert np.all(x0[~m0] == 0.0) and np.all(x1[~m1] == 0.0)


def test_solve_recovers_a_manufactured_solution():
    n0, nb = 8, 4
    p0, p1 = level_phis(n0, 32)
    flags = random_flags(n0 // nb, 32, 0.5)
    m0, m1 = leaf_mask0(flags, nb), leaf_mask1(flags, nb)
    rng = np.random.default_rng(32)
    s0, s1 = np.where(m0, rng.standard_normal(p0.shape), 0.0), np.where(m1, rng.standard_normal(p1.shape), 0.0)
    v0, v1 = volumes(n0)
    sm = v0 * s0[m0].sum() + v1 * s1[m1].sum()
    s0, s1 = np.where(m0, s0 - sm, 0.0), np.where(m1, s1 - sm, 0.0)
    b0, b1 = O.amr_apply(flags, nb, p0, p1, s0, s1, RN, RP)
    x0, x1, it, rel = O.amr_solve(flags, nb, p0, p1, b0, b1, RN, RP, rtol=1e-13)
    scale = max(np.abs(s0).max(), np.abs(s1).max())
    assert np.abs(x0 - s0).max() <= 1e-6 * scale and np.abs(x1 - s1).max() <= 1e-6 * scale


def test_solve_without_refinement_is_the_uniform_solve():
    n0, nb = 8, 4
    p0, p1 = level_phis(n0, 33)
    b0 = np.random.default_rng(33).standard_normal(p0.shape)
    none = np.zeros((2, 2, 2), np.uint8)
    x0, _, _, rel = O.amr_solve(none, nb, p0, p1, b0, np.zeros_like(p1), RN, RP, rtol=1e-13)
    b = b0 - b0.mean()
    ref = O.solve_jacobi_pcg(O.faces(p0, RN, RP), b, tol=1e-13)
    ref = ref[0] if isinstance(ref, tuple) else ref
    assert np.abs(x0 - ref).max() <= 1e-7 * np.abs(ref).max()
