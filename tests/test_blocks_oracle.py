"""Pins of the oracle's block-structured layout: scatter and gather invert each other,
guard cells of a linear field hold the field at the guard positions (its mirror image
across a wall), a guard cell equals the neighbouring block's cell it shadows, and the
block-by-block stencil on filled guards equals the grid stencil."""
import numpy as np
import pytest

import oracle as O
from paper_2312_11740_amd import problems as G


def centre_coords(n):
    return np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")   # k, j, i


@pytest.mark.parametrize("n,nb,g", [(8, 4, 1), (12, 4, 2), (16, 8, 1), (8, 8, 3), (6, 2, 2)])
def test_scatter_gather_roundtrip(n, nb, g):
    f = np.random.default_rng(n + nb + g).standard_normal((n, n, n))
    blk = O.blocks_scatter(f, nb, g)
    assert blk.shape == O.blocks_shape(n, nb, g)[:1] + (nb + 2 * g,) * 3
    assert np.array_equal(O.blocks_gather(blk, n, nb, g), f)
    # guards untouched by scatter
    inner = np.zeros_like(blk, dtype=bool)
    inner[:, g:g + nb, g:g + nb, g:g + nb] = True
    assert np.all(blk[~inner] == 0.0)


@pytest.mark.parametrize("n,nb,g", [(8, 4, 1), (12, 4, 2), (16, 8, 2), (6, 2, 2), (8, 8, 3)])
def test_guards_of_a_linear_field(n, nb, g):
    # f = a i + b j + c k (integers, exact); a guard at global position (I, J, K) must
    # hold f at (mirror(I), mirror(J), mirror(K)) with mirror(a) = -1 - a below 0 and
    # 2n - 1 - a at or above n
    K, J, I = centre_coords(n)
    f = (3.0 * I + 5.0 * J + 7.0 * K).astype(np.float64)
    blk = O.blocks_fill_guards(O.blocks_scatter(f, nb, g), n, nb, g)
    nbx = n // nb
    m = lambda a: -1 - a if a < 0 else (2 * n - 1 - a if a >= n else a)
    rng = np.random.default_rng(n * 31 + g)
    for _ in range(400):
        b = rng.integers(0, nbx ** 3)
        bi, bj, bk = b % nbx, (b // nbx) % nbx, b // (nbx * nbx)
        li, lj, lk = rng.integers(-g, nb + g, size=3)
        gi, gj, gk = m(bi * nb + li), m(bj * nb + lj), m(bk * nb + lk)
        assert blk[b, lk + g, lj + g, li + g] == 3.0 * gi + 5.0 * gj + 7.0 * gk


def test_guard_equals_the_neighbour_cell_it_shadows():
    n, nb, g = 12, 4, 2
    f = np.random.default_rng(3).standard_normal((n, n, n))
    blk = O.blocks_fill_guards(O.blocks_scatter(f, nb, g), n, nb, g)
    nbx = n // nb
    # block (1,1,1): its -x guard layer 1 is column nb-1 of block (0,1,1), its +z guard
    # layer 2 is plane 1 of block (1,1,2); a corner guard is the diagonal neighbour's cell
    b = 1 + nbx * (1 + nbx * 1)
    assert np.array_equal(blk[b, g:g + nb, g:g + nb, g - 1], f[nb:2 * nb, nb:2 * nb, nb - 1])
    assert np.array_equal(blk[b, g + nb + 1, g:g + nb, g:g + nb], f[2 * nb + 1, nb:2 * nb, nb:2 * nb])
    assert blk[b, 0, 0, 0] == f[nb - 2, nb - 2, nb - 2]


@pytest.mark.parametrize("n,nb,g", [(8, 4, 1), (16, 8, 1), (12, 4, 2), (16, 16, 1)])
def test_block_stencil_equals_grid_stencil(n, nb, g):
    phi = G.bubble_phi(n, [(0.45, 0.5, 0.55)], [0.27])
    fc = O.faces(phi, 1e-3, 1.0)
    x = np.random.default_rng(9).standard_normal((n, n, n))
    blk = O.blocks_fill_guards(O.blocks_scatter(x, nb, g), n, nb, g)
    y = O.blocks_gather(O.blocks_apply(fc, blk, nb, g), n, nb, g)
    ref = O.apply(fc, x)
    assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref))
    # without the guard fill the block boundaries are wrong
    y0 = O.blocks_gather(O.blocks_apply(fc, O.blocks_scatter(x, nb, g), nb, g), n, nb, g)
    if nb < n:
        assert np.max(np.abs(y0 - ref)) > 1e-3 * np.max(np.abs(ref))


def test_block_bad_arguments():
    f = np.zeros((8, 8, 8))
    for nb, g in [(3, 1), (4, -1), (4, 5), (0, 1)]:
        with pytest.raises((O.OracleError, ZeroDivisionError, ValueError)):
            O.blocks_scatter(f, nb, g)
