"""Block-structured layout on the GPU against the oracle: scatter, gather and the
guard-cell fill are copies (bit for bit), the block stencil uses the oracle's order of
operations (bit for bit), at sizes with one block, many blocks, wide guards, batches
and the 256^3 grid in 16^3 blocks."""
import numpy as np
import pytest

import oracle as O
from paper_2312_11740_amd import problems as G

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2312_11740_amd as M  # noqa: E402

DEV = "cuda:0"


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def to_host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("n,nb,g", [(16, 16, 1), (32, 8, 1), (32, 8, 2), (48, 16, 1),
                                    (24, 4, 3), (20, 10, 2)])
def test_layout_and_guards_match_oracle(n, nb, g):
    f = np.random.default_rng(n * 7 + nb + g).standard_normal((n, n, n))
    blk = M.blocks_scatter(to_dev(f), nb, g)
    ref = O.blocks_scatter(f, nb, g)
    assert np.array_equal(to_host(blk), ref)
    M.blocks_fill_guards(blk, n, nb, g)
    ref = O.blocks_fill_guards(ref, n, nb, g)
    assert np.array_equal(to_host(blk), ref)
    assert np.array_equal(to_host(M.blocks_gather(blk, n, nb, g)), f)


@pytest.mark.parametrize("n,nb,g", [(32, 8, 1), (48, 16, 2), (20, 10, 1)])
def test_block_stencil_matches_oracle(n, nb, g):
    phi = G.bubble_phi(n, [(0.45, 0.5, 0.55), (0.7, 0.3, 0.3)], [0.25, 0.12])
    x = np.random.default_rng(5).standard_normal((n, n, n))
    op = M.Operator(to_dev(phi), 1e-3, 1.0, 0.01)
    xb = M.blocks_fill_guards(M.blocks_scatter(to_dev(x), nb, g), n, nb, g)
    y = to_host(op.blocks_apply(xb, nb, g))
    fc = O.faces(phi, 1e-3, 1.0)
    ref = O.blocks_apply(fc, O.blocks_fill_guards(O.blocks_scatter(x, nb, g), n, nb, g), nb, g)
    assert np.array_equal(y, ref)
    # and it is the grid stencil of the same operator, block by block
    grid_y = to_host(op.apply(to_dev(x)))
    assert np.max(np.abs(to_host(M.blocks_gather(to_dev(y), n, nb, g)) - grid_y)) <= \
        1e-12 * np.max(np.abs(grid_y))


def test_batched_blocks():
    n, nb, g, B = 32, 16, 1, 3
    f = np.random.default_rng(8).standard_normal((B, n, n, n))
    blk = M.blocks_fill_guards(M.blocks_scatter(to_dev(f), nb, g), n, nb, g)
    got = to_host(blk)
    for b in range(B):
        assert np.array_equal(got[b], O.blocks_fill_guards(O.blocks_scatter(f[b], nb, g), n, nb, g))
    assert np.array_equal(to_host(M.blocks_gather(blk, n, nb, g)), f)


def test_blocks_full_size():
    # the 256^3 rising-bubble grid in 4096 blocks of 16^3 with one guard layer: every
    # value of the filled layout and of the block stencil against the oracle
    n, nb, g = 256, 16, 1
    pr = G.rising_bubble_problem(0, n=n)
    x = np.random.default_rng(6).standard_normal((n, n, n))
    op = M.Operator(to_dev(pr.phi), pr.rho_neg, pr.rho_pos, pr.sigma)
    xb = M.blocks_fill_guards(M.blocks_scatter(to_dev(x), nb, g), n, nb, g)
    ref = O.blocks_fill_guards(O.blocks_scatter(x, nb, g), n, nb, g)
    assert np.array_equal(to_host(xb), ref)
    y = to_host(op.blocks_apply(xb, nb, g))
    fc = O.faces(pr.phi, pr.rho_neg, pr.rho_pos)
    assert np.array_equal(y, O.blocks_apply(fc, ref, nb, g))
