"""The seeded input generators: determinism, the bubble placement rules, layout."""
import numpy as np
import pytest

from paper_2312_11740_amd import problems as G


def test_same_seed_same_bytes():
    a = G.many_bubbles_problem(n=32, count=5, seed=9)
    b = G.many_bubbles_problem(n=32, count=5, seed=9)
    assert a.phi.tobytes() == b.phi.tobytes() and a.f.tobytes() == b.f.tobytes()
    c = G.many_bubbles_problem(n=32, count=5, seed=10)
    assert c.f.tobytes() != a.f.tobytes()


@pytest.mark.parametrize("seed", [20000, 20001, 20063, 0, 10499])
def test_random_bubbles_rules(seed):
    pr = G.random_bubbles_problem(seed, n=64)
    h = 1.0 / 64
    assert 1 <= len(pr.radii) <= 8
    ratio = pr.rho_pos / pr.rho_neg
    assert 10.0 <= ratio <= 1000.0
    for (c, r) in zip(pr.centres, pr.radii):
        assert 0.05 <= r <= 0.15
        assert all(0.15 <= ci <= 0.85 for ci in c)
        assert all(ci - r >= 2 * h and ci + r <= 1 - 2 * h for ci in c)
    for a in range(len(pr.radii)):
        for b in range(a):
            gap = np.linalg.norm(np.subtract(pr.centres[a], pr.centres[b])) - pr.radii[a] - pr.radii[b]
            assert gap >= 4 * h
    assert abs(pr.f.mean()) < 1e-15 and pr.f.min() >= -1.01 and pr.f.max() <= 1.01


def test_many_bubbles_config():
    pr = G.many_bubbles_problem(n=128)
    assert len(pr.radii) == 20 and pr.rho_neg == 1e-3 and pr.rho_pos == 1.0 and pr.sigma == 0.01
    assert all(0.04 <= r <= 0.12 for r in pr.radii)


def test_phi_layout_x_fastest():
    n = 8
    phi = G.bubble_phi(n, [(0.1, 0.5, 0.9)], [0.0])
    # the minimum of |x - c| sits at i = 0 (x = 1/16), j = 3 or 4, k = 7
    k, j, i = np.unravel_index(np.argmin(phi), phi.shape)
    assert i == 0 and k == 7 and j in (3, 4)


def test_rising_bubble_sequence():
    a = G.rising_bubble_problem(0, n=32)
    b = G.rising_bubble_problem(99, n=32)
    assert a.centres[0] == (0.5, 0.5, 0.2)
    assert abs(b.centres[0][2] - (0.2 + 0.004 * 99)) < 1e-15
    assert a.rho_pos / a.rho_neg == pytest.approx(1000.0)


def test_single_bubble_rhs():
    pr = G.single_bubble_problem(32)
    assert pr.rho_neg == 1.0 and pr.rho_pos == 10.0 and pr.sigma == 0.0
    assert abs(pr.f.mean()) < 1e-13
