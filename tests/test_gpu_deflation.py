"""The deflation regions and their coarse matrix against their definitions: the regions
are the connected components (through faces) of the lighter phase's cells, numbered by
their smallest cell index with the first 32 kept (scipy.ndimage.label numbers components
in that order); E = Z^T A Z with Z the regions' indicator fields and A the oracle's
operator; problems with equal densities or a light phase above a quarter of the cells are
not deflated.  Deflated solves themselves are checked against the oracle by every solve
test (deflation is on by default)."""
import numpy as np
import pytest
from scipy import ndimage

import oracle as O
from paper_2312_11740_amd import problems as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2312_11740_amd as M  # noqa: E402

DEV = "cuda:0"


def expected(phi, rn, rp):
    n = phi.shape[0]
    if rn == rp:
        return np.zeros(phi.shape, np.uint8), 0
    light = phi <= 0 if rn < rp else phi > 0
    if np.count_nonzero(light) > n ** 3 // 4 + 64:
        return np.zeros(phi.shape, np.uint8), 0
    lab, num = ndimage.label(light, structure=ndimage.generate_binary_structure(3, 1))
    lab[lab > 32] = 0
    return lab.astype(np.uint8), min(num, 32)


def expected_e(phi, rn, rp, lab, k):
    fc = O.faces(phi, rn, rp)
    E = np.zeros((k, k))
    for j in range(k):
        az = O.apply(fc, (lab == j + 1).astype(np.float64))
        for i in range(k):
            E[i, j] = np.sum(az[lab == i + 1])
    return E


def check(op, cases):
    lab, ks, E = op.deflation_info()
    lab = lab.cpu().numpy()
    if lab.ndim == 3:
        lab = lab[None]
    for b, (phi, rn, rp) in enumerate(cases):
        le, ke = expected(phi, rn, rp)
        print("problem %d: %d regions (expected %d)" % (b, ks[b], ke), flush=True)
        assert ks[b] == ke
        assert np.array_equal(lab[b], le)
        if ke:
            Ee = expected_e(phi, rn, rp, le, ke)
            assert np.max(np.abs(E[b, :ke, :ke] - Ee)) <= 1e-12 * np.max(np.abs(Ee))
            assert np.all(E[b, ke:, :] == 0.0) and np.all(E[b, :, ke:] == 0.0)
            # negative definite (A is negative semi-definite, no region combination is
            # constant on the whole domain)
            assert np.max(np.linalg.eigvalsh(0.5 * (Ee + Ee.T))) < 0


def test_regions_of_random_bubble_problems():
    probs = [G.random_bubbles_problem(20000 + s, n=64) for s in range(3)]
    cases = [(q.phi, q.rho_neg, q.rho_pos) for q in probs]
    op = M.Operator(torch.from_numpy(np.stack([c[0] for c in cases])).to(DEV),
                    [c[1] for c in cases], [c[2] for c in cases], [q.sigma for q in probs])
    check(op, cases)


def test_regions_beyond_32_are_not_kept():
    n = 64
    rng = np.random.default_rng(7)
    cs = [tuple(rng.uniform(0.08, 0.92, 3)) for _ in range(45)]
    phi = G.bubble_phi(n, cs, [0.03] * len(cs))   # some overlap: fewer components than bubbles
    _, num = ndimage.label(phi <= 0, structure=ndimage.generate_binary_structure(3, 1))
    assert num > 32
    op = M.Operator(torch.from_numpy(phi).to(DEV), 1e-3, 1.0, 0.01)
    check(op, [(phi, 1e-3, 1.0)])


@pytest.mark.parametrize("rn,rp", [(1.0, 1.0), (1.0, 1e-3)])
def test_no_deflation_for_equal_densities_or_a_large_light_phase(rn, rp):
    """Equal densities: nothing to deflate; the light phase outside the bubbles (rho_pos
    smaller): more than a quarter of the cells, not deflated."""
    n = 32
    phi = G.bubble_phi(n, [(0.5, 0.45, 0.55)], [0.2])
    op = M.Operator(torch.from_numpy(phi).to(DEV), rn, rp, 0.01)
    check(op, [(phi, rn, rp)])
    f = np.random.default_rng(2).uniform(-1, 1, (n, n, n))
    p, infos = op.solve(torch.from_numpy(f).to(DEV), rtol=1e-10)
    assert infos[0].status == M.OK


def test_region_touching_the_walls_and_the_deflated_solve():
    """A bubble cut by two walls and one inside: two regions; the deflated and the plain
    solve reach the same solution (the oracle's)."""
    n = 48
    phi = G.bubble_phi(n, [(0.0, 0.0, 0.5), (0.6, 0.6, 0.6)], [0.3, 0.15])
    f = np.random.default_rng(3).uniform(-1, 1, (n, n, n))
    op = M.Operator(torch.from_numpy(phi).to(DEV), 1e-3, 1.0, 0.01)
    check(op, [(phi, 1e-3, 1.0)])
    fd = torch.from_numpy(f).to(DEV)
    pd, idf = op.solve(fd, rtol=1e-11, deflate=True)
    pp, ipl = op.solve(fd, rtol=1e-11, deflate=False)
    print("iterations deflated %d plain %d" % (idf[0].iters, ipl[0].iters), flush=True)
    od = O.pipeline(phi, f, 1e-3, 1.0, 0.01)
    po, _ = O.solve_mg_pcg(od["faces"], od["b"], tol=1e-13)
    for p in (pd, pp):
        ph = p.cpu().numpy()
        assert O.rel_residual(od["faces"], od["b"], ph) <= 1.05e-11
        assert np.linalg.norm(ph - po) / np.linalg.norm(po) <= 1e-8
    assert idf[0].iters < ipl[0].iters
