"""Pins of the CPU oracle of the learned-guess network (oracle/net.py)."""
import numpy as np
import pytest

from oracle import net as N


def test_param_count_and_packing():
    p = N.init_params(1)
    assert p.size == N.param_count() == 354577
    assert np.array_equal(N.pack(N.unpack(p)), p)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    a = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-8, 8, 20000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 65504.0]])
    ref = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(N.bf16(a), ref)


def test_conv_matches_scipy_correlate():
    from scipy import ndimage
    rng = np.random.default_rng(1)
    n, ci, co = 6, 3, 2
    x = rng.standard_normal((n, n, n, ci))
    w = rng.standard_normal((27, co, ci))
    b = rng.standard_normal(co)
    y = N.conv(x, w, b)
    for o in range(co):
        ref = np.full((n, n, n), b[o])
        for c in range(ci):
            k = w[:, o, c].reshape(3, 3, 3)        # tap index = 9 (dz+1) + 3 (dy+1) + dx+1
            ref += ndimage.correlate(x[..., c], k, mode="constant", cval=0.0)
        assert np.allclose(y[..., o], ref, rtol=1e-12, atol=1e-12)


def test_adjoint_pairs():
    rng = np.random.default_rng(2)
    n = 8
    x = rng.standard_normal((n, n, n, 5))
    w = rng.standard_normal((27, 3, 5))
    g = rng.standard_normal((n, n, n, 3))
    lhs = np.vdot(N.conv(x, w, np.zeros(3)), g)
    rhs = np.vdot(x, N.conv_dx(g, w))
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)
    dw, db = N.conv_dw(g, x)
    # <conv(x; w), g> is linear in w with gradient dw
    assert abs(np.vdot(dw, w) - lhs) < 1e-10 * abs(lhs)
    assert np.allclose(db, g.reshape(-1, 3).sum(axis=0))
    s = rng.standard_normal((n // 2, n // 2, n // 2, 2))
    t = rng.standard_normal((n, n, n, 2))
    assert abs(np.vdot(N.up(s), t) - np.vdot(s, N.up_back(t))) < 1e-10
    assert abs(np.vdot(N.pool(t), s) - np.vdot(t, N.pool_back(s))) < 1e-10


def _loss(params, x, t):
    y, c = N.forward(params, x, bf16_mode=False)
    return N.loss_and_dy(y, t), c


def test_gradient_matches_finite_differences():
    # central differences in plain FP64; steps small enough (1e-7 along unit-size
    # random directions) that no pre-activation crosses the relu kink
    n = 8
    rng = np.random.default_rng(3)
    p = N.init_params(4)
    p += 0.05 * rng.standard_normal(p.size)      # non-zero biases too
    x = rng.standard_normal((n, n, n, N.IN_CH))
    t = rng.standard_normal((n, n, n))
    t -= t.mean()
    (loss, dy), c = _loss(p, x, t)
    g = N.backward(p, c, dy, bf16_mode=False)
    eps = 1e-7
    P = N.unpack(np.arange(p.size, dtype=float))
    for name, ci, co in N.CONVS + [("head", N.HEAD_CI, 1)]:
        w, b = P[name]
        idx = np.concatenate([w.reshape(-1), b.reshape(-1)]).astype(int)
        v = np.zeros(p.size)
        v[idx] = rng.standard_normal(idx.size) / np.sqrt(idx.size)
        fd = (_loss(p + eps * v, x, t)[0][0] - _loss(p - eps * v, x, t)[0][0]) / (2 * eps)
        assert abs(fd - np.vdot(g, v)) <= 1e-6 * abs(fd) + 1e-8, name


def test_loss_is_zero_for_exact_prediction_up_to_a_constant():
    t = np.random.default_rng(5).standard_normal((8, 8, 8))
    t -= t.mean()
    loss, dy = N.loss_and_dy(t + 3.0, t)
    assert loss < 1e-28 and np.abs(dy).max() < 1e-13


def test_adam_matches_torch():
    """The oracle's Adam against torch.optim.Adam (a library routine) over 3 steps."""
    import torch
    rng = np.random.default_rng(3)
    w0 = rng.normal(size=50)
    gs = [rng.normal(size=50) for _ in range(3)]
    w = torch.tensor(w0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([w], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    ww, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    for t, g in enumerate(gs, start=1):
        opt.zero_grad()
        w.grad = torch.tensor(g)
        opt.step()
        ww, m, v = N.adam_step(ww, m, v, g, t, lr=1e-2)
        assert np.allclose(ww, w.detach().numpy(), rtol=0, atol=1e-14)


def test_coarsen_is_block_mean():
    rng = np.random.default_rng(4)
    a = rng.normal(size=(8, 8, 8))
    c = N.coarsen(a, 2)
    assert np.isclose(c[1, 2, 3], a[2:4, 4:6, 6:8].mean())
    assert np.isclose(c.mean(), a.mean())
    assert np.array_equal(N.coarsen(a, 1), a)


def test_trilinear_prolongation_properties():
    n, r = 6, 4
    # constants are kept everywhere, the identity at r = 1
    assert np.allclose(N.prolong_trilinear(np.full((n, n, n), 2.5), r), 2.5)
    rng = np.random.default_rng(5)
    c = rng.normal(size=(n, n, n))
    assert np.allclose(N.prolong_trilinear(c, 1), c)
    # an affine function of the cell centres is reproduced away from the walls
    xc = (np.arange(n) + 0.5) / n
    Z, Y, X = np.meshgrid(xc, xc, xc, indexing="ij")
    lin = 1.0 + 2.0 * X - 3.0 * Y + 0.5 * Z
    f = N.prolong_trilinear(lin, r)
    xf = (np.arange(n * r) + 0.5) / (n * r)
    Zf, Yf, Xf = np.meshgrid(xf, xf, xf, indexing="ij")
    exact = 1.0 + 2.0 * Xf - 3.0 * Yf + 0.5 * Zf
    inner = slice(r // 2, n * r - r // 2)
    assert np.allclose(f[inner, inner, inner], exact[inner, inner, inner], atol=1e-12)
    # the 1D weights at r = 2 are 3/4 and 1/4
    e = np.zeros((n, n, n))
    e[2, 2, 2] = 1.0
    p = N.prolong_trilinear(e, 2)
    assert np.isclose(p[5, 5, 5], 0.75 ** 3) and np.isclose(p[6, 5, 5], 0.25 * 0.75 ** 2)
