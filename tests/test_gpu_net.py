"""Parity of the BF16 matrix-core U-Net (learned initial guess) with the CPU oracle
that emulates the same BF16 rounding points, through the C ABI.

Two regimes.  (1) Exact: sparse weights of +-1, half-integer biases and integer inputs
keep every sum of the forward pass and of the activation gradients exactly
representable in FP32 (checked on the CPU for each case), so the GPU's FP32
accumulation in any order gives the oracle's exact values before each BF16 rounding:
the forward output must agree to FP32 rounding and the weight gradients, whose
reductions over cells do round in FP32, to 1e-5.  (2) Dense He-normal weights: a
10-layer network that stores BF16 activations amplifies any change of summation order
(an FP32-ulp change of one sum flips a BF16 rounding, which perturbs its neighbours in
the next layer, ...), so its output is only defined to the spread that the oracle
itself shows under FP32-level perturbations of its sums, about 3e-3 relative; the
tolerance there is 2e-2.
"""
import numpy as np
import pytest

import oracle as O
from oracle import net as N
from paper_2312_11740_amd import problems as G

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2312_11740_amd as M  # noqa: E402

DEV = "cuda:0"


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def to_host(t):
    torch.cuda.synchronize()
    return t.detach().float().cpu().numpy().astype(np.float64) if t.dtype == torch.bfloat16 \
        else t.detach().cpu().numpy()


def rel2(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def params_case(seed):
    """FP32-representable parameters: He-normal weights, small random biases."""
    p = N.init_params(seed)
    rng = np.random.default_rng(seed + 1000)
    P = N.unpack(p)
    for name, _, co in N.CONVS:
        P[name][1][:] = rng.normal(0.0, 0.05, co)
    P["head"][1][:] = 0.1
    return p.astype(np.float32).astype(np.float64)


def sparse_params(seed, nnz=3):
    """Exact-regime parameters: nnz weights of +-1 per output channel at random taps and
    input channels, biases in {0, 1/2, 1}, head weights in {+-1/2, +-1}."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, ci, co in N.CONVS:
        w = np.zeros((27, co, ci))
        for o in range(co):
            for _ in range(nnz):
                w[rng.integers(27), o, rng.integers(ci)] = rng.choice([-1.0, 1.0])
        parts += [w.reshape(-1), rng.choice([0.0, 0.5, 1.0], co)]
    parts += [rng.choice([-1.0, -0.5, 0.5, 1.0], N.HEAD_CI), np.array([0.25])]
    return np.concatenate(parts)


def input_case(n, batch, seed):
    rng = np.random.default_rng(seed)
    x = np.zeros((batch, n, n, n, 4))
    x[..., 0] = rng.uniform(-1.0, 0.0, (batch, n, n, n))
    x[..., 1] = rng.normal(0.0, 1.0, (batch, n, n, n))
    return N.bf16(x)


def int_input(n, batch, seed):
    rng = np.random.default_rng(seed)
    x = np.zeros((batch, n, n, n, 4))
    x[..., :2] = rng.integers(-3, 4, (batch, n, n, n, 2))
    return x


def grid_unit(a):
    """Largest power of two of which every value of a is a multiple."""
    nz = np.abs(np.asarray(a, dtype=np.float64))
    nz = nz[nz != 0]
    if nz.size == 0:
        return 1.0
    k = 30
    while not np.all(np.mod(nz / 2.0 ** k, 1.0) == 0):
        k -= 1
        assert k > -200
    return 2.0 ** k


def assert_exact_regime(params, x, dy):
    """Every FP32 sum of the forward convolutions and of the data gradients has terms on
    a common grid and a total below 2^24 grid units: no rounding in any order."""
    P = N.unpack(params)
    _, cache = N.forward(params, x, bf16_mode=True)
    trace = {}
    N.backward(params, cache, dy, bf16_mode=True, trace=trace)
    for name, _, _ in N.CONVS:
        inp, _, _ = cache[name]
        w, b = P[name]
        u = min(grid_unit(inp), grid_unit(b))
        assert N.conv(np.abs(inp), np.abs(w), np.abs(b)).max() < 2.0 ** 24 * u, name
        gz = trace[name]
        assert N.conv_dx(np.abs(gz), np.abs(w)).max() < 2.0 ** 24 * grid_unit(gz), name
    d1 = cache["d1"]
    hw, hb = P["head"]
    assert (np.abs(d1) @ np.abs(hw) + abs(hb[0])).max() < 2.0 ** 24 * min(grid_unit(d1), 0.25)


def make_net(n, batch, params):
    net = M.Net(n, batch, seed=0, device=DEV)
    net.set_params(params.astype(np.float32))
    return net


def test_param_count_and_roundtrip():
    net = M.Net(16, 1, seed=3, device=DEV)
    assert net.nparams == N.param_count()
    p = params_case(5)
    net.set_params(p.astype(np.float32))
    assert np.array_equal(net.get_params(), p.astype(np.float32))


def test_device_init_is_he_normal():
    net = M.Net(16, 1, seed=11, device=DEV)
    P = N.unpack(net.get_params().astype(np.float64))
    for name, ci, co in N.CONVS:
        w, b = P[name]
        assert np.all(b == 0.0)
        sd = np.sqrt(2.0 / (27 * ci))
        assert abs(w.std() / sd - 1.0) < 0.1 and abs(w.mean()) < 0.1 * sd, name


@pytest.mark.parametrize("n,batch,seed", [(16, 2, 0), (32, 1, 1), (16, 1, 2)])
def test_forward_exact_regime(n, batch, seed):
    params = sparse_params(seed)
    x = int_input(n, batch, seed)
    net = make_net(n, batch, params)
    y = to_host(net.forward(to_dev(x, torch.bfloat16)))
    for b in range(batch):
        assert_exact_regime(params, x[b], np.zeros((n, n, n)))
        y_ref, _ = N.forward(params, x[b], bf16_mode=True)
        e = np.max(np.abs(y[b] - y_ref)) / np.max(np.abs(y_ref))
        print("n=%d sample %d forward max rel %.2e" % (n, b, e), flush=True)
        assert e <= 1e-6


@pytest.mark.parametrize("n,batch", [(16, 2), (32, 1)])
def test_forward_dense_weights(n, batch):
    params = params_case(1)
    x = input_case(n, batch, 2)
    net = make_net(n, batch, params)
    y = to_host(net.forward(to_dev(x, torch.bfloat16)))
    for b in range(batch):
        y_ref, _ = N.forward(params, x[b], bf16_mode=True)
        e = rel2(y[b], y_ref)
        print("n=%d sample %d forward rel L2 %.2e" % (n, b, e), flush=True)
        assert e <= 2e-2


def test_loss_matches_oracle():
    n, batch = 16, 3
    rng = np.random.default_rng(7)
    y = rng.normal(size=(batch, n, n, n)).astype(np.float32)
    t = rng.normal(size=(batch, n, n, n))
    t -= t.mean(axis=(1, 2, 3), keepdims=True)
    t = t.astype(np.float32)
    net = M.Net(n, batch, device=DEV)
    lo, dy = net.loss(to_dev(y), to_dev(t))
    lo, dy = to_host(lo), to_host(dy)
    for b in range(batch):
        l_ref, dy_ref = N.loss_and_dy(y[b].astype(np.float64), t[b].astype(np.float64))
        assert abs(lo[b] - l_ref) <= 1e-5 * l_ref
        assert rel2(dy[b] * batch, dy_ref) <= 1e-5


def test_loss_zero_for_exact_prediction_up_to_a_constant():
    n = 16
    rng = np.random.default_rng(8)
    t = rng.normal(size=(1, n, n, n))
    t -= t.mean()
    net = M.Net(n, 1, device=DEV)
    lo, dy = net.loss(to_dev((t + 3.0).astype(np.float32)), to_dev(t.astype(np.float32)))
    assert to_host(lo)[0] < 1e-10
    assert np.max(np.abs(to_host(dy))) < 1e-5


@pytest.mark.parametrize("n,batch,seed", [(16, 2, 3), (32, 1, 4)])
def test_backward_exact_regime(n, batch, seed):
    params = sparse_params(seed)
    x = int_input(n, batch, seed)
    rng = np.random.default_rng(seed + 50)
    dy = rng.integers(-4, 5, (batch, n, n, n)) * 2.0 ** -6
    net = make_net(n, batch, params)
    net.forward(to_dev(x, torch.bfloat16))
    net.backward(to_dev(dy.astype(np.float32)))
    g = net.get_grads().astype(np.float64)
    g_ref = np.zeros_like(g)
    for b in range(batch):
        assert_exact_regime(params, x[b], dy[b])
        _, cache = N.forward(params, x[b], bf16_mode=True)
        g_ref += N.backward(params, cache, dy[b], bf16_mode=True)
    G_ = N.unpack(g)
    R = N.unpack(g_ref)
    for name in [c[0] for c in N.CONVS] + ["head"]:
        for part in (0, 1):
            e = rel2(G_[name][part], R[name][part])
            print("%s %s rel L2 %.2e" % (name, "w" if part == 0 else "b", e), flush=True)
            assert e <= 1e-5, (name, part, e)


def test_adam_update_rule():
    """Two steps against the published update, with the device's own gradients (read
    back) as g: a property of the update, not an oracle input."""
    n = 16
    params = params_case(9).astype(np.float32)
    x = input_case(n, 1, 10)
    rng = np.random.default_rng(11)
    t = rng.normal(size=(1, n, n, n))
    t = (t - t.mean()).astype(np.float32)
    net = make_net(n, 1, params.astype(np.float64))
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    w = params.astype(np.float64)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    xd, td = to_dev(x, torch.bfloat16), to_dev(t)
    for step in (1, 2):
        y = net.forward(xd)
        _, dy = net.loss(y, td)
        net.backward(dy)
        g = net.get_grads().astype(np.float64)
        net.adam(lr, b1, b2, eps)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g * g
        w = w - lr * (m / (1 - b1 ** step)) / (np.sqrt(v / (1 - b2 ** step)) + eps)
        got = net.get_params().astype(np.float64)
        assert np.max(np.abs(got - w)) <= 1e-6 + 1e-6 * np.max(np.abs(w)), step
        w = got   # FP32 state carries on


def problem_batch(n, seeds, ratio=None):
    phis, fs, rn, rp, sg = [], [], [], [], []
    for s in seeds:
        pr = G.random_bubbles_problem(s, n=n)
        phis.append(pr.phi)
        fs.append(pr.f)
        rn.append(pr.rho_neg if ratio is None else 1.0 / ratio)
        rp.append(pr.rho_pos)
        sg.append(pr.sigma)
    return np.stack(phis), np.stack(fs), rn, rp, sg


@pytest.mark.parametrize("nf,nn", [(32, 16), (64, 16)])
def test_features_and_targets_match_oracle(nf, nn):
    seeds = [3, 4]
    phi, f, rn, rp, sg = problem_batch(nf, seeds)
    op = M.Operator(to_dev(phi), rn, rp, sg)
    net = M.Net(nn, len(seeds), device=DEV)
    r = nf // nn
    p_ref = []
    for b in range(len(seeds)):
        p, _, _ = O.solve(phi[b], f[b], rn[b], rp[b], sg[b])
        p_ref.append(p)
    x, t, rms = net.features(op, to_dev(f), to_dev(np.stack(p_ref)))
    x, t, rms = to_host(x), to_host(t), to_host(rms)
    for b in range(len(seeds)):
        d = O.pipeline(phi[b], f[b], rn[b], rp[b], sg[b])
        inv_rho = np.where(phi[b] > 0, 1.0 / rp[b], 1.0 / rn[b])
        x_ref, rms_ref = N.learned_features(inv_rho, d["b"], r)
        assert abs(rms[b] - rms_ref) <= 1e-6 * rms_ref
        xr = N.bf16(x_ref)
        # one BF16 ulp at most (the GPU's b differs from the oracle's by rounding)
        assert np.all(np.abs(x[b] - xr) <= 2.0 ** -8 * np.abs(xr) + 1e-30)
        t_ref = N.coarsen(p_ref[b], r) * nn ** 2 / rms_ref
        assert rel2(t[b], t_ref) <= 1e-6


def oracle_guess(params, phi, f, rn, rp, sg, r, sweeps):
    """The learned guess written out from its definition (oracle arithmetic only)."""
    d = O.pipeline(phi, f, rn, rp, sg)
    inv_rho = np.where(phi > 0, 1.0 / rp, 1.0 / rn)
    x, rms = N.learned_features(inv_rho, d["b"], r)
    y, _ = N.forward(params, x, bf16_mode=True)
    nc = phi.shape[0] // r
    p = N.prolong_trilinear(y * rms / nc ** 2, r)
    p -= p.mean()
    # the multiple of p closest to the solution in the energy norm
    p *= np.dot(p.ravel(), d["b"].ravel()) / np.dot(p.ravel(), O.apply(d["faces"], p).ravel())
    for _ in range(sweeps):
        p = O.gs_colour(d["faces"], d["b"], p, 0)
        p = O.gs_colour(d["faces"], d["b"], p, 1)
    res = O.rel_residual(d["faces"], d["b"], p)
    return p, res, d


@pytest.mark.parametrize("nf,nn,sweeps", [(32, 16, 0), (32, 16, 2), (64, 16, 0), (64, 16, 2)])
def test_learned_guess_matches_oracle(nf, nn, sweeps):
    """r = nf / nn = 2 (the kernels' run-time coarsening factor) and r = 4 (the
    compile-time factor the 256^3 benchmark uses with the 64^3 network)."""
    seeds = [21, 22]
    phi, f, rn, rp, sg = problem_batch(nf, seeds)
    params = sparse_params(12)
    P = N.unpack(params)
    op = M.Operator(to_dev(phi), rn, rp, sg)
    net = make_net(nn, len(seeds), params)
    p, fell = op.learned_guess(net, to_dev(f), sweeps=sweeps)
    p = to_host(p)
    for b in range(len(seeds)):
        p_ref, res, _ = oracle_guess(params, phi[b], f[b], rn[b], rp[b], sg[b], nf // nn, sweeps)
        print("sample %d: oracle residual %.3f, fell back %d" % (b, res, fell[b]), flush=True)
        if abs(res - 1.0) < 1e-6:   # on the fallback threshold: either outcome is right
            assert fell[b] == 1 and np.all(p[b] == 0.0) or rel2(p[b], p_ref) <= 1e-3
        elif res > 1.0:
            assert fell[b] == 1 and np.all(p[b] == 0.0)
        else:
            assert fell[b] == 0
            assert rel2(p[b], p_ref) <= 1e-3


def test_non_finite_guess_falls_back_to_zero_and_solves():
    nf, nn = 32, 16
    phi, f, rn, rp, sg = problem_batch(nf, [31])
    params = params_case(13)
    P = N.unpack(params)
    P["head"][0][:] = 3.0e38   # overflows to inf in the head's FP32 sum
    op = M.Operator(to_dev(phi), rn, rp, sg)
    net = make_net(nn, 1, params.astype(np.float32).astype(np.float64))
    fd = to_dev(f)
    p0, fell = op.learned_guess(net, fd, sweeps=2)
    assert fell == [1] and torch.all(p0 == 0).item()
    p, info = op.solve(fd, p0)
    p_zero, info_zero = op.solve(fd)
    assert info[0].iters == info_zero[0].iters
    assert torch.equal(p, p_zero)


def test_training_reduces_loss_and_iterations():
    """A short training run on solver-generated 32^3 triples; the trained network's
    guess must cut the MG-PCG iterations of held-out problems below a zero start."""
    n = 32
    train_seeds, test_seeds = list(range(100, 132)), list(range(10000, 10008))
    phi, f, rn, rp, sg = problem_batch(n, train_seeds)
    op = M.Operator(to_dev(phi), rn, rp, sg)
    fd = to_dev(f)
    p, infos = op.solve(fd)
    assert all(i.status == 0 for i in infos)
    net = M.Net(n, len(train_seeds), seed=1, device=DEV)
    x, t, _ = net.features(op, fd, p)
    # 300 steps of 8 samples drawn from the 32 triples, in one mpp_net_train call
    losses = to_host(net.train(x, t, 300, 8, lr=1e-3, seed=2024)).mean(axis=1)
    print("loss first %.3f last %.3f" % (np.mean(losses[:10]), np.mean(losses[-10:])), flush=True)
    assert np.mean(losses[-20:]) < 0.7 * np.mean(losses[:10])
    phi2, f2, rn2, rp2, sg2 = problem_batch(n, test_seeds)
    op2 = M.Operator(to_dev(phi2), rn2, rp2, sg2)
    f2d = to_dev(f2)
    # the gain over plain MG-PCG (no deflation: deflating the bubble regions removes the
    # slow modes the guess mostly takes out, and then the guess does not pay)
    _, zero = op2.solve(f2d, deflate=False)
    net2 = M.Net(n, len(test_seeds), device=DEV)
    net2.set_params(net.get_params())
    g0, fell = op2.learned_guess(net2, f2d, sweeps=2)
    p2, learned = op2.solve(f2d, g0, deflate=False)
    it0 = np.mean([i.iters for i in zero])
    it1 = np.mean([i.iters for i in learned])
    print("held-out iterations: zero start %.2f, learned %.2f, fallbacks %d"
          % (it0, it1, sum(fell)), flush=True)
    assert all(i.status == 0 and i.rel_resid <= 1e-10 for i in learned)
    assert it1 < it0


def splitmix64_index(seed, q, count):
    """Output number q of the SplitMix64 stream started at seed (Steele, Lea & Flood 2014),
    mod count: the draw mpp_net_train documents, written out here from its definition."""
    m = 2 ** 64 - 1
    z = (seed + (q + 1) * 0x9E3779B97F4A7C15) & m
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    z ^= z >> 31
    return z % count


@pytest.mark.parametrize("seed", [0, 987654321])
def test_net_train_equals_the_four_call_sequence(seed):
    """mpp_net_train is the sequence draw / forward / loss / backward / Adam run by the
    library: the same steps made by separate calls on the same samples (drawn here from
    the documented generator) give the same parameters and losses, bit for bit, on a
    learning-rate schedule that changes every step."""
    n, count, batch, steps = 16, 6, 2, 4
    rng = np.random.default_rng(5)
    x = to_dev(input_case(n, count, 6), torch.bfloat16)
    t = rng.normal(size=(count, n, n, n))
    t = to_dev((t - t.mean(axis=(1, 2, 3), keepdims=True)).astype(np.float32))
    params = params_case(17)
    a = make_net(n, batch, params)
    b = make_net(n, batch, params)
    lo_a = to_host(a.train(x, t, steps, batch, lr=1e-3, lr_final=2e-4, seed=seed))
    lr0, lr1 = float(np.float32(1e-3)), float(np.float32(2e-4))
    lo_b = []
    for g in range(steps):
        idx = [splitmix64_index(seed, g * batch + j, count) if seed else (g * batch + j) % count
               for j in range(batch)]
        xi = x[torch.tensor(idx, device=DEV)].contiguous()
        ti = t[torch.tensor(idx, device=DEV)].contiguous()
        y = b.forward(xi)
        lo, dy = b.loss(y, ti)
        b.backward(dy)
        b.adam(lr0 * (lr1 / lr0) ** (g / (steps - 1)))
        lo_b.append(to_host(lo))
    assert np.array_equal(lo_a, np.stack(lo_b))
    assert np.array_equal(a.get_params(), b.get_params())
    assert not np.array_equal(a.get_params(), params.astype(np.float32))


def test_net_train_split_into_calls_equals_one_call():
    """first_step / total_steps: a run cut into calls continues the draw and the schedule."""
    n, count, batch = 16, 5, 2
    rng = np.random.default_rng(8)
    x = to_dev(input_case(n, count, 9), torch.bfloat16)
    t = rng.normal(size=(count, n, n, n))
    t = to_dev((t - t.mean(axis=(1, 2, 3), keepdims=True)).astype(np.float32))
    params = params_case(19)
    a, b = make_net(n, batch, params), make_net(n, batch, params)
    a.train(x, t, 5, batch, lr=1e-3, lr_final=1e-4, seed=77)
    b.train(x, t, 2, batch, lr=1e-3, lr_final=1e-4, seed=77, first_step=0, total_steps=5)
    b.train(x, t, 3, batch, lr=1e-3, lr_final=1e-4, seed=77, first_step=2, total_steps=5)
    assert np.array_equal(a.get_params(), b.get_params())


def test_net_train_rejects_a_batch_above_batch_max():
    n = 16
    net = M.Net(n, 2, device=DEV)
    x = torch.zeros((4, n, n, n, 4), dtype=torch.bfloat16, device=DEV)
    t = torch.zeros((4, n, n, n), dtype=torch.float32, device=DEV)
    with pytest.raises(M.MppError) as ei:
        net.train(x, t, 1, 3)
    assert ei.value.status == M.EINVAL


def test_weight_gradient_of_a_batch_above_512():
    """Batches above 512 samples (more weight-gradient partials than the fixed minimum the
    buffer holds; they once overran it): 600 copies of one sample give 600 times its
    gradient (exact regime: sparse weights, integer inputs)."""
    n, batch = 16, 600
    params = sparse_params(23)
    x1 = int_input(n, 1, 24)
    dy1 = np.random.default_rng(25).integers(-4, 5, (1, n, n, n)) * 2.0 ** -6
    one = make_net(n, 1, params)
    one.forward(to_dev(x1, torch.bfloat16))
    one.backward(to_dev(dy1.astype(np.float32)))
    g1 = one.get_grads().astype(np.float64)
    many = make_net(n, batch, params)
    xb = to_dev(x1, torch.bfloat16).expand(batch, n, n, n, 4).contiguous()
    dyb = to_dev(dy1.astype(np.float32)).expand(batch, n, n, n).contiguous()
    many.forward(xb)
    many.backward(dyb)
    g = many.get_grads().astype(np.float64)
    assert np.all(np.isfinite(g))
    # the per-sample sums are exact; adding 600 of them in FP32 rounds, by at most
    # (batch - 1) units of 2^-24 relative to the total
    assert np.max(np.abs(g - batch * g1)) <= batch * 2.0 ** -24 * np.max(np.abs(batch * g1))


def test_deflated_judge_keeps_the_guess_or_zero():
    """MPP_JUDGE_DEFLATED computes the same guess as the plain judge and only decides
    differently whether to keep it: each problem gets either that guess or zero; a
    deflated solve from the result meets the oracle."""
    nf, nn = 64, 16
    seeds = [41, 42, 43]
    phi, f, rn, rp, sg = problem_batch(nf, seeds)
    op = M.Operator(to_dev(phi), rn, rp, sg)
    net = make_net(nn, len(seeds), params_case(3))
    fd = to_dev(f)
    gp, fp = op.learned_guess(net, fd, sweeps=2, judge="plain")
    gd, fdj = op.learned_guess(net, fd, sweeps=2, judge="deflated")
    gp, gd = to_host(gp), to_host(gd)
    print("fallbacks plain %s deflated %s" % (fp, fdj), flush=True)
    for b in range(len(seeds)):
        if fdj[b]:
            assert np.all(gd[b] == 0.0)
        else:
            assert fp[b] == 0 and np.array_equal(gd[b], gp[b])
    p, infos = op.solve(fd, to_dev(gd), rtol=1e-10, mode="mixed")
    ph = to_host(p)
    for b in range(len(seeds)):
        d = O.pipeline(phi[b], f[b], rn[b], rp[b], sg[b])
        assert infos[b].status == M.OK
        assert O.rel_residual(d["faces"], d["b"], ph[b]) <= 1.05e-10
        po, _ = O.solve_mg_pcg(d["faces"], d["b"], tol=1e-13)
        assert rel2(ph[b], po) <= 1e-8


def test_solve_reuses_the_guess_right_hand_side():
    """mpp_solve_opts.reuse_rhs: a solve right after the learned guess on the same f takes
    the right-hand side that guess assembled, with the same bits as assembling it again;
    after any other call on the operator, or for another f, the solve assembles it."""
    nf, nn = 64, 16
    seeds = [41, 42]
    phi, f, rn, rp, sg = problem_batch(nf, seeds)
    op = M.Operator(to_dev(phi), rn, rp, sg)
    net = make_net(nn, len(seeds), params_case(3))
    fd = to_dev(f)
    g, fell = op.learned_guess(net, fd, sweeps=2, judge="deflated")
    g1, g2 = g.clone(), g.clone()
    p1, i1 = op.solve(fd, g1, rtol=1e-10, mode="mixed", reuse_rhs=True)   # taken from the guess
    p2, i2 = op.solve(fd, g2, rtol=1e-10, mode="mixed", reuse_rhs=True)   # assembled
    assert torch.equal(p1, p2)
    for a, b in zip(i1, i2):
        assert (a.iters, a.removed_mean, a.bnorm, a.rel_resid) == \
            (b.iters, b.removed_mean, b.bnorm, b.rel_resid)
    # a guess for f, then a solve for another right-hand side: assembled from that one
    f3 = fd * 0.5 + 1.0
    op.learned_guess(net, fd, sweeps=2, judge="deflated")
    p3, i3 = op.solve(f3, rtol=1e-10, mode="mixed", reuse_rhs=True)
    p4, i4 = op.solve(f3, rtol=1e-10, mode="mixed")
    assert torch.equal(p3, p4)
    assert [a.removed_mean for a in i3] == [a.removed_mean for a in i4]
    ph = to_host(p1)
    for b in range(len(seeds)):
        d = O.pipeline(phi[b], f[b], rn[b], rp[b], sg[b])
        assert i1[b].status == M.OK
        assert O.rel_residual(d["faces"], d["b"], ph[b]) <= 1.05e-10
