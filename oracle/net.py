"""FP64 CPU oracle of the learned initial guess (a small 3D U-Net) and its gradients.

TEST INFRASTRUCTURE ONLY (like the rest of `oracle/`): the reference for the GPU's
BF16 matrix-core network, never called by the library.

Not in the paper (which has no learned component): the network is the stated design
of the learned initial guess.  Architecture, fixed:

  in (4 channels: log10(1/rho)/3, b/rms(b), 0, 0) at n^3
  e1: conv 4->16, relu, conv 16->16, relu                      (n^3)
  pool (mean of 2x2x2) -> e2: conv 16->32, relu, conv 32->32, relu   (n/2)
  pool -> bott: conv 32->64, relu, conv 64->64, relu                 (n/4)
  up (nearest) -> concat [up, e2] (96) -> d2: conv 96->32, relu, conv 32->32, relu
  up -> concat [up, e1] (48) -> d1: conv 48->16, relu, conv 16->16, relu
  head: 1x1x1 conv 16->1 (no activation)

3x3x3 convolutions with zero padding.  Parameters, flattened in layer order, each conv
as W[tap][co][ci] (tap = 9 (dz+1) + 3 (dy+1) + (dx+1)) followed by bias[co]; the head
as W[0][ci] then its bias.  Fields are (n, n, n, channels) arrays indexed [z, y, x, c].

BF16 emulation (bf16=True) rounds, like the GPU, the weights, every stored activation
(after bias + relu, after pooling) and every activation gradient fed to a product to
bfloat16 (round to nearest even, via float32); sums are exact (FP64) and each result is
rounded to float32 before the bfloat16 rounding.  bf16=False is plain FP64 (used for the
finite-difference gradient pins).
"""
from __future__ import annotations

import numpy as np

CONVS = [  # (name, ci, co)
    ("e1a", 4, 16), ("e1b", 16, 16),
    ("e2a", 16, 32), ("e2b", 32, 32),
    ("b1", 32, 64), ("b2", 64, 64),
    ("d2a", 96, 32), ("d2b", 32, 32),
    ("d1a", 48, 16), ("d1b", 16, 16),
]
HEAD_CI = 16
IN_CH = 4


def param_count():
    return sum(27 * ci * co + co for _, ci, co in CONVS) + HEAD_CI + 1


def unpack(params):
    """Flat vector -> dict name -> (W[27, co, ci], bias[co]); 'head' -> (w[16], b[1])."""
    out, o = {}, 0
    for name, ci, co in CONVS:
        w = params[o:o + 27 * co * ci].reshape(27, co, ci)
        o += 27 * co * ci
        b = params[o:o + co]
        o += co
        out[name] = (w, b)
    out["head"] = (params[o:o + HEAD_CI], params[o + HEAD_CI:o + HEAD_CI + 1])
    assert o + HEAD_CI + 1 == params.size
    return out


def pack(grads):
    parts = []
    for name, ci, co in CONVS:
        parts += [grads[name][0].reshape(-1), grads[name][1].reshape(-1)]
    parts += [grads["head"][0].reshape(-1), grads["head"][1].reshape(-1)]
    return np.concatenate(parts)


def bf16(a):
    """Round to bfloat16 (nearest even) through float32; returns float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    r = np.where(np.isfinite(f), r, u & 0xFFFF0000)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def shift(x, dz, dy, dx):
    """s[z,y,x] = x[z+dz, y+dy, x+dx] with zeros outside."""
    n = x.shape[0]
    s = np.zeros_like(x)
    zs, zd = (slice(0, n - dz), slice(dz, n)) if dz >= 0 else (slice(-dz, n), slice(0, n + dz))
    ys, yd = (slice(0, n - dy), slice(dy, n)) if dy >= 0 else (slice(-dy, n), slice(0, n + dy))
    xs, xd = (slice(0, n - dx), slice(dx, n)) if dx >= 0 else (slice(-dx, n), slice(0, n + dx))
    s[zs, ys, xs] = x[zd, yd, xd]
    return s


def conv(x, w, b):
    """y[v, co] = b[co] + sum_tap sum_ci w[tap, co, ci] x[v + tap, ci] (zero padding)."""
    y = np.zeros(x.shape[:3] + (w.shape[1],))
    for t, (dz, dy, dx) in enumerate(TAPS):
        y += shift(x, dz, dy, dx) @ w[t].T
    return y + b


def conv_dx(dy_, w):
    """Adjoint of conv in x: dx[u, ci] = sum_tap sum_co w[tap, co, ci] dy[u - tap, co]."""
    dx = np.zeros(dy_.shape[:3] + (w.shape[2],))
    for t, (dz, dy, dxx) in enumerate(TAPS):
        dx += shift(dy_, -dz, -dy, -dxx) @ w[t]
    return dx


def conv_dw(dy_, x):
    """dw[tap, co, ci] = sum_v dy[v, co] x[v + tap, ci]; db[co] = sum_v dy[v, co]."""
    co, ci = dy_.shape[3], x.shape[3]
    dw = np.zeros((27, co, ci))
    g = dy_.reshape(-1, co)
    for t, (dz, dy, dx) in enumerate(TAPS):
        dw[t] = g.T @ shift(x, dz, dy, dx).reshape(-1, ci)
    return dw, g.sum(axis=0)


def pool(x):
    n = x.shape[0] // 2
    return x.reshape(n, 2, n, 2, n, 2, -1).mean(axis=(1, 3, 5))


def pool_back(g):
    return np.repeat(np.repeat(np.repeat(g, 2, 0), 2, 1), 2, 2) / 8.0


def up(x):
    return np.repeat(np.repeat(np.repeat(x, 2, 0), 2, 1), 2, 2)


def up_back(g):
    n = g.shape[0] // 2
    return g.reshape(n, 2, n, 2, n, 2, -1).sum(axis=(1, 3, 5))


def forward(params, x, bf16_mode=True):
    """x: (n, n, n, 4).  Returns (y (n, n, n), cache for backward)."""
    P = unpack(np.asarray(params, dtype=np.float64))
    R = bf16 if bf16_mode else (lambda a: a)
    Rf = (lambda a: bf16(f32(a))) if bf16_mode else (lambda a: a)
    Wr = {k: (R(v[0]), v[1]) for k, v in P.items()}   # weights rounded, biases FP32
    c = {"x": R(x)}

    def layer(name, inp):
        w, b = Wr[name]
        z = conv(inp, w, b)
        a = Rf(np.maximum(z, 0.0))
        c[name] = (inp, z, a)
        return a

    e1 = layer("e1b", layer("e1a", c["x"]))
    p1 = Rf(pool(e1))
    e2 = layer("e2b", layer("e2a", p1))
    p2 = Rf(pool(e2))
    bt = layer("b2", layer("b1", p2))
    u2 = np.concatenate([up(bt), e2], axis=3)
    d2 = layer("d2b", layer("d2a", u2))
    u1 = np.concatenate([up(d2), e1], axis=3)
    d1 = layer("d1b", layer("d1a", u1))
    hw, hb = Wr["head"]
    y = d1 @ hw + hb[0]
    if bf16_mode:
        y = f32(y)
    c["d1"] = d1
    c["W"] = Wr
    return y, c


def loss_and_dy(y, t):
    """Relative squared error of the zero-mean prediction: sum (y-mean(y)-t)^2 / sum t^2
    (t zero-mean); returns (loss, dloss/dy)."""
    e = (y - y.mean()) - t
    den = float(np.sum(t * t))
    loss = float(np.sum(e * e)) / den
    dy_ = 2.0 * (e - e.mean()) / den
    return loss, dy_


def backward(params, cache, dy_out, bf16_mode=True, trace=None):
    """Gradient of sum(dy_out * y) with respect to the flat parameter vector.  trace: an
    optional dict that receives each layer's pre-activation gradient (name -> gz)."""
    W = cache["W"]
    Rg = (lambda a: bf16(f32(a))) if bf16_mode else (lambda a: a)
    grads = {}
    d1 = cache["d1"]
    hw, hb = W["head"]
    grads["head"] = ((d1 * dy_out[..., None]).reshape(-1, HEAD_CI).sum(axis=0),
                     np.array([dy_out.sum()]))
    g = Rg(dy_out[..., None] * hw[None, None, None, :])

    def layer_back(name, g_a):
        inp, z, a = cache[name]
        gz = Rg(g_a * (z > 0))
        if trace is not None:
            trace[name] = gz
        w, b = W[name]
        dw, db = conv_dw(gz, inp)
        grads[name] = (dw, db)
        return Rg(conv_dx(gz, w))

    g = layer_back("d1a", layer_back("d1b", g))          # grad wrt u1 (48 ch)
    g_up1, g_e1 = g[..., :32], g[..., 32:]
    g = layer_back("d2a", layer_back("d2b", Rg(up_back(g_up1))))   # grad wrt u2 (96 ch)
    g_up2, g_e2 = g[..., :64], g[..., 64:]
    g = layer_back("b1", layer_back("b2", Rg(up_back(g_up2))))     # grad wrt p2
    g = Rg(g_e2 + pool_back(g))
    g = layer_back("e2a", layer_back("e2b", g))                    # grad wrt p1
    g = Rg(g_e1 + pool_back(g))
    layer_back("e1a", layer_back("e1b", g))
    return pack(grads)


def init_params(seed=0):
    """He-normal weights, zero biases (the reference initialisation; the GPU draws its
    own)."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, ci, co in CONVS:
        parts += [rng.normal(0.0, np.sqrt(2.0 / (27 * ci)), 27 * co * ci), np.zeros(co)]
    parts += [rng.normal(0.0, np.sqrt(1.0 / HEAD_CI), HEAD_CI), np.zeros(1)]
    return np.concatenate(parts)


def features(inv_rho, b):
    """Network input: log10(1/rho)/3 and b/rms(b), two zero channels; returns (x, rms)."""
    rms = float(np.sqrt(np.mean(b * b)))
    x = np.zeros(inv_rho.shape + (IN_CH,))
    x[..., 0] = np.log10(inv_rho) / 3.0
    x[..., 1] = b / rms if rms > 0 else 0.0
    return x, rms


def adam_step(w, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba, Algorithm 1) at step count t >= 1; returns new
    (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def coarsen(a, r):
    """Means over r^3 blocks of an (N, N, N) field, N = r n."""
    n = a.shape[0] // r
    return a.reshape(n, r, n, r, n, r).mean(axis=(1, 3, 5))


def _lin1d(N, n, r):
    """Interpolation matrix (N x n) of cell-centred linear interpolation, clamped."""
    P = np.zeros((N, n))
    for i in range(N):
        u = (i + 0.5) / r - 0.5
        i0 = int(np.floor(u))
        w = u - i0
        P[i, min(max(i0, 0), n - 1)] += 1.0 - w
        P[i, min(max(i0 + 1, 0), n - 1)] += w
    return P


def prolong_trilinear(c, r):
    """Trilinear interpolation of cell values to a grid r times finer (cell centres
    (i + 1/2)/(r n) in units of the domain; neighbours beyond a wall are the wall
    cell's value)."""
    n = c.shape[0]
    P = _lin1d(r * n, n, r)
    return np.einsum("ai,bj,ck,ijk->abc", P, P, P, c, optimize=True)


def learned_features(inv_rho, b, r):
    """Network inputs from the cell values of 1/rho and of the solver's right-hand
    side b at resolution r n ([z, y, x] arrays): block means, then features();
    returns (x, rms)."""
    return features(coarsen(inv_rho, r), coarsen(b, r))
