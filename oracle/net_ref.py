"""FP64 reference of the warm-start network (forward and backward).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The network is not part of the paper: it is the learned warm start of the
contact solve (an initial pressure field), and only the solve it seeds is
held to the paper's method.  This module fixes its definition in plain
NumPy so that the GPU forward/backward kernels can be checked against it;
it is pinned by central finite differences in tests/test_oracle_net.py.

Definition (NHWC, 16 channels everywhere, every convolution 3x3, stride 1,
zero "same" padding, weights W[tap][co][ci] with tap = 3 (dy+1) + (dx+1)):
  s0 = relu(c(relu(c(x))))                     HxW     (layers 0, 1)
  s1 = relu(c(relu(c(pool(s0)))))              H/2     (layers 2, 3)
  s2 = relu(c(relu(c(pool(s1)))))              H/4     (layers 4, 5)
  s3 = relu(c(relu(c(pool(s2)))))              H/8     (layers 6, 7)
  e2 = relu(c(up(s3)) + s2)                    H/4     (layer 8)
  e1 = relu(c(up(e2)) + s1)                    H/2     (layer 9)
  e0 = relu(c(up(e1)) + s0)                    HxW     (layer 10)
  z  = c(e0)[..., 0]                           HxW     (layer 11, no relu)
  q  = softplus(z);  p^ = q / mean(q)          per sample
  t^ = t / mean(t)                             per sample (t: solved pressure)
  loss = mean over the batch of sum (p^ - t^)^2 / sum t^^2
pool = 2x2 average, up = 2x2 nearest copy; c(.) includes the bias.
"""
from __future__ import annotations

import numpy as np

C = 16
NLAYER = 12
LAYER_PARAMS = 9 * C * C + C
NPARAM = NLAYER * LAYER_PARAMS


def unpack(params):
    params = np.asarray(params, dtype=np.float64)
    out = []
    for l in range(NLAYER):
        base = l * LAYER_PARAMS
        W = params[base:base + 9 * C * C].reshape(9, C, C)
        b = params[base + 9 * C * C:base + LAYER_PARAMS]
        out.append((W, b))
    return out


def init_params(seed=0):
    """He-style initialisation (the GPU trainer uses the same draws)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAM)
    for l in range(NLAYER):
        base = l * LAYER_PARAMS
        std = np.sqrt(2.0 / (9 * C))
        if l == NLAYER - 1:
            std *= 0.1
        p[base:base + 9 * C * C] = rng.standard_normal(9 * C * C) * std
    return p


def conv(x, W, b):
    """y[n,y,x,co] = b[co] + sum_{tap,ci} W[tap,co,ci] x[n, y+dy, x+dx, ci]."""
    n, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    y = np.broadcast_to(b, (n, H, Wd, C)).copy()
    for tap in range(9):
        dy, dx = tap // 3 - 1, tap % 3 - 1
        xs = xp[:, 1 + dy:1 + dy + H, 1 + dx:1 + dx + Wd, :]
        y += np.einsum("nhwi,oi->nhwo", xs, W[tap])
    return y


def conv_bwd(x, W, dy):
    """Gradients of conv w.r.t. x, W, b given dL/dy."""
    n, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dW = np.zeros_like(W)
    dxp = np.zeros_like(xp)
    for tap in range(9):
        dyy, dxx = tap // 3 - 1, tap % 3 - 1
        xs = xp[:, 1 + dyy:1 + dyy + H, 1 + dxx:1 + dxx + Wd, :]
        dW[tap] = np.einsum("nhwo,nhwi->oi", dy, xs)
        dxp[:, 1 + dyy:1 + dyy + H, 1 + dxx:1 + dxx + Wd, :] += np.einsum("nhwo,oi->nhwi", dy, W[tap])
    db = dy.sum(axis=(0, 1, 2))
    return dxp[:, 1:-1, 1:-1, :], dW, db


def pool(x):
    n, H, W, c = x.shape
    return x.reshape(n, H // 2, 2, W // 2, 2, c).mean(axis=(2, 4))


def pool_bwd(dy):
    return np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2) / 4.0


def up(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up_bwd(dy):
    n, H, W, c = dy.shape
    return dy.reshape(n, H // 2, 2, W // 2, 2, c).sum(axis=(2, 4))


def relu(a):
    return np.maximum(a, 0.0)


def softplus(z):
    return np.logaddexp(0.0, z)


def forward(params, x, keep=False):
    """x: (n, H, W, 16).  Returns z (n, H, W) [and the saved activations]."""
    L = unpack(params)
    a = {}
    a["x"] = x
    h = relu(conv(x, *L[0]))
    a["h0"] = h
    s0 = relu(conv(h, *L[1]))
    a["s0"] = s0
    p1 = pool(s0)
    a["p1"] = p1
    h = relu(conv(p1, *L[2]))
    a["h1"] = h
    s1 = relu(conv(h, *L[3]))
    a["s1"] = s1
    p2 = pool(s1)
    a["p2"] = p2
    h = relu(conv(p2, *L[4]))
    a["h2"] = h
    s2 = relu(conv(h, *L[5]))
    a["s2"] = s2
    p3 = pool(s2)
    a["p3"] = p3
    h = relu(conv(p3, *L[6]))
    a["h3"] = h
    s3 = relu(conv(h, *L[7]))
    a["s3"] = s3
    u2 = up(s3)
    a["u2"] = u2
    e2 = relu(conv(u2, *L[8]) + s2)
    a["e2"] = e2
    u1 = up(e2)
    a["u1"] = u1
    e1 = relu(conv(u1, *L[9]) + s1)
    a["e1"] = e1
    u0 = up(e1)
    a["u0"] = u0
    e0 = relu(conv(u0, *L[10]) + s0)
    a["e0"] = e0
    z = conv(e0, *L[11])[..., 0]
    return (z, a) if keep else z


def normalised_pressure(z):
    q = softplus(z)
    return q / q.mean(axis=(1, 2), keepdims=True)


def loss_and_dz(z, t):
    """loss = mean_n sum (p^ - t^)^2 / sum t^^2 and dloss/dz, t^ = t/mean(t)."""
    n = z.shape[0]
    t = t / t.mean(axis=(1, 2), keepdims=True)
    q = softplus(z)
    m = q.mean(axis=(1, 2), keepdims=True)
    ph = q / m
    tt = (t * t).sum(axis=(1, 2), keepdims=True)
    r = ph - t
    loss = float(((r * r).sum(axis=(1, 2), keepdims=True) / tt).mean())
    dph = 2.0 * r / tt / n
    npx = z.shape[1] * z.shape[2]
    # ph = q / m, m = sum q / npx:  dq = dph / m - sum(dph q) / (m^2 npx)
    dq = dph / m - (dph * q).sum(axis=(1, 2), keepdims=True) / (m * m * npx)
    dz = dq / (1.0 + np.exp(-z))
    return loss, dz


def backward(params, x, t):
    """loss and the full parameter gradient (flat, NPARAM)."""
    L = unpack(params)
    z, a = forward(params, x, keep=True)
    loss, dz = loss_and_dz(z, t)
    grads = [None] * NLAYER
    dy = np.zeros(z.shape + (C,))
    dy[..., 0] = dz
    d_e0, dW, db = conv_bwd(a["e0"], L[11][0], dy)
    grads[11] = (dW, db)
    # e0 = relu(conv(u0) + s0)
    da = d_e0 * (a["e0"] > 0)
    d_s0 = da.copy()
    d_u0, dW, db = conv_bwd(a["u0"], L[10][0], da)
    grads[10] = (dW, db)
    d_e1 = up_bwd(d_u0)
    da = d_e1 * (a["e1"] > 0)
    d_s1 = da.copy()
    d_u1, dW, db = conv_bwd(a["u1"], L[9][0], da)
    grads[9] = (dW, db)
    d_e2 = up_bwd(d_u1)
    da = d_e2 * (a["e2"] > 0)
    d_s2 = da.copy()
    d_u2, dW, db = conv_bwd(a["u2"], L[8][0], da)
    grads[8] = (dW, db)
    d_s3 = up_bwd(d_u2)
    # encoder, deepest first
    for lvl, (hk, sk, pk, l_a, l_b) in enumerate(
            [("h3", "s3", "p3", 6, 7), ("h2", "s2", "p2", 4, 5), ("h1", "s1", "p1", 2, 3)]):
        ds = {"s3": d_s3, "s2": d_s2, "s1": d_s1}[sk]
        da = ds * (a[sk] > 0)
        d_h, dW, db = conv_bwd(a[hk], L[l_b][0], da)
        grads[l_b] = (dW, db)
        da = d_h * (a[hk] > 0)
        d_p, dW, db = conv_bwd(a[pk], L[l_a][0], da)
        grads[l_a] = (dW, db)
        below = pool_bwd(d_p)
        if sk == "s3":
            d_s2 = d_s2 + below
        elif sk == "s2":
            d_s1 = d_s1 + below
        else:
            d_s0 = d_s0 + below
    da = d_s0 * (a["s0"] > 0)
    d_h, dW, db = conv_bwd(a["h0"], L[1][0], da)
    grads[1] = (dW, db)
    da = d_h * (a["h0"] > 0)
    _, dW, db = conv_bwd(a["x"], L[0][0], da)
    grads[0] = (dW, db)
    flat = np.concatenate([np.concatenate([g[0].ravel(), g[1]]) for g in grads])
    return loss, flat


# ---------------------------------------------------------------------------
# Input features and output interpolation of the warm start
# ---------------------------------------------------------------------------
GAP_SCALES = (0.005, 0.02, 0.08)


def features(f, G, L, h, E1, nu1, E2, nu2, F):
    """(G, G, 16) inputs: the gap to the lowest point of f, cell-averaged
    (N >= G) or repeated (N < G) onto G x G, clipped at three length
    scales s L; then log10(h/L)/3, log10(E1/E2)/2, 2 nu1, 2 nu2,
    log10(F/(E2* L^2))/4 and 1; the rest zero."""
    f = np.asarray(f, dtype=np.float64)
    N = f.shape[0]
    g = f - f.min()
    if N >= G:
        r = N // G
        g = g.reshape(G, r, G, r).mean(axis=(1, 3))
    else:
        r = G // N
        g = np.repeat(np.repeat(g, r, axis=0), r, axis=1)
    x = np.zeros((G, G, C))
    for c, s in enumerate(GAP_SCALES):
        x[..., c] = np.minimum(g / (s * L), 1.0)
    E2s = E2 / (1.0 - nu2 * nu2)
    scal = [np.log10(max(h, 1e-12) / L) / 3.0, np.log10(E1 / E2) / 2.0, 2.0 * nu1, 2.0 * nu2,
            np.log10(max(F, 1e-300) / (E2s * L * L)) / 4.0, 1.0]
    for c, v in enumerate(scal):
        x[..., 3 + c] = v
    return x


def prolong(z, N, cut=0.0):
    """Initial pressure on N x N from the head output z (G x G):
    q = softplus(z) / mean(q), zero below cut, then cell-centred bilinear
    interpolation with clamped edges (N >= G) or cell averages (N < G)."""
    z = np.asarray(z, dtype=np.float64)
    G = z.shape[0]
    q = softplus(z)
    q = q / q.mean()
    q = np.where(q < cut, 0.0, q)
    if N < G:
        r = G // N
        return q.reshape(N, r, N, r).mean(axis=(1, 3))
    s = (np.arange(N) + 0.5) * G / N - 0.5
    i0 = np.floor(s).astype(int)
    w = s - i0
    lo = np.clip(i0, 0, G - 1)
    hi = np.clip(i0 + 1, 0, G - 1)
    rows = (1 - w)[:, None] * q[lo, :] + w[:, None] * q[hi, :]
    return np.ascontiguousarray((1 - w)[None, :] * rows[:, lo] + w[None, :] * rows[:, hi])
