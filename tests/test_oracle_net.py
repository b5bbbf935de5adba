"""Pin of the FP64 warm-start network reference: its analytic gradient
equals central finite differences of its loss, and the building blocks
satisfy their adjoint identities (so a transposed or dropped term fails)."""
import numpy as np
import pytest

from oracle import net_ref as nr


def _problem(H=16, W=16, n=2, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, H, W, nr.C))
    t = rng.uniform(0.2, 2.0, (n, H, W))
    t /= t.mean(axis=(1, 2), keepdims=True)
    return x, t


def test_gradient_matches_central_differences():
    x, t = _problem()
    params = nr.init_params(3)
    params[nr.LAYER_PARAMS - nr.C:nr.LAYER_PARAMS] += 0.05   # nonzero biases
    loss, g = nr.backward(params, x, t)
    rng = np.random.default_rng(1)
    idx = rng.choice(nr.NPARAM, 60, replace=False)
    # include a few from every layer
    idx = np.concatenate([idx, [l * nr.LAYER_PARAMS + 7 for l in range(nr.NLAYER)],
                          [l * nr.LAYER_PARAMS + 9 * nr.C * nr.C + 2 for l in range(nr.NLAYER)]])
    h = 1e-6
    for i in idx:
        pp = params.copy()
        pp[i] += h
        lp, _ = nr.loss_and_dz(nr.forward(pp, x), t)
        pm = params.copy()
        pm[i] -= h
        lm, _ = nr.loss_and_dz(nr.forward(pm, x), t)
        fd = (lp - lm) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=2e-5, abs=1e-9), f"param {i}"


def test_conv_adjoint_identity():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 8, 8, nr.C))
    y = rng.standard_normal((1, 8, 8, nr.C))
    W = rng.standard_normal((9, nr.C, nr.C))
    b = np.zeros(nr.C)
    lhs = np.sum(nr.conv(x, W, b) * y)
    dx, _, _ = nr.conv_bwd(x, W, y)
    assert lhs == pytest.approx(np.sum(x * dx), rel=1e-12)


def test_pool_up_adjoints():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1, 8, 8, nr.C))
    y = rng.standard_normal((1, 4, 4, nr.C))
    assert np.sum(nr.pool(x) * y) == pytest.approx(np.sum(x * nr.pool_bwd(y)), rel=1e-12)
    assert np.sum(nr.up(y) * x) == pytest.approx(np.sum(y * nr.up_bwd(x)), rel=1e-12)


def test_conv_is_direct_correlation():
    """One output value written out by hand from the definition."""
    rng = np.random.default_rng(4)
    x = rng.standard_normal((1, 5, 5, nr.C))
    W = rng.standard_normal((9, nr.C, nr.C))
    b = rng.standard_normal(nr.C)
    y = nr.conv(x, W, b)
    yy, xx, co = 2, 0, 5
    val = b[co]
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if 0 <= yy + dy < 5 and 0 <= xx + dx < 5:
                val += np.dot(W[3 * (dy + 1) + dx + 1, co], x[0, yy + dy, xx + dx])
    assert y[0, yy, xx, co] == pytest.approx(val, rel=1e-13)


def test_normalised_output_has_unit_mean():
    z = np.random.default_rng(5).standard_normal((3, 8, 8))
    ph = nr.normalised_pressure(z)
    np.testing.assert_allclose(ph.mean(axis=(1, 2)), 1.0, rtol=1e-14)


def test_features_pins():
    """Flat profile: zero gap; a step of height 0.05 L: the three channels
    read 1, 1 and 0.625 outside; the scalars at round values."""
    G, L = 32, 2.0
    f = np.zeros((64, 64))
    f[:, 32:] = 0.05 * L
    x = nr.features(f, G, L, h=0.002, E1=100.0, nu1=0.25, E2=1.0, nu2=0.0, F=1e-4 * L * L)
    assert np.all(x[:, :16, :3] == 0.0)
    np.testing.assert_allclose(x[:, 16:, 0], 1.0)
    np.testing.assert_allclose(x[:, 16:, 1], 1.0)
    np.testing.assert_allclose(x[:, 16:, 2], 0.625)
    np.testing.assert_allclose(x[0, 0, 3:9], [-1.0, 1.0, 0.5, 0.0, -1.0, 1.0])
    assert np.all(x[..., 9:] == 0.0)
    # coarser profile than the grid: repeated cells
    x2 = nr.features(f[::4, ::4], G, L, 0.002, 100.0, 0.25, 1.0, 0.0, 1e-4 * L * L)
    np.testing.assert_array_equal(x2[..., :3], x[..., :3])


def test_prolong_pins():
    """Constant field -> constant 1; a field linear in the cell-centre
    coordinate is reproduced exactly away from the clamped edge; the
    N < G branch averages; cut zeroes small values."""
    G = 16
    np.testing.assert_allclose(nr.prolong(np.full((G, G), 0.3), 64), 1.0)
    # choose z so that softplus(z) is linear in y: z = log(expm1(q))
    yc = np.arange(G) + 0.5
    q = np.repeat((1.0 + 0.1 * yc)[:, None], G, axis=1)
    z = np.log(np.expm1(q))
    p = nr.prolong(z, 64)
    yf = (np.arange(64) + 0.5) * G / 64
    interior = (yf > 0.5) & (yf < G - 0.5)
    expect = (1.0 + 0.1 * yf) / q.mean()
    np.testing.assert_allclose(p[interior, 5], expect[interior], rtol=1e-12)
    pc = nr.prolong(z, 4)
    np.testing.assert_allclose(pc.mean(), 1.0, rtol=1e-12)
    np.testing.assert_allclose(pc[:, 0], [(q[4 * i:4 * i + 4, :4] / q.mean()).mean() for i in range(4)],
                               rtol=1e-12)
    zz = np.array([[-10.0, 5.0], [5.0, 5.0]]).repeat(8, 0).repeat(8, 1)
    assert np.all(nr.prolong(zz, 16, cut=0.01)[:8, :8] == 0.0)


def test_loss_zero_at_match_and_scale_invariant():
    """softplus(z) proportional to t gives zero loss and zero gradient;
    scaling t by a constant leaves loss and gradient unchanged."""
    rng = np.random.default_rng(5)
    t = rng.uniform(0.1, 3.0, (2, 8, 8))
    z = np.log(np.expm1(0.7 * t))
    loss, dz = nr.loss_and_dz(z, t)
    assert loss < 1e-28 and np.abs(dz).max() < 1e-14
    z2 = rng.standard_normal((2, 8, 8))
    l1, d1 = nr.loss_and_dz(z2, t)
    l2, d2 = nr.loss_and_dz(z2, 123.0 * t)
    assert abs(l1 - l2) < 1e-14 * l1 and np.allclose(d1, d2, rtol=1e-12, atol=0)
