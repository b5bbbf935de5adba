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
