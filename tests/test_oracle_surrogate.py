"""Pins of the surrogate oracle: every layer against an independent definition."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import surrogate as NN


def test_conv3x3_matches_library_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 7, 9, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    z = NN.conv3x3(x, w, b)
    for bi in range(2):
        for o in range(4):
            ref = sum(correlate2d(x[bi, :, :, i], w[o, :, :, i], mode="same") for i in range(3)) + b[o]
            assert np.allclose(z[bi, :, :, o], ref, rtol=1e-13, atol=1e-13)


def _fd(f, x, eps=1e-6):
    g = np.zeros_like(x)
    it = np.nditer(x, flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        old = x[i]
        x[i] = old + eps
        hi = f()
        x[i] = old - eps
        lo = f()
        x[i] = old
        g[i] = (hi - lo) / (2 * eps)
    return g


def test_conv3x3_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 4, 5, 2))
    w = rng.standard_normal((3, 3, 3, 2))
    r = rng.standard_normal((2, 4, 5, 3))
    loss = lambda: float(np.sum(r * NN.conv3x3(x, w)))
    gx = _fd(loss, x)
    gw = _fd(loss, w)
    assert np.allclose(NN.conv3x3_dgrad(r, w), gx, rtol=1e-7, atol=1e-8)
    assert np.allclose(NN.conv3x3_wgrad(x, r), gw, rtol=1e-7, atol=1e-8)


def test_pool_and_upsample_adjoints_and_values():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 6, 8, 3))
    y = rng.standard_normal((2, 3, 4, 3))
    assert np.sum(NN.avgpool2(x) * y) == pytest.approx(np.sum(x * NN.avgpool2_grad(y)), rel=1e-13)
    assert np.sum(NN.upsample2(y) * x) == pytest.approx(np.sum(y * NN.upsample2_grad(x)), rel=1e-13)
    assert NN.avgpool2(x)[1, 2, 3, 1] == pytest.approx(np.mean(x[1, 4:6, 6:8, 1]), rel=1e-15)
    up = NN.upsample2(y)
    assert up[0, 5, 7, 2] == y[0, 2, 3, 2] and up[1, 4, 6, 0] == y[1, 2, 3, 0]


def test_patchify_index_convention():
    rng = np.random.default_rng(3)
    f = rng.standard_normal((2, 8, 8, 3))
    p = NN.patchify4(f)
    for b, Y, X, py, px, c in [(0, 0, 0, 0, 0, 0), (1, 1, 0, 3, 2, 1), (0, 1, 1, 1, 3, 2), (1, 0, 1, 2, 0, 0)]:
        assert p[b, Y, X, (py * 4 + px) * 3 + c] == f[b, 4 * Y + py, 4 * X + px, c]
    h = rng.standard_normal((2, 2, 2, 16))
    u = NN.unpatchify4(h)
    for b, Y, X, py, px in [(0, 0, 0, 0, 0), (1, 1, 0, 3, 2), (0, 1, 1, 1, 3)]:
        assert u[b, 4 * Y + py, 4 * X + px] == h[b, Y, X, py * 4 + px]


def test_network_gradients_match_finite_differences():
    """Directional derivatives of the MSE loss along random directions confined to each
    parameter tensor (a wrong gradient in any single tensor fails its own direction)."""
    spec = NN.NetSpec(n=64, width=(4, 4, 8, 8, 8))
    rng = np.random.default_rng(4)
    p = spec.init(5)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    q = rng.uniform(0.1, 2.0, (2, 64, 64)) * 1e6
    v = np.exp(0.5 * rng.standard_normal((2, 64, 64)))
    m = 1.0 + 0.05 * rng.uniform(-1, 1, (2, 64, 64))
    t = rng.standard_normal((2, 64, 64))
    _, g, _ = NN.loss_and_grads(spec, p, q, v, m, t)
    for k in spec.shapes():
        d = rng.standard_normal(p[k].shape)
        eps = 1e-6
        p0 = p[k]
        p[k] = p0 + eps * d
        hi = NN.mse(NN.forward(spec, p, q, v, m)[0], t)
        p[k] = p0 - eps * d
        lo = NN.mse(NN.forward(spec, p, q, v, m)[0], t)
        p[k] = p0
        fd = (hi - lo) / (2 * eps)
        an = float(np.sum(g[k] * d))
        assert an == pytest.approx(fd, rel=1e-6, abs=1e-12), k


def test_param_count_and_flat_roundtrip():
    spec = NN.NetSpec()
    p = spec.init(0)
    flat = spec.flatten(p)
    assert flat.size == spec.param_count()
    assert 0.8e6 < flat.size < 1.2e6  # about one million parameters
    back = spec.unflatten(flat)
    assert all(np.array_equal(back[k], p[k]) for k in p)


def test_adam_first_steps_closed_form():
    rng = np.random.default_rng(6)
    g = rng.standard_normal(7)
    opt = NN.Adam(lr=0.01)
    p = {"w": np.zeros(7)}
    opt.step(p, {"w": g})
    # bias-corrected first moments are g and g^2: the step is lr * g / (|g| + eps)
    assert np.allclose(p["w"], -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14)
    # second step with gradient h, by hand
    h = rng.standard_normal(7)
    opt.step(p, {"w": h})
    m = 0.9 * 0.1 * g + 0.1 * h
    v = 0.999 * 0.001 * g * g + 0.001 * h * h
    step2 = 0.01 * (m / (1 - 0.81)) / (np.sqrt(v / (1 - 0.999 ** 2)) + 1e-8)
    assert np.allclose(p["w"], -0.01 * g / (np.abs(g) + 1e-8) - step2, rtol=1e-12)
