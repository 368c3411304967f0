"""Pins of the reference U-Net: convolution against a library routine, the
whole-network gradient against central finite differences (FP64), and the
closed form of Adam's first step."""
import numpy as np
import pytest
from scipy.signal import correlate

from oracle import convnet


def test_conv_matches_scipy_correlate_and_stride():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((1, 5, 6, 4, 1))
    W = rng.standard_normal((27, 1, 1))
    y = convnet.conv(x, W, np.zeros(1), 3, 1)
    ref = correlate(np.pad(x[0, ..., 0], 1), W[:, 0, 0].reshape(3, 3, 3), mode="valid")
    assert np.allclose(y[0, ..., 0], ref, atol=1e-12)
    y2 = convnet.conv(x, W, np.zeros(1), 3, 2)
    assert y2.shape[1:4] == (3, 3, 2)
    assert np.allclose(y2[0, ..., 0], ref[::2, ::2, ::2], atol=1e-12)
    # channel mixing is a matrix product per tap
    x3 = rng.standard_normal((2, 3, 3, 3, 4))
    W1 = rng.standard_normal((1, 4, 5))
    assert np.allclose(convnet.conv(x3, W1, np.ones(5), 1, 1), x3 @ W1[0] + 1.0)


@pytest.mark.parametrize("levels", [1, 3])
def test_network_gradient_matches_finite_differences(levels):
    rng = np.random.default_rng(1 + levels)
    specs = convnet.layer_specs(levels, 3, 4, 4)
    n = convnet.param_count(specs)
    params = 0.4 * rng.standard_normal(n)
    x = rng.standard_normal((2, 4, 5, 3, 4))
    y, cache = convnet.forward(params, specs, levels, x)
    dy = rng.standard_normal(y.shape)
    g = convnet.backward(params, specs, levels, cache, dy)
    for idx in rng.choice(n, 40, replace=False):
        e = np.zeros(n); e[idx] = 1e-6
        fp = np.sum(convnet.forward(params + e, specs, levels, x)[0] * dy)
        fm = np.sum(convnet.forward(params - e, specs, levels, x)[0] * dy)
        fd = (fp - fm) / 2e-6
        assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, g[idx])


def test_adam_first_step_is_signed_learning_rate():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    p1, m, v = convnet.adam(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=1e-12)
    assert np.allclose(p1, p - 0.01 * np.sign(g), atol=1e-9)
