"""Pins of the FP64 reference network (no GPU): the convolution against an
independent correlation routine, the analytic gradient against central
finite differences, GELU against its closed form at special points, and the
parameter count."""
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import cnn


def test_parameter_count():
    # 4->16, 16->16, 16->16, 16->2 with 3x3x3 kernels and biases
    assert cnn.n_params() == (4 * 16 * 27 + 16) + 2 * (16 * 16 * 27 + 16) + (16 * 2 * 27 + 2) == 16466


def test_conv_matches_ndimage_correlate():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 5, 6, 7))
    W = rng.standard_normal((2, 3, 3, 3, 3))
    b = rng.standard_normal(2)
    out = cnn.conv3d(x, W, b)
    for o in range(2):
        ref = b[o] + sum(ndimage.correlate(x[c], W[o, c], mode="constant", cval=0.0) for c in range(3))
        assert np.allclose(out[o], ref, rtol=1e-12, atol=1e-12)


def test_gelu_special_values():
    assert cnn.gelu(np.array(0.0)) == 0.0
    assert cnn.gelu(np.array(1.0)) == pytest.approx(0.8413447460685429, abs=1e-15)  # Phi(1)
    assert cnn.gelu_grad(np.array(0.0)) == pytest.approx(0.5)
    x = np.linspace(-4, 4, 41)
    e = 1e-6
    assert np.allclose((cnn.gelu(x + e) - cnn.gelu(x - e)) / (2 * e), cnn.gelu_grad(x), atol=1e-8)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    theta = 0.2 * rng.standard_normal(cnn.n_params())
    x = rng.standard_normal((4, 4, 5, 3))
    t = rng.standard_normal((2, 4, 5, 3))
    loss, g = cnn.loss_and_grad(theta, x, t)
    for k in rng.choice(cnn.n_params(), 40, replace=False):
        e = 1e-5
        tp, tm = theta.copy(), theta.copy()
        tp[k] += e
        tm[k] -= e
        fd = (cnn.loss_and_grad(tp, x, t)[0] - cnn.loss_and_grad(tm, x, t)[0]) / (2 * e)
        assert fd == pytest.approx(g[k], rel=1e-5, abs=1e-9)


def test_adam_first_step_is_signed_lr():
    """With bias correction, the first Adam step moves every parameter by lr
    against the sign of its gradient (up to eps)."""
    rng = np.random.default_rng(2)
    th = rng.standard_normal(10)
    g = rng.standard_normal(10)
    new, m, v = cnn.adam_step(th, np.zeros(10), np.zeros(10), g, 1, lr=1e-3)
    assert np.allclose(new - th, -1e-3 * np.sign(g), rtol=1e-6)
