"""Pins of the oracle warm-start network: convolution against scipy's correlate
(the library definition), stride-2 as subsampling, gradients against finite
differences."""
import numpy as np
from scipy import signal

from oracle import cnn


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 9, 7, 3))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    out = cnn.conv3x3(x, w, b, 1)
    ref = np.zeros((2, 9, 7, 4))
    for bb in range(2):
        for co in range(4):
            acc = np.full((9, 7), b[co])
            for ci in range(3):
                acc += signal.correlate(x[bb, :, :, ci], w[co, :, :, ci], mode="same")
            ref[bb, :, :, co] = acc
    assert np.allclose(out, ref, atol=1e-12)
    s2 = cnn.conv3x3(x, w, b, 2)
    assert s2.shape == (2, 5, 4, 4)
    assert np.allclose(s2, out[:, ::2, ::2], atol=1e-12)


def test_conv_backward_finite_differences():
    rng = np.random.default_rng(1)
    for stride in (1, 2):
        x = rng.standard_normal((2, 6, 5, 3))
        w = rng.standard_normal((4, 3, 3, 3))
        b = rng.standard_normal(4)
        dout = rng.standard_normal(cnn.conv3x3(x, w, b, stride).shape)
        dx, dw, db = cnn.conv3x3_backward(x, w, stride, dout)
        f = lambda xx, ww, bb: float(np.sum(dout * cnn.conv3x3(xx, ww, bb, stride)))
        eps = 1e-6
        for idx in [(0, 0, 0, 0), (1, 3, 2, 1), (0, 5, 4, 2)]:
            xp_, xm_ = x.copy(), x.copy()
            xp_[idx] += eps
            xm_[idx] -= eps
            assert abs((f(xp_, w, b) - f(xm_, w, b)) / (2 * eps) - dx[idx]) < 1e-6
        for idx in [(0, 0, 0, 0), (3, 2, 1, 2), (1, 1, 2, 0)]:
            wp_, wm_ = w.copy(), w.copy()
            wp_[idx] += eps
            wm_[idx] -= eps
            assert abs((f(x, wp_, b) - f(x, wm_, b)) / (2 * eps) - dw[idx]) < 1e-6
        assert np.allclose(db, dout.sum(axis=(0, 1, 2)))


def test_network_gradient_finite_differences():
    rng = np.random.default_rng(2)
    params = [(0.3 * rng.standard_normal((co, 3, 3, ci)), 0.1 * rng.standard_normal(co))
              for ci, co, _, _ in cnn.LAYERS]
    # narrow the network for speed: keep shapes, small spatial size
    x = rng.standard_normal((1, 8, 8, 2))
    label = rng.standard_normal((1, 2, 2, 1))
    out, acts = cnn.forward(params, x)
    loss, dout = cnn.mse(out, label, 0.5)
    grads = cnn.backward(params, acts, dout)
    eps = 1e-6
    for li, idx in [(0, (3, 1, 1, 0)), (1, (5, 2, 0, 7)), (2, (0, 1, 2, 31)), (3, (0, 0, 1, 4))]:
        w, b = params[li]
        wp_ = w.copy(); wp_[idx] += eps
        wm_ = w.copy(); wm_[idx] -= eps
        pp = list(params); pp[li] = (wp_, b)
        pm = list(params); pm[li] = (wm_, b)
        lp_ = cnn.mse(cnn.forward(pp, x)[0], label, 0.5)[0]
        lm_ = cnn.mse(cnn.forward(pm, x)[0], label, 0.5)[0]
        assert abs((lp_ - lm_) / (2 * eps) - grads[li][0][idx]) < 1e-5 * max(1.0, abs(grads[li][0][idx]))
