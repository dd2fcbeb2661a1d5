"""Pins for the FP64 CNN reference (CPU only)."""
import numpy as np
import scipy.signal

from oracle import cnn


def test_conv_matches_scipy_correlate2d():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((2, 3, 7, 9))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    Y = cnn.conv(X, W, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(scipy.signal.correlate2d(X[n, c], W[o, c], mode="same")
                             for c in range(3))
            assert np.max(np.abs(Y[n, o] - ref)) < 1e-12


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    params = cnn.init_params(rng, channels=(5, 4, 4, 3, 1))
    for p in params[1::2]:
        p += rng.standard_normal(p.shape) * 0.1    # nonzero biases
    X = rng.standard_normal((2, 5, 6, 5))
    T = rng.standard_normal((2, 1, 6, 5)) * 2.0     # some residuals beyond the Huber knee
    L, grads, _ = cnn.loss_and_grad(params, X, T)
    h = 1e-6
    for k, p in enumerate(params):
        flat = p.reshape(-1)
        idx = rng.choice(flat.size, min(6, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            Lp, _, _ = cnn.loss_and_grad(params, X, T)
            flat[i] = old - h
            Lm, _, _ = cnn.loss_and_grad(params, X, T)
            flat[i] = old
            fd = (Lp - Lm) / (2 * h)
            g = grads[k].reshape(-1)[i]
            assert abs(fd - g) <= 1e-6 * max(1.0, abs(fd)), (k, i, fd, g)


def test_adam_first_step_closed_form():
    p = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -4.0, 0.0])]
    m = [np.zeros(3)]
    v = [np.zeros(3)]
    cnn.adam_step(p, g, m, v, t=1, lr=0.1)
    # first step: m_hat = g, v_hat = g^2 -> step -lr*sign(g) (eps negligible)
    assert np.allclose(p[0], [0.9, -1.9, 3.0], atol=1e-7)
