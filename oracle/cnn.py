"""FP64 reference of the flip-proposal CNN (forward, loss, backward, Adam).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The network is not part of the paper: the paper contrasts PNGF's exact
evaluations with surrogate models (Introduction; Discussion).  Here a small
CNN only *ranks* pixels; every accepted flip is still decided by an exact PNGF
evaluation.  Definitions (written out plainly):

    conv(X, W, b)[n, o, y, x] = b[o] + sum_{c, ky, kx} W[o, c, ky, kx]
                                       X[n, c, y + ky - 1, x + kx - 1]
    (3x3 cross-correlation, zero padding, stride 1)

    Z1 = conv(X, W1, b1), A1 = relu(Z1)       7 -> 32 channels
    Z2 = conv(A1, W2, b2), A2 = relu(Z2)     32 -> 32
    Z3 = conv(A2, W3, b3), A3 = relu(Z3)     32 -> 32
    Y  = conv(A3, W4, b4)                     32 -> 1   (flip priority)

    loss = mean over pixels of huber(Y - T), huber(r) = r^2/2 (|r| <= 1),
           |r| - 1/2 otherwise.

    Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
    w -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Inputs (``features``), per design pixel m of an H x W design region, from
the current PNGF state (field E on the design, output row R', the Green
function's diagonal G_mm, outputs x_f, objective f = sum_f c_f |x_f|^2):

    0  design bit
    1  Re E[m] / max|E|        2  Im E[m] / max|E|
    3  Re R'[m] / max|R'|      4  Im R'[m] / max|R'|
    5  |G_mm| / max|G_mm|
    6  asinh(df_lin[m] / (1e-3 f)), the flip's objective change with the
       denominator of eq. lru_eobj_rs set to 1 (first-order field change
       dx = k0^2 delta_m E[m] R'[m]):
       df_lin = sum_f c_f (|x_f + dx_f|^2 - |x_f|^2).
E, R' and G_mm are taken at the first frequency.

Pins: tests/test_oracle_cnn.py checks conv against scipy.signal.correlate2d
summed over input channels, every gradient against central finite
differences, and Adam's first step against its closed form (a step of -lr per
coordinate with a nonzero gradient).  ``features`` is a plain composition of
pinned quantities (E: full solves; R': the adjoint-sensitivity pin of
output_row; G_mm: green_dd).
"""
from __future__ import annotations

import numpy as np

CHANNELS = (7, 32, 32, 32, 1)
FEATURE_SCALE = 1e-3


def init_params(rng, channels=CHANNELS):
    """He-normal weights, zero biases, as float64 arrays."""
    params = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        std = np.sqrt(2.0 / (cin * 9))
        params.append(rng.standard_normal((cout, cin, 3, 3)) * std)
        params.append(np.zeros(cout))
    return params


def conv(X, W, b):
    N, C, H, Wd = X.shape
    O = W.shape[0]
    Xp = np.zeros((N, C, H + 2, Wd + 2))
    Xp[:, :, 1:-1, 1:-1] = X
    Y = np.zeros((N, O, H, Wd)) + b[None, :, None, None]
    for ky in range(3):
        for kx in range(3):
            patch = Xp[:, :, ky:ky + H, kx:kx + Wd]            # N C H W
            Y += np.einsum("oc,nchw->nohw", W[:, :, ky, kx], patch)
    return Y


def conv_backward(X, W, dY):
    """Gradients of conv w.r.t. X, W, b given dL/dY."""
    N, C, H, Wd = X.shape
    Xp = np.zeros((N, C, H + 2, Wd + 2))
    Xp[:, :, 1:-1, 1:-1] = X
    dW = np.zeros_like(W)
    dXp = np.zeros_like(Xp)
    for ky in range(3):
        for kx in range(3):
            patch = Xp[:, :, ky:ky + H, kx:kx + Wd]
            dW[:, :, ky, kx] = np.einsum("nohw,nchw->oc", dY, patch)
            dXp[:, :, ky:ky + H, kx:kx + Wd] += np.einsum("oc,nohw->nchw", W[:, :, ky, kx], dY)
    db = dY.sum(axis=(0, 2, 3))
    return dXp[:, :, 1:-1, 1:-1], dW, db


def forward(params, X):
    """Returns (Y, cache) for the 4-layer network."""
    cache = []
    A = X
    nl = len(params) // 2
    for l in range(nl):
        W, b = params[2 * l], params[2 * l + 1]
        Z = conv(A, W, b)
        cache.append((A, Z))
        A = np.maximum(Z, 0.0) if l < nl - 1 else Z
    return A, cache


def huber(R):
    a = np.abs(R)
    return np.where(a <= 1.0, 0.5 * R * R, a - 0.5)


def loss_and_grad(params, X, T):
    """Mean Huber loss and its gradients w.r.t. every parameter."""
    Y, cache = forward(params, X)
    R = Y - T
    L = float(np.mean(huber(R)))
    dY = np.clip(R, -1.0, 1.0) / R.size
    grads = [None] * len(params)
    nl = len(params) // 2
    d = dY
    for l in reversed(range(nl)):
        A, Z = cache[l]
        if l < nl - 1:
            d = d * (Z > 0)
        dA, dW, db = conv_backward(A, params[2 * l], d)
        grads[2 * l], grads[2 * l + 1] = dW, db
        d = dA
    return L, grads, Y


def adam_step(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in place; t is the 1-based step count."""
    for k in range(len(params)):
        m[k] = b1 * m[k] + (1 - b1) * grads[k]
        v[k] = b2 * v[k] + (1 - b2) * grads[k] ** 2
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        params[k] -= lr * mh / (np.sqrt(vh) + eps)


def features(prob, bits):
    """The seven input channels [7, n_d] of the design ``bits`` (FP64)."""
    from .green import green_dd, output_row, pngf_state
    from .fdfd import objective_norms
    bits = np.asarray(bits, dtype=np.uint8)
    F = prob.nfreq
    delta = np.where(bits != 0, -1.0, 1.0) * (prob.eps_hi - prob.eps_lo)
    xs, f, df = [], 0.0, np.zeros(prob.n_d)
    E0 = R0 = None
    norms = objective_norms(prob)
    for fi in range(F):
        E, x = pngf_state(prob, bits, fi)
        R = output_row(prob, bits, fi)
        if fi == 0:
            E0, R0 = E, R
        c = 1.0 / (F * norms[fi])
        dx = prob.k0[fi] ** 2 * delta * E * R
        f += c * abs(x) ** 2
        df += c * (np.abs(x + dx) ** 2 - abs(x) ** 2)
    g = np.abs(np.diag(green_dd(prob, 0)))
    ae, ar = np.abs(E0).max(), np.abs(R0).max()
    return np.stack([bits.astype(np.float64), E0.real / ae, E0.imag / ae,
                     R0.real / ar, R0.imag / ar, g / g.max(),
                     np.arcsinh(df / (FEATURE_SCALE * f))])
