"""Training data and training loop of the flip-proposal CNN.

Every number here comes from libpngf: the exact objective changes (the PNGF
candidate scores of eq. lru_eobj_rs, FP64), the CNN inputs, and the network's
forward/backward/Adam kernels.  This module only chooses which states to log,
shuffles and batches.

Training pairs: at a state of a search trajectory, the inputs are the seven
per-pixel channels of ``Handle.features`` and the target of pixel m is
asinh(df_m / (s f)) with df_m the exact objective change of flipping m, f the
current objective and s = 1e-3 (a signed log-like scale: improving flips of
0.1 % of f map to about 0.9, large ones grow logarithmically).
"""
from __future__ import annotations

import numpy as np

TARGET_SCALE = 1e-3


def target_from_df(df, f, scale=TARGET_SCALE):
    return np.arcsinh(np.asarray(df) / (scale * f)).astype(np.float32)


def design_hw(prob):
    return int(prob.design_side), int(prob.design_side)


def log_state(h, prob):
    """(X [7,H,W], T [1,H,W]) of the handle's current state."""
    H, W = design_hw(prob)
    f, _ = h.evaluate()
    fnew = h.score_flips(np.arange(h.n_d, dtype=np.int32))
    X = h.features().reshape(-1, H, W)
    T = target_from_df(fnew - f, f).reshape(1, H, W)
    return X, T


def log_trajectory(h, prob, bits0, accepted, every=8):
    """Pairs at every `every`-th state along an accepted-flip sequence."""
    h.set_design(bits0)
    X, T = [], []
    acc = np.asarray(accepted, dtype=np.int32)
    for a in range(0, len(acc) + 1, every):
        x, t = log_state(h, prob)
        X.append(x)
        T.append(t)
        if a < len(acc):
            h.accept_flips(acc[a:a + every])
    return X, T


def greedy_trajectory(h, bits0, max_steps, eta=1e-9):
    """Exact steepest ascent: accept the best improving flip until none."""
    h.set_design(bits0)
    cand = np.arange(h.n_d, dtype=np.int32)
    seq = []
    for _ in range(max_steps):
        f, _ = h.evaluate()
        fnew = h.score_flips(cand)
        i = int(np.argmax(fnew))
        if not fnew[i] - f > eta * f:
            break
        h.accept_flips([i])
        seq.append(i)
    return np.asarray(seq, dtype=np.int32)


def collect(h, prob, every=8, greedy=True, greedy_steps=4096):
    """Training pairs of one problem: its DBS trajectory (and optionally its
    exact steepest-ascent trajectory, the states the learned search visits)."""
    h.set_design(prob.init_bits)
    r = h.dbs_run(prob.perms)
    X, T = log_trajectory(h, prob, prob.init_bits, r["accepted"], every)
    if greedy:
        seq = greedy_trajectory(h, prob.init_bits, greedy_steps)
        x2, t2 = log_trajectory(h, prob, prob.init_bits, seq, every)
        X += x2
        T += t2
    return X, T


def train(model, X, T, epochs=20, batch=32, lr=1e-3, seed=0, log=None):
    """Minibatch Adam over the logged pairs; returns the per-epoch mean loss."""
    X = np.ascontiguousarray(np.stack(X), dtype=np.float32)
    T = np.ascontiguousarray(np.stack(T), dtype=np.float32)
    n = X.shape[0]
    batch = min(batch, model.max_batch)
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        order = rng.permutation(n)
        tot, cnt = 0.0, 0
        for b0 in range(0, n, batch):
            idx = order[b0:b0 + batch]
            loss, _ = model.train_step(X[idx], T[idx], lr)
            tot += loss * len(idx)
            cnt += len(idx)
        hist.append(tot / cnt)
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4f}")
    return hist
