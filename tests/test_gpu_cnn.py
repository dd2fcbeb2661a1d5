"""Flip-proposal CNN kernels on the GPU vs the FP64 oracle (oracle/cnn.py),
and the learned search's exactness.

The network runs with BF16 operands on the matrix cores and FP32
accumulation.  BF16 has unit roundoff u = 2^-8 (about 3.9e-3); each product
of two rounded operands carries at most about 2u relative error and the FP32
accumulation adds nothing comparable, so a layer's output is within a few u of
the FP64 result in the 2-norm, and four layers stay within about 5u = 2e-2.
That is the bar for the forward output.  Gradients are pinned exactly on
data where BF16 rounding is exact, and loosely on generic data.
"""
import numpy as np
import pytest

import oracle
import oracle.cnn as ocnn
import workloads
import paper_2501_18054_amd as P
from gpu_util import say

pytestmark = pytest.mark.gpu

BF16_TOL = 2e-2
C0 = ocnn.CHANNELS[0]


def _nrel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _params(seed, bias=0.1):
    rng = np.random.default_rng(seed)
    ps = ocnn.init_params(rng)
    for k in range(1, len(ps), 2):
        ps[k] = bias * rng.standard_normal(ps[k].shape)
    # the model holds float32 masters: the oracle uses exactly those values
    return [np.float32(p).astype(np.float64) for p in ps]


def _flat(ps):
    return np.concatenate([p.ravel() for p in ps]).astype(np.float32)


@pytest.mark.parametrize("H,W,N", [(7, 21, 3), (5, 16, 1), (12, 33, 4)])
def test_forward_matches_oracle(H, W, N):
    say(f"cnn forward H={H} W={W} N={N}")
    m = P.Model(H, W, max_batch=4, seed=1)
    ps = _params(10 + H)
    m.set_params(_flat(ps))
    rng = np.random.default_rng(H * W)
    X = rng.standard_normal((N, C0, H, W)).astype(np.float32)
    Y = m.forward(X)
    Yo, _ = ocnn.forward(ps, X.astype(np.float64))
    assert Y.shape == Yo.shape
    assert _nrel(Y, Yo) < BF16_TOL
    m.close()


def test_initial_params_are_he_normal():
    m = P.Model(8, 8, max_batch=1, seed=5)
    ps = m.unflatten(m.get_params())
    for l, cin in enumerate(ocnn.CHANNELS[:-1]):
        W, b = ps[2 * l], ps[2 * l + 1]
        std = np.sqrt(2.0 / (9 * cin))
        assert abs(W.std() / std - 1.0) < 0.25
        assert np.all(b == 0)
    m.close()


def _bf16_exact(a):
    """True if every value is a float32 whose low 16 bits are zero (BF16)."""
    a = np.asarray(a, np.float64)
    f = a.astype(np.float32)
    return bool(np.array_equal(f.astype(np.float64), a)
                and not np.any(f.view(np.uint32) & 0xFFFF))


def _exact_case(seed, H, W, N, taps=(4, 4, 4, 8)):
    """A network and batch on which BF16 rounding is exact everywhere.

    Sparse weights in {+-1/2, +-1} (`taps` nonzeros per output channel),
    inputs in {0, 1/4, 1/2, 3/4}, first-layer biases in eighths, targets at
    Y -+ 1/2 and N H W a power of two: every value the kernels round to BF16
    (inputs, activations, output gradients of every layer) then has at most 8
    significant bits, and every FP32 sum is exact, so the GPU result must equal
    the FP64 oracle's up to FP32 storage.  Returns None if some value of this
    draw has more bits (checked here, on the CPU)."""
    rng = np.random.default_rng(seed)
    ch = ocnn.CHANNELS
    ps = []
    for l, (cin, cout) in enumerate(zip(ch[:-1], ch[1:])):
        Wl = np.zeros((cout, cin * 9))
        for o in range(cout):
            idx = rng.choice(cin * 9, taps[l], replace=False)
            Wl[o, idx] = rng.choice([-1.0, -0.5, 0.5, 1.0], taps[l])
        ps += [Wl.reshape(cout, cin, 3, 3),
               rng.integers(-2, 3, cout) / 8.0 if l == 0 else np.zeros(cout)]
    X = rng.integers(0, 4, (N, C0, H, W)) / 4.0
    Y, cache = ocnn.forward(ps, X)
    T = Y - 0.5 * rng.choice([-1.0, 1.0], Y.shape)
    ok = _bf16_exact(X)
    for _, Z in cache:
        ok = ok and _bf16_exact(np.maximum(Z, 0.0))
    d = np.clip(Y - T, -1.0, 1.0) / Y.size
    ok = ok and _bf16_exact(d)
    for l in reversed(range(4)):
        A, Z = cache[l]
        if l < 3:
            d = d * (Z > 0)
        ok = ok and _bf16_exact(d)
        d = ocnn.conv_backward(A, ps[2 * l], d)[0]
    return (ps, X, T) if ok else None


@pytest.mark.parametrize("H,W,N", [(16, 8, 1), (4, 32, 2), (8, 16, 4)])
def test_gradients_exact_on_bf16_exact_data(H, W, N):
    case = None
    for seed in range(40):
        case = _exact_case(seed, H, W, N)
        if case:
            break
    assert case is not None
    ps, X, T = case
    say(f"cnn exact grads H={H} W={W} N={N} seed={seed}")
    m = P.Model(H, W, max_batch=N, seed=2)
    m.set_params(_flat(ps))
    loss, g = m.train_step(X.astype(np.float32), T.astype(np.float32), lr=0.0, want_grads=True)
    Lo, go, Yo = ocnn.loss_and_grad(ps, X, T)
    assert loss == Lo
    assert np.array_equal(m.forward(X.astype(np.float32)), Yo.astype(np.float32))
    for k, (a, b) in enumerate(zip(m.unflatten(g), go)):
        assert np.max(np.abs(a - b)) <= 1e-6 * max(np.max(np.abs(b)), 1e-30), \
            f"parameter tensor {k}"
        assert np.count_nonzero(b) > 0


def test_gradients_random_data():
    """Generic data: the sums behind a gradient cancel (terms of both signs
    over every pixel), so BF16's relative error on the terms (a few u) becomes
    a larger error relative to the result, about sqrt(#terms) u for random
    signs; the bar is 0.1 in the 2-norm per tensor.  Exactness of the index
    arithmetic is pinned by the BF16-exact cases above."""
    H, W, N = 9, 20, 3
    say(f"cnn train_step grads H={H} W={W} N={N}")
    m = P.Model(H, W, max_batch=N, seed=2)
    ps = _params(3)
    m.set_params(_flat(ps))
    rng = np.random.default_rng(4)
    X = rng.standard_normal((N, C0, H, W)).astype(np.float32)
    T = (2.0 * rng.standard_normal((N, 1, H, W))).astype(np.float32)
    loss, g = m.train_step(X, T, lr=0.0, want_grads=True)
    Lo, go, _ = ocnn.loss_and_grad(ps, X.astype(np.float64), T.astype(np.float64))
    assert abs(loss - Lo) < BF16_TOL * Lo
    for k, (a, b) in enumerate(zip(m.unflatten(g), go)):
        assert _nrel(a, b) < 0.1, f"parameter tensor {k}"
    # lr = 0 leaves the parameters untouched
    assert np.array_equal(m.get_params(), _flat(ps))
    m.close()


def test_adam_first_step():
    """Adam's first step is -lr g / (|g| + eps) (the bias corrections
    cancel).  On BF16-exact data the gradient is exact, so every coordinate
    must take exactly that step from the oracle's gradient, up to FP32
    rounding of the update (a few ulp of the weight)."""
    H, W, N = 8, 16, 2
    ps, X, T = _exact_case(0, H, W, N)
    say("cnn adam step")
    m = P.Model(H, W, max_batch=N, seed=3)
    w0 = _flat(ps)
    m.set_params(w0)
    lr = 1e-3
    m.train_step(X.astype(np.float32), T.astype(np.float32), lr=lr)
    w1 = m.get_params().astype(np.float64)
    _, go, _ = ocnn.loss_and_grad(ps, X, T)
    g = np.concatenate([x.ravel() for x in go])
    want = w0.astype(np.float64) - lr * g / (np.abs(g) + 1e-8)
    tol = 4 * np.finfo(np.float32).eps * np.abs(w0) + 1e-5 * lr
    assert np.all(np.abs(w1 - want) <= tol)
    assert np.count_nonzero(g) > 0.3 * g.size
    m.close()


def test_training_tracks_oracle_training():
    """Fit a random teacher network: the same Adam steps from the same
    initial weights on the same batches, on the GPU (BF16 operands) and in the
    FP64 oracle.  Each epoch's mean loss agrees within 25 %, and the loss falls
    below 30 % of its first-epoch value."""
    H = W = 8
    N, n_img, epochs, lr = 8, 64, 12, 2e-3
    say("cnn training vs oracle training")
    rng = np.random.default_rng(11)
    teacher = _params(12, bias=0.05)
    X = rng.standard_normal((n_img, C0, H, W)).astype(np.float32)
    T = ocnn.forward(teacher, X.astype(np.float64))[0].astype(np.float32)
    ps = [np.float32(p).astype(np.float64) for p in ocnn.init_params(np.random.default_rng(13))]
    m = P.Model(H, W, max_batch=N, seed=0)
    m.set_params(_flat(ps))
    mo = [np.zeros_like(p) for p in ps]
    vo = [np.zeros_like(p) for p in ps]
    t = 0
    gpu, ref = [], []
    for ep in range(epochs):
        lg = lo = 0.0
        for i in range(0, n_img, N):
            xb, tb = X[i:i + N], T[i:i + N]
            lg += m.train_step(xb, tb, lr=lr)[0]
            L, g, _ = ocnn.loss_and_grad(ps, xb.astype(np.float64), tb.astype(np.float64))
            t += 1
            ocnn.adam_step(ps, g, mo, vo, t, lr=lr)
            lo += L
        gpu.append(lg)
        ref.append(lo)
    assert ref[-1] < 0.3 * ref[0]
    for a, b in zip(gpu, ref):
        assert abs(a - b) < 0.25 * b
    m.close()


def test_model_errors():
    with pytest.raises(P.PngfError):
        P.Model(100, 100)          # more than 8192 pixels
    m = P.Model(4, 4, max_batch=2)
    with pytest.raises(P.PngfError):
        m.forward(np.zeros((3, C0, 4, 4), np.float32))   # beyond max_batch
    m.close()


# ----------------------------------------------------------------- features
def test_features_match_oracle():
    p = workloads.config0()
    h = P.Handle(p).bind(P.default_options())
    rng = np.random.default_rng(5)
    for bits in (p.init_bits, (rng.random(p.n_d) < 0.5).astype(np.uint8)):
        say("config0 features")
        h.set_design(bits)
        X = h.features()
        Xo = ocnn.features(p, bits)
        assert X.shape == Xo.shape == (C0, p.n_d)
        assert np.all(np.abs(X - Xo) <= 1e-6 * np.maximum(1.0, np.abs(Xo)))
    h.close()


# ----------------------------------------------------------- learned search
def _oracle_f(p, bits):
    xs = [oracle.pngf_state(p, bits, fi)[1] for fi in range(p.nfreq)]
    return oracle.objective(p, xs)


def _oracle_steepest(p, bits, eta=1e-9, cap=400):
    bits = bits.copy()
    seq = []
    for _ in range(cap):
        f = _oracle_f(p, bits)
        fs = oracle.score_all(p, bits)
        i = int(np.argmax(fs))
        if not fs[i] - f > eta * f:
            break
        bits[i] ^= 1
        seq.append(i)
    return seq, bits


def test_learned_full_k_is_exact_steepest_ascent():
    """With k = N_d every pixel is scored exactly, so whatever the network
    says the search is exact steepest ascent."""
    p = workloads.config0()
    h = P.Handle(p).bind(P.default_options())
    m = P.Model(p.design_side, p.design_side, max_batch=1, seed=21)
    say("config0 learned search k = n_d")
    h.set_design(p.init_bits)
    r = h.learned_dbs_run(m, k=p.n_d, max_accepts=400)
    seq, bits = _oracle_steepest(p, p.init_bits)
    assert r["converged"]
    assert list(r["accepted"]) == seq
    assert abs(r["f_final"] - _oracle_f(p, bits)) < 1e-10 * r["f_final"]
    m.close()
    h.close()


@pytest.mark.parametrize("use_model,k", [(True, 1), (True, 7), (False, 7), (False, 100)])
def test_ranked_search_accepts_only_exact_improvements(use_model, k):
    """Every accepted flip is an exact improvement (full re-solves), the
    final design is a local optimum, and the evaluation count is consistent:
    between N_d (the final state scans the whole ranking) and N_d per state."""
    p = workloads.config0()
    h = P.Handle(p).bind(P.default_options())
    m = P.Model(p.design_side, p.design_side, max_batch=1, seed=22) if use_model else None
    say(f"config0 ranked search model={use_model} k={k}")
    h.set_design(p.init_bits)
    r = h.learned_dbs_run(m, k=k, max_accepts=400)
    assert r["converged"]
    bits = p.init_bits.copy()
    f = _oracle_f(p, bits)
    for j, i in enumerate(r["accepted"]):
        bits[i] ^= 1
        fn = _oracle_f(p, bits)
        assert fn - f > 1e-9 * f * (1 - 1e-6)
        assert abs(r["f_trace"][j] - fn) < 1e-10 * fn
        f = fn
    fs = oracle.score_all(p, bits)
    assert np.all(fs - f <= 1e-9 * f * (1 + 1e-6))
    n = r["n_accepted"]
    assert p.n_d <= r["attempts"] <= (n + 1) * p.n_d
    assert r["attempts"] >= min(k, p.n_d) * (n + 1)
    if m is not None:
        m.close()
    h.close()


def test_learned_rejects_bad_arguments():
    p = workloads.config0()
    h = P.Handle(p).bind(P.default_options())
    h.set_design(p.init_bits)
    m = P.Model(p.design_side, p.design_side + 1, max_batch=1)
    with pytest.raises(P.PngfError):
        h.learned_dbs_run(m, k=4)      # image size differs from the design
    m.close()
    m = P.Model(p.design_side, p.design_side, max_batch=1)
    with pytest.raises(P.PngfError):
        h.learned_dbs_run(m, k=0)
    with pytest.raises(P.PngfError):
        h.learned_dbs_run(m, k=p.n_d + 1)
    m.close()
    h.close()
