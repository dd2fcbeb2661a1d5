"""Learned flip proposal, A/B on the eight held-out problems of the
256x256 / 40x40 family (N_d = 1600): the network is trained on the GPU from
(state, exact objective change) pairs logged on eight training problems, then
the ranked search runs on unseen seeds with and without it.

What is asserted (the gain and its price):
  * training is bit-for-bit reproducible (fixed-order gradient reductions):
    two fresh networks trained on the same pairs end with identical weights;
  * every accepted flip is an exact improvement: on the first held-out seed
    the trace is re-checked at every state by the FP64 plain path, and on
    every seed the final objective equals a full sparse re-solve (oracle);
  * over the eight held-out seeds the trained ranking needs well under 60 %
    of the exact evaluations of DBS run to convergence, and under half of
    those of the same ranked search driven by the first-order change, while
    its final objective averages at least 95 % of DBS's (each run ends in a
    local optimum of its own).  An untrained network is compared on the first
    seed.
Wall time is reported, not asserted: on the GPU, DBS scores every candidate
in the same pass as the accept, so fewer evaluations do not mean less time.
"""
import numpy as np
import pytest

import oracle
import workloads
import paper_2501_18054_amd as P
from paper_2501_18054_amd import learned
from gpu_util import say

pytestmark = pytest.mark.gpu

N_TRAIN = 8
EVAL_SEED = workloads.CONFIG3_EVAL_SEEDS[0]
K = 4


@pytest.fixture(scope="module")
def pairs():
    X, T = [], []
    for s in workloads.CONFIG3_TRAIN_SEEDS[:N_TRAIN]:
        say(f"log training pairs, seed {s}")
        p = workloads.config3_problem(s)
        h = P.Handle(p).bind(P.default_options(max_accepts=8192, max_sweeps=8))
        x, t = learned.collect(h, p, every=4, greedy=True)
        X += x
        T += t
        h.close()
    return X, T


@pytest.fixture(scope="module")
def trained(pairs):
    X, T = pairs
    say(f"train on {len(X)} states")
    m = P.Model(40, 40, max_batch=32, seed=0)
    hist = learned.train(m, X, T, epochs=40, batch=32, lr=1e-3)
    assert hist[-1] < 0.8 * hist[0]
    return m


def test_training_is_bit_reproducible(pairs):
    X, T = pairs
    say("train two fresh networks on the same pairs")
    out = []
    for _ in range(2):
        m = P.Model(40, 40, max_batch=32, seed=7)
        hist = learned.train(m, X[:96], T[:96], epochs=3, batch=32, lr=1e-3, seed=3)
        out.append((m.get_params(), hist))
        m.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]


def _replay_exact(h, p, r):
    """Each accepted flip improved f by more than eta f at its state (FP64
    plain path scores), and the trace is the objective after each flip."""
    h.set_design(p.init_bits)
    f, _ = h.evaluate()
    for j, i in enumerate(r["accepted"]):
        fn = h.score_flips([i])[0]
        assert fn - f > 1e-9 * f
        assert abs(fn - r["f_trace"][j]) <= 1e-12 * fn
        h.accept_flips([i])
        f = fn
    return f


def test_learned_ab_on_held_out_seeds(trained):
    rows = []
    for j, seed in enumerate(workloads.CONFIG3_EVAL_SEEDS):
        p = workloads.config3_problem(seed, n_sweeps=30)
        h = P.Handle(p).bind(P.default_options(max_accepts=8192, max_sweeps=30))
        say(f"DBS to convergence, seed {seed}")
        h.set_design(p.init_bits)
        dbs = h.dbs_run(p.perms)
        assert dbs["converged"]
        models = [("trained", trained), ("first_order", None)]
        if j == 0:
            models.append(("untrained", P.Model(40, 40, max_batch=1, seed=99)))
        runs = {}
        for name, model in models:
            say(f"ranked search ({name}), k = {K}, seed {seed}")
            h.set_design(p.init_bits)
            runs[name] = h.learned_dbs_run(model, k=K, max_accepts=8192)
            assert runs[name]["converged"]
        lr = runs["trained"]
        print(f"[learned A/B] seed {seed}: DBS {dbs['attempts']} evals, f {dbs['f_final']:.6g}; "
              + "; ".join(f"{n}: {r['attempts']} evals, f {r['f_final']:.6g}"
                          for n, r in runs.items()), flush=True)
        if j == 0:
            say("replay the trained run's accepts")
            f_end = _replay_exact(h, p, lr)
            assert abs(f_end - lr["f_final"]) <= 1e-10 * lr["f_final"]
            assert lr["attempts"] < 0.5 * runs["untrained"]["attempts"]
        bits = p.init_bits.copy()
        for i in lr["accepted"]:
            bits[i] ^= 1
        xs = [oracle.pngf_state(p, bits, fi)[1] for fi in range(p.nfreq)]
        fo = oracle.objective(p, xs)
        assert abs(lr["f_final"] - fo) <= 1e-10 * fo
        rows.append((dbs["attempts"], dbs["f_final"], lr["attempts"], lr["f_final"],
                     runs["first_order"]["attempts"]))
        h.close()
    a = np.asarray(rows, dtype=np.float64)
    ratio = a[:, 3] / a[:, 1]
    print(f"[learned A/B] trained/DBS evaluations {a[:, 2].sum() / a[:, 0].sum():.3f}, "
          f"trained/first-order {a[:, 2].sum() / a[:, 4].sum():.3f}, objective ratio "
          f"mean {ratio.mean():.4f} min {ratio.min():.4f} max {ratio.max():.4f}", flush=True)
    # the gain, and what it costs in objective
    assert a[:, 2].sum() < 0.6 * a[:, 0].sum()
    assert a[:, 2].sum() < 0.5 * a[:, 4].sum()
    assert ratio.mean() >= 0.95
