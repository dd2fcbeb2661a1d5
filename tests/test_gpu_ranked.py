"""Ranked search on the device (pngf_learned_dbs_run with chunks of one pixel):
at every state the pixels are ranked (by the network, or by the first-order
change) and the first improving pixel of the ranking is accepted; the
ranking, the key selection and the step run on the device for every form.

  * FP64 plain: identical, accept for accept, to a host loop built from the
    public calls (features, network forward, exact scores of every
    candidate, first improving pixel in ranked order, Sherman-Morrison
    accept);
  * mixed (FP32 steps, FP64 decisions inside the error band) and R-form: the
    ranking is computed from each form's own state, so trajectories may part
    from the FP64 one where two ranked scores nearly tie; what is asserted is
    that every accepted flip is an exact improvement (replayed on an FP64
    handle), that the final objective equals the oracle's full re-solve to
    1e-10, and that the converged design is a single-flip local optimum
    (every flip scored in FP64: none improves).
"""
import numpy as np
import pytest

import oracle
import workloads
import paper_2501_18054_amd as P
from gpu_util import say

pytestmark = pytest.mark.gpu

ETA = 1e-9


def _host_ranked(h, p, model, max_acc):
    """The ranked-search policy from the public calls (reference)."""
    H = W = p.design_side
    h.set_design(p.init_bits)
    cand = np.arange(h.n_d, dtype=np.int32)
    acc, ftr = [], []
    for _ in range(max_acc):
        f, _ = h.evaluate()
        X = h.features().reshape(1, 7, H, W)
        s = (model.forward(X) if model is not None else X[:, 6]).ravel()
        order = np.lexsort((np.arange(s.size), -s))   # best first, ties by pixel id
        fn = h.score_flips(cand)
        imp = fn[order] - f > ETA * f
        if not imp.any():
            break
        m = int(order[np.argmax(imp)])
        h.accept_flips([m])
        acc.append(m)
        ftr.append(fn[m])
    return acc, np.asarray(ftr)


@pytest.mark.parametrize("ranker", ["first_order", "network"])
def test_ranked_plain_equals_host_loop(ranker):
    p = workloads.config3_problem(workloads.CONFIG3_EVAL_SEEDS[1])
    say(f"ranked search FP64 vs host loop ({ranker})")
    h = P.Handle(p).bind(P.default_options(max_accepts=4096, max_sweeps=2))
    model = P.Model(40, 40, max_batch=1, seed=5) if ranker == "network" else None
    want, wtr = _host_ranked(h, p, model, 48)
    h.set_design(p.init_bits)
    r = h.learned_dbs_run(model, k=1, max_accepts=48)
    assert r["accepted"].tolist() == want
    assert np.max(np.abs(r["f_trace"] - wtr) / wtr) < 1e-12
    if model is not None:
        model.close()
    h.close()


def _exact_checks(p, r):
    """Every accept improves f by more than eta f at its state (FP64
    handle), the final objective equals the oracle's, and the final design is
    a single-flip local optimum."""
    h = P.Handle(p).bind(P.default_options(max_accepts=64, max_sweeps=2))
    h.set_design(p.init_bits)
    f, _ = h.evaluate()
    for j, m in enumerate(r["accepted"]):
        fn = h.score_flips([m])[0]
        assert fn - f > ETA * f, j
        h.accept_flips([m])
        f = fn
    bits = p.init_bits.copy()
    for m in r["accepted"]:
        bits[m] ^= 1
    xs = [oracle.field(p, bits, fi) @ p.w[0] for fi in range(p.nfreq)]
    fo = oracle.objective(p, np.asarray(xs)[:, None])
    assert abs(r["f_final"] - fo) <= 1e-10 * fo
    if r["converged"]:
        fn = h.score_flips(np.arange(h.n_d, dtype=np.int32))
        assert not np.any(fn - fo > ETA * fo)
    h.close()


@pytest.mark.parametrize("form", ["plain", "mixed", "rform"])
@pytest.mark.parametrize("which", ["config1", "broadband"])
def test_ranked_forms_exact_and_converged(form, which):
    p = (workloads.config3_problem(workloads.CONFIG3_EVAL_SEEDS[2]) if which == "config1"
         else workloads.config4_scaled())
    prec = {"plain": P.PNGF_FP64_PLAIN, "mixed": P.PNGF_MIXED, "rform": P.PNGF_RFORM}[form]
    say(f"ranked search to convergence, {which}, {form}")
    h = P.Handle(p).bind(P.default_options(precision=prec, max_accepts=8192, max_sweeps=2))
    h.set_design(p.init_bits)
    r = h.learned_dbs_run(None, k=1, max_accepts=8192)
    assert r["converged"]
    assert r["n_accepted"] > 10
    h.close()
    _exact_checks(p, r)


def test_ranked_rejects_bad_arguments():
    p = workloads.config0()
    say("ranked search argument checks")
    h = P.Handle(p).bind(P.default_options(max_accepts=16, max_sweeps=1))
    h.set_design(p.init_bits)
    with pytest.raises(P.PngfError):
        h.learned_dbs_run(None, k=1, max_accepts=17)   # beyond the bound log capacity
    r = h.learned_dbs_run(None, k=1, max_accepts=0)
    assert r["n_accepted"] == 0 and not r["converged"]
    h.close()
