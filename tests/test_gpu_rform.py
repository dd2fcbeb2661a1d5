"""R-form search (FP64 reduced scoring: T0 = C^-1 G plus a panel of the
columns p = T[:, m], every candidate scored from diag(T), E, R') vs the
oracle's FP64 trajectory.

Bar: identical accepted-flip sequence and attempt count, per-step objectives
within 1e-10 relative, fields of the final design within 1e-10 of a fresh
full solve.  Small panel capacities force many folds of the panel into T0;
k_refresh re-anchors the state on an FP64 C^-1 (alone and between folds).
"""
import numpy as np
import pytest

import oracle
import workloads
import paper_2501_18054_amd as P
from gpu_util import say, golden, rel

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _rform(p, **kw):
    opts = P.default_options(precision=P.PNGF_RFORM, max_accepts=8192, max_sweeps=8, **kw)
    h = P.Handle(p).bind(opts)
    h.set_design(p.init_bits)
    return h, h.dbs_run(p.perms)


def _check(res, g):
    assert res["accepted"].tolist() == [a[2] for a in g["accepted"]]
    assert res["attempts"] == g["attempts"]
    assert rel(res["f_trace"], [a[3] for a in g["accepted"]]) < TOL
    assert abs(res["f_final"] - g["f_final"]) < TOL * g["f_final"]


def _final_bits(p, res):
    bits = p.init_bits.copy()
    for m in res["accepted"]:
        bits[m] ^= 1
    return bits


def test_rform_config0_identical():
    p = workloads.config0()
    say("config0 rform")
    h, res = _rform(p)
    _check(res, golden(0))
    # the calls that need C^-1 first bring it to the final design
    bits = _final_bits(p, res)
    cands = np.array([0, 7, 55, 99], np.int32)
    assert rel(h.score_flips(cands), oracle.score_all(p, bits, cands)) < TOL
    h.close()


@pytest.mark.parametrize("k_fold,k_refresh", [(0, 0), (7, 0), (64, 0), (0, 32), (16, 40)])
def test_rform_config1_identical(k_fold, k_refresh):
    g = golden(1)
    if g is None:
        pytest.skip("golden trajectory for workload 1 not generated")
    p = workloads.config1()
    say(f"config1 rform panel capacity {k_fold or 512}, re-anchor every {k_refresh}")
    h, res = _rform(p, k_fold=k_fold, k_refresh=k_refresh)
    _check(res, g)
    f, x, E = h.evaluate(fields=True)
    Eo, xo = oracle.pngf_state(p, _final_bits(p, res), 0)
    assert rel(E[0], Eo) < TOL
    assert abs(f - g["f_final"]) < TOL * g["f_final"]
    # a second run from the same start repeats itself
    h.set_design(p.init_bits)
    res2 = h.dbs_run(p.perms)
    assert res2["accepted"].tolist() == res["accepted"].tolist()
    h.close()


def test_rform_multifrequency_tiny():
    p = workloads.tiny(seed=51, n=24, npml=4, side=5, nfreq=3, n_sweeps=4)
    say("tiny 3-frequency rform")
    r = oracle.dbs(p)
    h, res = _rform(p, k_fold=3)
    assert res["accepted"].tolist() == [a[2] for a in r.accepted]
    assert res["attempts"] == r.attempts
    assert res["converged"] == r.converged
    assert abs(res["f_final"] - r.f_final) < TOL * r.f_final
    h.close()


def test_rform_then_accept_flips():
    """accept_flips after an R-form run starts from the run's final design."""
    p = workloads.config0()
    say("config0 rform then accept_flips")
    h, res = _rform(p)
    bits = _final_bits(p, res)
    h.accept_flips([3, 40])
    bits[3] ^= 1
    bits[40] ^= 1
    f, x, E = h.evaluate(fields=True)
    Eo, xo = oracle.pngf_state(p, bits, 0)
    assert rel(E[0], Eo) < TOL
    h.close()


def test_rform_not_batched():
    p = workloads.config0()
    h = P.Handle(p).bind(P.default_options(precision=P.PNGF_RFORM))
    with pytest.raises(P.PngfError):
        P.Batch([h])
    h.close()
