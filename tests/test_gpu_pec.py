"""Perfectly conducting (PEC) pixels on the GPU path vs the oracle.

The library runs a PEC problem as the transposed j-form (the kernels see
G - I and kappa = -1); the oracle solves the full FDFD system with Ez = 0 on
the conducting nodes.  Bar: fields z (total field on open pixels, equivalent
current on conducting ones) within 1e-10 of the oracle's; the accepted-flip
sequence and attempt count of every form identical to the oracle's, with
objectives within 1e-10 relative (1e-6 for the FP32-derived per-step values
of the mixed form).
"""
import numpy as np
import pytest

import oracle
import workloads
import paper_2501_18054_amd as P
from gpu_util import say, golden, rel

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def metal():
    return workloads.metal()


def _bits_after(p, acc):
    bits = p.init_bits.copy()
    for m in acc:
        bits[m] ^= 1
    return bits


def test_pec_initial_state_and_scores(metal):
    p = metal
    say("metal initial state fp64")
    h = P.Handle(p).bind(P.default_options())
    h.set_design(p.init_bits)
    f, x, Z = h.evaluate(fields=True)
    zo, xo = oracle.pec_state(p, p.init_bits, 0)
    assert rel(Z[0], zo) < TOL
    assert abs(x[0] - xo) < TOL * abs(xo)
    cands = np.array([0, 1, 100, 287, 288, 575], np.int32)
    assert rel(h.score_flips(cands), oracle.score_all(p, p.init_bits, cands)) < TOL
    # accepting flips (both directions) keeps the state exact
    flips = [5, 77, 300, 301]
    h.accept_flips(flips)
    bits = _bits_after(p, flips)
    f, x, Z = h.evaluate(fields=True)
    zo, xo = oracle.pec_state(p, bits, 0)
    assert rel(Z[0], zo) < TOL
    h.refresh()
    f2, x2, Z2 = h.evaluate(fields=True)
    assert rel(Z2[0], zo) < TOL
    h.close()


@pytest.mark.parametrize("form", ["plain", "mixed", "rform"])
def test_pec_dbs_identical_to_oracle(metal, form):
    p = metal
    g = golden("metal")
    if g is None:
        pytest.skip("golden trajectory of the metal workload not generated")
    prec = {"plain": P.PNGF_FP64_PLAIN, "mixed": P.PNGF_MIXED, "rform": P.PNGF_RFORM}[form]
    say(f"metal dbs {form}")
    # The R-form re-anchors on a fresh FP64 inverse every 32 accepts: its
    # incremental updates of E, R' and tau drift to ~5e-10 in f over the
    # 390 accepts without it (FP64 CPU replay of the same updates).
    kw = {"k_refresh": 32} if form in ("mixed", "rform") else {}
    h = P.Handle(p).bind(P.default_options(precision=prec, max_accepts=4096, max_sweeps=8,
                                           **kw))
    h.set_design(p.init_bits)
    res = h.dbs_run(p.perms)
    assert res["accepted"].tolist() == [a[2] for a in g["accepted"]]
    assert res["attempts"] == g["attempts"]
    tol = 1e-6 if form == "mixed" else TOL
    assert rel(res["f_trace"], [a[3] for a in g["accepted"]]) < tol
    assert abs(res["f_final"] - g["f_final"]) < TOL * g["f_final"]
    f, x, Z = h.evaluate(fields=True)
    zo, xo = oracle.pec_state(p, _bits_after(p, res["accepted"]), 0)
    assert rel(Z[0], zo) < TOL
    h.close()


@pytest.mark.parametrize("form", ["plain", "mixed", "rform"])
def test_pec_multifrequency_tiny(form):
    p = workloads.tiny_metal(seed=31, n=22, side=5, nfreq=3, n_sweeps=4)
    prec = {"plain": P.PNGF_FP64_PLAIN, "mixed": P.PNGF_MIXED, "rform": P.PNGF_RFORM}[form]
    say(f"tiny 3-frequency metal {form}")
    r = oracle.dbs(p)
    h = P.Handle(p).bind(P.default_options(precision=prec, max_accepts=512, max_sweeps=8,
                                           k_fold=3))
    h.set_design(p.init_bits)
    res = h.dbs_run(p.perms)
    assert res["accepted"].tolist() == [a[2] for a in r.accepted]
    assert res["attempts"] == r.attempts
    assert res["converged"] == r.converged
    assert abs(res["f_final"] - r.f_final) < TOL * r.f_final
    h.close()


def test_pec_batch_equals_solo():
    import torch
    stream = torch.cuda.Stream()
    probs = [workloads.tiny_metal(seed=s, n=24, side=6, nfreq=1 + s % 2, n_sweeps=6)
             for s in (41, 42, 43)]
    say("metal batch vs solo")
    opts = P.default_options(max_accepts=1024, max_sweeps=6)
    hs = [P.Handle(p).bind(opts, stream=stream) for p in probs]
    solo = []
    for h, p in zip(hs, probs):
        h.set_design(p.init_bits)
        solo.append(h.dbs_run(p.perms))
    for h, p in zip(hs, probs):
        h.set_design(p.init_bits)
    b = P.Batch(hs)
    out = b.dbs_run([p.perms for p in probs])
    for r, s in zip(out, solo):
        assert r["accepted"].tolist() == s["accepted"].tolist()
        assert abs(r["f_final"] - s["f_final"]) <= 1e-12 * abs(s["f_final"])
    b.close()
    for h in hs:
        h.close()


@pytest.mark.parametrize("fill", [0, 1])
def test_pec_all_open_or_all_metal_start(fill):
    """Degenerate start designs: no conductor (C = I) and every pixel a
    conductor (C^-1 is the inverse of the whole G block)."""
    p = workloads.tiny_metal(seed=33, n=22, side=5, nfreq=2, n_sweeps=3)
    p.init_bits[:] = fill
    say(f"tiny metal, every pixel {fill}")
    r = oracle.dbs(p)
    h = P.Handle(p).bind(P.default_options(max_accepts=512, max_sweeps=4))
    h.set_design(p.init_bits)
    f0, x0, Z0 = h.evaluate(fields=True)
    zo, xo = oracle.pec_state(p, p.init_bits, 0)
    assert rel(Z0[0], zo) < TOL
    res = h.dbs_run(p.perms)
    assert res["accepted"].tolist() == [a[2] for a in r.accepted]
    assert res["attempts"] == r.attempts
    assert abs(res["f_final"] - r.f_final) < TOL * r.f_final
    h.close()
