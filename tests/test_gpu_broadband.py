"""The broadband setting of workload 4 (eight frequencies over 0.9-1.1 f0,
lambda0/25 grid, 16-cell PML, mean over frequencies) at a size the oracle can
search (workloads.config4_scaled: 160x160 grid, 24x24 design), every form vs
the oracle's golden trajectory.

Bar: identical accepted-flip sequence and attempt count; per-step objectives
within 1e-10 relative for the FP64 forms and 1e-6 for the mixed form (FP32
scores), its final objective within 1e-10 after the FP64 re-formation;
gradients within 1e-10 of the oracle's adjoint gradient; the batched run of
the same problem equal to the solo run.
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
def prob():
    return workloads.config4_scaled()


@pytest.fixture(scope="module")
def gold():
    g = golden("config4_scaled")
    if g is None:
        pytest.skip("golden trajectory of the broadband workload not generated")
    return g


@pytest.mark.parametrize("form", ["plain", "mixed", "rform"])
def test_broadband_identical(prob, gold, form):
    p = prob
    prec = {"plain": P.PNGF_FP64_PLAIN, "mixed": P.PNGF_MIXED, "rform": P.PNGF_RFORM}[form]
    say(f"broadband 8 frequencies {form}")
    h = P.Handle(p).bind(P.default_options(precision=prec, max_accepts=4096, max_sweeps=4))
    h.set_design(p.init_bits)
    res = h.dbs_run(p.perms)
    assert res["accepted"].tolist() == [a[2] for a in gold["accepted"]]
    assert res["attempts"] == gold["attempts"]
    tol = 1e-6 if form == "mixed" else TOL
    assert rel(res["f_trace"], [a[3] for a in gold["accepted"]]) < tol
    assert abs(res["f_final"] - gold["f_final"]) < TOL * gold["f_final"]
    h.close()


def test_broadband_gradient_and_batch(prob, gold):
    import torch
    p = prob
    say("broadband gradient and batch of one")
    stream = torch.cuda.Stream()
    h = P.Handle(p).bind(P.default_options(precision=P.PNGF_MIXED, max_accepts=4096,
                                           max_sweeps=4), stream=stream)
    h.set_design(p.init_bits)
    solo = h.dbs_run(p.perms)
    h.set_design(p.init_bits)
    b = P.Batch([h])
    out = b.dbs_run([p.perms])[0]
    assert out["accepted"].tolist() == solo["accepted"].tolist()
    assert abs(out["f_final"] - solo["f_final"]) <= 1e-12 * solo["f_final"]
    b.close()
    h.close()
    h = P.Handle(p).bind(P.default_options())
    h.set_design(p.init_bits)
    assert rel(h.gradient(), oracle.gradient(p, p.init_bits)) < TOL
    h.close()
