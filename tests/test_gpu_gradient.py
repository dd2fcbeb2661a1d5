"""Objective gradient df/d eps_m (pngf_gradient) vs the oracle's adjoint
gradient on full solves.  Bar: max-norm error within 1e-10 of max|grad|, at
the initial design and after a search in every form."""
import numpy as np
import pytest

import oracle
import workloads
import paper_2501_18054_amd as P
from gpu_util import say, rel

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.mark.parametrize("prec", [P.PNGF_FP64_PLAIN, P.PNGF_MIXED, P.PNGF_RFORM])
def test_gradient_matches_oracle(prec):
    p = workloads.tiny(seed=61, n=26, npml=4, side=6, nfreq=2, n_sweeps=2)
    say(f"gradient, precision {prec}")
    h = P.Handle(p).bind(P.default_options(precision=prec, max_accepts=256, max_sweeps=4))
    h.set_design(p.init_bits)
    assert rel(h.gradient(), oracle.gradient(p, p.init_bits)) < TOL
    res = h.dbs_run(p.perms)
    bits = p.init_bits.copy()
    for m in res["accepted"]:
        bits[m] ^= 1
    assert rel(h.gradient(), oracle.gradient(p, bits)) < TOL
    h.close()


def test_gradient_config0():
    p = workloads.config0()
    say("gradient config0")
    h = P.Handle(p).bind(P.default_options())
    h.set_design(p.init_bits)
    assert rel(h.gradient(), oracle.gradient(p, p.init_bits)) < TOL
    h.close()


def test_gradient_rejects_pec():
    p = workloads.tiny_metal(seed=62, n=20, side=3)
    h = P.Handle(p).bind(P.default_options())
    h.set_design(p.init_bits)
    with pytest.raises(P.PngfError) as e:
        h.gradient()
    assert e.value.code == -1
    h.close()
