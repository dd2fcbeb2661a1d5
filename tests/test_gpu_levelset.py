"""Sparse multi-pixel updates (pngf_flip_set) and the level-set driver that
uses them with the O(N_d) gradient (Supplementary Notes 5 and 6), vs the
oracle's full solves.  Bar: fields and objectives within 1e-10 of the oracle
after every update; gradients within 1e-10 (max-norm relative)."""
import numpy as np
import pytest

import oracle
import workloads
import paper_2501_18054_amd as P
from paper_2501_18054_amd import levelset
from gpu_util import say, rel

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _f_oracle(p, bits):
    return oracle.objective(p, [oracle.pngf_state(p, bits, fi)[1] for fi in range(p.nfreq)])


@pytest.mark.parametrize("prec", [P.PNGF_FP64_PLAIN, P.PNGF_RFORM])
def test_flip_set_matches_oracle(prec):
    p = workloads.config0()
    say(f"flip_set config0 precision {prec}")
    h = P.Handle(p).bind(P.default_options(precision=prec, max_sweeps=2))
    h.set_design(p.init_bits)
    if prec == P.PNGF_RFORM:
        res = h.dbs_run(p.perms)          # leaves C^-1 behind the design
        bits = p.init_bits.copy()
        for m in res["accepted"]:
            bits[m] ^= 1
    else:
        bits = p.init_bits.copy()
    rng = np.random.default_rng(3)
    pix = rng.choice(p.n_d, 70, replace=False).astype(np.int32)   # two blocks (64 + 6)
    h.flip_set(pix)
    bits[pix] ^= 1
    f, x, E = h.evaluate(fields=True)
    Eo, xo = oracle.pngf_state(p, bits, 0)
    assert rel(E[0], Eo) < TOL
    assert abs(f - _f_oracle(p, bits)) < TOL * f
    h.flip_set(pix[:5])
    bits[pix[:5]] ^= 1
    assert rel(h.evaluate(fields=True)[2][0], oracle.pngf_state(p, bits, 0)[0]) < TOL
    cands = np.arange(0, p.n_d, 9, dtype=np.int32)
    assert rel(h.score_flips(cands), oracle.score_all(p, bits, cands)) < TOL
    h.close()


def test_flip_set_errors():
    p = workloads.config0()
    h = P.Handle(p).bind(P.default_options())
    h.set_design(p.init_bits)
    with pytest.raises(P.PngfError):
        h.flip_set([3, 3])
    with pytest.raises(P.PngfError):
        h.flip_set([p.n_d])
    h.close()
    h = P.Handle(p).bind(P.default_options(precision=P.PNGF_MIXED))
    h.set_design(p.init_bits)
    with pytest.raises(P.PngfError):
        h.flip_set([1])
    h.close()


def test_levelset_run_states_are_exact():
    p = workloads.config0()
    say("level-set run config0")
    h = P.Handle(p).bind(P.default_options())
    hist = levelset.run(h, p.init_bits, p.design_side, iters=8)
    assert len(hist["f"]) >= 2, "expected at least one accepted level-set step"
    assert all(b > a for a, b in zip(hist["f"], hist["f"][1:]))
    for bits, f in zip(hist["bits"], hist["f"]):
        assert abs(f - _f_oracle(p, bits)) < TOL * f
    final = hist["bits"][-1]
    assert rel(h.gradient(), oracle.gradient(p, final)) < TOL
    assert rel(h.evaluate(fields=True)[2][0], oracle.pngf_state(p, final, 0)[0]) < TOL
    h.close()
