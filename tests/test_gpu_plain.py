"""FP64 plain path on the GPU vs the CPU oracle (full sparse re-solves).

Bars: fields <= 1e-10 relative, objectives <= 1e-10 relative, and the
identical accepted-flip sequence (pixels, positions, attempts) on workloads
0 and 1.
"""
import numpy as np
import pytest

import oracle
import workloads
import paper_2501_18054_amd as P
from gpu_util import say, golden, rel

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-10


@pytest.fixture(scope="module")
def cfg0():
    p = workloads.config0()
    h = P.Handle(p).bind(P.default_options(max_accepts=4096, max_sweeps=8, timing=True))
    yield p, h
    h.close()


def _oracle_state(p, bits):
    Es, xs = [], []
    for fi in range(p.nfreq):
        E, x = oracle.pngf_state(p, bits, fi)
        Es.append(E)
        xs.append(x)
    return np.array(Es), np.array(xs), oracle.objective(p, xs)


def test_initial_state_matches_oracle(cfg0):
    p, h = cfg0
    say("config0 set_design + evaluate")
    h.set_design(p.init_bits)
    f, x, E = h.evaluate(fields=True)
    Eo, xo, fo = _oracle_state(p, p.init_bits)
    assert rel(E, Eo) < FIELD_TOL
    assert rel(x, xo) < FIELD_TOL
    assert abs(f - fo) < FIELD_TOL * fo


def test_score_all_candidates_matches_full_resolve(cfg0):
    p, h = cfg0
    say("config0 score_flips all")
    h.set_design(p.init_bits)
    fs = h.score_flips(np.arange(p.n_d))
    fo = oracle.score_all(p, p.init_bits)
    assert rel(fs, fo) < FIELD_TOL
    # a ragged subset in arbitrary order, including a repeated id
    sub = np.array([97, 3, 3, 50, 0, 99], np.int32)
    fs2 = h.score_flips(sub)
    assert rel(fs2, fo[sub]) < FIELD_TOL


def test_accept_flips_matches_fresh_solve(cfg0):
    p, h = cfg0
    say("config0 accept_flips x5 + evaluate")
    h.set_design(p.init_bits)
    flips = [5, 17, 5, 88, 42]
    h.accept_flips(flips)
    bits = p.init_bits.copy()
    for m in flips:
        bits[m] ^= 1
    f, x, E = h.evaluate(fields=True)
    Eo, xo, fo = _oracle_state(p, bits)
    assert rel(E, Eo) < FIELD_TOL
    assert abs(f - fo) < FIELD_TOL * fo
    say("config0 refresh")
    h.refresh()
    f2, x2, E2 = h.evaluate(fields=True)
    assert rel(E2, Eo) < FIELD_TOL


def test_invalid_arguments(cfg0):
    p, h = cfg0
    say("config0 invalid args")
    h.set_design(p.init_bits)
    with pytest.raises(P.PngfError):
        h.score_flips([p.n_d])
    with pytest.raises(P.PngfError):
        h.accept_flips([-1])
    with pytest.raises(P.PngfError):
        h.dbs_run(np.zeros((1, p.n_d), np.int32))   # not a permutation
    # the handle still works after rejected calls
    assert np.isfinite(h.score_flips([0])[0])


def _check_against_golden(p, h, g, res):
    acc = [a[2] for a in g["accepted"]]
    assert res["accepted"].tolist() == acc
    assert res["attempts"] == g["attempts"]
    assert res["converged"] == g["converged"]
    assert res["sweeps"] == g["sweeps"]
    ftr = np.array([a[3] for a in g["accepted"]])
    assert rel(res["f_trace"], ftr) < FIELD_TOL
    assert abs(res["f_initial"] - g["f0"]) < FIELD_TOL * g["f0"]


def test_dbs_config0_identical_to_oracle(cfg0):
    p, h = cfg0
    g = golden(0)
    say("config0 dbs_run")
    h.set_design(p.init_bits)
    res = h.dbs_run(p.perms)
    _check_against_golden(p, h, g, res)
    bits = p.init_bits.copy()
    for m in res["accepted"]:
        bits[m] ^= 1
    f, x, E = h.evaluate(fields=True)
    Eo, xo, fo = _oracle_state(p, bits)
    assert rel(E, Eo) < FIELD_TOL
    t, n = h.kernel_times("accept")
    assert n >= res["n_accepted"] and t > 0


def test_dbs_multifrequency_tiny_matches_oracle():
    p = workloads.tiny(seed=31, n=24, npml=4, side=5, nfreq=3, n_sweeps=4)
    say("tiny 3-frequency dbs_run")
    r = oracle.dbs(p)
    h = P.Handle(p).bind(P.default_options(max_accepts=512, max_sweeps=8))
    h.set_design(p.init_bits)
    res = h.dbs_run(p.perms)
    assert res["accepted"].tolist() == [a[2] for a in r.accepted]
    assert res["attempts"] == r.attempts
    assert res["converged"] == r.converged
    assert abs(res["f_final"] - r.f_final) < FIELD_TOL * r.f_final
    h.close()


def test_dbs_single_pixel_and_cap():
    """N_d = 1 (degenerate) and an accept cap of 1."""
    p = workloads.tiny(seed=32, n=16, npml=3, side=1, n_sweeps=3)
    say("single-pixel dbs_run")
    r = oracle.dbs(p)
    h = P.Handle(p).bind(P.default_options(max_accepts=8, max_sweeps=4))
    h.set_design(p.init_bits)
    res = h.dbs_run(p.perms)
    assert res["accepted"].tolist() == [a[2] for a in r.accepted]
    assert res["attempts"] == r.attempts
    h.close()
    p = workloads.tiny(seed=33, n=24, npml=4, side=6, n_sweeps=2)
    say("accept cap 1")
    h = P.Handle(p).bind(P.default_options(max_accepts=1, max_sweeps=2))
    h.set_design(p.init_bits)
    res = h.dbs_run(p.perms)
    r = oracle.dbs(p)
    assert res["n_accepted"] == 1
    assert res["accepted"][0] == r.accepted[0][2]
    h.close()


def test_dbs_ragged_rows_npl2():
    """N_d = 17^2 = 289 (two row tiles of 256 plus a ragged tail)."""
    p = workloads.tiny(seed=34, n=40, npml=6, side=17, n_sweeps=1)
    say("ragged 17x17 dbs_run")
    r = oracle.dbs(p, workers=4)
    h = P.Handle(p).bind(P.default_options(max_accepts=2048, max_sweeps=2))
    h.set_design(p.init_bits)
    res = h.dbs_run(p.perms)
    assert res["accepted"].tolist() == [a[2] for a in r.accepted]
    assert res["attempts"] == r.attempts
    h.close()


def test_dbs_config1_identical_to_oracle():
    g = golden(1)
    if g is None:
        pytest.skip("golden trajectory for workload 1 not generated")
    p = workloads.config1()
    say("config1 precompute + dbs_run FP64")
    h = P.Handle(p).bind(P.default_options(max_accepts=8192, max_sweeps=8))
    h.set_design(p.init_bits)
    res = h.dbs_run(p.perms)
    _check_against_golden(p, h, g, res)
    bits = p.init_bits.copy()
    for m in res["accepted"]:
        bits[m] ^= 1
    f, x, E = h.evaluate(fields=True)
    Eo, xo, fo = _oracle_state(p, bits)
    assert rel(E, Eo) < FIELD_TOL
    assert abs(f - fo) < FIELD_TOL * fo
    h.close()
