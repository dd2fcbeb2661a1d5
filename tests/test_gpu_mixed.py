"""Mixed-precision path (complex-FP32 matrices, deferred Sherman-Morrison
panel, FP64 re-inversion, error band) vs the oracle's FP64 trajectory.

Bar: identical accepted-flip sequence and attempt count; per-step objectives
within 1e-6 relative (they are FP32-derived); the final objective, re-formed in
FP64, within 1e-10 relative.
"""
import numpy as np
import pytest

import oracle
import workloads
import paper_2501_18054_amd as P
from gpu_util import say, golden, rel

pytestmark = pytest.mark.gpu

OBJ_TOL = 1e-6


def _mixed(p, **kw):
    opts = P.default_options(precision=P.PNGF_MIXED, max_accepts=8192, max_sweeps=8, **kw)
    h = P.Handle(p).bind(opts)
    h.set_design(p.init_bits)
    return h, h.dbs_run(p.perms)


def _check(res, acc, attempts, ftr, f_final):
    assert res["accepted"].tolist() == acc
    assert res["attempts"] == attempts
    assert rel(res["f_trace"], ftr) < OBJ_TOL
    assert abs(res["f_final"] - f_final) < 1e-10 * f_final


def test_mixed_config0_identical():
    p = workloads.config0()
    g = golden(0)
    say("config0 mixed k_refresh=32")
    h, res = _mixed(p, k_refresh=32)
    _check(res, [a[2] for a in g["accepted"]], g["attempts"],
           [a[3] for a in g["accepted"]], g["f_final"])
    assert res["n_refresh"] >= 1
    h.close()


@pytest.mark.parametrize("k_refresh,k_fold", [(32, 0), (12, 0), (0, 0), (0, 8), (64, 5)])
def test_mixed_config1_identical(k_refresh, k_fold):
    g = golden(1)
    if g is None:
        pytest.skip("golden trajectory for workload 1 not generated")
    p = workloads.config1()
    say(f"config1 mixed k_refresh={k_refresh} k_fold={k_fold}")
    h, res = _mixed(p, k_refresh=k_refresh, k_fold=k_fold)
    _check(res, [a[2] for a in g["accepted"]], g["attempts"],
           [a[3] for a in g["accepted"]], g["f_final"])
    if k_refresh == 32:
        assert res["n_refresh"] >= len(g["accepted"]) // 32
    # the FP64 state re-formed at the end matches a fresh oracle solve
    bits = p.init_bits.copy()
    for m in res["accepted"]:
        bits[m] ^= 1
    f, x, E = h.evaluate(fields=True)
    Eo, xo = oracle.pngf_state(p, bits, 0)
    assert rel(E[0], Eo) < 1e-10
    h.close()


def test_mixed_multifrequency_tiny():
    p = workloads.tiny(seed=51, n=24, npml=4, side=5, nfreq=3, n_sweeps=4)
    say("tiny 3-frequency mixed")
    r = oracle.dbs(p)
    h, res = _mixed(p, k_refresh=8, k_fold=3)
    assert res["accepted"].tolist() == [a[2] for a in r.accepted]
    assert res["attempts"] == r.attempts
    assert res["converged"] == r.converged
    assert abs(res["f_final"] - r.f_final) < 1e-10 * r.f_final
    h.close()


def test_mixed_then_plain_calls():
    """After a mixed run the FP64 state is current: score_flips agrees with
    the oracle's full re-solves."""
    p = workloads.config0()
    say("config0 mixed then score_flips")
    h, res = _mixed(p, k_refresh=16)
    bits = p.init_bits.copy()
    for m in res["accepted"]:
        bits[m] ^= 1
    cands = np.array([0, 7, 55, 99], np.int32)
    fs = h.score_flips(cands)
    fo = oracle.score_all(p, bits, cands)
    assert rel(fs, fo) < 1e-10
    h.close()


@pytest.mark.parametrize("wl,k_refresh,k_fold", [("config1", 32, 0), ("config1", 12, 0),
                                                   ("config1", 0, 8), ("config0", 32, 0),
                                                   ("metal", 32, 0)])
def test_persistent_batches_equal_step_launches(wl, k_refresh, k_fold):
    """One launch per batch (rows of C0^-1 held in registers, grid barriers
    between steps; with a periodic refresh, each refresh queued behind its
    batch before the host reads the batch's state, its flip list padded to
    k_refresh columns) against one kernel per step, on one handle: the same
    arithmetic, so bit-identical searches, and a second persistent search
    identical to the first."""
    p = getattr(workloads, wl)()
    say(f"{wl} mixed persistent vs per-step launches, k_refresh={k_refresh} k_fold={k_fold}")
    h = P.Handle(p)
    out = []
    for step_launches in (False, True, False):
        h.bind(P.default_options(precision=P.PNGF_MIXED, max_accepts=8192, max_sweeps=8,
                                 k_refresh=k_refresh, k_fold=k_fold,
                                 step_launches=step_launches))
        h.set_design(p.init_bits)
        out.append(h.dbs_run(p.perms))
    for r in out[1:]:
        assert r["accepted"].tolist() == out[0]["accepted"].tolist()
        assert r["attempts"] == out[0]["attempts"]
        assert r["n_refresh"] == out[0]["n_refresh"]
        assert r["f_trace"].tolist() == out[0]["f_trace"].tolist()
        assert r["f_final"] == out[0]["f_final"]
    h.close()


def test_persistent_barrier_time_out_is_reported_and_recoverable():
    """Failure handling of the persistent search, forced from the host: with
    barrier waits bounded to a single poll the workgroups give up at the
    first barrier (every kernel still exits), the search fails with
    PNGF_ENUMERIC, and after set_design the handle searches normally again."""
    g = golden(1)
    if g is None:
        pytest.skip("golden trajectory for workload 1 not generated")
    p = workloads.config1()
    say("config1 persistent search with one-poll barrier waits (expected to fail cleanly)")
    h = P.Handle(p).bind(P.default_options(precision=P.PNGF_MIXED, max_accepts=8192,
                                           max_sweeps=8))
    h.set_persist_spin(1)
    h.set_design(p.init_bits)
    with pytest.raises(P.PngfError, match="timed out") as e:
        h.dbs_run(p.perms)
    assert e.value.code == -3   # PNGF_ENUMERIC
    say("config1 persistent search after the time-out")
    h.set_persist_spin(1 << 20)
    h.set_design(p.init_bits)
    res = h.dbs_run(p.perms)
    _check(res, [a[2] for a in g["accepted"]], g["attempts"],
           [a[3] for a in g["accepted"]], g["f_final"])
    h.close()


@pytest.mark.parametrize("step_launches", [False, True])
def test_singular_refresh_recovery(step_launches):
    """Recovery from a singular block-Woodbury refresh, forced from the host
    for the first two refreshes: the search re-inverts C^-1 instead (the
    persistent search learns it at its next launch, which runs no step) and
    still follows the oracle's trajectory."""
    g = golden(1)
    if g is None:
        pytest.skip("golden trajectory for workload 1 not generated")
    p = workloads.config1()
    say(f"config1 mixed, first two refreshes forced singular, step_launches={step_launches}")
    h = P.Handle(p).bind(P.default_options(precision=P.PNGF_MIXED, max_accepts=8192,
                                           max_sweeps=8, step_launches=step_launches))
    h.set_design(p.init_bits)
    h.force_singular_refresh(2)
    res = h.dbs_run(p.perms)
    _check(res, [a[2] for a in g["accepted"]], g["attempts"],
           [a[3] for a in g["accepted"]], g["f_final"])
    h.close()


@pytest.mark.parametrize("precision", ["mixed", "plain"])
def test_search_after_failed_unpivoted_check(precision):
    """set_design returns with its inverse queued; the search's start checks
    it.  With the check forced to fail (zero tolerance) the search must run
    on the pivot-searched inverse: the start state is formed again after the
    re-inversion, so the trajectory, its initial objective and the final
    fields equal the oracle's."""
    g = golden(1)
    if g is None:
        pytest.skip("golden trajectory for workload 1 not generated")
    p = workloads.config1()
    prec = P.PNGF_MIXED if precision == "mixed" else P.PNGF_FP64_PLAIN
    say(f"config1 {precision} search straight after a failed unpivoted check")
    h = P.Handle(p).bind(P.default_options(precision=prec, k_refresh=32, max_accepts=8192,
                                           max_sweeps=8))
    h.set_inverse_check(0.0)
    h.set_design(p.init_bits)
    res = h.dbs_run(p.perms)
    assert h.inverse_stats() == (0, 1)
    tol = OBJ_TOL if precision == "mixed" else 1e-10
    _check(res, [a[2] for a in g["accepted"]], g["attempts"],
           [a[3] for a in g["accepted"]], g["f_final"])
    assert rel(res["f_trace"], [a[3] for a in g["accepted"]]) < tol
    assert abs(res["f_initial"] - g["f0"]) < 1e-10 * abs(g["f0"])
    bits = p.init_bits.copy()
    for m in res["accepted"]:
        bits[m] ^= 1
    f, x, E = h.evaluate(fields=True)
    Eo, xo = oracle.pngf_state(p, bits, 0)
    assert rel(E[0], Eo) < 1e-10
    h.close()
