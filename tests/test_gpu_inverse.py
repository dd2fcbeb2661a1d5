"""The FP64 initial inverse on every path and pivot-search shape vs the oracle.

An inversion first runs blocked Gauss-Jordan on 64-column panels without row
exchanges, checked by a probe residual; it falls back to the pivot search
when that check fails (forced here with a zero tolerance) and always uses the
pivot search with PNGF_FLAG_PIVOT_SEARCH.  The pivot search of a 16-column
panel is partial pivoting over every candidate row in one workgroup up to
1024 rows; above that, tournament levels across the chip (groups of 64
rows, then merges of four groups' proposals) first thin the candidates to at
most 1024, and past 64 level-0 groups (n_S > 4096) a merge level runs too.
The number of eps_hi pixels n_S picks the shape (and the ragged last panel
of either path), so designs with n_S on either side of every boundary are
set on workload 1 (N_d = 1600), a 66 x 66 design (N_d = 4356) and a 96 x 96
design (N_d = 9216), and the fields compared with the oracle's sparse FDFD
solve.  Bar: E and x within 1e-10 relative, as for the other FP64 states.
"""
import numpy as np
import pytest

import oracle
import workloads
import paper_2501_18054_amd as P
from gpu_util import say, rel

pytestmark = pytest.mark.gpu

TOL = 1e-10
MODES = ("unpivoted", "pivot_search", "fallback")


def _check(p, h, ns, seed, mode):
    h.bind(P.default_options(pivot_search=(mode == "pivot_search")))
    h.set_inverse_check(0.0 if mode == "fallback" else 1e-12)
    order = np.random.default_rng(seed).permutation(p.n_d)
    bits = np.zeros(p.n_d, np.uint8)
    bits[order[:ns]] = 1
    say(f"N_d = {p.n_d} initial inverse, n_S = {ns}, {mode}")
    n0, p0 = h.inverse_stats()
    h.set_design(bits)
    n1, p1 = h.inverse_stats()
    if mode == "unpivoted":
        assert (n1 - n0, p1 - p0) == (1, 0)
    else:
        assert (n1 - n0, p1 - p0) == (0, 1)
    f, x, E = h.evaluate(fields=True)
    Eo, xo = oracle.pngf_state(p, bits, 0)
    assert rel(E[0], Eo) < TOL
    assert abs(x[0] - xo) < TOL * abs(xo)


@pytest.fixture(scope="module")
def cfg1():
    p = workloads.config1()
    h = P.Handle(p)
    yield p, h
    h.close()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("ns", [1, 15, 63, 64, 65, 257, 1023, 1024, 1025, 1600])
def test_inverse_at_every_shape(cfg1, ns, mode):
    p, h = cfg1
    _check(p, h, ns, 1000 + ns, mode)


@pytest.fixture(scope="module")
def big():
    # 66 x 66 design (N_d = 4356): the level-0 tournament in front of the
    # partial pivoting, and one merge level past 4096 rows
    p = workloads.tiny(seed=7, n=88, npml=8, side=66, n_sweeps=1)
    h = P.Handle(p)
    yield p, h
    h.close()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("ns", [2048, 2049, 4096, 4097, 4356])
def test_inverse_with_tournament_levels(big, ns, mode):
    p, h = big
    _check(p, h, ns, 2000 + ns, mode)


@pytest.fixture(scope="module")
def huge():
    # 96 x 96 design (N_d = 9216): more tournament groups, merge levels
    p = workloads.tiny(seed=8, n=118, npml=8, side=96, n_sweeps=1)
    h = P.Handle(p)
    yield p, h
    h.close()


@pytest.mark.parametrize("mode", ["unpivoted", "pivot_search"])
@pytest.mark.parametrize("ns", [8193, 9216])
def test_inverse_at_large_n(huge, ns, mode):
    p, h = huge
    _check(p, h, ns, 3000 + ns, mode)
