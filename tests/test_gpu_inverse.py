"""The FP64 initial inverse at every tournament shape vs the oracle.

The pivot search of a 16-column panel works on groups of 64 candidate rows,
one per wave, and merges the proposals of four groups at a time: one wave
alone for n_S <= 64; level 0 across the chip and the merges in one workgroup
of up to 16 waves for n_S <= 4096; above that merge levels across the chip
too.  The number of eps_hi pixels n_S picks the shape, so designs with n_S on
either side of every boundary (ragged last panels included) are set on
workload 1 (N_d = 1600) and on a 66 x 66 design (N_d = 4356), and the fields
compared with the oracle's sparse FDFD solve.  Bar: E and x within 1e-10
relative, as for the other FP64 states.
"""
import numpy as np
import pytest

import oracle
import workloads
import paper_2501_18054_amd as P
from gpu_util import say, rel

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def cfg1():
    p = workloads.config1()
    h = P.Handle(p).bind(P.default_options())
    yield p, h
    h.close()


@pytest.mark.parametrize("ns", [1, 15, 63, 64, 65, 257, 1023, 1024, 1025, 1600])
def test_inverse_at_tournament_shapes(cfg1, ns):
    p, h = cfg1
    order = np.random.default_rng(1000 + ns).permutation(p.n_d)
    bits = np.zeros(p.n_d, np.uint8)
    bits[order[:ns]] = 1
    say(f"config1 initial inverse, n_S = {ns}")
    h.set_design(bits)
    f, x, E = h.evaluate(fields=True)
    Eo, xo = oracle.pngf_state(p, bits, 0)
    assert rel(E[0], Eo) < TOL
    assert abs(x[0] - xo) < TOL * abs(xo)


@pytest.fixture(scope="module")
def big():
    # 66 x 66 design (N_d = 4356): past 64 level-0 groups the first merge
    # level also runs across the chip
    p = workloads.tiny(seed=7, n=88, npml=8, side=66, n_sweeps=1)
    h = P.Handle(p).bind(P.default_options())
    yield p, h
    h.close()


@pytest.mark.parametrize("ns", [4097, 4356])
def test_inverse_with_chip_wide_merge_level(big, ns):
    p, h = big
    order = np.random.default_rng(2000 + ns).permutation(p.n_d)
    bits = np.zeros(p.n_d, np.uint8)
    bits[order[:ns]] = 1
    say(f"N_d = {p.n_d} initial inverse, n_S = {ns}")
    h.set_design(bits)
    f, x, E = h.evaluate(fields=True)
    Eo, xo = oracle.pngf_state(p, bits, 0)
    assert rel(E[0], Eo) < TOL
    assert abs(x[0] - xo) < TOL * abs(xo)
