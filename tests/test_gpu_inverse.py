"""The FP64 initial inverse at every tournament shape vs the oracle.

The pivot search of a 16-column panel runs in one workgroup (one wave per
64 candidate rows, merged four groups at a time) while the eps_hi block has at
most 1024 pixels, and as multi-workgroup levels of 1024 rows above that.  The
number of eps_hi pixels n_S picks the shape, so designs with n_S on either side
of every boundary (one wave, 64, 16 waves = 1024, ragged last panels) are set
on workload 1 (N_d = 1600) and the fields compared with the oracle's sparse
FDFD solve.  Bar: E and x within 1e-10 relative, as for the other FP64 states.
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
