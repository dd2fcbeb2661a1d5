"""Host logic of the level-set driver, on the CPU: a stand-in handle answers
with the oracle's full solves, so the driver's own steps (velocity from the
gradient, narrow band, accept/undo, step control) are checked without a GPU."""
import numpy as np

import oracle
import workloads
from paper_2501_18054_amd import levelset


class OracleHandle:
    def __init__(self, p):
        self.p = p
        self.bits = None
        self.updates = []

    def _f(self):
        return oracle.objective(self.p, [oracle.pngf_state(self.p, self.bits, fi)[1]
                                         for fi in range(self.p.nfreq)])

    def set_design(self, bits):
        self.bits = np.array(bits, dtype=np.uint8)

    def evaluate(self):
        return (self._f(),)

    def gradient(self):
        return oracle.gradient(self.p, self.bits)

    def flip_set(self, pix):
        pix = np.asarray(pix)
        assert len(np.unique(pix)) == len(pix)
        self.bits[pix] ^= 1
        self.updates.append(len(pix))


def test_levelset_driver_ascends_with_sparse_updates():
    p = workloads.tiny(seed=33, n=26, npml=4, side=8, nfreq=1)
    h = OracleHandle(p)
    hist = levelset.run(h, p.init_bits, 8, iters=6)
    assert len(hist["f"]) >= 2
    assert all(b > a for a, b in zip(hist["f"], hist["f"][1:]))
    # each accepted design is the handle's design at that point, and the
    # updates touch few pixels (the narrow band), not the whole region
    assert np.array_equal(hist["bits"][-1], h.bits)
    assert max(h.updates) < p.n_d // 2
    for bits, f in zip(hist["bits"], hist["f"]):
        h2 = OracleHandle(p)
        h2.set_design(bits)
        assert abs(h2.evaluate()[0] - f) < 1e-12 * f


def test_phi_from_bits_and_band():
    bits = np.array([0, 1, 1, 0], np.uint8)
    phi = levelset.phi_from_bits(bits, 2)
    assert np.array_equal(phi > 0, bits.reshape(2, 2) == 1)
    b = np.zeros((4, 4), np.uint8)
    b[1:3, 1:3] = 1
    band = levelset.boundary_band(b.ravel(), 4)
    assert band[1:3, 1:3].all()                 # every pixel of the block touches the outside
    assert band.sum() == 4 + 8                  # plus the 8 outside neighbours of the block
    assert not band[0, 0] and not band[3, 3]
