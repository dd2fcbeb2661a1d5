"""Searches over tiles of pixels flipped together (rank-M updates, M up to 64)
vs the oracle's tile search with full re-solves.

Bar: identical accepted-tile sequence, attempt count and convergence; per-step
objectives within 1e-10 relative; fields of the final design within 1e-10 of
a fresh full solve.  Tile sizes cover the three kernel instantiations
(M <= 16, <= 32, <= 64), ragged edge tiles and mirror-tied tile pairs.
"""
import numpy as np
import pytest

import oracle
import workloads
import paper_2501_18054_amd as P
from gpu_util import say, golden, rel

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _final_bits(p, acc):
    bits = p.init_bits.copy()
    for t in acc:
        row = p.tiles[t]
        bits[row[row >= 0]] ^= 1
    return bits


def _run(p, **kw):
    m = p.tiles.shape[1]
    h = P.Handle(p).bind(P.default_options(max_accepts=1024, max_sweeps=8, max_tile=m, **kw))
    h.set_design(p.init_bits)
    return h, h.tile_dbs_run(p.tiles, p.tile_perms)


def test_tiles_config1_identical():
    g = golden("tiles1")
    if g is None:
        pytest.skip("golden trajectory of the tile workload not generated")
    p = workloads.tiles1()
    say("tiles1 (4x4 tiles of workload 1)")
    h, res = _run(p)
    assert res["accepted"].tolist() == [a[2] for a in g["accepted"]]
    assert res["attempts"] == g["attempts"]
    assert res["converged"] == g["converged"]
    assert rel(res["f_trace"], [a[3] for a in g["accepted"]]) < TOL
    assert abs(res["f_final"] - g["f_final"]) < TOL * g["f_final"]
    f, x, E = h.evaluate(fields=True)
    Eo, xo = oracle.pngf_state(p, _final_bits(p, res["accepted"]), 0)
    assert rel(E[0], Eo) < TOL
    h.close()


@pytest.mark.parametrize("a,mirror,nfreq", [(2, True, 2), (3, False, 1), (4, True, 1),
                                            (8, False, 2)])
def test_tiles_tiny_vs_oracle(a, mirror, nfreq):
    p = workloads.with_tiles(workloads.tiny(seed=70 + a, n=30, npml=4, side=12, nfreq=nfreq,
                                            n_sweeps=4), a, mirror=mirror)
    say(f"tiny tiles a={a} mirror={mirror} M={p.tiles.shape[1]} F={nfreq}")
    r = oracle.dbs(p, perms=p.tile_perms, tiles=p.tiles)
    h, res = _run(p)
    assert res["accepted"].tolist() == [t for (_, _, t, _) in r.accepted]
    assert res["attempts"] == r.attempts
    assert res["converged"] == r.converged
    if r.accepted:
        assert rel(res["f_trace"], [fo for (_, _, _, fo) in r.accepted]) < TOL
    assert abs(res["f_final"] - r.f_final) < TOL * r.f_final
    h.close()


def test_tiles_pec():
    p = workloads.with_tiles(workloads.tiny_metal(seed=81, n=28, side=10, n_sweeps=4), 2)
    say("tiny metal tiles a=2")
    r = oracle.dbs(p, perms=p.tile_perms, tiles=p.tiles)
    h, res = _run(p)
    assert res["accepted"].tolist() == [t for (_, _, t, _) in r.accepted]
    assert res["attempts"] == r.attempts
    assert abs(res["f_final"] - r.f_final) < TOL * r.f_final
    f, x, Z = h.evaluate(fields=True)
    zo, xo = oracle.pec_state(p, _final_bits(p, res["accepted"]), 0)
    assert rel(Z[0], zo) < TOL
    assert abs(x[0] - xo) < TOL * abs(xo)
    h.close()


def test_tiles_errors():
    p = workloads.with_tiles(workloads.tiny(seed=90, n=20, npml=4, side=4, n_sweeps=2), 2)
    h = P.Handle(p).bind(P.default_options(max_tile=4))
    h.set_design(p.init_bits)
    bad = p.tiles.copy()
    bad[0, 0] = -1            # padding before a pixel id
    with pytest.raises(P.PngfError):
        h.tile_dbs_run(bad, p.tile_perms)
    bad = p.tiles.copy()
    bad[1, 1] = bad[1, 0]     # repeated pixel inside a tile
    with pytest.raises(P.PngfError):
        h.tile_dbs_run(bad, p.tile_perms)
    with pytest.raises(P.PngfError):
        h.tile_dbs_run(np.hstack([p.tiles, p.tiles]), p.tile_perms)   # M > max_tile
    h.close()
    h = P.Handle(p).bind(P.default_options())          # max_tile = 0
    h.set_design(p.init_bits)
    with pytest.raises(P.PngfError):
        h.tile_dbs_run(p.tiles, p.tile_perms)
    h.close()
    with pytest.raises(P.PngfError):                     # tiles need the FP64 plain form
        P.Handle(p).bind(P.default_options(precision=P.PNGF_MIXED, max_tile=4))


def test_tile_covering_the_whole_design():
    """One tile of every pixel (3x3 design): the search flips the whole
    design at once or nothing."""
    p = workloads.with_tiles(workloads.tiny(seed=91, n=20, npml=4, side=3, n_sweeps=3), 3)
    assert p.tiles.shape == (1, 9)
    say("single tile over the whole design")
    r = oracle.dbs(p, perms=p.tile_perms, tiles=p.tiles)
    h, res = _run(p)
    assert res["accepted"].tolist() == [t for (_, _, t, _) in r.accepted]
    assert res["attempts"] == r.attempts
    assert res["converged"] == r.converged
    assert abs(res["f_final"] - r.f_final) < TOL * r.f_final
    h.close()
