"""Pins for the oracle's direct binary search (CPU only).

Checked by independent full solves: each accepted flip improves by more than
eta*f at its state, each position skipped between two accepts does not, and a
converged design is a single-flip local optimum.
"""
import numpy as np

import oracle
from oracle.dbs import ETA
import workloads


def _replay_checks(p, res):
    bits = p.init_bits.copy()
    f = oracle.objective(p, [oracle.pngf_state(p, bits, fi)[1] for fi in range(p.nfreq)])
    assert abs(f - res.f0) < 1e-12 * f
    cursor = (0, 0)
    for (s, q, m, fnew) in res.accepted:
        # positions from the cursor up to (but excluding) the accept
        skipped = []
        cs, cq = cursor
        while (cs, cq) != (s, q):
            skipped.append(int(p.perms[cs, cq]))
            cq += 1
            if cq == p.n_d:
                cs, cq = cs + 1, 0
        if skipped:
            fs = oracle.score_all(p, bits, skipped)
            assert np.all(fs - f <= ETA * f)
        b2 = bits.copy()
        b2[m] ^= 1
        f2 = oracle.objective(p, [oracle.pngf_state(p, b2, fi)[1] for fi in range(p.nfreq)])
        assert abs(f2 - fnew) < 1e-12 * f2
        assert f2 - f > ETA * f
        bits, f = b2, f2
        cursor = (s, q + 1) if q + 1 < p.n_d else (s + 1, 0)
    assert np.array_equal(bits, res.bits)
    return bits, f


def test_dbs_invariants_tiny():
    p = workloads.tiny(seed=11, n=20, npml=4, side=4, n_sweeps=6)
    res = oracle.dbs(p)
    assert res.accepted, "expected at least one accepted flip"
    bits, f = _replay_checks(p, res)
    if res.converged:
        fs = oracle.score_all(p, bits)
        assert np.all(fs - f <= ETA * f)


def test_dbs_multifrequency_invariants():
    p = workloads.tiny(seed=12, n=20, npml=4, side=3, nfreq=3, n_sweeps=4)
    res = oracle.dbs(p)
    _replay_checks(p, res)


def test_dbs_pool_matches_sequential():
    p = workloads.tiny(seed=13, n=20, npml=4, side=4, n_sweeps=2)
    r1 = oracle.dbs(p)
    r2 = oracle.dbs(p, workers=3)
    assert [a[:3] for a in r1.accepted] == [a[:3] for a in r2.accepted]
    assert r1.attempts == r2.attempts


def test_dbs_config0_converges_to_local_optimum_after_sweeps():
    """Config 0, one sweep: invariants hold at full size."""
    p = workloads.config0()
    res = oracle.dbs(p)
    _replay_checks(p, res)


def test_tile_dbs_with_single_pixel_tiles_is_pixel_dbs():
    """1x1 tiles in pixel order reduce the tile search to the pixel search."""
    p = workloads.tiny(seed=14, n=20, npml=4, side=3, n_sweeps=3)
    tiles = workloads.tile_groups(3, 1)
    assert np.array_equal(tiles[:, 0], np.arange(p.n_d))
    r1 = oracle.dbs(p)
    r2 = oracle.dbs(p, perms=p.perms, tiles=tiles)
    assert r1.accepted == r2.accepted and r1.attempts == r2.attempts


def test_tile_dbs_invariants():
    """2x2 tiles of a 5x5 region (ragged edge tiles) and mirror-tied tiles:
    every accepted tile improves, every skipped one does not, a converged
    design is a single-tile local optimum (independent full solves)."""
    for mirror in (False, True):
        p = workloads.with_tiles(workloads.tiny(seed=15, n=22, npml=4, side=5, n_sweeps=4),
                                 2, mirror=mirror)
        res = oracle.dbs(p, perms=p.tile_perms, tiles=p.tiles)
        assert res.accepted
        bits = p.init_bits.copy()
        f = res.f0
        cursor = (0, 0)
        nt = p.tiles.shape[0]
        for (s, q, t, fnew) in res.accepted:
            skipped = []
            cs, cq = cursor
            while (cs, cq) != (s, q):
                skipped.append(int(p.tile_perms[cs, cq]))
                cq += 1
                if cq == nt:
                    cs, cq = cs + 1, 0
            if skipped:
                fs = oracle.score_all(p, bits, skipped, tiles=p.tiles)
                assert np.all(fs - f <= ETA * f)
            row = p.tiles[t]
            bits[row[row >= 0]] ^= 1
            f2 = oracle.objective(p, [oracle.pngf_state(p, bits, fi)[1]
                                      for fi in range(p.nfreq)])
            assert abs(f2 - fnew) < 1e-12 * f2 and f2 - f > ETA * f
            f = f2
            cursor = (s, q + 1) if q + 1 < nt else (s + 1, 0)
        assert np.array_equal(bits, res.bits)
        if res.converged:
            assert np.all(oracle.score_all(p, bits, tiles=p.tiles) - f <= ETA * f)
