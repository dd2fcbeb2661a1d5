"""C-ABI library checks that need no GPU: it loads, exports every symbol the
header declares, and its host precompute matches the oracle."""
import re
import os

import numpy as np
import pytest

import oracle
from oracle.green import background
import workloads
import paper_2501_18054_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    text = open(os.path.join(ROOT, "include", "pngf.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(pngf_\w+)\s*\(", text, re.M)))


def test_library_exports_header_symbols():
    L = P.lib()
    syms = _header_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(P.EXPORTS), "binding and header disagree"
    assert b"gfx950" in L.pngf_version()


def test_precompute_matches_oracle_config0():
    p = workloads.config0()
    h = P.Handle(p)
    G, b, god, xb = h.get_precompute(0)
    Go = oracle.green_dd(p, 0)
    Godo = oracle.green_od(p, 0)
    _, bo, xbo = background(p, 0)
    assert np.abs(G - Go).max() < 1e-11 * np.abs(Go).max()
    assert np.abs(G - G.T).max() == 0.0
    assert np.abs(b - bo).max() < 1e-11 * np.abs(bo).max()
    assert np.abs(god - Godo[0]).max() < 1e-11 * np.abs(Godo).max()
    assert abs(xb - xbo) < 1e-11 * abs(xbo)
    h.close()


def test_precompute_matches_oracle_multifreq_ragged():
    """Three frequencies, a 5x5 design (ragged against every tile size)."""
    p = workloads.tiny(seed=21, n=30, npml=5, side=5, nfreq=3)
    h = P.Handle(p)
    assert (h.n_d, h.nfreq) == (25, 3)
    for fi in range(3):
        G, b, god, xb = h.get_precompute(fi)
        Go = oracle.green_dd(p, fi)
        _, bo, xbo = background(p, fi)
        assert np.abs(G - Go).max() < 1e-11 * np.abs(Go).max()
        assert np.abs(b - bo).max() < 1e-11 * np.abs(bo).max()
        assert abs(xb - xbo) < 1e-11 * abs(xbo)
    h.close()


def test_precompute_matches_oracle_config1_sampled():
    p = workloads.config1()
    h = P.Handle(p)
    assert h.n_d == 1600
    G, b, god, xb = h.get_precompute(0)
    rng = np.random.default_rng(5)
    cols = rng.choice(1600, 8, replace=False)
    Gc = oracle.green_dd(p, 0, cols)
    assert np.abs(G[:, cols] - Gc).max() < 1e-10 * np.abs(Gc).max()
    _, bo, xbo = background(p, 0)
    assert np.abs(b - bo).max() < 1e-10 * np.abs(bo).max()
    assert abs(xb - xbo) < 1e-10 * abs(xbo)
    Godo = oracle.green_od(p, 0)
    assert np.abs(god - Godo[0]).max() < 1e-10 * np.abs(Godo).max()
    h.close()


def test_single_pixel_design():
    p = workloads.tiny(seed=4, n=16, npml=3, side=1)
    h = P.Handle(p)
    G, b, god, xb = h.get_precompute(0)
    assert G.shape == (1, 1)
    assert abs(G[0, 0] - oracle.green_dd(p, 0)[0, 0]) < 1e-12 * abs(G[0, 0])
    h.close()


def test_precompute_rejects_mask_in_pml():
    p = workloads.tiny(seed=4, n=16, npml=3, side=1)
    p.design_mask[:] = 0
    p.design_mask[1, 1] = 1
    with pytest.raises(P.PngfError) as e:
        P.Handle(p)
    assert e.value.code == -1


def test_precompute_rejects_empty_design_and_bad_nobj():
    p = workloads.tiny(seed=4, n=16, npml=3, side=1)
    p.design_mask[:] = 0
    with pytest.raises(P.PngfError):
        P.Handle(p)
    p = workloads.tiny(seed=4, n=16, npml=3, side=1)
    p.w = np.vstack([p.w, p.w])
    with pytest.raises(P.PngfError):
        P.Handle(p)


def test_unbound_calls_fail_cleanly():
    p = workloads.tiny(seed=4, n=16, npml=3, side=2)
    h = P.Handle(p)
    with pytest.raises(P.PngfError) as e:
        h.set_design(np.zeros(4, np.uint8))
    assert e.value.code == -5
    h.close()


def test_precompute_pec_pixels():
    """PEC pixels share the environment's G, b, G_OD, x_b; an unknown pixel
    kind is rejected."""
    p = workloads.tiny_metal(seed=8, n=20, side=3)
    h = P.Handle(p)
    G, b, god, xb = h.get_precompute(0)
    assert np.max(np.abs(G - oracle.green_dd(p, 0))) < 1e-10 * np.max(np.abs(G))
    h.close()
    p.pixel_kind = 7
    with pytest.raises(P.PngfError) as e:
        P.Handle(p)
    assert e.value.code == -1


def test_objective_norm_matches_oracle():
    """Mean-transmission normalizers (vacuum transmission per frequency) from
    the library's own elimination against the oracle's sparse vacuum solves;
    other objectives keep obj_norm."""
    p = workloads.config4_scaled()
    h = P.Handle(p)
    want = oracle.objective_norms(p)
    for fi in range(p.nfreq):
        assert abs(h.objective_norm(fi) - want[fi]) < 1e-11 * want[fi]
    h.close()
    p = workloads.tiny(seed=4, n=16, npml=3, side=2, nfreq=2)
    p.obj_norm = np.array([2.0, 0.5])
    h = P.Handle(p)
    assert [h.objective_norm(0), h.objective_norm(1)] == [2.0, 0.5]
    with pytest.raises(P.PngfError):
        h.objective_norm(2)
    h.close()


@pytest.mark.parametrize("shape", ["ring", "ell", "holes"])
def test_precompute_irregular_design_masks(shape):
    """The nested-dissection precompute on design regions that are not
    rectangles (a ring around an exterior island, an L, a block with interior
    exterior cells): G, b, G_OD and x_b against the oracle's column solves."""
    p = workloads.tiny(seed=6, n=34, npml=5, side=12, nfreq=2)
    i0, j0 = p.design_origin
    m = p.design_mask
    if shape == "ring":
        m[j0 + 4:j0 + 8, i0 + 4:i0 + 8] = 0
    elif shape == "ell":
        m[j0:j0 + 6, i0 + 6:i0 + 12] = 0
    else:
        m[j0 + 2, i0 + 3] = 0
        m[j0 + 7:j0 + 9, i0 + 8] = 0
        m[j0 + 5, i0 + 5:i0 + 7] = 0
    nd = int(m.sum())
    p.init_bits = p.init_bits[:nd]
    p.perms = np.stack([np.random.default_rng(1).permutation(nd).astype(np.int32)])
    h = P.Handle(p)
    assert h.n_d == nd
    for fi in range(2):
        G, b, god, xb = h.get_precompute(fi)
        Go = oracle.green_dd(p, fi)
        _, bo, xbo = background(p, fi)
        assert np.abs(G - Go).max() < 1e-11 * np.abs(Go).max()
        assert np.abs(G - G.T).max() == 0.0
        assert np.abs(b - bo).max() < 1e-11 * np.abs(bo).max()
        assert abs(xb - xbo) < 1e-11 * abs(xbo)
        Godo = oracle.green_od(p, fi)
        assert np.abs(god - Godo[0]).max() < 1e-11 * np.abs(Godo).max()
    h.close()
