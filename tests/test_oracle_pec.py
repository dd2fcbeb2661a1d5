"""Pins for the oracle's perfectly conducting (PEC) pixels (CPU only).

A PEC pixel is Ez = 0 on its node in the full FDFD system (oracle.fdfd
pec_system).  These tests tie that definition to what the paper fixes:

* it is the limit of an ever larger conductivity (Supplementary Note 1 takes
  sigma -> infinity), approached at the rate 1/sigma;
* the current that replaces the conductors (current equivalence, Results,
  Numerical Green's functions) satisfies the paper's discrete equation
  [(I - P) + P G] j = P e_inc (eq. currequiv_j_disc), with G, e_inc and the
  output projection taken from the oracle's independently pinned Green
  function columns;
* one and two conducting pixels reduce to closed forms;
* direct binary search over PEC pixels keeps the search invariants.
"""
import numpy as np
import scipy.sparse as sp

import oracle
import oracle.fdfd as fd
from oracle.dbs import ETA
from oracle.green import background
import workloads


def _pieces(p, fi=0):
    G = oracle.green_dd(p, fi)
    God = oracle.green_od(p, fi)
    _, b, xb = background(p, fi)
    return G, God[0], b, xb


def _lossy_solve(p, bits, s):
    """Full solve with the conducting pixels replaced by eps = eps_lo + i s."""
    k0 = p.k0[0]
    eps = fd.total_eps(p, np.zeros(p.n_d, np.uint8))
    L, scale = fd.assemble(p.nx, p.ny, p.npml, p.h, eps, k0)
    d = np.zeros(p.nx * p.ny, dtype=np.complex128)
    d[p.design_indices()[bits != 0]] = k0 * k0 * 1j * s
    L = sp.csc_matrix(L + sp.diags(d))
    return fd.Solver(L, scale).solve(fd.rhs(p.src[0], k0))


def test_pec_is_the_large_conductivity_limit():
    p = workloads.tiny_metal(seed=21, n=24, side=4)
    bits = np.array([1, 0, 1, 1, 0, 0, 1, 0, 1, 1, 0, 0, 0, 1, 0, 1], np.uint8)
    E = oracle.field(p, bits, 0)
    scale = np.max(np.abs(E))
    errs = [np.max(np.abs(_lossy_solve(p, bits, s) - E)) / scale for s in (1e4, 1e5, 1e6)]
    # first-order convergence: each decade of conductivity gains a decade
    assert 7.0 < errs[0] / errs[1] < 13.0
    assert 7.0 < errs[1] / errs[2] < 13.0
    assert errs[2] < 1e-5
    assert np.all(E[p.design_indices()[bits != 0]] == 0)


def test_current_satisfies_the_paper_j_form():
    """[(I-P) + P G] j = P e_inc and x = x_inc + G_obj j in the paper's sign
    convention (field = e_inc - G j), where G_obj = -G_OD."""
    p = workloads.tiny_metal(seed=22, n=22, side=4)
    G, God, b, xb = _pieces(p)
    rng = np.random.default_rng(7)
    for _ in range(3):
        bits = (rng.random(p.n_d) < 0.5).astype(np.uint8)
        P = np.diag(bits.astype(float))
        E, j = oracle.equivalent_current(p, bits, 0)
        C = (np.eye(p.n_d) - P) + P @ G
        lhs = C @ j
        assert np.max(np.abs(lhs - P @ b)) < 1e-10 * np.max(np.abs(b))
        x = xb + (-God) @ j
        xf = complex(p.w[0] @ E)
        assert abs(x - xf) < 1e-10 * abs(xf)
        # the field on the design region is e_inc - G j, zero on conductors
        ed = b - G @ j
        assert np.max(np.abs(ed - E[p.design_indices()])) < 1e-10 * np.max(np.abs(b))


def test_single_pec_pixel_closed_form():
    """One conductor m: G_mm j_m = b_m, E_D = b - G[:, m] j_m,
    x = x_b - G_OD[m] j_m."""
    p = workloads.tiny_metal(seed=23, n=20, side=3)
    G, God, b, xb = _pieces(p)
    for m in (0, 4, 8):
        bits = np.zeros(p.n_d, np.uint8)
        bits[m] = 1
        jm = b[m] / G[m, m]
        Ed = b - G[:, m] * jm
        x = xb - God[m] * jm
        z, xf = oracle.pec_state(p, bits, 0)
        zref = Ed.copy()
        zref[m] = jm
        assert np.max(np.abs(z - zref)) < 1e-11 * np.max(np.abs(zref))
        assert abs(x - xf) < 1e-11 * abs(xf)


def test_two_pec_pixels_closed_form():
    """Two conductors a, c: the 2x2 system G_SS j_S = b_S by Cramer's rule."""
    p = workloads.tiny_metal(seed=24, n=20, side=3)
    G, God, b, xb = _pieces(p)
    a, c = 1, 7
    bits = np.zeros(p.n_d, np.uint8)
    bits[[a, c]] = 1
    det = G[a, a] * G[c, c] - G[a, c] * G[c, a]
    ja = (b[a] * G[c, c] - b[c] * G[a, c]) / det
    jc = (b[c] * G[a, a] - b[a] * G[c, a]) / det
    Ed = b - G[:, a] * ja - G[:, c] * jc
    z, xf = oracle.pec_state(p, bits, 0)
    assert abs(z[a] - ja) < 1e-11 * abs(ja) and abs(z[c] - jc) < 1e-11 * abs(jc)
    others = np.setdiff1d(np.arange(p.n_d), [a, c])
    assert np.max(np.abs(z[others] - Ed[others])) < 1e-11 * np.max(np.abs(Ed))
    assert abs(xb - God[a] * ja - God[c] * jc - xf) < 1e-11 * abs(xf)


def test_no_conductor_is_the_background():
    p = workloads.tiny_metal(seed=25, n=20, side=3)
    _, God, b, xb = _pieces(p)
    z, x = oracle.pec_state(p, np.zeros(p.n_d, np.uint8), 0)
    assert np.max(np.abs(z - b)) < 1e-12 * np.max(np.abs(b))
    assert abs(x - xb) < 1e-12 * abs(xb)


def test_pec_dbs_invariants():
    """Every accept improves by more than eta f, every skipped position does
    not, and a converged design is a single-flip local optimum (independent
    full solves, two frequencies)."""
    p = workloads.tiny_metal(seed=26, n=20, side=4, nfreq=2, n_sweeps=5)
    res = oracle.dbs(p)
    assert res.accepted
    bits = p.init_bits.copy()
    f = res.f0
    cursor = (0, 0)
    for (s, q, m, fnew) in res.accepted:
        skipped = []
        cs, cq = cursor
        while (cs, cq) != (s, q):
            skipped.append(int(p.perms[cs, cq]))
            cq += 1
            if cq == p.n_d:
                cs, cq = cs + 1, 0
        if skipped:
            assert np.all(oracle.score_all(p, bits, skipped) - f <= ETA * f)
        bits[m] ^= 1
        xs = [oracle.pec_state(p, bits, fi)[1] for fi in range(p.nfreq)]
        f2 = oracle.objective(p, xs)
        assert abs(f2 - fnew) < 1e-12 * f2 and f2 - f > ETA * f
        f = f2
        cursor = (s, q + 1) if q + 1 < p.n_d else (s + 1, 0)
    if res.converged:
        assert np.all(oracle.score_all(p, bits) - f <= ETA * f)
