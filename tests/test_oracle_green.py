"""Pins for the oracle's Green function, projections and PNGF equivalence.

The PNGF reduced system (I - k0^2 G_DD diag(deps)) E_D = b with
x = x_b + k0^2 G_OD diag(deps) E_D must reproduce the full FDFD solve exactly
(Results, Numerical Green's functions: no approximation).  These tests check
the oracle's G_DD, G_OD, b, x_b (each from full solves) against full solves of
other designs, closed forms and reciprocity.
"""
import itertools

import numpy as np
import pytest

import oracle
import oracle.fdfd as fd
from oracle.green import background
import workloads


def _pieces(p, fi=0):
    G = oracle.green_dd(p, fi)
    God = oracle.green_od(p, fi)
    _, b, xb = background(p, fi)
    return G, God, b, xb


def test_reciprocity():
    """G_DD (column solves, no symmetry assumed) is complex symmetric, and the
    transposed-solve G_OD equals minus the design restriction of the adjoint
    field L_b^-1 w (reciprocity)."""
    p = workloads.config0()
    G, God, _, _ = _pieces(p)
    assert np.max(np.abs(G - G.T)) < 1e-12 * np.max(np.abs(G))
    eps = fd.total_eps(p, np.zeros(p.n_d, np.uint8))
    L, s = fd.assemble(p.nx, p.ny, p.npml, p.h, eps, p.k0[0])
    y = fd.Solver(L, s).solve(p.w[0].astype(complex))
    adj = -y[p.design_indices()]
    assert np.max(np.abs(God[0] - adj)) < 1e-12 * np.max(np.abs(adj))


def test_output_row_is_adjoint_sensitivity():
    """dx/d eps_m = k0^2 E[m] R'[m]: central finite differences of full
    solves in which only pixel m's permittivity moves by +-h (first-order
    perturbation of L E = i k0 J, whose eps term is +k0^2 eps)."""
    p = workloads.config0()
    rng = np.random.default_rng(3)
    bits = (rng.random(p.n_d) < 0.4).astype(np.uint8)
    R = oracle.output_row(p, bits, 0)
    E, _ = oracle.pngf_state(p, bits, 0)
    idx = p.design_indices()
    k0 = p.k0[0]
    hstep = 1e-4
    for m in (0, 37, 99):
        xs = []
        for sgn in (1.0, -1.0):
            eps = fd.total_eps(p, bits).ravel().copy()
            eps[idx[m]] += sgn * hstep
            Ef = fd.solve(p.nx, p.ny, p.npml, p.h, eps.reshape(p.ny, p.nx), k0, p.src[0])
            xs.append(complex(p.w[0] @ Ef))
        fdx = (xs[0] - xs[1]) / (2 * hstep)
        pred = k0 ** 2 * E[m] * R[m]
        assert abs(fdx - pred) < 1e-6 * abs(pred)
    # background design: the output row is G_OD
    R0 = oracle.output_row(p, np.zeros(p.n_d, np.uint8), 0)
    assert np.max(np.abs(R0 - oracle.green_od(p, 0)[0])) < 1e-12 * np.max(np.abs(R0))


def test_single_pixel_closed_form():
    """One-pixel region: E = b / (1 - k0^2 deps G11), x = x_b + k0^2 G_O1 deps E."""
    p = workloads.tiny(seed=5, n=20, npml=4, side=1)
    G, God, b, xb = _pieces(p)
    k0 = p.k0[0]
    for bit in (0, 1):
        deps = bit * (p.eps_hi - p.eps_lo)
        E = b[0] / (1.0 - k0 * k0 * deps * G[0, 0])
        x = xb + k0 * k0 * God[0, 0] * deps * E
        Ef, xf = oracle.pngf_state(p, np.array([bit], np.uint8), 0)
        assert abs(E - Ef[0]) < 1e-11 * abs(Ef[0])
        assert abs(x - xf) < 1e-11 * abs(xf)
    # zero contrast leaves the background untouched
    Ef, xf = oracle.pngf_state(p, np.array([0], np.uint8), 0)
    assert abs(Ef[0] - b[0]) < 1e-12 * abs(b[0]) and abs(xf - xb) < 1e-12 * abs(xb)


def test_two_pixel_closed_form():
    """2x2 region with two pixels set: the explicit 2x2 inverse (Cramer) of
    I - k0^2 G D on the active pair reproduces the full solve."""
    p = workloads.tiny(seed=6, n=20, npml=4, side=2)
    G, God, b, xb = _pieces(p)
    k0 = p.k0[0]
    d = p.eps_hi - p.eps_lo
    bits = np.array([1, 0, 0, 1], np.uint8)
    a, c = 0, 3
    # active rows/cols a, c: E_a, E_c solve a 2x2 system; others follow
    m11 = 1 - k0 * k0 * d * G[a, a]
    m12 = -k0 * k0 * d * G[a, c]
    m21 = -k0 * k0 * d * G[c, a]
    m22 = 1 - k0 * k0 * d * G[c, c]
    det = m11 * m22 - m12 * m21
    Ea = (m22 * b[a] - m12 * b[c]) / det
    Ec = (m11 * b[c] - m21 * b[a]) / det
    E = b + k0 * k0 * d * (G[:, a] * Ea + G[:, c] * Ec)
    x = xb + k0 * k0 * d * (God[0, a] * Ea + God[0, c] * Ec)
    Ef, xf = oracle.pngf_state(p, bits, 0)
    assert np.max(np.abs(E - Ef)) < 1e-11 * np.max(np.abs(Ef))
    assert abs(x - xf) < 1e-11 * abs(xf)


def test_enumerate_3x3():
    """All 2^9 designs of a 3x3 region: the reduced N_d system gives the same
    objective as the full FDFD solve."""
    p = workloads.tiny(seed=7, n=20, npml=4, side=3)
    G, God, b, xb = _pieces(p)
    k0 = p.k0[0]
    worst = 0.0
    for combo in itertools.product((0, 1), repeat=9):
        bits = np.array(combo, np.uint8)
        D = np.diag(bits * (p.eps_hi - p.eps_lo))
        E = np.linalg.solve(np.eye(9) - k0 * k0 * G @ D, b)
        x = xb + k0 * k0 * (God @ D @ E)[0]
        _, xf = oracle.pngf_state(p, bits, 0)
        worst = max(worst, abs(abs(x) ** 2 - abs(xf) ** 2) / abs(xf) ** 2)
    assert worst < 1e-10


def test_green_config1_sampled_columns():
    """Config-1 size: sampled G_DD columns are symmetric with their rows."""
    p = workloads.config1()
    rng = np.random.default_rng(0)
    cols = rng.choice(p.n_d, 6, replace=False)
    Gc = oracle.green_dd(p, 0, cols)
    sub = Gc[cols, :]
    assert np.max(np.abs(sub - sub.T)) < 1e-11 * np.max(np.abs(sub))
