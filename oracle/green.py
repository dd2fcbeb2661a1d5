"""Design-region Green function and output projection by full solves, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definitions (Results, Precomputation: G = B^T A^-1 B over the optimization
region, G_obj = W^T A^-1 B, x_inc = W^T e_inc), written in the field form
used throughout, with the background operator L_b (design cells at eps_lo):

    G_DD = -(L_b^-1)[D, D],   G_OD = -w^T L_b^-1[:, D],
    E_b = L_b^-1 (i k0 J),    b = E_b[D],   x_b = w^T E_b .

With these, the full system (L_b + k0^2 P_D^T diag(deps) P_D) E = i k0 J is
equivalent to (I - k0^2 G_DD diag(deps)) E_D = b and
x = x_b + k0^2 G_OD diag(deps) E_D (Supplementary Note 4, C = I + Y G, with
the sign of G fixed by the field form).

Every quantity here is computed column by column from its definition; no
symmetry is assumed (G_OD uses a transposed solve, not reciprocity).

Pins: reciprocity G_DD = G_DD^T and G_OD against the adjoint-solve rows
(tests/test_oracle_green.py::test_reciprocity), the one- and two-pixel closed
forms (::test_single_pixel_closed_form, ::test_two_pixel_closed_form) and the
exhaustive enumeration of a 3x3 region (::test_enumerate_3x3).
"""
from __future__ import annotations

import numpy as np

from .fdfd import Solver, assemble, rhs, total_eps


def _background_solver(prob, fi):
    eps = total_eps(prob, np.zeros(prob.n_d, dtype=np.uint8))
    L, scale = assemble(prob.nx, prob.ny, prob.npml, prob.h, eps, prob.k0[fi])
    return Solver(L, scale)


def green_dd(prob, fi, cols=None, solver=None):
    """Columns ``cols`` (pixel ids) of G_DD = -(L_b^-1)[D, D] at frequency fi."""
    S = solver or _background_solver(prob, fi)
    idx = prob.design_indices()
    cols = np.arange(prob.n_d) if cols is None else np.asarray(cols)
    N = prob.nx * prob.ny
    out = np.empty((prob.n_d, len(cols)), dtype=np.complex128)
    step = 64
    for c0 in range(0, len(cols), step):
        cc = cols[c0:c0 + step]
        B = np.zeros((N, len(cc)), dtype=np.complex128)
        B[idx[cc], np.arange(len(cc))] = 1.0
        X = S.solve(B)
        out[:, c0:c0 + len(cc)] = -X[idx, :]
    return out


def green_od(prob, fi, solver=None):
    """G_OD = -w^T L_b^-1[:, D] (1 x N_d) via a transposed solve of L_b."""
    S = solver or _background_solver(prob, fi)
    idx = prob.design_indices()
    # L^-1 = A^-1 diag(scale) with A = diag(scale) L, so w^T L^-1 =
    # (A^-T w)^T diag(scale).
    w = prob.w[0].astype(np.complex128)
    y = S.lu.solve(w, trans="T")
    r = w - S.A.T @ y
    y = y + S.lu.solve(r, trans="T")
    row = y * S.scale
    return -row[idx][None, :]


def background(prob, fi, solver=None):
    """(E_b full field, b = E_b[D], x_b = w^T E_b) at frequency fi."""
    S = solver or _background_solver(prob, fi)
    Eb = S.solve(rhs(prob.src[fi], prob.k0[fi]))
    idx = prob.design_indices()
    return Eb, Eb[idx].copy(), complex(prob.w[0] @ Eb)


def output_row(prob, bits, fi):
    """R'_D = -w^T L(eps)^-1[:, D] for the current design (1-D, N_d) by a
    transposed solve of the full operator of that design.

    It is the output row of the PNGF state: a small change d of the
    permittivity of pixel m changes x by k0^2 d E[m] R'[m] to first order
    (adjoint sensitivity; pinned by central finite differences in
    tests/test_oracle_green.py::test_output_row_is_adjoint_sensitivity), and
    for the background design it equals G_OD."""
    eps = total_eps(prob, bits)
    L, scale = assemble(prob.nx, prob.ny, prob.npml, prob.h, eps, prob.k0[fi])
    S = Solver(L, scale)
    idx = prob.design_indices()
    w = prob.w[0].astype(np.complex128)
    y = S.lu.solve(w, trans="T")
    r = w - S.A.T @ y
    y = y + S.lu.solve(r, trans="T")
    return -(y * S.scale)[idx]


def equivalent_current(prob, bits, fi):
    """(E full field, j on the design pixels) for a design of PEC pixels.

    Current equivalence (Results, Numerical Green's functions; Supplementary
    Note 1): the conductors are replaced by a current on their nodes that,
    radiating in the background environment, gives the same field.  From the
    Dirichlet solution E of the full system, that current is the residual of
    the background operator, j = (L_b E - i k0 J) restricted to the design,
    in the paper's sign convention (field = e_inc - G j with G = G_DD =
    -(L_b^-1)[D, D]): it vanishes on open pixels and E_D = b - G_DD j holds
    by construction."""
    from .fdfd import field, rhs
    E = field(prob, bits, fi)
    eps = total_eps(prob, np.zeros(prob.n_d, dtype=np.uint8))
    Lb, _ = assemble(prob.nx, prob.ny, prob.npml, prob.h, eps, prob.k0[fi])
    r = Lb @ E - rhs(prob.src[fi], prob.k0[fi])
    return E, r[prob.design_indices()].copy()


def pec_state(prob, bits, fi):
    """(z, x) of a PEC design: z = E_D on open pixels and the equivalent
    current j (see equivalent_current) on conducting pixels, x = w^T E."""
    E, j = equivalent_current(prob, bits, fi)
    idx = prob.design_indices()
    on = np.asarray(bits) != 0
    z = np.where(on, j, E[idx])
    return z, complex(prob.w[0] @ E)


def pngf_state(prob, bits, fi):
    """(E_D, x) for design ``bits`` at frequency fi, from one full solve."""
    from .fdfd import field
    E = field(prob, bits, fi)
    idx = prob.design_indices()
    return E[idx].copy(), complex(prob.w[0] @ E)
