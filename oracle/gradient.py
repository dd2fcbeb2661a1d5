"""Objective gradient with respect to the pixel permittivities, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Supplementary Note 5 obtains df/d eps_r over the whole design region from the
state of the current design; its chain rule (eq. supp_grad_chainrule) is

    df/d eps_m = 2 Re[ (df/dx) (dx/dy) (dy/d eps_m) ],

with the Wirtinger derivative df/dx = conj(x) for f = |x|^2.  Here every factor
comes from its plain definition on the full FDFD system L(eps) E = i k0 J,
x = w^T E: differentiating L E = i k0 J gives dE/d eps_m = -L^-1 (dL/d eps_m) E
with dL/d eps_m = k0^2 e_m e_m^T (the operator's diagonal holds k0^2 eps), so

    dx/d eps_m = -k0^2 (w^T L^-1)[m] E[m],

one forward and one adjoint (transposed) sparse solve per frequency, i.e. the
conventional adjoint method on the full simulation domain.  With the mean over
frequencies of |x_f|^2 / norm_f:

    df/d eps_m = sum_f 2 Re[conj(x_f) dx_f/d eps_m] / (F norm_f).

Pin: central finite differences of full re-solves in a continuous eps_m,
converging at second order (tests/test_oracle_gradient.py).
"""
from __future__ import annotations

import numpy as np

from .fdfd import Solver, assemble, rhs, total_eps, objective_norms


def gradient(prob, bits):
    """df/d eps_m for every design pixel m at the design ``bits``."""
    eps = total_eps(prob, bits)
    idx = prob.design_indices()
    g = np.zeros(prob.n_d)
    w = prob.w[0].astype(np.complex128)
    norms = objective_norms(prob)
    for fi in range(prob.nfreq):
        k0 = prob.k0[fi]
        L, scale = assemble(prob.nx, prob.ny, prob.npml, prob.h, eps, k0)
        S = Solver(L, scale)
        E = S.solve(rhs(prob.src[fi], k0))
        x = complex(w @ E)
        # w^T L^-1 = (A^-T w)^T diag(scale) with A = diag(scale) L
        y = S.lu.solve(w, trans="T")
        y = y + S.lu.solve(w - S.A.T @ y, trans="T")
        adj = (y * scale)[idx]
        dx = -k0 * k0 * adj * E[idx]
        g += 2.0 * np.real(np.conj(x) * dx) / (prob.nfreq * norms[fi])
    return g
