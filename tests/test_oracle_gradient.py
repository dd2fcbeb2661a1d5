"""Pin of the oracle's objective gradient (CPU only): central finite
differences of full re-solves in a continuous pixel permittivity, whose error
falls at second order in the step."""
import numpy as np
import scipy.sparse as sp

import oracle
import oracle.fdfd as fd
import workloads


def _f_with(p, bits, m, d):
    """Objective with pixel m's permittivity shifted by d (full solves)."""
    xs = []
    eps = fd.total_eps(p, bits).ravel().copy()
    eps[p.design_indices()[m]] += d
    for fi in range(p.nfreq):
        L, scale = fd.assemble(p.nx, p.ny, p.npml, p.h, eps, p.k0[fi])
        E = fd.Solver(L, scale).solve(fd.rhs(p.src[fi], p.k0[fi]))
        xs.append(p.w[0] @ E)
    return oracle.objective(p, xs)


def test_gradient_matches_central_differences():
    p = workloads.tiny(seed=17, n=22, npml=4, side=4, nfreq=2)
    bits = p.init_bits
    g = oracle.gradient(p, bits)
    for m in (0, 5, 10, 15):
        errs = []
        for hstep in (1e-2, 5e-3):
            fd_m = (_f_with(p, bits, m, hstep) - _f_with(p, bits, m, -hstep)) / (2 * hstep)
            errs.append(abs(fd_m - g[m]))
        assert errs[1] < 1e-6 * np.max(np.abs(g))
        # second order: halving the step quarters the error (when resolvable)
        if errs[0] > 1e-9 * np.max(np.abs(g)):
            assert 2.5 < errs[0] / errs[1] < 6.0
