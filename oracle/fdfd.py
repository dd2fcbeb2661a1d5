"""2D TM (Ez) FDFD operator with SC-PML and sparse direct solves, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Discrete problem (the paper fixes only "FDFD on a Yee grid with PML";
Supplementary Note 2 gives A = -i w diag(eps) + (i/w) D^H diag(1/mu) D^E for the
time convention e^{+i w t}).  For Ez in 2D with c0 = eps0 = mu0 = 1, lengths in
lambda0 and w = k0, eliminating H gives (lap + k0^2 eps) Ez = i k0 Jz, i.e. the
paper's A equals -(i/k0) times this operator.  We solve

    (L E)_ij = [ (E_{i+1,j}-E_ij)/s_x(i+1/2) - (E_ij-E_{i-1,j})/s_x(i-1/2) ]
               / (h^2 s_x(i))  + (same along y)  + k0^2 eps_ij E_ij
             = i k0 J_ij ,

with Ez = 0 beyond the grid (Dirichlet) and the PML stretch
    d(u) = max(0, npml - u, u - (N-1-npml)) / npml     (u in cell units)
    sigma(u) = sigma_max d(u)^3,  sigma_max = -(m+1) ln(R) / (2 npml h),
    m = 3, R = 1e-8,  s(u) = 1 - i sigma(u)/k0,
so outgoing waves (e^{-i kappa x}) decay inside the layer.

Pins: the 1D closed-form discrete Green function and PML attenuation
(tests/test_oracle_fdfd.py::test_1d_closed_form), the exact discrete energy
balance of the 5-point stencil (::test_energy_balance), the reflection against
a 4x larger domain (::test_pml_reflection), dense inversion of the same matrix
on a tiny grid (::test_dense_bruteforce), symmetry of the scaled operator
(::test_operator_symmetric).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

PML_ORDER = 3
PML_R = 1e-8


def pml_profile(u, n: int, npml: int, h: float):
    """Normalized PML depth d(u) in [0, ...) for position u (cell units)."""
    u = np.asarray(u, dtype=np.float64)
    if npml <= 0:
        return np.zeros_like(u)
    d = np.maximum(0.0, np.maximum(npml - u, u - (n - 1 - npml)))
    return d / npml


def stretch(u, n: int, npml: int, h: float, k0: float):
    """Complex coordinate stretch s(u) = 1 - i sigma(u) / k0."""
    d = pml_profile(u, n, npml, h)
    if npml <= 0:
        return np.ones_like(d, dtype=np.complex128)
    sigma_max = -(PML_ORDER + 1) * math.log(PML_R) / (2.0 * npml * h)
    sigma = sigma_max * d ** PML_ORDER
    return 1.0 - 1j * sigma / k0


def assemble(nx, ny, npml, h, eps, k0, periodic_y=False, pml_y=True):
    """Return (L, scale): sparse L (unsymmetric form above) and the row scale.

    ``scale`` = s_x(i) s_y(j) per node; diag(scale) @ L is complex symmetric.
    ``periodic_y`` and ``pml_y`` are test-only options (1D checks).
    """
    eps = np.asarray(eps, dtype=np.float64).reshape(ny, nx)
    npml_y = npml if pml_y else 0
    ii = np.arange(nx, dtype=np.float64)
    jj = np.arange(ny, dtype=np.float64)
    sx_n = stretch(ii, nx, npml, h, k0)
    sx_p = stretch(ii + 0.5, nx, npml, h, k0)
    sx_m = stretch(ii - 0.5, nx, npml, h, k0)
    sy_n = stretch(jj, ny, npml_y, h, k0)
    sy_p = stretch(jj + 0.5, ny, npml_y, h, k0)
    sy_m = stretch(jj - 0.5, ny, npml_y, h, k0)
    N = nx * ny
    inv_h2 = 1.0 / (h * h)
    I, Jg = np.meshgrid(np.arange(nx), np.arange(ny))      # [j, i] grids
    node = (Jg * nx + I).ravel()
    # coefficient of E_{i+1,j}, E_{i-1,j}, E_{i,j+1}, E_{i,j-1} in row (i, j)
    cxp = (inv_h2 / (sx_n * sx_p))[None, :].repeat(ny, 0).ravel()
    cxm = (inv_h2 / (sx_n * sx_m))[None, :].repeat(ny, 0).ravel()
    cyp = (inv_h2 / (sy_n * sy_p))[:, None].repeat(nx, 1).ravel()
    cym = (inv_h2 / (sy_n * sy_m))[:, None].repeat(nx, 1).ravel()
    diag = k0 * k0 * eps.ravel() - cxp - cxm - cyp - cym
    Ir, Jr = I.ravel(), Jg.ravel()
    rows, cols, vals = [node], [node], [diag.astype(np.complex128)]
    # x neighbours: Dirichlet (drop links leaving the grid)
    m = Ir + 1 < nx
    rows.append(node[m]); cols.append(node[m] + 1); vals.append(cxp[m])
    m = Ir - 1 >= 0
    rows.append(node[m]); cols.append(node[m] - 1); vals.append(cxm[m])
    if periodic_y:
        rows.append(node); cols.append(((Jr + 1) % ny) * nx + Ir); vals.append(cyp)
        rows.append(node); cols.append(((Jr - 1) % ny) * nx + Ir); vals.append(cym)
    else:
        m = Jr + 1 < ny
        rows.append(node[m]); cols.append(node[m] + nx); vals.append(cyp[m])
        m = Jr - 1 >= 0
        rows.append(node[m]); cols.append(node[m] - nx); vals.append(cym[m])
    L = sp.csc_matrix((np.concatenate(vals).astype(np.complex128),
                       (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    L.sum_duplicates()
    scale = np.outer(sy_n, sx_n).ravel()
    return L, scale


def rhs(J, k0):
    """Right-hand side i k0 J of L E = i k0 J."""
    return 1j * k0 * np.asarray(J, dtype=np.complex128)


class Solver:
    """Sparse LU of the symmetrized operator diag(scale) L, with refinement."""

    def __init__(self, L, scale, permc_spec="COLAMD"):
        self.scale = scale
        self.A = sp.diags(scale) @ L
        self.A = sp.csc_matrix(self.A)
        self.lu = spla.splu(self.A, permc_spec=permc_spec)

    def solve(self, b, refine=1):
        """Solve L x = b (b may be 1D or 2D column block)."""
        sb = (self.scale[:, None] * b) if b.ndim == 2 else self.scale * b
        x = self.lu.solve(sb)
        for _ in range(refine):
            r = sb - self.A @ x
            x = x + self.lu.solve(r)
        return x


def solve(nx, ny, npml, h, eps, k0, J, refine=1, permc_spec="COLAMD"):
    L, scale = assemble(nx, ny, npml, h, eps, k0)
    return Solver(L, scale, permc_spec).solve(rhs(J, k0), refine)


def total_eps(prob, bits):
    """Permittivity map with design bits applied (background + design)."""
    eps = prob.eps_static.copy().ravel()
    idx = prob.design_indices()
    eps[idx] = np.where(np.asarray(bits) != 0, prob.eps_hi, prob.eps_lo)
    return eps.reshape(prob.ny, prob.nx)


PEC = 1


def metal_nodes(prob, bits):
    """Flat node ids of the design pixels that are perfect conductors (empty
    unless the problem has PEC pixels)."""
    if getattr(prob, "pixel_kind", 0) != PEC:
        return np.zeros(0, dtype=np.int64)
    return prob.design_indices()[np.asarray(bits) != 0]


def pec_system(L, b, nodes):
    """Impose Ez = 0 on ``nodes`` (perfect electric conductor, the sigma ->
    infinity limit of Results, Numerical Green's functions): with K the
    diagonal 0/1 mask of the free nodes, K L K + (I - K) and K b.  The rows
    and columns of the conductor nodes become identity rows and columns, the
    rest of the system is untouched, and symmetry is kept."""
    N = L.shape[0]
    keep = np.ones(N)
    keep[np.asarray(nodes, dtype=np.int64)] = 0.0
    K = sp.diags(keep)
    Lp = sp.csc_matrix(K @ L @ K + sp.diags(1.0 - keep))
    return Lp, keep * b


def total_operator(prob, bits, fi):
    """(L, scale, right-hand side) of the full system of design ``bits`` at
    frequency fi: dielectric pixels enter through eps, PEC pixels as Ez = 0."""
    k0 = prob.k0[fi]
    b = rhs(prob.src[fi], k0)
    if getattr(prob, "pixel_kind", 0) == PEC:
        eps = total_eps(prob, np.zeros(prob.n_d, dtype=np.uint8))
        L, scale = assemble(prob.nx, prob.ny, prob.npml, prob.h, eps, k0)
        L, b = pec_system(L, b, metal_nodes(prob, bits))
        return L, scale, b
    L, scale = assemble(prob.nx, prob.ny, prob.npml, prob.h, total_eps(prob, bits), k0)
    return L, scale, b


def field(prob, bits, fi, refine=1):
    """Full-domain Ez at frequency index fi for the design ``bits``."""
    L, scale, b = total_operator(prob, bits, fi)
    return Solver(L, scale).solve(b, refine)


MEAN_TRANSMISSION = 2


def objective_norms(prob):
    """Per-frequency normalizers norm_f of the objective.

    ``obj_norm`` as given; for the mean-transmission objective each is further
    multiplied by the vacuum transmission |w^T E_vac,f|^2, where E_vac,f is the
    field of the same source on the same grid and PML with eps = 1 everywhere
    (no static features, no design).  This reads the paper's per-frequency
    transmission objectives (Supplementary Notes, Objective functions for
    design studies: a transmission coefficient per frequency, combined by a
    mean) as power transmitted relative to empty space.  Computed once per
    problem object and kept on it."""
    base = np.asarray(prob.obj_norm, dtype=np.float64)
    if int(prob.objective_kind) != MEAN_TRANSMISSION:
        return base
    cached = prob.__dict__.get("_oracle_vacuum_norms")
    if cached is None:
        one = np.ones((prob.ny, prob.nx))
        t = np.empty(prob.nfreq)
        for fi in range(prob.nfreq):
            E = solve(prob.nx, prob.ny, prob.npml, prob.h, one, prob.k0[fi], prob.src[fi])
            t[fi] = abs(prob.w[0] @ E) ** 2
        cached = t
        prob.__dict__["_oracle_vacuum_norms"] = cached
    return base * cached


def objective(prob, xs):
    """f = mean over frequencies of |x_f|^2 / norm_f (x_f = w^T E_f, N_obj=1).

    Covers the point intensity |Ez|^2, the Gaussian-overlap intensity
    |sum_y w(y) Ez(x_out, y)|^2 (no conjugate, no h factor) and the mean
    transmission normalized by vacuum (``objective_norms``); all three are to
    be maximized.
    """
    xs = np.asarray(xs, dtype=np.complex128).reshape(prob.nfreq, -1)
    return float(np.mean(np.abs(xs[:, 0]) ** 2 / objective_norms(prob)))
