"""Direct binary search with a full sparse re-solve per candidate, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Direct binary search (Results, Direct binary search optimization): start from
an initial design; flip one tile at a time in a random order; keep the flip if
the objective improves, otherwise try another tile; the search has converged
when every possible flip has been tried without improvement.  Readings taken
where the paper is silent:

* the visiting order of sweep s is the explicit permutation perms[s]; after an
  accepted flip the search continues with the next position of the same
  sweep; a sweep that ends starts the next permutation at position 0;
* "improves" means f' - f > eta * f with eta = 1e-9 (f >= 0 is maximized);
* converged = one whole sweep without an accepted flip; the run also stops
  after len(perms) sweeps;
* an "attempted flip" is one visited position (each costs one evaluation).

Every candidate objective f' is obtained by assembling the FDFD operator of
the candidate design and solving it (sparse LU + one refinement step) at every
frequency; PEC pixels enter that operator as Ez = 0 on their nodes.  Candidates ahead of the cursor may be evaluated speculatively in a
process pool; the decisions are those of the sequential loop.

Pins: tests/test_oracle_dbs.py checks, by independent full solves, that every
accepted flip improves by more than eta*f, that every skipped position between
two accepts does not, and that the converged design is a single-flip local
optimum (every flip enumerated).
"""
from __future__ import annotations

from dataclasses import dataclass, field as dfield
import os

import numpy as np
import scipy.sparse as sp

from .fdfd import Solver, assemble, rhs, total_eps, objective, metal_nodes, pec_system, PEC

ETA = 1e-9

_W = {}


def _base_ops(prob):
    """Background operators per frequency (design cells at eps_lo)."""
    eps = total_eps(prob, np.zeros(prob.n_d, dtype=np.uint8))
    ops = []
    for fi in range(prob.nfreq):
        L, scale = assemble(prob.nx, prob.ny, prob.npml, prob.h, eps, prob.k0[fi])
        ops.append((L, scale))
    return ops


def _eval_bits(prob, ops, bits):
    """Objective and outputs x_f of design ``bits`` by full solves."""
    idx = prob.design_indices()
    deps = np.where(np.asarray(bits) != 0, prob.eps_hi - prob.eps_lo, 0.0)
    xs = np.empty(prob.nfreq, dtype=np.complex128)
    N = prob.nx * prob.ny
    metal = metal_nodes(prob, bits)
    for fi, (Lb, scale) in enumerate(ops):
        k0 = prob.k0[fi]
        b = rhs(prob.src[fi], k0)
        if getattr(prob, "pixel_kind", 0) == PEC:
            L, b = pec_system(Lb, b, metal)
        else:
            d = np.zeros(N, dtype=np.complex128)
            d[idx] = k0 * k0 * deps
            L = sp.csc_matrix(Lb + sp.diags(d))
        E = Solver(L, scale).solve(b)
        xs[fi] = prob.w[0] @ E
    return objective(prob, xs), xs


def _worker_init(prob):
    # one BLAS thread per worker process: the pool provides the parallelism
    try:
        from threadpoolctl import threadpool_limits
        _W["limits"] = threadpool_limits(1)
    except ImportError:
        pass
    _W["prob"] = prob
    _W["ops"] = _base_ops(prob)


def _worker_eval(bits):
    return _eval_bits(_W["prob"], _W["ops"], bits)[0]


@dataclass
class DBSResult:
    accepted: list = dfield(default_factory=list)   # (sweep, pos, pixel, f_new)
    f0: float = 0.0
    f_final: float = 0.0
    bits: np.ndarray = None
    attempts: int = 0
    sweeps: int = 0
    converged: bool = False
    near_ties: list = dfield(default_factory=list)  # (sweep, pos, pixel, margin)


def _flip(bits, cand, tiles):
    """Copy of bits with candidate ``cand`` flipped: one pixel, or every pixel
    of tile ``cand`` when ``tiles`` ((n_tiles, M), -1 padded) is given."""
    b = bits.copy()
    if tiles is None:
        b[cand] ^= 1
    else:
        row = np.asarray(tiles[cand])
        b[row[row >= 0]] ^= 1
    return b


def score_all(prob, bits, cands=None, workers=1, tiles=None):
    """f' for flipping each candidate (full re-solve each); returns array.
    Candidates are pixels, or tiles of pixels flipped together."""
    bits = np.asarray(bits, dtype=np.uint8)
    n = prob.n_d if tiles is None else len(tiles)
    cands = np.arange(n) if cands is None else np.asarray(cands)
    designs = [_flip(bits, m, tiles) for m in cands]
    if workers <= 1:
        ops = _base_ops(prob)
        return np.array([_eval_bits(prob, ops, b)[0] for b in designs])
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers, _worker_init, (prob,)) as pool:
        return np.array(pool.map(_worker_eval, designs, chunksize=1))


def dbs(prob, bits0=None, perms=None, eta=ETA, workers=1, tie_band=1e-7,
        progress=None, tiles=None, max_accepts=None):
    """Run DBS on ``prob``; returns a DBSResult.  With ``tiles`` ((n_tiles, M)
    pixel ids, -1 padded) a candidate is a tile whose pixels all flip
    together (a rank-M update in the paper's terms, eq. lru_dcn), ``perms``
    order the tiles and the accepted entries name tiles.  With
    ``max_accepts`` the search stops right after that many accepted flips
    (attempts counted up to and including the last accepted one)."""
    bits = np.array(prob.init_bits if bits0 is None else bits0, dtype=np.uint8)
    perms = prob.perms if perms is None else np.asarray(perms)
    ops = _base_ops(prob)
    f, _ = _eval_bits(prob, ops, bits)
    res = DBSResult(f0=f)
    pool = None
    if workers > 1:
        import multiprocessing as mp
        pool = mp.get_context("fork").Pool(workers, _worker_init, (prob,))
    try:
        for s in range(perms.shape[0]):
            res.sweeps = s + 1
            any_acc = False
            pos = 0
            n = perms.shape[1]
            while pos < n:
                width = workers if pool is not None else 1
                batch = list(range(pos, min(n, pos + width)))
                designs = [_flip(bits, perms[s, q], tiles) for q in batch]
                if pool is not None:
                    fs = pool.map(_worker_eval, designs, chunksize=1)
                else:
                    fs = [_eval_bits(prob, ops, designs[0])[0]]
                taken = None
                for q, fn in zip(batch, fs):
                    res.attempts += 1
                    margin = (fn - f) / f - eta if f != 0 else fn - f
                    if abs(margin) < tie_band:
                        res.near_ties.append((s, q, int(perms[s, q]), margin))
                    if fn - f > eta * f:
                        taken = (q, fn)
                        break
                if taken is None:
                    pos = batch[-1] + 1
                    if progress is not None:
                        progress(res)
                    continue
                q, fn = taken
                m = int(perms[s, q])
                bits = _flip(bits, m, tiles)
                f = fn
                res.accepted.append((s, q, m, fn))
                any_acc = True
                pos = q + 1
                if progress is not None:
                    progress(res)
                if max_accepts is not None and len(res.accepted) >= max_accepts:
                    break
            if max_accepts is not None and len(res.accepted) >= max_accepts:
                break
            if not any_acc:
                res.converged = True
                break
    finally:
        if pool is not None:
            pool.close()
            pool.join()
    res.f_final = f
    res.bits = bits
    return res
