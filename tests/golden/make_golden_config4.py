"""Writes the golden values of the large broadband workload (640x640 grid,
80x80 design, eight frequencies) from the CPU oracle (full sparse re-solves).

Calls only ``oracle`` and ``workloads``.  One candidate costs eight sparse LU
solves of a 409,600-node system, so the search is cut after a fixed number of
accepted flips (the GPU run uses the same cap).  Usage:
    python tests/golden/make_golden_config4.py [--workers N] [--accepts K]
Writes tests/golden/config4_golden.json with
  * the per-frequency normalizers (vacuum transmission);
  * at the initial design: f, x_f, and E_f at 256 sampled pixels together
    with max |E_f| over the design region, for all eight frequencies;
  * f' of 32 sampled candidate flips at the initial design;
  * the accepted flips (sweep, position, pixel, f_new), attempts and near-ties
    of the search capped at K accepts;
  * at the design it ends in: f, x_f and the sampled E_f.
"""
import argparse
import json
import os
import sys
import time

for _v in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads  # noqa: E402

N_FIELD_SAMPLES = 256
N_CAND_SAMPLES = 32


def fields(p, bits, pix, workers):
    """(f, x [F], E at pix [F, len(pix)], max |E| over D [F]) by full solves,
    the frequencies in a process pool."""
    import multiprocessing as mp
    idx = p.design_indices()
    with mp.get_context("fork").Pool(min(workers, p.nfreq)) as pool:
        Es = pool.starmap(oracle.field, [(p, bits, fi) for fi in range(p.nfreq)])
    xs = np.array([p.w[0] @ E for E in Es])
    ED = np.array([E[idx] for E in Es])
    return (oracle.objective(p, xs[:, None]), xs, ED[:, pix], np.abs(ED).max(axis=1))


def cplx(a):
    a = np.asarray(a)
    return [[float(v.real), float(v.imag)] for v in a.ravel()]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=7)
    ap.add_argument("--accepts", type=int, default=16)
    a = ap.parse_args()
    p = workloads.config4()
    t0 = time.time()
    rng = np.random.Generator(np.random.PCG64([4, 4444]))
    pix = np.sort(rng.choice(p.n_d, N_FIELD_SAMPLES, replace=False))
    cands = np.sort(rng.choice(p.n_d, N_CAND_SAMPLES, replace=False))
    norms = oracle.objective_norms(p)
    f0, x0, E0, emax0 = fields(p, p.init_bits, pix, a.workers)
    print(f"initial fields: f0 {f0:.6e}, {time.time()-t0:.0f}s", flush=True)
    fc = oracle.score_all(p, p.init_bits, cands, workers=a.workers)
    print(f"candidates: {time.time()-t0:.0f}s", flush=True)
    last = [time.time()]

    def prog(res):
        if time.time() - last[0] > 60:
            last[0] = time.time()
            print(f"dbs: {len(res.accepted)} accepts, {res.attempts} attempts, "
                  f"{time.time()-t0:.0f}s", flush=True)
    res = oracle.dbs(p, workers=a.workers, progress=prog, max_accepts=a.accepts)
    f1, x1, E1, emax1 = fields(p, res.bits, pix, a.workers)
    assert abs(f1 - res.f_final) <= 1e-12 * abs(f1)
    out = {
        "workload": p.name, "seed": p.seed, "eta": oracle.dbs.__globals__["ETA"],
        "norms": [float(v) for v in norms],
        "sample_pixels": [int(v) for v in pix],
        "initial": {"f": f0, "x": cplx(x0), "E": cplx(E0), "E_max": [float(v) for v in emax0]},
        "candidates": [int(v) for v in cands],
        "candidate_f": [float(v) for v in fc],
        "max_accepts": a.accepts,
        "accepted": [[int(s), int(q), int(m), float(f)] for (s, q, m, f) in res.accepted],
        "attempts": res.attempts,
        "near_ties": [[int(s), int(q), int(m), float(g)] for (s, q, m, g) in res.near_ties],
        "final": {"f": f1, "x": cplx(x1), "E": cplx(E1), "E_max": [float(v) for v in emax1]},
        "oracle_seconds": time.time() - t0, "workers": a.workers,
    }
    with open(os.path.join(HERE, "config4_golden.json"), "w") as fh:
        json.dump(out, fh, indent=0)
    print(f"done: {len(res.accepted)} accepts, {res.attempts} attempts, "
          f"f {f0:.6e} -> {f1:.6e}, {time.time()-t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
