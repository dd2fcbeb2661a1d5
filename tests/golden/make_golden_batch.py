"""Writes oracle golden values for a batch of problems of the batching
workload (seeded problems of uneven size and frequency count), from full
sparse re-solves.

Calls only ``oracle`` and ``workloads``.  The problems cover every search
kernel a batch dispatches: design sides 17-56 (N_d 289-3136) with one to four
frequencies.  Each search is cut after a fixed number of accepted flips (the
GPU runs use the same cap).  Usage:
    python tests/golden/make_golden_batch.py [--workers N] [--accepts K]
Writes tests/golden/batch_config2.json: per problem its seed, the accepted
flips (sweep, position, pixel, f_new), attempts, f0, and at the design the
search ends in f, x_f and E_f at 64 sampled pixels with max |E_f| over the
design region.
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

# (seed, N_d, frequencies): 1009 (289, 4), 1002 (625, 3), 1031 (1369, 1),
# 1038 (1600, 4), 1017 (2401, 1), 1029 (3136, 4)
SEEDS = (1009, 1002, 1031, 1038, 1017, 1029)
N_FIELD_SAMPLES = 64


def cplx(a):
    a = np.asarray(a)
    return [[float(v.real), float(v.imag)] for v in a.ravel()]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=7)
    ap.add_argument("--accepts", type=int, default=24)
    a = ap.parse_args()
    out = {"eta": oracle.dbs.__globals__["ETA"], "max_accepts": a.accepts, "problems": []}
    t0 = time.time()
    for seed in SEEDS:
        p = workloads.config2_problem(seed)
        res = oracle.dbs(p, workers=a.workers, max_accepts=a.accepts)
        rng = np.random.Generator(np.random.PCG64([seed, 2222]))
        pix = np.sort(rng.choice(p.n_d, min(N_FIELD_SAMPLES, p.n_d), replace=False))
        idx = p.design_indices()
        Es = [oracle.field(p, res.bits, fi) for fi in range(p.nfreq)]
        xs = np.array([p.w[0] @ E for E in Es])
        ED = np.array([E[idx] for E in Es])
        f1 = oracle.objective(p, xs[:, None])
        assert abs(f1 - res.f_final) <= 1e-12 * abs(f1)
        out["problems"].append({
            "seed": seed, "n_d": p.n_d, "nfreq": p.nfreq, "f0": res.f0, "f_final": f1,
            "accepted": [[int(s), int(q), int(m), float(f)] for (s, q, m, f) in res.accepted],
            "attempts": res.attempts, "sweeps": res.sweeps, "converged": res.converged,
            "near_ties": [[int(s), int(q), int(m), float(g)] for (s, q, m, g) in res.near_ties],
            "x": cplx(xs), "sample_pixels": [int(v) for v in pix], "E": cplx(ED[:, pix]),
            "E_max": [float(v) for v in np.abs(ED).max(axis=1)]})
        print(f"seed {seed}: N_d {p.n_d}, F {p.nfreq}: {len(res.accepted)} accepts, "
              f"{res.attempts} attempts, f {res.f0:.6e} -> {f1:.6e}, {time.time()-t0:.0f}s",
              flush=True)
    out["oracle_seconds"] = time.time() - t0
    with open(os.path.join(HERE, "batch_config2.json"), "w") as fh:
        json.dump(out, fh, indent=0)


if __name__ == "__main__":
    main()
