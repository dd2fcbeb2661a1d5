"""Writes the golden DBS trajectories from the CPU oracle (full re-solves).

Calls only ``oracle`` and ``workloads``.  Usage:
    python tests/golden/make_golden.py 0 [1] [metal] [tiles1] [config4_scaled] [--workers N]
Writes tests/golden/dbs_config{i}.json (dbs_metal.json for the PEC-pixel
workload ``workloads.metal()``, dbs_tiles1.json for the 4x4-tile search
``workloads.tiles1()``, whose accepted entries name tiles, dbs_config4_scaled.json
for the eight-frequency ``workloads.config4_scaled()``) with the accepted flips
(sweep, position, pixel, f_new), the initial and final objective, the number
of attempted flips, and any near-ties within 1e-7 of the acceptance threshold.
"""
import argparse
import json
import os
import sys
import time

# one BLAS / OpenMP thread per process: parallelism comes from the worker pool
for _v in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("configs", nargs="+")
    ap.add_argument("--workers", type=int, default=1)
    a = ap.parse_args()
    for c in a.configs:
        named = {"metal": workloads.metal, "tiles1": workloads.tiles1,
                 "config4_scaled": workloads.config4_scaled}
        p = named[c]() if c in named else workloads.make_config(int(c))
        tag = c if c in named else f"config{c}"
        tk = {} if p.tiles is None else {"perms": p.tile_perms, "tiles": p.tiles}
        t0 = time.time()
        last = [t0]

        def prog(res):
            if time.time() - last[0] > 30:
                last[0] = time.time()
                print(f"{tag}: {len(res.accepted)} accepts, "
                      f"{res.attempts} attempts, {time.time()-t0:.0f}s", flush=True)
        res = oracle.dbs(p, workers=a.workers, progress=prog, **tk)
        out = {
            "workload": p.name, "seed": p.seed, "eta": oracle.dbs.__globals__["ETA"],
            "f0": res.f0, "f_final": res.f_final, "attempts": res.attempts,
            "sweeps": res.sweeps, "converged": res.converged,
            "accepted": [[int(s), int(q), int(m), float(f)] for (s, q, m, f) in res.accepted],
            "near_ties": [[int(s), int(q), int(m), float(g)] for (s, q, m, g) in res.near_ties],
            "oracle_seconds": time.time() - t0, "workers": a.workers,
        }
        with open(os.path.join(HERE, f"dbs_{tag}.json"), "w") as fh:
            json.dump(out, fh, indent=0)
        print(f"{tag}: done {len(res.accepted)} accepts, {res.attempts} attempts, "
              f"f {res.f0:.6e} -> {res.f_final:.6e}, {time.time()-t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
