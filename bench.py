"""Benchmark of the PNGF hot path on one MI355X.

A step is one complete direct-binary-search run on the 256x256 / 40x40-pixel
workload (N_d = 1600, five sweeps): initial inverse, scoring of every
candidate, selection, Sherman-Morrison accepts until convergence or the sweep
cap.  `value` is attempted flip evaluations per second over the K timed runs
(time-to-design is ms_per_step).  Inputs (G, b, G_OD, x_b) are resident in
HBM before timing starts; the host precompute is reported separately.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

def log(msg):
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


METRIC = "flip evals/s + time-to-design, mixed vs FP64 plain, ≤1e-6 rel objective err"
HBM_PEAK_GBS = 8000.0


def cpu_baseline(prob, seconds_target=15.0):
    """Oracle (full sparse re-solve per candidate) on the host cores, on a
    bounded sample: candidate evaluations at the initial design, evaluated by
    a process pool over the available cores."""
    import numpy as np
    import oracle
    cores = len(os.sched_getaffinity(0))
    workers = max(1, min(cores, 16))
    n = 2 * workers
    cands = np.arange(n)
    t0 = time.perf_counter()
    oracle.score_all(prob, prob.init_bits, cands, workers=workers)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "flip evals/s", "cores": workers, "kind": "oracle",
            "sample": f"{n} candidate flips of the initial design, each a full sparse "
                      f"LU re-solve of the {prob.nx}x{prob.ny} FDFD system; {dt:.1f} s wall"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py: this build measures one GPU only (the hot path runs on one "
              "MI355X); multi-GPU runs are not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads
    import paper_2501_18054_amd as P

    prob = workloads.config1()
    cpu = None
    if not a.no_cpu_baseline:
        # before any GPU initialization: the oracle's process pool forks
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(prob)
        log(f"cpu baseline: {cpu['value']:.3f} flip evals/s on {cpu['cores']} cores")
    log("precompute (host) ...")
    t0 = time.perf_counter()
    h = P.Handle(prob)
    t_pre = time.perf_counter() - t0
    log(f"precompute done in {t_pre:.1f} s; binding")
    h.bind(P.default_options(max_accepts=8192, max_sweeps=8, timing=True))
    stream = torch.cuda.current_stream()

    def one_run():
        h.set_design(prob.init_bits)
        return h.dbs_run(prob.perms)

    for w in range(a.warmup):
        r = one_run()
        log(f"warmup run {w}: {r['n_accepted']} accepts, {r['attempts']} attempts")
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    for k in range(a.steps):
        results.append(one_run())
        log(f"timed run {k} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    attempts = sum(r["attempts"] for r in results)
    accepts = sum(r["n_accepted"] for r in results)
    ms_step = 1e3 * dt / a.steps
    t_acc, n_acc = h.kernel_times("accept")
    t_sc, n_sc = h.kernel_times("score")
    nd = h.n_d
    bytes_accept = 3.0 * nd * nd * 16.0          # read+write C^-1, read G (c128)
    avg_acc_ms = t_acc / max(n_acc, 1)
    achieved = bytes_accept / (avg_acc_ms * 1e-3) / 1e9
    r0 = results[-1]
    out = {
        "metric": METRIC,
        "value": attempts / dt,
        "unit": "flip evals/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c128 (f64)", "data": "synthetic",
        "config": {"workload": "2D TM FDFD 256x256, 12-cell PML, 40x40 design (N_d=1600), "
                               "eps {1,11.7}, Gaussian line source -> Gaussian overlap, 5 sweeps",
                   "precision": "fp64_plain", "n_d": nd, "sweeps": r0["sweeps"]},
        "time_to_design_ms": ms_step,
        "accepts_per_run": r0["n_accepted"], "attempts_per_run": r0["attempts"],
        "f_initial": r0["f_initial"], "f_final": r0["f_final"],
        "precompute_s": t_pre,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_accept_rescore", "avg_ms": avg_acc_ms,
                     "bytes_per_launch": bytes_accept},
        "kernels": {"accept_rescore_avg_us": 1e3 * avg_acc_ms, "accept_launches": n_acc,
                    "score_avg_us": 1e3 * t_sc / max(n_sc, 1)},
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    h.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
