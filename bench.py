"""Benchmark of the PNGF hot path on one MI355X.

A step is one complete direct-binary-search run on the 256x256 grid /
40x40-pixel workload (N_d = 1600, eps in {1, 11.7}, Gaussian line source to a
Gaussian-overlap output, five sweeps): the FP64 initial inverse of the start
design, scoring of every candidate, selection, accepts and refreshes until the
sweep cap or convergence.  Every form runs on the same resident input and must
reproduce the same accepted sequence:

  * mixed (headline `value`): complex-FP32 C0^-1 with a deferred panel, FP64
    refresh every 32 accepts, FP64 decisions inside the FP32 error band;
  * plain: FP64 C^-1 with a fused Sherman-Morrison accept + rescore per step;
  * mixed_drift: as mixed, refreshing only when the FP64 residual drifts;
  * rform: FP64 reduced scoring from T0 = C^-1 G and a panel of T columns;
  * learned: the ranked exact search driven by a CNN trained here on other
    seeds (exact evaluations counted; training is not timed);
  * tiles: the same workload searched over 4x4-pixel tiles (rank-16 updates;
    its own sequence, not comparable with the pixel search);
  * broadband (a separate workload): eight frequencies over a 20% band on a
    160x160 grid with a 24x24 design, plain against mixed (refresh every 32
    accepts, or only on drift);
  * batch (a separate workload): 24 problems of the batching family
    advanced together, one launch per step, against the same problems run
    one after the other.

`value` is attempted flip evaluations per second of the mixed form over the K
timed runs and ms_per_step its time-to-design.  Inputs (G, b, G_OD, x_b) are
resident in HBM before timing starts; the host precompute is reported
separately.  Per-kernel times are HIP events recorded around every launch on
the library's stream during the timed runs (events come from a reused pool).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--no-learned] [--no-batch]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "flip evals/s + time-to-design, mixed vs FP64 plain, ≤1e-6 rel objective err"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
KERNELS = ("score", "select", "accept", "lu", "other", "fold", "mixed_q", "wood")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "mixed_persist_n1600_traffic.json")
C4_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "mixed_step_n6400_f8_traffic.json")
STEP_SOURCE = os.path.join(ROOT, "paper_2501_18054_amd", "csrc", "step_kernels.hip")


def log(msg):
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def cpu_baseline(prob):
    """Oracle (full sparse re-solve per candidate) on the host cores, on a
    bounded sample: candidate evaluations at the initial design, by a process
    pool over the available cores (at most 16)."""
    import numpy as np
    import oracle
    cores = len(os.sched_getaffinity(0))
    workers = max(1, min(cores, 16))
    n = 8 * workers
    cands = np.arange(n)
    t0 = time.perf_counter()
    oracle.score_all(prob, prob.init_bits, cands, workers=workers)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "flip evals/s", "cores": workers, "kind": "oracle",
            "sample": f"{n} candidate flips of the initial design, each a full sparse "
                      f"LU re-solve of the {prob.nx}x{prob.ny} FDFD system; {dt:.1f} s wall"}


def oracle_candidate_seconds(prob, n_cand, workers):
    """Wall seconds of the oracle per candidate flip of prob at its initial
    design (every frequency a full sparse LU re-solve), from n_cand sampled
    candidates scored by a pool of `workers` processes: the extrapolation base
    for workloads whose oracle search would take hours."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(7)
    cands = np.sort(rng.choice(prob.n_d, n_cand, replace=False))
    t0 = time.perf_counter()
    oracle.score_all(prob, prob.init_bits, cands, workers=workers)
    return (time.perf_counter() - t0) / n_cand


_POOL = {}


def _pool_init():
    """One BLAS thread per forked worker: the pool supplies the parallelism.
    The oracle (and with it scipy's own BLAS) is loaded first, so the limit
    covers every BLAS library the sparse solves use."""
    import oracle  # noqa: F401
    try:
        from threadpoolctl import threadpool_limits
        _POOL["limits"] = threadpool_limits(1)
    except ImportError:
        pass


def _one_candidate(args):
    """Oracle seconds for one candidate flip of one problem (pool task)."""
    import numpy as np
    import oracle
    prob, cand = args
    t0 = time.perf_counter()
    oracle.score_all(prob, prob.init_bits, np.array([cand]), workers=1)
    return time.perf_counter() - t0


def oracle_batch_seconds(probs, workers):
    """Oracle seconds of one candidate flip of each problem (every frequency a
    full sparse re-solve), the problems spread over a process pool."""
    import multiprocessing as mp
    with mp.get_context("fork").Pool(workers, _pool_init) as pool:
        return pool.map(_one_candidate, [(p, p.n_d // 2) for p in probs], chunksize=1)


def cpu_pform_baseline(prob, G, b, god, xb, norm, budget_s=12.0):
    """FP64 PNGF on the host cores (numpy / OpenBLAS), the class of the
    paper's own CPU implementation: C^-1 of the initial design by LAPACK, then
    direct binary search in visiting order, each attempted flip scored in
    O(N_d) from the current C^-1 (eq. lru_eobj_rs: tau_m = (C^-1 G)[m,m] from
    row m of C^-1 and of G, by reciprocity), each accept a Sherman-Morrison
    rank-1 update of C^-1 (eq. lru_woodbury) and of E and R'.  Candidates
    are scored 64 at a time in visiting order (the first improving one wins,
    the rest of its block is discarded and not counted).  Runs the first
    sweeps of the trajectory until budget_s; returns evaluations per second
    and the accepted pixels (to check against the GPU's)."""
    import numpy as np
    nd = G.shape[0]
    k2d = prob.k0[0] ** 2 * (prob.eps_hi - prob.eps_lo)
    bits = prob.init_bits.astype(np.uint8).copy()
    t0 = time.perf_counter()
    d = k2d * bits
    C = np.eye(nd, dtype=np.complex128) - G * d[None, :]
    Ci = np.linalg.inv(C)
    E = Ci @ b
    R = god + k2d * (Ci @ (G @ (bits * god)))
    x = xb + np.sum(god * d * E)
    f = abs(x) ** 2 / norm
    t_inv = time.perf_counter() - t0
    acc, evals = [], 0
    t1 = time.perf_counter()
    eta = 1e-9
    for s in range(prob.perms.shape[0]):
        pos = 0
        while pos < nd and time.perf_counter() - t1 < budget_s:
            blk = prob.perms[s, pos:pos + 64]
            delta = np.where(bits[blk] != 0, -1.0, 1.0) * k2d
            tau = np.einsum("ij,ij->i", Ci[blk], G[blk])
            dx = delta * E[blk] * R[blk] / (1.0 - delta * tau)
            fn = np.abs(x + dx) ** 2 / norm
            ok = np.flatnonzero(fn - f > eta * f)
            if ok.size == 0:
                evals += blk.size
                pos += blk.size
                continue
            j = int(ok[0])
            evals += j + 1
            m = int(blk[j])
            a = delta[j] / (1.0 - delta[j] * tau[j])
            p = Ci @ G[m]
            q = Ci[m].copy()
            Ci += a * np.outer(p, q)
            Em, Rm = E[m], R[m]
            E += a * Em * p
            R += a * Rm * p
            x += a * Em * Rm
            f = abs(x) ** 2 / norm
            bits[m] ^= 1
            acc.append(m)
            pos += j + 1
        if time.perf_counter() - t1 >= budget_s:
            break
    dt = time.perf_counter() - t1
    return {"value": evals / dt, "unit": "flip evals/s", "evals": evals, "accepts": len(acc),
            "seconds": dt, "initial_inverse_s": t_inv}, acc


def run_form(h, prob, opts, steps, warmup, name):
    import torch
    h.bind(opts)

    def one_run():
        h.set_design(prob.init_bits)
        return h.dbs_run(prob.perms)

    for w in range(warmup):
        r = one_run()
        log(f"{name}: warmup {w}: {r['n_accepted']} accepts, {r['attempts']} attempts, "
            f"{r['n_refresh']} refreshes")
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    for k in range(steps):
        results.append(one_run())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log(f"{name}: {steps} timed runs in {dt:.3f} s")
    kt = {k: h.kernel_times(k) for k in KERNELS}   # the last timed run
    return results, dt, kt


def summarize(results, dt, steps):
    attempts = sum(r["attempts"] for r in results)
    r0 = results[-1]
    return {"flip_evals_per_s": attempts / dt, "time_to_design_ms": 1e3 * dt / steps,
            "accepts": r0["n_accepted"], "attempts": r0["attempts"], "sweeps": r0["sweeps"],
            "refreshes": r0["n_refresh"], "band_decisions": r0["n_verified"],
            "f_final": r0["f_final"], "f_initial": r0["f_initial"]}


def kernel_table(kt, nd, ns, form, accepts):
    """Average launch time (us) and the algorithmic rate of each kernel class.

    Algorithmic work per launch (N_d pixels, n_S pixels at eps_hi):
      accept  plain 3 N_d^2 16 B (read + write C^-1, read G); mixed N_d^2 8 B
              (C0^-1 stream); rform (k_avg + 8) N_d 16 B (T0 row, panel,
              vectors), k_avg = accepts / 2
      score   2 N_d^2 16 B
      lu      rform: the T0 build, 8 N_d^2 n_S flop; otherwise the inversion,
              8 n_S^2 N_d flop (K^-1 and the Z rows)
      wood    2 x 8 N_d^2 k flop with k = 32 changed pixels
    """
    out = {}
    for k, (tms, n) in kt.items():
        if n == 0:
            continue
        e = {"launches": n, "total_ms": tms, "avg_us": 1e3 * tms / n}
        b = fl = None
        if k == "accept":
            b = {"plain": 3 * nd * nd * 16.0, "mixed": nd * nd * 8.0,
                 "rform": (accepts / 2 + 8) * nd * 16.0}[form]
        elif k == "score":
            b = 2 * nd * nd * 16.0
        elif k == "lu":
            fl = 8.0 * nd * nd * ns if form == "rform" else 8.0 * ns * ns * nd
        elif k == "wood":
            fl = 2 * 8.0 * nd * nd * 32
        if b is not None:
            e["bytes_per_launch"] = b
            e["GB_s"] = b / (tms / n * 1e-3) / 1e9
        if fl is not None:
            e["flop_per_launch"] = fl
            e["TFLOP_s"] = fl / (tms / n * 1e-3) / 1e12
        out[k] = e
    return out


# the mixed step kernel the headline workload runs (one frequency, N_d <= 2048:
# a batch of steps per launch, rows of C0^-1 resident in registers); its unit
# of work is one accepted flip
HEAD_STEP_KERNEL = "k_mixed_persist"


def traffic_for(kernel_name, path=None):
    """Counter-measured HBM bytes per unit of work of a step kernel from the
    committed rocprofv3 summary, or None if it was taken from another version
    of the kernel source."""
    path = path or TRAFFIC_FILE
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    with open(STEP_SOURCE, "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()
    if t.get("source_sha256") != digest or t.get("kernel") != kernel_name:
        return None
    return t["fetch_bytes"] + t["write_bytes"]


def tile_form(P, h, steps, warmup):
    """The same workload searched over 100 tiles of 4x4 pixels (M = 16, rank-16
    Woodbury scores and accepts, FP64 P-form), on the handle's resident
    inputs.  A step is one complete tile search from the start design."""
    import torch
    import workloads
    pt = workloads.tiles1()
    m = pt.tiles.shape[1]
    h.bind(P.default_options(max_accepts=8192, max_sweeps=8, max_tile=m, timing=True))

    def one_run():
        h.set_design(pt.init_bits)
        return h.tile_dbs_run(pt.tiles, pt.tile_perms)

    for _ in range(warmup):
        one_run()
    torch.cuda.synchronize()
    res = []
    t0 = time.perf_counter()
    for _ in range(steps):
        res.append(one_run())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    r = res[-1]
    nd = h.n_d
    out = {"tiles": int(pt.tiles.shape[0]), "M": int(m),
           "tile_evals_per_s": sum(x["attempts"] for x in res) / dt,
           "time_to_design_ms": 1e3 * dt / steps, "accepts": r["n_accepted"],
           "attempts": r["attempts"], "converged": r["converged"], "f_final": r["f_final"]}
    tms, n = h.kernel_times("tile")
    if n:
        # one scoring pass reads every tile's rows of C^-1 and G: 2 N_d^2 16 B
        out["tile_score_avg_us"] = 1e3 * tms / n
        out["tile_score_GB_s"] = 2 * nd * nd * 16.0 / (tms / n * 1e-3) / 1e9
    wms, wn = h.kernel_times("wood")
    if wn:
        out["woodbury_accept_avg_us"] = 1e3 * wms / wn
    log(f"tiles: {out['accepts']} accepts, {out['attempts']} attempts, "
        f"{out['time_to_design_ms']:.1f} ms per design")
    return out


def broadband_form(P, steps, warmup):
    """Workload 4's eight-frequency setting at reduced size (160x160 grid,
    24x24 design): plain FP64 and mixed forms from the same start design; one
    launch per step covers all eight frequencies."""
    import workloads
    pb = workloads.config4_scaled()
    t0 = time.perf_counter()
    hb = P.Handle(pb)
    t_pre = time.perf_counter() - t0
    hb.bind(P.default_options())
    hb.set_design(pb.init_bits)
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        hb.set_design(pb.init_bits)
    torch.cuda.synchronize()
    t_inv = (time.perf_counter() - t0) / 3
    out = {"n_d": hb.n_d, "frequencies": pb.nfreq, "precompute_s": t_pre,
           "set_design_ms": 1e3 * t_inv}
    seqs = {}
    for name, kw in (("plain", {}), ("mixed", dict(precision=P.PNGF_MIXED, k_refresh=32)),
                     ("mixed_drift", dict(precision=P.PNGF_MIXED, k_refresh=0))):
        opts = P.default_options(max_accepts=8192, max_sweeps=8, timing=True, **kw)
        res, dt, kt = run_form(hb, pb, opts, steps, warmup, "broadband " + name)
        s = summarize(res, dt, steps)
        out[name] = {k: s[k] for k in ("flip_evals_per_s", "time_to_design_ms", "accepts",
                                       "attempts", "f_final", "refreshes")}
        # per-kernel times of the last run; bytes are those of one frequency
        out[name]["kernels"] = {k: {"launches": n, "total_ms": tms, "avg_us": 1e3 * tms / n}
                                for k, (tms, n) in kt.items() if n}
        seqs[name] = res[-1]["accepted"]
    out["same_sequence"] = bool(seqs["plain"].tolist() == seqs["mixed"].tolist() ==
                                seqs["mixed_drift"].tolist())
    out["objective_rel_err"] = abs(out["mixed"]["f_final"] - out["plain"]["f_final"]) / \
        out["plain"]["f_final"]
    hb.close()
    return out


# the mixed step kernel of the eight-frequency N_d = 6400 workload (one launch
# per step; every launch streams the complex-FP32 C0^-1 of all frequencies)
C4_STEP_KERNEL = "k_mixed_step"
C4_WORKLOAD = ("2D TM FDFD 640x640, 16-cell PML, h = lambda0/25, 80x80 design (N_d=6400), "
               "eps {1,11.7}, 8 frequencies over 0.9-1.1 f0, Gaussian line source -> "
               "vacuum-normalized mean Gaussian-mode transmission, to convergence (<= 20 sweeps)")


def config4_learned(P, hb, p, c4, train_seeds=(41, 42)):
    """The combined form on workload 4: the mixed form (complex-FP32 steps,
    FP64 decisions in the error band, FP64 refresh every 32 accepts), all
    eight frequencies in every launch, driven by the learned proposal (the
    first improving pixel of the network's ranking of each state, ranked on
    the device).  The network is trained first (not timed) on pairs logged
    from two other seeds of the same workload.  Every accept is an exact
    improvement; the objective of the design it reaches is re-evaluated from
    a fresh FP64 inverse."""
    import numpy as np
    import torch
    import workloads
    from paper_2501_18054_amd import learned
    t0 = time.perf_counter()
    X, T = [], []
    for s in train_seeds:
        q = workloads.config4(seed=s)
        hq = P.Handle(q).bind(P.default_options(max_accepts=16384, max_sweeps=20))
        x, t = learned.collect(hq, q, every=4, greedy=True)
        X += x
        T += t
        hq.close()
    model = P.Model(80, 80, max_batch=8, seed=0)
    hist = learned.train(model, X, T, epochs=20, batch=8, lr=1e-3)
    t_train = time.perf_counter() - t0
    log(f"config4 learned: trained on {len(X)} states in {t_train:.1f} s "
        f"(loss {hist[0]:.3f} -> {hist[-1]:.3f})")
    out = {"train_s": t_train, "train_seeds": list(train_seeds)}
    hb.bind(P.default_options(precision=P.PNGF_MIXED, k_refresh=32, max_accepts=16384,
                              max_sweeps=20))
    hb.set_design(p.init_bits)
    hb.learned_dbs_run(model, k=1, max_accepts=16384)
    res = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 2
    for _ in range(reps):
        hb.set_design(p.init_bits)
        res.append(hb.learned_dbs_run(model, k=1, max_accepts=16384))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    r = res[-1]
    bits = p.init_bits.copy()
    for m in r["accepted"]:
        bits[m] ^= 1
    hb.bind(P.default_options(max_accepts=64, max_sweeps=1))
    hb.set_design(bits)
    f64, _ = hb.evaluate()
    hb.bind(P.default_options(precision=P.PNGF_MIXED, k_refresh=32, max_accepts=16384,
                              max_sweeps=20))
    hb.set_design(p.init_bits)
    t1 = time.perf_counter()
    r1 = hb.learned_dbs_run(None, k=1, max_accepts=16384)
    torch.cuda.synchronize()
    t_fo = time.perf_counter() - t1
    model.close()
    fp = c4["plain"]["f_final"]
    out.update({"time_to_design_ms": 1e3 * dt, "exact_evals": r["attempts"],
                "exact_evals_per_s": r["attempts"] / dt, "accepts": r["n_accepted"],
                "converged": r["converged"], "f_final": r["f_final"],
                "objective_rel_err_vs_fp64_eval": abs(r["f_final"] - f64) / f64,
                "objective_rel_to_plain_dbs": r["f_final"] / fp,
                "exact_evals_rel_to_plain_dbs": r["attempts"] / c4["plain"]["attempts"],
                "speedup_vs_plain_dbs": c4["plain"]["time_to_design_ms"] / (1e3 * dt),
                "timed_runs": reps,
                "first_order_ranking": {"time_to_design_ms": 1e3 * t_fo,
                                        "exact_evals": r1["attempts"], "accepts": r1["n_accepted"],
                                        "f_final": r1["f_final"]}})
    log(f"config4 learned mixed: {r['n_accepted']} accepts, {r['attempts']} exact evals, "
        f"f {r['f_final']:.6g} ({out['objective_rel_to_plain_dbs']:.4f} of plain DBS), "
        f"{1e3 * dt:.0f} ms per design")
    return out


def config4_form(P, learned=True):
    """Workload 4 at full size: 640x640 grid, 80x80 design (N_d = 6400),
    eight frequencies, vacuum-normalized mean transmission.  Each form runs
    the search from the same start design until a whole sweep keeps nothing
    or 20 sweeps; plain FP64 once, the mixed form (FP64 refresh every 32
    accepts) and the R-form twice; then one mixed run with events around
    every kernel class for the roofline of its step kernel."""
    import torch
    import workloads
    p = workloads.config4()
    t0 = time.perf_counter()
    hb = P.Handle(p)
    out = {"n_d": hb.n_d, "frequencies": p.nfreq, "precompute_s": hb.precompute_seconds(),
           "precompute_wall_s": time.perf_counter() - t0}
    seqs = {}
    for name, kw, reps in (("mixed", dict(precision=P.PNGF_MIXED, k_refresh=32), 2),
                           ("mixed_drift", dict(precision=P.PNGF_MIXED, k_refresh=0), 2),
                           ("rform", dict(precision=P.PNGF_RFORM), 2),
                           ("plain", {}, 1)):
        opts = P.default_options(max_accepts=16384, max_sweeps=20, timing_steps=True, **kw)
        hb.bind(opts)
        hb.set_design(p.init_bits)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hb.set_design(p.init_bits)
        torch.cuda.synchronize()
        t_inv = time.perf_counter() - t0
        res = []
        t0 = time.perf_counter()
        for _ in range(reps):
            hb.set_design(p.init_bits)
            res.append(hb.dbs_run(p.perms))
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        r = res[-1]
        out[name] = {"time_to_design_ms": 1e3 * dt, "flip_evals_per_s": r["attempts"] / dt,
                     "accepts": r["n_accepted"], "attempts": r["attempts"],
                     "sweeps": r["sweeps"], "converged": r["converged"],
                     "refreshes": r["n_refresh"], "band_decisions": r["n_verified"],
                     "f_initial": r["f_initial"], "f_final": r["f_final"],
                     "initial_inverse_ms": 1e3 * t_inv, "timed_runs": reps}
        seqs[name] = r["accepted"]
        log(f"config4 {name}: {r['n_accepted']} accepts, {r['attempts']} attempts, "
            f"{r['sweeps']} sweeps, {1e3 * dt:.0f} ms per design")
    out["same_sequence"] = bool(seqs["plain"].tolist() == seqs["mixed"].tolist() ==
                                seqs["mixed_drift"].tolist() == seqs["rform"].tolist())
    fp = out["plain"]["f_final"]
    out["objective_rel_err_mixed_drift_vs_plain"] = abs(out["mixed_drift"]["f_final"] - fp) / fp
    out["objective_rel_err_mixed_vs_plain"] = abs(out["mixed"]["f_final"] - fp) / fp
    out["objective_rel_err_rform_vs_plain"] = abs(out["rform"]["f_final"] - fp) / fp
    if learned:
        out["learned_mixed"] = config4_learned(P, hb, p, out)
    # per-class times of one mixed run (events on every launch)
    hb.bind(P.default_options(precision=P.PNGF_MIXED, k_refresh=32, max_accepts=16384,
                              max_sweeps=20, timing=True))
    hb.set_design(p.init_bits)
    r = hb.dbs_run(p.perms)
    nd, F = hb.n_d, p.nfreq
    kt = {k: hb.kernel_times(k) for k in KERNELS}
    ks = {k: {"launches": n, "total_ms": tms, "avg_us": 1e3 * tms / n}
          for k, (tms, n) in kt.items() if n}
    out["mixed"]["kernels"] = ks
    # the step kernel: every launch that accepts streams C0^-1 of every
    # frequency once (F N_d^2 8 B); launches are counted per accepted flip
    tms, n = kt["accept"]
    if n:
        per = tms / n * 1e-3
        achieved = F * nd * nd * 8.0 / per / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                           "traffic": traffic_for(C4_STEP_KERNEL, C4_TRAFFIC_FILE),
                           "kernel": C4_STEP_KERNEL, "avg_us": 1e6 * per,
                           "per": "accepted flip", "bytes_per_unit": F * nd * nd * 8.0}
    hb.close()
    return out


def learned_form(P, h, prob, steps, k=4):
    """Train the proposal network on other seeds of the same family (not
    timed), then time the ranked exact search on this workload."""
    import torch
    import workloads
    from paper_2501_18054_amd import learned
    t0 = time.perf_counter()
    X, T = [], []
    for s in workloads.CONFIG3_TRAIN_SEEDS[:6]:
        p = workloads.config3_problem(s)
        hh = P.Handle(p).bind(P.default_options(max_accepts=8192, max_sweeps=8))
        x, t = learned.collect(hh, p, every=4, greedy=True)
        X += x
        T += t
        hh.close()
    side = prob.design_side
    model = P.Model(side, side, max_batch=32, seed=0)
    hist = learned.train(model, X, T, epochs=40, batch=32, lr=1e-3)
    t_train = time.perf_counter() - t0
    log(f"learned: trained on {len(X)} states in {t_train:.1f} s (loss {hist[0]:.3f} -> "
        f"{hist[-1]:.3f})")
    h.bind(P.default_options(max_accepts=8192, max_sweeps=8))
    h.set_design(prob.init_bits)
    h.learned_dbs_run(model, k=k)
    torch.cuda.synchronize()
    res = []
    t0 = time.perf_counter()
    for _ in range(steps):
        h.set_design(prob.init_bits)
        res.append(h.learned_dbs_run(model, k=k))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    r = res[-1]
    model.close()
    return {"exact_evals_per_s": sum(x["attempts"] for x in res) / dt,
            "time_to_design_ms": 1e3 * dt / steps, "exact_evals": r["attempts"],
            "accepts": r["n_accepted"], "converged": r["converged"], "k": k,
            "f_final": r["f_final"], "train_s": t_train, "train_states": len(X)}


def batch_form(P, steps, probs):
    """The batching workload (48 problems, uneven N_d 256-3136, 1-4
    frequencies, mixed form): one launch per step over all of them (hipGraph
    replays, autotuned launch shape) against the same problems run one after
    the other.  Both include each problem's FP64 initial inverse."""
    import torch
    stream = torch.cuda.Stream()
    opts = P.default_options(precision=P.PNGF_MIXED, k_refresh=32, max_accepts=8192,
                             max_sweeps=20)
    hs = [P.Handle(p).bind(opts, stream=stream) for p in probs]

    def solo():
        return [(h.set_design(p.init_bits), h.dbs_run(p.perms))[1] for h, p in zip(hs, probs)]

    b = P.Batch(hs)

    def batched(tune=False):
        for h, p in zip(hs, probs):
            h.set_design(p.init_bits)
        return b.dbs_run([p.perms for p in probs], autotune=tune)

    solo()
    batched(tune=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        rs = solo()
    torch.cuda.synchronize()
    t_solo = (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    for _ in range(steps):
        rb = batched()
    torch.cuda.synchronize()
    t_b = (time.perf_counter() - t0) / steps
    att = sum(r["attempts"] for r in rb)
    same = all(x["accepted"].tolist() == y["accepted"].tolist() for x, y in zip(rb, rs))
    out = {"problems": len(probs), "n_d": [h.n_d for h in hs],
           "attempts_per_problem": [int(r["attempts"]) for r in rb],
           "frequencies": [p.nfreq for p in probs], "attempts": att,
           "batched_ms": 1e3 * t_b, "solo_ms": 1e3 * t_solo,
           "batched_flip_evals_per_s": att / t_b, "solo_flip_evals_per_s": att / t_solo,
           "ms_per_batched_step": b.ms_per_step(), "tuning": b.tuning(),
           "same_sequences_as_solo": same}
    b.close()
    for h in hs:
        h.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-config4", action="store_true")
    ap.add_argument("--config4-only", action="store_true",
                    help="run only the 640x640 / N_d 6400 / 8-frequency leg (for profiling)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py: measures one GPU only (the hot path runs on one MI355X); "
              "multi-GPU runs are not supported", file=sys.stderr)
        sys.exit(2)

    if a.config4_only:
        import torch  # noqa: F401
        import paper_2501_18054_amd as P
        c4 = config4_form(P, learned=not a.no_learned)
        m = c4["mixed"]
        print(json.dumps({
            "metric": METRIC, "value": m["flip_evals_per_s"], "unit": "flip evals/s",
            "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": m["time_to_design_ms"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "c64 + f64", "data": "synthetic",
            "config": {"workload": C4_WORKLOAD, "n_d": c4["n_d"]},
            "roofline": c4.get("roofline"), "forms": {"config4": c4}}))
        return

    import workloads
    prob = workloads.config1()
    probs2 = [workloads.config2_problem(s) for s in range(1000, 1048)]
    cpu = None
    extra_cpu = {}
    workers = max(1, min(len(os.sched_getaffinity(0)), 16))
    if not a.no_cpu_baseline:
        # before any GPU initialization: the oracle's process pools fork
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(prob)
        log(f"cpu baseline: {cpu['value']:.3f} flip evals/s on {cpu['cores']} cores")
        if not a.no_config4:
            log("oracle per-candidate time, workload 4 ...")
            c4 = workloads.config4()
            extra_cpu["oracle_config4_candidate_s"] = oracle_candidate_seconds(c4, workers,
                                                                               workers)
        log("oracle per-candidate time, batching workload ...")
        extra_cpu["oracle_config2_candidate_s"] = oracle_batch_seconds(probs2, workers)

    import torch  # noqa: F401
    import paper_2501_18054_amd as P
    log("precompute (host) ...")
    t0 = time.perf_counter()
    h = P.Handle(prob)
    t_pre = time.perf_counter() - t0
    log(f"precompute done in {t_pre:.2f} s")
    if not a.no_cpu_baseline:
        log("cpu baseline (FP64 P-form PNGF, numpy) ...")
        G, b, god, xb = h.get_precompute(0)
        pf, pf_acc = cpu_pform_baseline(prob, G, b, god, xb, h.objective_norm(0))
        del G
        try:
            import threadpoolctl
            pf["cores"] = max(i["num_threads"] for i in threadpoolctl.threadpool_info())
        except Exception:
            pf["cores"] = len(os.sched_getaffinity(0))
        pf["kind"] = "cpu-pngf"
        pf["sample"] = (f"FP64 P-form PNGF (numpy/OpenBLAS) on the 256x256 workload: the "
                        f"first {pf['evals']} attempted flips ({pf['accepts']} accepts) of "
                        f"the search in {pf['seconds']:.1f} s, after a {pf['initial_inverse_s']:.2f} s "
                        f"LAPACK initial inverse")
        extra_cpu["pform_config1"] = pf
        extra_cpu["_pform_accepted"] = pf_acc
        log(f"cpu P-form: {pf['value']:.0f} flip evals/s on {pf['cores']} threads")
    nd = h.n_d
    ns = int(prob.init_bits.sum())
    forms = {}
    seqs = {}
    for name, kw in (("plain", {}),
                     ("mixed", dict(precision=P.PNGF_MIXED, k_refresh=32)),
                     ("mixed_drift", dict(precision=P.PNGF_MIXED, k_refresh=0)),
                     ("rform", dict(precision=P.PNGF_RFORM))):
        # timed runs: HIP events around the step launches only (the value and
        # the roofline); then one run with events around every kernel class
        # for the per-class table (its events cost time on every launch)
        opts = P.default_options(max_accepts=8192, max_sweeps=8, timing_steps=True, **kw)
        res, dt, kt = run_form(h, prob, opts, a.steps, a.warmup, name)
        opts_d = P.default_options(max_accepts=8192, max_sweeps=8, timing=True, **kw)
        _, _, kt_d = run_form(h, prob, opts_d, 1, 0, name + " (events on every class)")
        kt_d["accept"] = kt["accept"]
        s = summarize(res, dt, a.steps)
        form = "mixed" if name.startswith("mixed") else name
        s["kernels"] = kernel_table(kt_d, nd, ns, form, s["accepts"])
        seqs[name] = res[-1]["accepted"]
        forms[name] = s
    forms["tiles"] = tile_form(P, h, a.steps, a.warmup)
    forms["broadband"] = broadband_form(P, a.steps, a.warmup)
    if not a.no_config4:
        log("workload 4 (640x640, N_d 6400, 8 frequencies) ...")
        forms["config4"] = config4_form(P, learned=not a.no_learned)
    ref = forms["plain"]
    for name in ("mixed", "mixed_drift", "rform"):
        f = forms[name]
        f["same_sequence_as_plain"] = bool(len(seqs[name]) == len(seqs["plain"]) and
                                           (seqs[name] == seqs["plain"]).all())
        f["objective_rel_err_vs_plain"] = abs(f["f_final"] - ref["f_final"]) / ref["f_final"]
    if not a.no_batch:
        log("batch ...")
        forms["batch"] = batch_form(P, 1, probs2)
        log(f"batch: {forms['batch']['batched_ms']:.1f} ms batched vs "
            f"{forms['batch']['solo_ms']:.1f} ms one after the other")
    if not a.no_learned:
        forms["learned"] = learned_form(P, h, prob, a.steps)
        forms["learned"]["objective_rel_to_plain"] = forms["learned"]["f_final"] / ref["f_final"]
    head = forms["mixed"]
    ks = head["kernels"]
    dom = max(ks, key=lambda k: ks[k]["total_ms"])
    if "GB_s" in ks[dom]:
        roof = {"bound": "hbm", "achieved": ks[dom]["GB_s"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ks[dom]["GB_s"] / HBM_PEAK_GBS,
                "traffic": traffic_for(HEAD_STEP_KERNEL) if dom == "accept" else None}
    else:
        roof = {"bound": "mfma", "achieved": ks[dom].get("TFLOP_s"), "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": (ks[dom].get("TFLOP_s") or 0.0) / FP64_PEAK_TFLOPS,
                "traffic": None}
    roof.update({"kernel": {"accept": HEAD_STEP_KERNEL}.get(dom, dom),
                 "avg_us": ks[dom]["avg_us"]})
    if dom == "accept":
        # one launch runs a batch of steps: achieved, traffic and avg_us are
        # per accepted flip (the launch's share)
        roof["per"] = "accepted flip"
    out = {
        "metric": METRIC,
        "value": head["flip_evals_per_s"],
        "unit": "flip evals/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": head["time_to_design_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 + f64", "data": "synthetic",
        "config": {"workload": "2D TM FDFD 256x256, 12-cell PML, 40x40 design (N_d=1600), "
                               "eps {1,11.7}, Gaussian line source -> Gaussian overlap, "
                               "5 sweeps; mixed form: FP64 refresh every 32 accepts",
                   "n_d": nd},
        "objective_rel_err_vs_plain": head["objective_rel_err_vs_plain"],
        "precompute_s": t_pre,
        "roofline": roof,
        "forms": forms,
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
        more = {}
        if "pform_config1" in extra_cpu:
            pf = dict(extra_cpu["pform_config1"])
            acc = extra_cpu["_pform_accepted"]
            gpu_acc = seqs["plain"].tolist()
            pf["same_accepts_as_gpu"] = bool(acc == gpu_acc[:len(acc)])
            more["pform_config1"] = pf
        if "oracle_config4_candidate_s" in extra_cpu and "config4" in forms:
            tc = extra_cpu["oracle_config4_candidate_s"]
            c4 = forms["config4"]
            more["oracle_config4_extrapolated"] = {
                "kind": "oracle", "cores": workers, "candidate_s": tc,
                "sample": f"{workers} candidate flips of workload 4's initial design in a "
                          f"pool of {workers} processes, each eight sparse LU re-solves of "
                          f"the 409,600-node system; extrapolated to the searches' attempts",
                "plain_search_s": tc * c4["plain"]["attempts"],
                "flip_evals_per_s": 1.0 / tc}
        if "oracle_config2_candidate_s" in extra_cpu and "batch" in forms:
            ts = extra_cpu["oracle_config2_candidate_s"]
            bt = forms["batch"]
            att = bt["attempts_per_problem"]
            more["oracle_config2_extrapolated"] = {
                "kind": "oracle", "cores": workers,
                "sample": "one candidate flip of each of the 48 problems (all its "
                          "frequencies re-solved), the problems over a process pool; "
                          "extrapolated to each problem's attempts in the batched run",
                "search_s": float(sum(t * n for t, n in zip(ts, att))),
                "serial_candidate_s_total": float(sum(ts))}
        out["cpu_baselines"] = more
    h.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
