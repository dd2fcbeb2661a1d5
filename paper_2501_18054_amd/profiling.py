"""Counter-measured memory traffic of a kernel, for the roofline report.

Two rocprofv3 counter runs of the benchmark (FETCH_SIZE, then WRITE_SIZE,
in KiB per dispatch) give the bytes a kernel moves between L2 and the memory
fabric.  Each counter is scaled by what it reads for a plain device-to-device
copy of known size (``copy``), and the result is written to profiles/ as a
short summary plus a JSON record that bench.py uses while the kernel source
is unchanged.

    rocprofv3 --pmc FETCH_SIZE -d OUT/cf -o run -- python -m paper_2501_18054_amd.profiling copy
    rocprofv3 --pmc WRITE_SIZE -d OUT/cw -o run -- python -m paper_2501_18054_amd.profiling copy
    rocprofv3 --pmc FETCH_SIZE -d OUT/bf -o run -- python bench.py ...
    rocprofv3 --pmc WRITE_SIZE -d OUT/bw -o run -- python bench.py ...
    python -m paper_2501_18054_amd.profiling summarize --dir OUT --kernel k_mixed_step ...

Matrix-core utilization of the MFMA kernels from one counter pass
(SQ_INSTS_VALU_MFMA_MOPS_F64/F32/BF16, SQ_INSTS_VALU_FMA_F64,
SQ_VALU_MFMA_BUSY_CYCLES, GRBM_GUI_ACTIVE):

    python -m paper_2501_18054_amd.profiling mfma --dir OUT/c1 --workload ... --out ...

The initial FP64 inverse of a workload alone, for its kernel times and
counters (``inverse``).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics

COPY_BYTES = 256 << 20
COPY_REPS = 5
HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def copy():
    import torch
    x = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(COPY_REPS):
        y.copy_(x)
    torch.cuda.synchronize()
    print(f"copied {COPY_REPS} x {COPY_BYTES} bytes", flush=True)


def _counter_rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    rows = []
    for f in files:
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def _per_dispatch(rows, counter, name_part):
    """Counter value (summed over its instances) per dispatch of kernels whose
    name contains name_part."""
    acc = {}
    for r in rows:
        if r.get("Counter_Name") != counter or name_part not in r.get("Kernel_Name", ""):
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        acc[key] = acc.get(key, 0.0) + float(r["Counter_Value"])
    return list(acc.values())


def summarize(a):
    cf = _per_dispatch(_counter_rows(os.path.join(a.dir, "cf")), "FETCH_SIZE", a.copy_kernel)
    cw = _per_dispatch(_counter_rows(os.path.join(a.dir, "cw")), "WRITE_SIZE", a.copy_kernel)
    bf = _per_dispatch(_counter_rows(os.path.join(a.dir, "bf")), "FETCH_SIZE", a.kernel)
    bw = _per_dispatch(_counter_rows(os.path.join(a.dir, "bw")), "WRITE_SIZE", a.kernel)
    kib = COPY_BYTES / 1024.0
    f_fetch = kib / statistics.median(cf)
    f_write = kib / statistics.median(cw)
    if a.units:
        # a launch covers a variable number of units (a batch of steps): the
        # run's total over its number of units
        bf_w = bf
        fetch = sum(bf) * 1024.0 * f_fetch / a.units
        write = sum(bw) * 1024.0 * f_write / a.units
    else:
        # launches that did work (the others found the search paused or finished)
        thr = 0.05 * max(bf)
        bf_w = [v for v in bf if v > thr]
        fetch = statistics.mean(bf_w) * 1024.0 * f_fetch
        write = statistics.median(bw) * 1024.0 * f_write
    per = a.unit_name if a.units else "launch"
    with open(a.source, "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()
    rec = {"kernel": a.kernel, "workload": a.workload, "per": per, "units": a.units or None,
           "fetch_bytes_per_launch": fetch if not a.units else None,
           "write_bytes_per_launch": write if not a.units else None,
           "fetch_bytes": fetch, "write_bytes": write, "algorithmic_bytes": a.alg_bytes,
           "algorithmic_bytes_per_launch": a.alg_bytes,
           "copy_scale_fetch": f_fetch, "copy_scale_write": f_write,
           "dispatches_fetch": len(bf_w), "dispatches_write": len(bw),
           "source": os.path.relpath(a.source, ROOT), "source_sha256": digest}
    base = os.path.join(ROOT, "profiles", a.out)
    with open(base + ".json", "w") as fh:
        json.dump(rec, fh, indent=1)
    with open(base + ".md", "w") as fh:
        fh.write(f"# Memory traffic of `{a.kernel}`: {a.workload}\n\n")
        fh.write("Commands (repository root, one MI355X, each counter in its own run):\n\n")
        for c in a.commands:
            fh.write(f"    {c}\n")
        fh.write("\n| quantity | value |\n|---|---|\n")
        fh.write(f"| copy calibration: FETCH_SIZE scale | {f_fetch:.4f} |\n")
        fh.write(f"| copy calibration: WRITE_SIZE scale | {f_write:.4f} |\n")
        fh.write(f"| working dispatches counted | {len(bf_w)} (fetch), {len(bw)} (write) |\n")
        if a.units:
            fh.write(f"| units ({per}) in the counted run | {a.units} |\n")
        fh.write(f"| fetched bytes per {per} | {fetch / 1e6:.3f} MB |\n")
        fh.write(f"| written bytes per {per} | {write / 1e6:.3f} MB |\n")
        fh.write(f"| algorithmic bytes per {per} | {a.alg_bytes / 1e6:.2f} MB |\n")
        fh.write(f"| traffic / algorithmic | {(fetch + write) / a.alg_bytes:.3f} |\n")
    print(json.dumps(rec, indent=1))


# dense peaks of MI355X (TFLOP/s) for the fraction columns
PEAK_TFLOPS = {"F64": 78.6, "F32": 157.3, "BF16": 2500.0}
SIMDS = 256 * 4


def _kname(n):
    n = n.replace("pngf::", "").replace("void ", "")
    i = n.find("(")
    return n[:i] if i > 0 else n


def mfma(a):
    """Per-kernel matrix-core and FP64-VALU work from one counter pass:
    SQ_INSTS_VALU_MFMA_MOPS_* count 512 FLOP each, SQ_INSTS_VALU_FMA_F64 one
    wave-wide FP64 FMA (64 lanes x 2 FLOP); SQ_VALU_MFMA_BUSY_CYCLES over
    GRBM_GUI_ACTIVE x SIMDs is the matrix cores' busy fraction while the
    kernel ran.  Durations are the dispatches' own timestamps."""
    rows = _counter_rows(a.dir)
    disp = {}
    for r in rows:
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        d = disp.setdefault(key, {"name": _kname(r["Kernel_Name"]),
                                  "ns": float(r["End_Timestamp"]) - float(r["Start_Timestamp"])})
        c = r["Counter_Name"]
        v = float(r["Counter_Value"])
        if c == "GRBM_GUI_ACTIVE":
            d[c] = max(d.get(c, 0.0), v)
        else:
            d[c] = d.get(c, 0.0) + v
    agg = {}
    for d in disp.values():
        g = agg.setdefault(d["name"], {"n": 0, "ns": 0.0, "F64": 0.0, "F32": 0.0, "BF16": 0.0,
                                       "valu64": 0.0, "busy": 0.0, "active": 0.0})
        g["n"] += 1
        g["ns"] += d["ns"]
        g["F64"] += 512.0 * d.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0)
        g["F32"] += 512.0 * d.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0)
        g["BF16"] += 512.0 * d.get("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0.0)
        g["valu64"] += 128.0 * d.get("SQ_INSTS_VALU_FMA_F64", 0.0)
        g["busy"] += d.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0)
        g["active"] += d.get("GRBM_GUI_ACTIVE", 0.0) * SIMDS
    keep = [(k, g) for k, g in agg.items()
            if g["F64"] + g["F32"] + g["BF16"] + g["valu64"] > 0.0]
    keep.sort(key=lambda kg: -kg[1]["ns"])
    out = []
    out.append(f"# Matrix-core and FP64-VALU work per kernel: {a.workload}\n\n")
    out.append("Command (repository root, one MI355X, one counter pass):\n\n")
    for c in a.commands:
        out.append(f"    {c}\n")
    out.append("\nFLOP from the counters (MFMA: 512 per SQ_INSTS_VALU_MFMA_MOPS_* count; FP64 "
               "VALU: 128 per wave-wide SQ_INSTS_VALU_FMA_F64), divided by the dispatches' "
               "own durations; peaks: FP64 78.6, FP32 157.3, BF16 2500 TFLOP/s (dense). "
               "MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE x 1024 SIMDs). "
               "Dispatches run one at a time under counter collection.\n\n")
    out.append("| kernel | launches | total ms | MFMA F64 TFLOP/s (of peak) | MFMA F32 TFLOP/s | "
               "MFMA BF16 TFLOP/s | VALU F64 TFLOP/s | MFMA busy |\n|---|---|---|---|---|---|---|---|\n")
    for k, g in keep:
        t = g["ns"] * 1e-9
        def rate(x, peak=None):
            if x <= 0.0:
                return "-"
            r = x / t / 1e12
            return f"{r:.2f} ({100.0 * r / peak:.1f}%)" if peak else f"{r:.2f}"
        busy = f"{100.0 * g['busy'] / g['active']:.1f}%" if g["active"] > 0 else "-"
        out.append(f"| `{k}` | {g['n']} | {g['ns'] / 1e6:.2f} | {rate(g['F64'], PEAK_TFLOPS['F64'])} | "
                   f"{rate(g['F32'], PEAK_TFLOPS['F32'])} | {rate(g['BF16'], PEAK_TFLOPS['BF16'])} | "
                   f"{rate(g['valu64'], PEAK_TFLOPS['F64'])} | {busy} |\n")
    f64 = sum(g["F64"] + g["valu64"] for _, g in keep)
    kns = sum(g["ns"] for _, g in keep)
    out.append(f"\nAll kernels: {f64 / 1e9:.1f} GFLOP of FP64 (matrix cores and vector ALUs) in "
               f"{kns / 1e6:.2f} ms of kernel time ({f64 / kns / 1e3:.2f} TFLOP/s).\n")
    if a.units > 0 and a.wall_ms > 0.0:
        per = f64 / a.units
        r = per / (a.wall_ms * 1e-3) / 1e12
        out.append(f"Per {a.unit_name}: {per / 1e9:.1f} GFLOP of FP64; over its wall time without "
                   f"counters, {a.wall_ms:.2f} ms, that is {r:.1f} TFLOP/s, "
                   f"{100.0 * r / PEAK_TFLOPS['F64']:.1f}% of the FP64 peak.\n")
    text = "".join(out)
    with open(os.path.join(ROOT, "profiles", a.out + ".md"), "w") as fh:
        fh.write(text)
    print(text)


def inverse(a):
    """The FP64 initial inverse of a workload, a.reps times after one warm-up
    (pngf_set_design: index lists, inversion, fields); prints one JSON line
    with the wall times and the inversion's FLOP count 8 n_S^2 N_d per
    frequency (Gauss-Jordan on the S block and C^-1[Z,S])."""
    import sys
    import time
    import torch
    sys.path.insert(0, ROOT)
    import workloads
    import paper_2501_18054_amd as P
    p = getattr(workloads, a.workload)()
    h = P.Handle(p).bind(P.default_options(pivot_search=a.pivot_search))
    h.set_design(p.init_bits)
    torch.cuda.synchronize()
    ts = []
    for _ in range(a.reps):
        t0 = time.perf_counter()
        h.set_design(p.init_bits)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    ns = int(p.init_bits.sum())
    print(json.dumps({"workload": a.workload, "n_d": int(p.n_d), "n_s": ns, "nfreq": int(p.nfreq),
                      "pivot_search": a.pivot_search, "reps": a.reps,
                      "ms_min": 1e3 * min(ts), "ms_median": 1e3 * statistics.median(ts),
                      "inversions": h.inverse_stats(),
                      "flop": 8.0 * ns * ns * p.n_d * p.nfreq}), flush=True)
    h.close()


def stats(a):
    """Kernel-time table from a rocprofv3 --kernel-trace --stats CSV run."""
    files = glob.glob(os.path.join(a.dir, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no kernel_stats.csv under {a.dir}")
    rows = []
    with open(files[0]) as fh:
        rows = list(csv.DictReader(fh))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"# Kernel-time summary: {a.workload}\n\n",
           "Command (repository root, one MI355X):\n\n"]
    for c in a.commands:
        out.append(f"    {c}\n")
    if a.note:
        out.append("\n" + a.note + "\n")
    out.append("\n| kernel | launches | total ms | avg us | share |\n|---|---|---|---|---|\n")
    for r in rows[:a.top]:
        t = float(r["TotalDurationNs"])
        n = int(float(r["Calls"]))
        out.append(f"| `{_kname(r['Name'])}` | {n} | {t / 1e6:.2f} | {t / n / 1e3:.2f} | "
                   f"{100.0 * t / tot:.1f}% |\n")
    out.append(f"\nTotal kernel time {tot / 1e9:.3f} s.\n")
    text = "".join(out)
    with open(os.path.join(ROOT, "profiles", a.out + ".md"), "w") as fh:
        fh.write(text)
    print(text)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    sub.add_parser("copy")
    st = sub.add_parser("stats")
    st.add_argument("--dir", required=True)
    st.add_argument("--workload", required=True)
    st.add_argument("--out", required=True)
    st.add_argument("--note", default="")
    st.add_argument("--top", type=int, default=30)
    st.add_argument("--commands", nargs="*", default=[])
    mf = sub.add_parser("mfma")
    mf.add_argument("--dir", required=True)
    mf.add_argument("--workload", required=True)
    mf.add_argument("--out", required=True)
    mf.add_argument("--commands", nargs="*", default=[])
    mf.add_argument("--units", type=int, default=0)
    mf.add_argument("--unit-name", default="unit")
    mf.add_argument("--wall-ms", type=float, default=0.0,
                    help="wall time of one unit without counters, for the FP64 rate")
    iv = sub.add_parser("inverse")
    iv.add_argument("--workload", required=True)
    iv.add_argument("--reps", type=int, default=3)
    iv.add_argument("--pivot-search", action="store_true")
    s = sub.add_parser("summarize")
    s.add_argument("--dir", required=True)
    s.add_argument("--kernel", required=True)
    s.add_argument("--copy-kernel", default="copy")
    s.add_argument("--workload", required=True)
    s.add_argument("--alg-bytes", type=float, required=True)
    s.add_argument("--source", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--commands", nargs="*", default=[])
    s.add_argument("--units", type=int, default=0,
                   help="divide the run's totals by this many units of work (0: per launch)")
    s.add_argument("--unit-name", default="unit")
    a = ap.parse_args()
    if a.cmd == "copy":
        copy()
    elif a.cmd == "mfma":
        mfma(a)
    elif a.cmd == "inverse":
        inverse(a)
    elif a.cmd == "stats":
        stats(a)
    else:
        summarize(a)


if __name__ == "__main__":
    main()
