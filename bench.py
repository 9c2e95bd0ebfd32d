#!/usr/bin/env python3
"""Benchmark of the BCGS QR hot path on one MI355X.

A step is one complete economic QR factorization X = Q R (every block
column: projections, block updates, intra-block Cholesky QR / TSQR,
reductions) of the synthetic workload, with X already resident in HBM.

Default workload: m = 4,194,304 rows, n = 256 columns, block size s = 16,
X = U diag(logspace(0, -8, 256)) V^T (kappa = 1e8), FP64.  The headline
variant is BCGSI+P-1S; BCGSI+ and BCGSI+P-2S are timed on the same X for
the speedups.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload tall|tall-k6|sweep]
"""

import argparse
import json
import math
import os
import sys
import time

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_PEAK_TFS = 78.6           # MI355X FP64 (vector and matrix), TFLOP/s
METRIC = ("BCGSI+P-1S GB/s & %HBM peak vs BCGSI+, m=4M n=256 fp64; "
          "p99 latency")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def chunked_gram(A, B=None, chunk=1 << 16):
    """A^T B on the device as a pairwise sum of per-chunk products."""
    import torch
    B = A if B is None else B
    parts = [A[i:i + chunk].t() @ B[i:i + chunk]
             for i in range(0, A.shape[0], chunk)]
    while len(parts) > 1:
        nxt = [parts[i] + parts[i + 1] for i in range(0, len(parts) - 1, 2)]
        if len(parts) % 2:
            nxt.append(parts[-1])
        parts = nxt
    return parts[0]


def accuracy(X, Q, R, chunk=1 << 16):
    """LOO ||Q^T Q - I||_2 and ||X - QR||_2 / ||X||_2 (section 1)."""
    import torch
    n = Q.shape[1]
    G = chunked_gram(Q) - torch.eye(n, dtype=Q.dtype, device=Q.device)
    loo = torch.linalg.eigvalsh(0.5 * (G + G.t())).abs().max().item()
    parts = []
    for i in range(0, X.shape[0], chunk):
        E = X[i:i + chunk] - Q[i:i + chunk] @ R
        parts.append(E.t() @ E)
    GE = torch.stack(parts).sum(0)
    GX = chunked_gram(X)
    num = torch.linalg.eigvalsh(0.5 * (GE + GE.t())).abs().max().sqrt().item()
    den = torch.linalg.eigvalsh(0.5 * (GX + GX.t())).abs().max().sqrt().item()
    return loo, num / den


def time_variant(X, s, variant, steps, warmup, Q, R):
    import torch
    from paper_2507_21791_amd import bcgs
    m, n = X.shape
    ws = bcgs.Workspace(m, n, s, variant, "fp64", X.device)
    for _ in range(warmup):
        bcgs.qr(X, s, variant, Q=Q, R=R, ws=ws)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    bcgs.profile_start(stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        bcgs.qr(X, s, variant, Q=Q, R=R, ws=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    recs = bcgs.profile_stop(stream)
    ms = e0.elapsed_time(e1) / steps
    info = ws.info()
    return ms, recs, info


def aggregate(recs, steps):
    """Per (kind, tag) totals per step."""
    agg = {}
    for r in recs:
        key = (r["kind"], r["tag"])
        a = agg.setdefault(key, {"kind": r["kind"], "tag": r["tag"], "n": 0,
                                 "ms": 0.0, "bytes": 0.0, "flops": 0.0})
        a["n"] += 1
        a["ms"] += r["ms"]
        a["bytes"] += r["bytes"]
        a["flops"] += r["flops"]
    for a in agg.values():
        for k in ("n", "ms", "bytes", "flops"):
            a[k] /= steps
    return sorted(agg.values(), key=lambda a: -a["ms"])


def kernel_name(kind, tag):
    if kind == "pass" and tag >= 1000000000:
        # tag 1WPBSTTPPN: waves, workgroups per CU, tile buffers, both
        # partial-sum areas, tile rows, Gram pairs per wave, B blocks
        nw, pc = (tag // 100000000) % 10, (tag // 10000000) % 10
        nbuf, scr2 = (tag // 1000000) % 10, (tag // 100000) % 10
        tr, maxp, ntb = (tag // 1000) % 100, (tag // 10) % 100, tag % 10
        cap = {(64, 4): 64, (64, 8): 128, (32, 4): 128, (32, 8): 272,
               (16, 4): 272, (16, 8): 272}.get((tr, nw), 0)
        gram = "true" if ntb else "false"
        if pc == 2:
            return (f"pass16_kernel<{tr}, {nbuf}, {cap}, {maxp}, {gram}, "
                    f"{max(ntb, 1)}>")
        return (f"pass16_deep_kernel<{tr}, {nbuf}, {cap}, {nw}, "
                f"{'true' if scr2 else 'false'}, {maxp}, {gram}, "
                f"{max(ntb, 1)}>")
    if kind == "pass":
        t = "float" if tag >= 1000 else "double"
        gram, ntb, maxa = (tag // 100) % 10, (tag // 10) % 10, tag % 10
        return (f"pass_kernel<{t},{'true' if gram else 'false'},{ntb},"
                f"{maxa}>")
    return {"reduce": "gram_reduce_kernel", "epilogue": "epilogue_kernel",
            "tsqr_leaf": "tsqr_leaf_kernel<double>",
            "tsqr_node": "tsqr_node_kernel", "tsqr_down": "tsqr_down_kernel",
            "tsqr_apply": "tsqr_apply_kernel<double>",
            "other": "fill_kernel"}.get(kind, kind)


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None when the summary is missing or
    was taken from different kernel sources."""
    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", "p1s_tall_hbm_traffic.txt")
    try:
        from paper_2507_21791_amd.prof_summary import source_digest
        lines = open(path).read().splitlines()
    except OSError:
        return None
    digest = [l.split(":")[1].strip() for l in lines
              if l.startswith("# kernel sources digest:")]
    if not digest or digest[0] != source_digest(root):
        return None
    want = kernel.replace(" ", "")
    for l in lines:
        if l.startswith("#") or l.startswith("  "):
            continue
        parts = l.rsplit(None, 4)
        if len(parts) == 5 and parts[0].replace(" ", "") == want:
            return float(parts[4]) * 1e9
    return None


def by_name(agg):
    """Per-step totals of every kernel, merged by name, slowest first."""
    out = {}
    for a in agg:
        k = kernel_name(a["kind"], a["tag"])
        o = out.setdefault(k, {"name": k, "launches": 0.0, "ms": 0.0,
                               "gb": 0.0, "gflop": 0.0})
        o["launches"] += a["n"]
        o["ms"] += a["ms"]
        o["gb"] += a["bytes"] / 1e9
        o["gflop"] += a["flops"] / 1e9
    rows = sorted(out.values(), key=lambda o: -o["ms"])
    for o in rows:
        o["ms"] = round(o["ms"], 4)
        o["gb"] = round(o["gb"], 3)
        o["gflop"] = round(o["gflop"], 2)
    return rows


def roofline(dom):
    t_hbm = dom["bytes"] / (HBM_PEAK_GBS * 1e9)
    t_fp = dom["flops"] / (FP64_PEAK_TFS * 1e12)
    per_launch_ms = dom["ms"] / dom["n"]
    traffic = measured_traffic(kernel_name(dom["kind"], dom["tag"]))
    if t_fp >= t_hbm:
        achieved = dom["flops"] / dom["n"] / (per_launch_ms * 1e-3) / 1e12
        return {"bound": "mfma", "achieved": round(achieved, 3),
                "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFS, 4), "traffic": traffic,
                "kernel": kernel_name(dom["kind"], dom["tag"]),
                "launches_per_step": dom["n"],
                "avg_launch_ms": round(per_launch_ms, 4),
                "algorithmic_bytes": dom["bytes"] / dom["n"],
                "hbm_gbs": round(dom["bytes"] / dom["n"] /
                                 (per_launch_ms * 1e-3) / 1e9, 1)}
    achieved = dom["bytes"] / dom["n"] / (per_launch_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": kernel_name(dom["kind"], dom["tag"]),
            "launches_per_step": dom["n"],
            "avg_launch_ms": round(per_launch_ms, 4)}


def cpu_baseline(Xd, s, rows, model_bytes_full, m_full):
    """The oracle (as it stands) on the first `rows` rows of the same X."""
    import numpy as np
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()
                       if p.get("internal_api") in ("openblas", "mkl",
                                                    "blis")] or [1])
    except Exception:
        threads = os.cpu_count()
    Xs = np.asfortranarray(Xd[:rows].cpu().numpy())
    t0 = time.perf_counter()
    r = oracle.qr(Xs, s, "p-1s")
    dt = time.perf_counter() - t0
    bytes_sample = model_bytes_full * rows / m_full
    return {"value": round(bytes_sample / dt / 1e9, 3), "unit": "GB/s",
            "cores": threads, "kind": "oracle",
            "sample": (f"BCGSI+P-1S oracle (numpy FP64) on the first {rows} "
                       f"rows of the same X ({rows}x{Xd.shape[1]}, s={s}); "
                       f"{dt:.2f} s; GB/s under the same algorithmic byte "
                       f"model scaled to the sample"),
            "seconds": round(dt, 3),
            "breakdown": None if r.breakdown is None else r.breakdown.block}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="tall")
    ap.add_argument("--m", type=int, default=None)
    ap.add_argument("--s", type=int, default=None)
    ap.add_argument("--variants", default="p-1s,bcgsi+,p-2s")
    ap.add_argument("--cpu-rows", type=int, default=1 << 20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (counter "
                         "calibration for rocprofv3 --pmc runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; "
                          "--gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_2507_21791_amd import bcgs, workloads as W
    bcgs.lib()                    # raises if the HIP library is not built
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    w = dict(W.WORKLOADS[args.workload])
    if args.m:
        w["m"] = args.m
    if args.s:
        w["s"] = args.s
    m, n, s = w["m"], w["n"], w["s"]
    log(f"[bench] generating {args.workload} X: m={m} n={n} s={s}")
    X = W.make_device(args.workload, m=m)
    torch.cuda.synchronize()
    Q = bcgs.empty_fortran(m, n, torch.float64, "cuda")
    R = bcgs.empty_fortran(n, n, torch.float64, "cuda")

    if args.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        src.fill_(1.0)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] copy calibration: 3 x 1 GiB device copies done")

    results = {}
    variants = args.variants.split(",")
    for v in variants:
        log(f"[bench] timing {v}: {args.warmup} warmup + {args.steps} steps")
        ms, recs, info = time_variant(X, s, v, args.steps, args.warmup, Q, R)
        agg = aggregate(recs, args.steps)
        model_bytes = sum(a["bytes"] for a in agg)
        model_flops = sum(a["flops"] for a in agg)
        res = {"ms": round(ms, 4), "model_gb": round(model_bytes / 1e9, 3),
               "gbs": round(model_bytes / (ms * 1e-3) / 1e9, 1),
               "tflops": round(model_flops / (ms * 1e-3) / 1e12, 2),
               "status": info.status, "syncs": info.syncs,
               "kernels": by_name(agg),
               "_agg": agg}
        if not args.no_check:
            loo, resid = accuracy(X, Q, R)
            res["loo"] = loo
            res["residual"] = resid
        log(f"[bench] {v}: {ms:.3f} ms  {res['gbs']} GB/s  "
            f"{res['tflops']} TF/s  status={info.status} "
            f"loo={res.get('loo')}")
        results[v] = res

    head = results[variants[0]]
    dom = head["_agg"][0]
    out = {
        "metric": METRIC,
        "value": head["gbs"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": (f"{args.workload}: m={m} n={n} s={s} "
                                f"kappa=1e{w['decades']} FP64, variant "
                                f"{variants[0]}"),
                   "m": m, "n": n, "s": s, "variant": variants[0]},
        "hbm_frac": round(head["gbs"] / HBM_PEAK_GBS, 4),
        "roofline": roofline(dom),
    }
    if "bcgsi+" in results and variants[0] != "bcgsi+":
        out["speedup_vs_bcgsi+"] = round(results["bcgsi+"]["ms"] / head["ms"], 3)
    if "p-2s" in results and "bcgsi+" in results:
        out["speedup_p2s_vs_bcgsi+"] = round(
            results["bcgsi+"]["ms"] / results["p-2s"]["ms"], 3)
    out["variants"] = {k: {kk: vv for kk, vv in r.items() if kk != "_agg"}
                       for k, r in results.items()}
    out["p99_latency_ms"] = None
    if not args.no_cpu:
        rows = min(args.cpu_rows, m)
        log(f"[bench] cpu baseline: oracle on {rows} rows")
        out["cpu_baseline"] = cpu_baseline(X, s, rows,
                                           head["model_gb"] * 1e9, m)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
