#!/usr/bin/env python3
"""Benchmark of the BCGS QR hot path on one MI355X.

A step is one complete economic QR factorization X = Q R (every block
column: projections, block updates, intra-block Cholesky QR / TSQR,
reductions) of the synthetic workload, with X already resident in HBM.

Default workload: m = 4,194,304 rows, n = 256 columns, block size s = 16,
X = U diag(logspace(0, -8, 256)) V^T (kappa = 1e8), FP64.  The headline
variant is BCGSI+P-1S; BCGSI+, BCGSI+P-2S, BCGS-PIPI+ and BCGSI+1s are
timed on the same X for the speedups.  Then the batched workload (256
uneven problems in one graph launch) and the served stream (Poisson
arrivals through the request queue, p50/p99), and the oracle on a sample
of X as the CPU baseline.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload tall|tall-k6|sweep]
"""

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_PEAK_TFS = 78.6           # MI355X FP64 (vector and matrix), TFLOP/s
METRIC = ("BCGSI+P-1S GB/s & %HBM peak vs BCGSI+, m=4M n=256 fp64; "
          "p99 latency")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


_CHECKER = None


def accuracy(X, Q, R):
    """LOO ||Q^T Q - I||_2 and ||X - QR||_2 / ||X||_2 (section 1), by the
    library's device checker (Gram matrices on the GPU, the 2-norms of the
    three n x n symmetric matrices on the host)."""
    import torch
    from paper_2507_21791_amd import bcgs
    global _CHECKER
    if _CHECKER is None:
        _CHECKER = bcgs.Checker()
    prec = "fp64" if X.dtype == torch.float64 else "fp32-bulk"
    return _CHECKER(X, Q, R, prec)


def time_variant(X, s, variant, steps, warmup, Q, R, precision="fp64"):
    """Times `steps` factorizations with HIP events only between steps (no
    per-launch events), then
    the same number of steps again with the library's per-launch events on
    the launch stream, which give the per-kernel durations the roofline
    uses.  Returns (ms per step of the plain run, per-launch records of the
    profiled run, info, per-step ms of the plain run, ms per step of the
    profiled run)."""
    import torch
    from paper_2507_21791_amd import bcgs
    m, n = X.shape
    ws = bcgs.Workspace(m, n, s, variant, precision, X.device)
    for _ in range(warmup):
        bcgs.qr(X, s, variant, precision, Q=Q, R=R, ws=ws)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for k in range(steps):
        bcgs.qr(X, s, variant, precision, Q=Q, R=R, ws=ws)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[steps]) / steps
    per_step = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
    # profiled steps: per-launch HIP events on the launch stream
    bcgs.profile_start(stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for k in range(steps):
        bcgs.qr(X, s, variant, precision, Q=Q, R=R, ws=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    recs = bcgs.profile_stop(stream)
    ms_prof = e0.elapsed_time(e1) / steps
    info = ws.info()
    return ms, recs, info, per_step, ms_prof


def copy_bandwidth(nbytes=1 << 31, reps=5):
    """Measured device-to-device copy rate (bytes read + written per
    second, GB/s): the practical streaming ceiling of this GPU."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def aggregate(recs, steps):
    """Per-kernel (kind, name) totals per step.  Names come from the
    library: the kernel and its template arguments as rocprofv3 prints
    them, so they match the profile summaries."""
    agg = {}
    for r in recs:
        key = (r["kind"], r["name"])
        a = agg.setdefault(key, {"kind": r["kind"], "name": r["name"],
                                 "tag": r["tag"], "n": 0, "ms": 0.0,
                                 "bytes": 0.0, "flops": 0.0})
        a["n"] += 1
        a["ms"] += r["ms"]
        a["bytes"] += r["bytes"]
        a["flops"] += r["flops"]
    for a in agg.values():
        for k in ("n", "ms", "bytes", "flops"):
            a[k] /= steps
    return sorted(agg.values(), key=lambda a: -a["ms"])


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
    digest = [l.split(":")[1].split()[0] for l in lines
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
        k = a["name"]
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
    traffic = measured_traffic(dom["name"])
    if t_fp >= t_hbm:
        achieved = dom["flops"] / dom["n"] / (per_launch_ms * 1e-3) / 1e12
        return {"bound": "mfma", "achieved": round(achieved, 3),
                "peak": FP64_PEAK_TFS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFS, 4), "traffic": traffic,
                "kernel": dom["name"],
                "launches_per_step": dom["n"],
                "avg_launch_ms": round(per_launch_ms, 4),
                "algorithmic_bytes": dom["bytes"] / dom["n"],
                "hbm_gbs": round(dom["bytes"] / dom["n"] /
                                 (per_launch_ms * 1e-3) / 1e9, 1)}
    achieved = dom["bytes"] / dom["n"] / (per_launch_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": dom["name"],
            "launches_per_step": dom["n"],
            "avg_launch_ms": round(per_launch_ms, 4),
            "algorithmic_bytes": dom["bytes"] / dom["n"]}


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


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
            "cores": threads, "cpu_model": cpu_model(), "kind": "oracle",
            "sample": (f"BCGSI+P-1S oracle (numpy FP64) on the first {rows} "
                       f"rows of the same X ({rows}x{Xd.shape[1]}, s={s}); "
                       f"{dt:.2f} s; GB/s under the same algorithmic byte "
                       f"model scaled to the sample"),
            "seconds": round(dt, 3),
            "breakdown": None if r.breakdown is None else r.breakdown.block}


def bench_fp32_bulk(m, n, s, steps, warmup, fp64_ms):
    """P-1S in the FP32-bulk form on the tall shape with kappa = 1e3 (inside
    Table 1's u kappa^2 <= 1 with u = 2^-24), X rounded to binary32; LOO and
    residual of the result in FP64, and the time against the FP64 form."""
    import torch
    from paper_2507_21791_amd import bcgs, workloads as W
    X64 = W.conditioned_device(m, n, 3, seed=2)
    X = torch.empty((n, m), dtype=torch.float32, device="cuda").t()
    X.copy_(X64)
    del X64
    Q = bcgs.empty_fortran(m, n, torch.float32, "cuda")
    R = bcgs.empty_fortran(n, n, torch.float64, "cuda")
    ms, recs, info, _, _ = time_variant(X, s, "p-1s", steps, warmup, Q, R,
                                        "fp32-bulk")
    agg = aggregate(recs, steps)
    model_bytes = sum(a["bytes"] for a in agg)
    loo, resid = accuracy(X, Q, R)
    out = {"workload": f"m={m} n={n} s={s} kappa=1e3, P-1S, FP32-bulk",
           "ms": round(ms, 4), "model_gb": round(model_bytes / 1e9, 3),
           "gbs": round(model_bytes / (ms * 1e-3) / 1e9, 1),
           "speedup_vs_fp64": round(fp64_ms / ms, 3),
           "status": info.status, "loo": loo, "residual": resid,
           "kernels": by_name(agg)[:6]}
    log(f"[bench] fp32-bulk: {ms:.3f} ms {out['gbs']} GB/s status="
        f"{info.status} loo={loo:.3g} residual={resid:.3g}")
    del X, Q, R
    torch.cuda.empty_cache()
    return out


def bench_small():
    """The accuracy case (m = 2000, n = 80, s = 8, kappa = 1e6; seed 1):
    LOO, residual and R against the sign-normalized Householder QR of the
    same X (numpy/LAPACK on the host) for each variant, with the time of
    one factorization (latency: the problem is cache resident)."""
    import torch
    from paper_2507_21791_amd import bcgs, workloads as W
    w = W.WORKLOADS["small"]
    Xh = W.make_host("small")
    Qh, Rh = np.linalg.qr(Xh, mode="reduced")
    d = np.where(np.diag(Rh) < 0, -1.0, 1.0)
    Rh = d[:, None] * Rh
    X = bcgs.empty_fortran(w["m"], w["n"], torch.float64, "cuda")
    X.copy_(torch.from_numpy(np.asfortranarray(Xh)))
    out = {"workload": (f"small: m={w['m']} n={w['n']} s={w['s']} "
                        f"kappa=1e{w['decades']} FP64"), "variants": {}}
    for v in ("bcgsi+", "p-2s", "p-1s"):
        Q, R, ws = bcgs.qr(X, w["s"], v)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            bcgs.qr(X, w["s"], v, Q=Q, R=R, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        info = ws.info()
        loo, res = accuracy(X, Q, R)
        rerr = float(np.linalg.norm(R.cpu().numpy() - Rh) /
                     np.linalg.norm(Rh))
        out["variants"][v] = {"status": info.status, "loo": loo,
                              "residual": res, "r_vs_householder": rerr,
                              "ms": round(e0.elapsed_time(e1) / 10, 4)}
    log(f"[bench] small: {out}")
    return out


def bench_twin(steps, warmup):
    """The kappa = 1e6 twin of the tall workload (same shape and seed):
    time and accuracy of P-1S, P-2S and BCGSI+, where every variant meets
    its Table 1 assumption."""
    import torch
    from paper_2507_21791_amd import bcgs, workloads as W
    w = W.WORKLOADS["tall-k6"]
    X = W.make_device("tall-k6")
    Q = bcgs.empty_fortran(w["m"], w["n"], torch.float64, "cuda")
    R = bcgs.empty_fortran(w["n"], w["n"], torch.float64, "cuda")
    out = {"workload": (f"tall-k6: m={w['m']} n={w['n']} s={w['s']} "
                        "kappa=1e6 FP64"), "variants": {}}
    for v in ("p-1s", "p-2s", "bcgsi+"):
        ms, recs, info, _, _ = time_variant(X, w["s"], v, steps, warmup, Q,
                                            R)
        gb = sum(r["bytes"] for r in recs) / steps / 1e9
        loo, res = accuracy(X, Q, R)
        out["variants"][v] = {"ms": round(ms, 4),
                              "gbs": round(gb / (ms * 1e-3), 1),
                              "status": info.status, "loo": loo,
                              "residual": res}
    bi = out["variants"]["bcgsi+"]["ms"]
    out["speedups_vs_bcgsi+"] = {v: round(bi / r["ms"], 3)
                                 for v, r in out["variants"].items()}
    log(f"[bench] tall-k6: {out}")
    del X, Q, R
    torch.cuda.empty_cache()
    return out


def bench_sweep(steps, warmup, sizes=(4, 8, 16, 32, 64), ld_pad=16):
    """The block-size sweep (m = 2^20, n = 512, kappa about 1.05, seed 3):
    time, algorithmic GB/s and TFLOP/s of P-1S, P-2S and BCGSI+ for each
    block size s, with X and Q stored with leading dimension m + ld_pad as
    in the headline run."""
    import torch
    from paper_2507_21791_amd import bcgs, workloads as W
    w = W.WORKLOADS["sweep"]
    m, n = w["m"], w["n"]
    X0 = W.make_device("sweep")
    X = bcgs.empty_fortran(m, n, torch.float64, "cuda", ld=m + ld_pad)
    X.copy_(X0)
    del X0
    Q = bcgs.empty_fortran(m, n, torch.float64, "cuda", ld=m + ld_pad)
    R = bcgs.empty_fortran(n, n, torch.float64, "cuda")
    rows = []
    for s in sizes:
        row = {"s": s}
        for v in ("p-1s", "p-2s", "bcgsi+"):
            ms, recs, info, _, _ = time_variant(X, s, v, steps, warmup, Q, R)
            gb = sum(r["bytes"] for r in recs) / steps / 1e9
            tf = sum(r["flops"] for r in recs) / steps / 1e12
            row[v] = {"ms": round(ms, 3), "gbs": round(gb / (ms * 1e-3), 1),
                      "tflops": round(tf / (ms * 1e-3), 2),
                      "status": info.status}
        row["p-1s_vs_bcgsi+"] = round(row["bcgsi+"]["ms"] /
                                      row["p-1s"]["ms"], 3)
        log(f"[bench] sweep s={s}: {row}")
        rows.append(row)
    del X, Q, R
    torch.cuda.empty_cache()
    return {"workload": (f"sweep: m={m} n={n} kappa~1.05 FP64, leading "
                         f"dimension m + {ld_pad}, {steps} timed steps each"),
            "rows": rows}


def _time_batched(batch, reps, mode):
    """ms per launch of bcgs_qr_batched in `mode` (None: the default graph
    launch; "persistent"), after one untimed launch (capture / upload)."""
    import torch
    from paper_2507_21791_amd import bcgs
    old = os.environ.pop("BCGS_BATCH_MODE", None)
    if mode:
        os.environ["BCGS_BATCH_MODE"] = mode
    try:
        stream = torch.cuda.current_stream()
        bcgs.qr_batched(batch)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            bcgs.qr_batched(batch)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    finally:
        os.environ.pop("BCGS_BATCH_MODE", None)
        if old is not None:
            os.environ["BCGS_BATCH_MODE"] = old


def bench_batched(count, reps):
    """The batched workload (uneven problems, P-1S, FP64): autotune, then
    time `reps` rounds of one batched launch (the graph launch and the
    persistent kernel) against the same problems launched one after
    another on one stream.  Then every instance's loss of orthogonality and
    residual by the device checker; the instances that broke down or miss
    10 n u on either measure run again as BCGSI+P-2S (Table 1: O(u) under
    u kappa <= 1 instead of u kappa^2 <= 1) in one batched launch, and the
    throughput counts the instances whose final result meets 10 n u."""
    import torch
    from paper_2507_21791_amd import bcgs, workloads as W
    specs = W.batched_specs(count)
    log(f"[bench] batched: generating {count} problems")
    Xs = [W.conditioned_device(p["m"], p["n"], p["decades"], p["seed"])
          for p in specs]
    torch.cuda.synchronize()
    items = [(X, p["s"], "p-1s", "fp64") for X, p in zip(Xs, specs)]
    batch = bcgs.Batch(items)
    t0 = time.perf_counter()
    bcgs.autotune(batch)
    tune_s = time.perf_counter() - t0
    log(f"[bench] batched: autotune {tune_s:.2f} s")
    stream = torch.cuda.current_stream()
    wss = [bcgs.Workspace(p["m"], p["n"], p["s"], "p-1s") for p in specs]
    outs = [(Q, R) for (_, Q, R, *_r) in batch.items]

    def one_by_one():
        for (X, s, v, pr), ws, (Q, R) in zip(items, wss, outs):
            bcgs.qr(X, s, v, pr, Q=Q, R=R, ws=ws)

    # algorithmic bytes of the whole batch, from the launch records
    one_by_one()
    torch.cuda.synchronize()
    bcgs.profile_start(stream)
    one_by_one()
    model_bytes = sum(r["bytes"] for r in bcgs.profile_stop(stream))
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        one_by_one()
    e1.record(stream)
    torch.cuda.synchronize()
    ms_single = e0.elapsed_time(e1) / reps
    fp_single = [int(_bits_sum(R)) for _, R in outs]
    ms_persist = _time_batched(batch, reps, "persistent")
    fp_persist = [int(_bits_sum(R)) for _, R in outs]
    ms_graph = _time_batched(batch, reps, None)
    fp_graph = [int(_bits_sum(R)) for _, R in outs]
    ms_batch = min(ms_graph, ms_persist)
    res = batch.results()
    U = 2.0 ** -53
    chk = bcgs.Checker()

    def measures(b, idx):
        """(status, loo, residual) of problem idx of batch b."""
        X, Q, R = b.items[idx][0], b.items[idx][1], b.items[idx][2]
        info = b.results()[idx][2]
        if info.status != 0:
            return info.status, None, None
        return (0,) + chk(X, Q, R)

    first = [measures(batch, i) for i in range(count)]
    torch.cuda.synchronize()
    e0.record(stream)
    for (X, s, v, pr), (Q, R) in zip(items, outs):
        chk.grams(X, Q, R)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_check = e0.elapsed_time(e1)
    good = lambda m, n: m[0] == 0 and m[1] <= 10 * n * U and \
        m[2] <= 10 * n * U
    redo = [i for i, p in enumerate(specs) if not good(first[i], p["n"])]
    final = list(first)
    ms_rerun = 0.0
    if redo:
        again = bcgs.Batch([(Xs[i], specs[i]["s"], "p-2s", "fp64")
                            for i in redo])
        ms_rerun = _time_batched(again, reps, None)
        for j, i in enumerate(redo):
            final[i] = measures(again, j)
    ok = [i for i, p in enumerate(specs) if good(final[i], p["n"])]
    loos = [final[i][1] for i in ok]
    ress = [final[i][2] for i in ok]
    out = {"workload": (f"{count} problems, m U[10000,200000], n in "
                        "{32,64,128,256}, s in {8,16}, kappa 1e2..1e10, "
                        "P-1S FP64"),
           "ms_batched": round(ms_batch, 3),
           "ms_graph": round(ms_graph, 3),
           "ms_persistent": round(ms_persist, 3),
           "ms_one_by_one": round(ms_single, 3),
           "speedup": round(ms_single / ms_batch, 3),
           "bitwise_equal_graph_persistent_alone": fp_single == fp_graph ==
           fp_persist,
           "problems_per_s": round(count / (ms_batch * 1e-3), 1),
           "model_gb": round(model_bytes / 1e9, 3),
           "gbs": round(model_bytes / (ms_batch * 1e-3) / 1e9, 1),
           "autotune_s": round(tune_s, 2),
           "breakdowns": sum(1 for _, _, info in res if info.status != 0),
           "p1s_accurate": sum(1 for i, p in enumerate(specs)
                               if good(first[i], p["n"])),
           "rerun_as_p2s": len(redo),
           "ms_rerun_p2s": round(ms_rerun, 3),
           "ms_check_all": round(ms_check, 3),
           "accurate_final": len(ok),
           "accurate_per_s": round(len(ok) / ((ms_batch + ms_rerun) * 1e-3),
                                   1),
           "accurate_per_s_with_check": round(
               len(ok) / ((ms_batch + ms_rerun + ms_check) * 1e-3), 1),
           "loo_max": max(loos, default=None),
           "residual_max": max(ress, default=None),
           "accuracy_bar": "loo and residual <= 10 n u (device checker)"}
    log(f"[bench] batched: {out}")
    del Xs, batch, wss, outs
    torch.cuda.empty_cache()
    return out


class _RawDevice:
    """A device buffer the library handed out (queue-allocated outputs), as
    an object torch.as_tensor accepts (__cuda_array_interface__)."""

    def __init__(self, ptr, nelems, typestr):
        self.__cuda_array_interface__ = {
            "shape": (nelems,), "typestr": typestr, "data": (ptr, False),
            "version": 3, "strides": None}


def _bits_sum(t):
    """Sum of the bit patterns of a column-major tensor with ld = rows (an
    exact, order-independent fingerprint; int64 wraps)."""
    import torch
    it = torch.int64 if t.element_size() == 8 else torch.int32
    return t.t().contiguous().view(it).sum(dtype=torch.int64)


def _fingerprint(r, m, n, precision):
    """Device fingerprints (Q bits, R bits) of a finished request."""
    import torch
    if r["Q"] is not None:
        return _bits_sum(r["Q"]), _bits_sum(r["R"])
    qt = "<f8" if precision == "fp64" else "<f4"
    q = torch.as_tensor(_RawDevice(r["Q_ptr"], m * n, qt), device="cuda")
    rr = torch.as_tensor(_RawDevice(r["R_ptr"], n * n, "<f8"), device="cuda")
    it = torch.int64 if precision == "fp64" else torch.int32
    return (q.view(it).sum(dtype=torch.int64),
            rr.view(torch.int64).sum(dtype=torch.int64))


def bench_served(nreq, rate, precision, pool, pool32, admission="shortest",
                 inflight=2, budget=96 << 30, arena=64 << 30):
    """Poisson arrivals at `rate` req/s of P-1S requests drawn from the
    device pool, through the library's request queue (continuous batching,
    queue-allocated outputs, a request that breaks down rerun once as
    P-2S).  Latency = completion - submission (the submitter submits at
    each arrival time).

    Accuracy of every result: each finished request's Q and R are
    fingerprinted on the device (sums of their bit patterns) before its
    outputs go back to the arena.  After the stream, every distinct (pool
    input, variant that produced the result) is factorized alone through
    bcgs_qr_ex, timed, fingerprinted and measured by the device checker
    (loss of orthogonality, relative residual); a served result whose
    fingerprints equal its lone run's carries that run's measures.
    Slowdown = latency / the lone run's time."""
    import threading
    import torch
    from paper_2507_21791_amd import bcgs, workloads as W
    trace = W.served_trace(nreq, rate, len(pool))
    src = pool if precision == "fp64" else pool32
    q = bcgs.Queue(hbm_budget_bytes=budget, max_inflight=inflight,
                   output_arena_bytes=arena, retry_variant="p-2s",
                   admission=admission)
    tickets = [None] * nreq

    def submitter():
        t0 = time.perf_counter()
        for i, (arr, k) in enumerate(trace):
            d = arr - (time.perf_counter() - t0)
            if d > 0:
                time.sleep(d)
            tickets[i] = q.submit(src[k][0], 16, "p-1s", precision,
                                  outputs="queue")

    th = threading.Thread(target=submitter)
    th.start()
    res = [None] * nreq
    fps = [None] * nreq
    fp_ok = True
    for i in range(nreq):
        while tickets[i] is None:
            time.sleep(0.0002)
        r = q.wait(tickets[i])
        if r["status"] == 0 and fp_ok:
            X = src[trace[i][1]][0]
            try:
                fps[i] = _fingerprint(r, X.shape[0], X.shape[1], precision)
            except Exception as e:      # no device-array import in torch
                log(f"[bench] served: fingerprints unavailable ({e})")
                fp_ok = False
        q.free(r["Q_ptr"])
        q.free(r["R_ptr"])
        res[i] = r
    th.join()
    q.close()
    lat = np.array([r["t_done"] - r["t_submit"] for r in res]) * 1e3
    span = max(r["t_done"] for r in res) - min(r["t_submit"] for r in res)
    fps = [None if f is None else (int(f[0]), int(f[1])) for f in fps]
    # lone runs of every distinct (input, variant) the stream produced
    chk = bcgs.Checker()
    lone = {}
    for i, r in enumerate(res):
        key = (trace[i][1], r["variant"])
        if r["status"] != 0 or key in lone:
            continue
        X = src[key[0]][0]
        Q, R, ws = bcgs.qr(X, 16, key[1], precision)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            bcgs.qr(X, 16, key[1], precision, Q=Q, R=R, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        fq, fr = _bits_sum(Q), _bits_sum(R)
        loo, resid = chk(X, Q, R, precision)
        lone[key] = {"ms": e0.elapsed_time(e1) / 3,
                     "fp": (int(fq), int(fr)), "loo": loo, "res": resid}
        del Q, R, ws
    ok = [i for i, r in enumerate(res) if r["status"] == 0]
    same = [i for i in ok
            if fps[i] == lone[(trace[i][1], res[i]["variant"])]["fp"]]
    loos = [lone[(trace[i][1], res[i]["variant"])]["loo"] for i in same]
    ress = [lone[(trace[i][1], res[i]["variant"])]["res"] for i in same]
    slow = np.array([lat[i] / lone[(trace[i][1], res[i]["variant"])]["ms"]
                     for i in ok])
    alone = np.array([lone[(trace[i][1], res[i]["variant"])]["ms"]
                      for i in ok])
    small = alone <= np.median(alone)
    lat_ok = lat[ok]
    pct = lambda a, p: round(float(np.percentile(a, p)), 3) if len(a) else None
    out = {"rate_per_s": rate, "requests": nreq, "precision": precision,
           "admission": admission, "inflight": inflight,
           "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
           "p99_over_p50": round(float(np.percentile(lat, 99) /
                                       np.percentile(lat, 50)), 2),
           "slowdown_p50": pct(slow, 50), "slowdown_p99": pct(slow, 99),
           "small_half_p50_ms": pct(lat_ok[small], 50),
           "small_half_p99_ms": pct(lat_ok[small], 99),
           "large_half_p50_ms": pct(lat_ok[~small], 50),
           "large_half_p99_ms": pct(lat_ok[~small], 99),
           "alone_ms_p50": pct(alone, 50), "alone_ms_p99": pct(alone, 99),
           "throughput_per_s": round(nreq / span, 1),
           "retried_as_p2s": int(sum(1 for r in res if r["attempts"] > 1)),
           "breakdowns": int(sum(1 for r in res if r["status"] == 2)),
           "errors": int(sum(1 for r in res if r["status"] not in (0, 2))),
           "results_checked": len(same),
           "results_differing_from_lone": len(ok) - len(same),
           "loo_max": max(loos, default=None),
           "loo_median": float(np.median(loos)) if loos else None,
           "residual_max": max(ress, default=None),
           "distinct_lone_runs": len(lone)}
    log(f"[bench] served: {out}")
    return out


def served_pool(count):
    import torch
    from paper_2507_21791_amd import workloads as W
    specs = W.served_pool_specs(count)
    log(f"[bench] served: generating a pool of {count} inputs")
    pool, pool32 = [], []
    for p in specs:
        X = W.conditioned_device(p["m"], p["n"], p["decades"], p["seed"])
        pool.append((X, p))
        X32 = torch.empty((p["n"], p["m"]), dtype=torch.float32,
                          device="cuda").t()
        X32.copy_(X)
        pool32.append((X32, p))
    torch.cuda.synchronize()
    return pool, pool32


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="tall")
    ap.add_argument("--m", type=int, default=None)
    ap.add_argument("--s", type=int, default=None)
    ap.add_argument("--variants", default="p-1s,bcgsi+,p-2s,pipi+,bcgsi+1s")
    ap.add_argument("--cpu-rows", type=int, default=1 << 20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-small", action="store_true")
    ap.add_argument("--ld-pad", type=int, default=16,
                    help="leading dimension of X and Q = m + LD_PAD")
    ap.add_argument("--no-twin", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--sweep-steps", type=int, default=3)
    ap.add_argument("--batched-count", type=int, default=256)
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--served-n", type=int, default=1000)
    ap.add_argument("--served-pool", type=int, default=64)
    ap.add_argument("--served-inflight", type=int, default=2)
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
    ld = m + args.ld_pad
    if args.ld_pad:
        Xp = bcgs.empty_fortran(m, n, torch.float64, "cuda", ld=ld)
        Xp.copy_(X)
        del X
        X = Xp
    torch.cuda.synchronize()
    Q = bcgs.empty_fortran(m, n, torch.float64, "cuda", ld=ld)
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
        ms, recs, info, steps_ms, ms_prof = time_variant(
            X, s, v, args.steps, args.warmup, Q, R)
        agg = aggregate(recs, args.steps)
        model_bytes = sum(a["bytes"] for a in agg)
        model_flops = sum(a["flops"] for a in agg)
        steps_ms = sorted(steps_ms)
        res = {"ms": round(ms, 4),
               "ms_profiled": round(ms_prof, 4),
               "step_ms_median": round(float(np.median(steps_ms)), 4),
               "step_ms_p99": round(float(np.percentile(steps_ms, 99)), 4),
               "model_gb": round(model_bytes / 1e9, 3),
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
                                f"{variants[0]}, X and Q column-major "
                                f"with leading dimension {ld}"),
                   "m": m, "n": n, "s": s, "variant": variants[0],
                   "ld": ld},
        "hbm_frac": round(head["gbs"] / HBM_PEAK_GBS, 4),
        "fp64_frac": round(head["tflops"] / FP64_PEAK_TFS, 4),
        "roofline": roofline(dom),
    }
    if "bcgsi+" in results and variants[0] != "bcgsi+":
        out["speedup_vs_bcgsi+"] = round(results["bcgsi+"]["ms"] / head["ms"], 3)
    if "p-2s" in results and "bcgsi+" in results:
        out["speedup_p2s_vs_bcgsi+"] = round(
            results["bcgsi+"]["ms"] / results["p-2s"]["ms"], 3)
    if "bcgsi+" in results:
        # every variant against BCGSI+ on the same X (Table 2's comparison
        # on one GPU), with its status and LOO in "variants"
        out["speedups_vs_bcgsi+"] = {
            v: round(results["bcgsi+"]["ms"] / r["ms"], 3)
            for v, r in results.items()}
    out["variants"] = {k: {kk: vv for kk, vv in r.items() if kk != "_agg"}
                       for k, r in results.items()}
    out["p99_latency_ms"] = None
    cgbs = copy_bandwidth()
    out["copy_gbs"] = round(cgbs, 1)
    out["frac_of_copy"] = round(head["gbs"] / cgbs, 4)
    log(f"[bench] device copy {cgbs:.1f} GB/s; P-1S at "
        f"{head['gbs'] / cgbs:.3f} of it")
    rows = min(args.cpu_rows, m)
    Xhead = None if args.no_cpu else X[:rows].cpu()
    del X, Q, R
    torch.cuda.empty_cache()
    if not args.no_fp32:
        out["fp32_bulk"] = bench_fp32_bulk(m, n, s, args.steps, args.warmup,
                                           head["ms"])
    if not args.no_small:
        out["small"] = bench_small()
    if not args.no_twin:
        out["tall_k6"] = bench_twin(args.steps, args.warmup)
    if not args.no_sweep:
        out["sweep"] = bench_sweep(args.sweep_steps, 1, ld_pad=args.ld_pad)
    if not args.no_batched:
        out["batched"] = bench_batched(args.batched_count, 3)
    if not args.no_served:
        pool, pool32 = served_pool(args.served_pool)
        # 2000/s: far above capacity, so throughput is the capacity and the
        # latencies include the backlog; then half of that measured
        # capacity: the latency under a load the queue sustains (the
        # headline p99), with both admission orders
        k = args.served_inflight
        over = bench_served(args.served_n, 2000.0, "fp64", pool, pool32,
                            inflight=k)
        half = round(0.5 * over["throughput_per_s"])
        served = [over,
                  bench_served(args.served_n, half, "fp64", pool, pool32,
                               inflight=k),
                  bench_served(args.served_n, half, "fp64", pool, pool32,
                               admission="arrival", inflight=k),
                  bench_served(args.served_n, 2000.0, "fp32-bulk", pool,
                               pool32, inflight=k)]
        out["served"] = {
            "workload": (f"Poisson arrivals, P-1S, s=16, pool of "
                         f"{args.served_pool} device-resident inputs (m "
                         "log-uniform 4096..2^21, n 16..512, kappa "
                         "1e2..1e8) drawn with replacement; every result "
                         "fingerprinted and matched to a lone run measured "
                         "by the device checker"),
            "runs": served}
        out["p99_latency_ms"] = served[1]["p99_ms"]
        out["p99_latency_load"] = (f"fp64 requests at {half}/s (half of "
                                   "the capacity measured at 2000/s), "
                                   "shortest-first admission with aging")
        del pool, pool32
        torch.cuda.empty_cache()
    if not args.no_cpu:
        log(f"[bench] cpu baseline: oracle on {rows} rows")
        out["cpu_baseline"] = cpu_baseline(Xhead, s, rows,
                                           head["model_gb"] * 1e9, m)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
