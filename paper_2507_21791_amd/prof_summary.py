"""Condense rocprofv3 CSV output into the short text summaries kept under
profiles/.

    python -m paper_2507_21791_amd.prof_summary trace  <dir> <prefix> "<cmd>"
    python -m paper_2507_21791_amd.prof_summary counters <fetch_dir>
           <write_dir> <prefix> "<cmd>"
    python -m paper_2507_21791_amd.prof_summary requests <read_dir>
           <write_dir> "<cmd>"
    python -m paper_2507_21791_amd.prof_summary sq <dir> "<cmd>" ...

`trace` reads <dir>/<prefix>_kernel_trace.csv (a --kernel-trace run) and
prints per-kernel launch counts and durations for this library's kernels
(the input generation by torch/rocBLAS/rocSOLVER is summed on one line).

`requests` reads two runs of the TCC_EA0 request-size counters (reads of
32, 64 and 128 bytes; writes of 64 bytes or else 32) and prints the bytes
they imply per launch, with no calibration: a check of the scale factors
that `counters` derives.

`counters` reads the FETCH_SIZE and WRITE_SIZE runs (one counter per run)
and prints the per-launch HBM traffic of every library kernel, scaled by
what the same counters read for the plain 1 GiB device copies that
`bench.py --copy-calibration` performs (copyBuffer dispatches with 131072
work-items).  The scale factors make the counters comparable to bytes.
"""

import csv
import hashlib
import os
import re
import sys
from collections import OrderedDict, defaultdict

GIB_KIB = 1 << 20


def short_name(name):
    n = re.sub(r"\(.*", "", name)
    n = n.replace("void ", "").replace("bcgs::", "")
    n = n.replace("p16::", "").replace("tq::", "tsqr_")
    n = n.replace("tw::", "tsqr_wave_").replace("ck::", "check_")
    return n.strip()


def ours(name):
    return "bcgs::" in name


# sources of the dominant kernel (the s <= 16 streaming pass)
PASS_SOURCES = ("pass16_impl.h", "pass16.hip", "pass16_reg.hip", "common.h")


def source_digest(root):
    """sha256 over the sources of the s <= 16 pass kernels, to tell whether
    their counters are stale."""
    h = hashlib.sha256()
    cdir = os.path.join(root, "paper_2507_21791_amd", "csrc")
    for f in PASS_SOURCES:
        with open(os.path.join(cdir, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    with open(os.path.join(root, "include", "bcgs.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def trace(d, prefix, cmd):
    rows = list(csv.DictReader(open(os.path.join(
        d, f"{prefix}_kernel_trace.csv"))))
    agg = OrderedDict()
    other_ns, other_n = 0, 0
    for r in rows:
        dt = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        if not ours(r["Kernel_Name"]):
            other_ns += dt
            other_n += 1
            continue
        k = short_name(r["Kernel_Name"])
        a = agg.setdefault(k, [0, 0, None, 0])
        a[0] += 1
        a[1] += dt
        a[2] = dt if a[2] is None else min(a[2], dt)
        a[3] = max(a[3], dt)
    out = [f"# rocprofv3 kernel trace summary", f"# command: {cmd}",
           "# library kernels, sorted by total time (all launches in the run)",
           f"{'kernel':52s} {'calls':>6s} {'total_ms':>10s} {'avg_us':>10s}"
           f" {'min_us':>9s} {'max_us':>9s}"]
    for k, (n, tot, lo, hi) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        out.append(f"{k:52s} {n:6d} {tot / 1e6:10.3f} {tot / n / 1e3:10.1f}"
                   f" {lo / 1e3:9.1f} {hi / 1e3:9.1f}")
    out.append(f"{'(input generation and copies: torch/rocBLAS/rocSOLVER)':52s}"
               f" {other_n:6d} {other_ns / 1e6:10.3f}")
    return "\n".join(out)


def _counter(d, name):
    f = [x for x in os.listdir(d) if x.endswith("counter_collection.csv")][0]
    res = []
    for r in csv.DictReader(open(os.path.join(d, f))):
        if r["Counter_Name"] == name:
            res.append((r["Kernel_Name"], int(r["Grid_Size"]),
                        float(r["Counter_Value"])))
    return res


def counters(dfetch, dwrite, prefix, cmd, root):
    fe = _counter(dfetch, "FETCH_SIZE")
    wr = _counter(dwrite, "WRITE_SIZE")
    cal = {}
    for tag, rows in (("FETCH_SIZE", fe), ("WRITE_SIZE", wr)):
        # the calibration copies run before the first library kernel (the
        # bench's own copy-rate measurement, 2 GiB copies, comes after it)
        first = next((i for i, (n, g, v) in enumerate(rows) if ours(n)),
                     len(rows))
        vals = [v for n, g, v in rows[:first]
                if "copyBuffer" in n and g == 131072]
        vals = [v for v in vals if v > 0.25 * GIB_KIB]
        vals = vals[-3:]
        cal[tag] = GIB_KIB / (sum(vals) / len(vals)) if vals else float("nan")
    per = defaultdict(lambda: [0, 0.0, 0.0])
    seq = []
    for (n, g, f), (n2, g2, w) in zip(
            [x for x in fe if ours(x[0])], [x for x in wr if ours(x[0])]):
        k = short_name(n)
        a = per[k]
        a[0] += 1
        fb = f * 1024 * cal["FETCH_SIZE"]
        wb = w * 1024 * cal["WRITE_SIZE"]
        a[1] += fb
        a[2] += wb
        seq.append((k, fb, wb))
    out = ["# rocprofv3 HBM traffic summary (FETCH_SIZE run, then WRITE_SIZE "
           "run)", f"# command (twice, --pmc FETCH_SIZE / --pmc WRITE_SIZE): "
           f"{cmd}",
           f"# kernel sources digest: {source_digest(root)} (s <= 16 pass sources)",
           "# calibration: 1 GiB plain device copy reads "
           f"{GIB_KIB / cal['FETCH_SIZE']:.0f} KiB FETCH_SIZE and "
           f"{GIB_KIB / cal['WRITE_SIZE']:.0f} KiB WRITE_SIZE;",
           f"# scale factors FETCH x{cal['FETCH_SIZE']:.4f}, "
           f"WRITE x{cal['WRITE_SIZE']:.4f}",
           "# per-launch averages in GB (1e9 bytes) after scaling",
           f"{'kernel':52s} {'calls':>6s} {'read_GB':>9s} {'write_GB':>9s}"
           f" {'total_GB':>9s}"]
    for k, (n, fb, wb) in sorted(per.items(), key=lambda kv: -(kv[1][1] +
                                                               kv[1][2])):
        out.append(f"{k:52s} {n:6d} {fb / n / 1e9:9.4f} {wb / n / 1e9:9.4f}"
                   f" {(fb + wb) / n / 1e9:9.4f}")
    out.append("# launch sequence of the last factorization "
               "(kernel, read_GB, write_GB)")
    last = [i for i, (k, _, _) in enumerate(seq) if k == "fill_kernel"]
    start = last[-1] if last else 0
    for k, fb, wb in seq[start:]:
        out.append(f"  {k:50s} {fb / 1e9:9.4f} {wb / 1e9:9.4f}")
    return "\n".join(out)


RD_COUNTERS = ("TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum",
               "TCC_EA0_RDREQ_128B_sum", "TCC_EA0_RDREQ_sum")
WR_COUNTERS = ("TCC_EA0_WRREQ_64B_sum", "TCC_EA0_WRREQ_sum")


def _dispatches(d, names):
    """{dispatch id: (kernel, grid, {counter: value})} in dispatch order."""
    f = [x for x in os.listdir(d) if x.endswith("counter_collection.csv")][0]
    out = OrderedDict()
    for r in csv.DictReader(open(os.path.join(d, f))):
        if names is not None and r["Counter_Name"] not in names:
            continue
        k = out.setdefault(int(r["Dispatch_Id"]),
                           (r["Kernel_Name"], int(r["Grid_Size"]), {}))
        k[2][r["Counter_Name"]] = float(r["Counter_Value"])
    return out


def requests(drd, dwrite, cmd):
    """HBM bytes from the L2-to-memory request counts by size (no
    calibration): reads 32, 64 or 128 bytes, writes 64 bytes or else 32."""
    rd = _dispatches(drd, RD_COUNTERS)
    wr = _dispatches(dwrite, WR_COUNTERS)
    per = defaultdict(lambda: [0, 0.0, 0.0, 0.0])
    copies = []
    for (i, (n, g, c)), (j, (n2, g2, w)) in zip(rd.items(), wr.items()):
        rb = (32 * c["TCC_EA0_RDREQ_32B_sum"] + 64 * c["TCC_EA0_RDREQ_64B_sum"]
              + 128 * c["TCC_EA0_RDREQ_128B_sum"])
        w64 = w["TCC_EA0_WRREQ_64B_sum"]
        wb = 64 * w64 + 32 * (w["TCC_EA0_WRREQ_sum"] - w64)
        if ours(n):
            a = per[short_name(n)]
            a[0] += 1
            a[1] += rb
            a[2] += wb
            a[3] += c["TCC_EA0_RDREQ_128B_sum"] / max(1.0, c["TCC_EA0_RDREQ_sum"])
        elif "copyBuffer" in n and g == 131072 and not per:
            copies.append((rb, wb))
    out = ["# rocprofv3 HBM request summary (TCC_EA0 read / write request "
           "counts by size, two runs)",
           f"# command (twice, --pmc {' '.join(RD_COUNTERS)} / --pmc "
           f"{' '.join(WR_COUNTERS)}): {cmd}"]
    for rb, wb in copies[-3:]:
        out.append(f"# plain 1 GiB device copy: read {rb / 2**30:.4f} GiB, "
                   f"written {wb / 2**30:.4f} GiB")
    out += ["# per-launch averages in GB (1e9 bytes); rd128 = share of read "
            "requests that are 128 bytes",
            f"{'kernel':52s} {'calls':>6s} {'read_GB':>9s} {'write_GB':>9s}"
            f" {'total_GB':>9s} {'rd128':>6s}"]
    for k, (n, rb, wb, f128) in sorted(per.items(),
                                       key=lambda kv: -(kv[1][1] + kv[1][2])):
        out.append(f"{k:52s} {n:6d} {rb / n / 1e9:9.4f} {wb / n / 1e9:9.4f}"
                   f" {(rb + wb) / n / 1e9:9.4f} {f128 / n:6.3f}")
    return "\n".join(out)


def sq(dirs, cmds):
    """Per-launch SQ counters of the library's streaming passes from one or
    more --pmc runs (each run holds at most 8 SQ counters).  MFMA busy is
    given as a share of the cycles of all SIMDs over the kernel's duration
    (SQ_BUSY_CYCLES counts one per shader engine and cycle: 32 on this
    GPU, each with 32 SIMDs), wait and issue counts per wave."""
    per = defaultdict(lambda: defaultdict(list))
    for d in dirs:
        for i, (n, g, c) in _dispatches(d, None).items():
            if ours(n) and "pass" in n:
                for k, v in c.items():
                    per[short_name(n)][k].append(v)
    out = ["# rocprofv3 SQ counter summary of the streaming passes",
           *[f"# command: {c}" for c in cmds],
           "# per-launch means; busy = SQ_VALU_MFMA_BUSY_CYCLES / (1024 SIMDs"
           " x SQ_BUSY_CYCLES / 32); wait_inst, wait_any: share of"
           " SQ_WAVE_CYCLES; instructions per wave (SQ_WAVES waves)"]
    for k, c in sorted(per.items()):
        m = {kk: sum(v) / len(v) for kk, v in c.items()}
        parts = [f"launches={len(next(iter(c.values())))}"]
        if "SQ_VALU_MFMA_BUSY_CYCLES" in m and "SQ_BUSY_CYCLES" in m:
            parts.append("mfma_busy=%.3f" % (m["SQ_VALU_MFMA_BUSY_CYCLES"] /
                                            (1024 * m["SQ_BUSY_CYCLES"] / 32)))
        for w in ("SQ_WAIT_INST_ANY", "SQ_WAIT_ANY"):
            if w in m and "SQ_WAVE_CYCLES" in m:
                parts.append("%s=%.3f" % (w.lower()[3:], m[w] /
                                          m["SQ_WAVE_CYCLES"]))
        if "SQ_WAVES" in m:
            for w in ("SQ_INSTS_MFMA", "SQ_INSTS_VALU", "SQ_INSTS_SALU",
                      "SQ_INSTS_LDS"):
                if w in m:
                    parts.append("%s/wave=%.0f" % (w.lower()[9:],
                                                   m[w] / m["SQ_WAVES"]))
        if "SQ_LDS_BANK_CONFLICT" in m:
            parts.append("lds_bank_conflict=%.3g" % m["SQ_LDS_BANK_CONFLICT"])
        out.append(k)
        out.append("    " + "  ".join(parts))
    return "\n".join(out)


def main(argv):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if argv[1] == "trace":
        print(trace(argv[2], argv[3], argv[4]))
    elif argv[1] == "counters":
        print(counters(argv[2], argv[3], argv[4], argv[5], root))
    elif argv[1] == "requests":
        print(requests(argv[2], argv[3], argv[4]))
    elif argv[1] == "sq":
        # sq <dir1> <cmd1> [<dir2> <cmd2> ...]
        print(sq(argv[2::2], argv[3::2]))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv)
