"""Host logic of the measurement: the profile summaries' byte models on
synthetic counter files, and the kernel names of the built library.  No
GPU."""

import csv
import os

import pytest

import bench
from paper_2507_21791_amd import prof_summary as P

from kernel_names import library_kernel_names


def _write_counters(d, rows):
    """rows: (dispatch, kernel, grid, {counter: value})"""
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w",
              newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Grid_Size",
                    "Counter_Name", "Counter_Value"])
        for dsp, name, grid, vals in rows:
            for c, v in vals.items():
                w.writerow([dsp, name, grid, c, v])


K = "void bcgs::p16::pass16_s2_kernel<double, 16, 2, 256, 7, true, 2, false>(bcgs::p16::ArgsT<double>)"
COPY = "__amd_rocclr_copyBuffer"
GIB = 1 << 30


def test_counter_scaling_uses_copies_before_the_library(tmp_path):
    """The calibration copies are the 1 GiB copies before the first library
    kernel; later copies (the copy-rate measurement, 2 GiB) are ignored."""
    kib = 1 << 20                     # 1 GiB in KiB
    fetch = [(1, COPY, 131072, {"FETCH_SIZE": 4 * kib}),      # input copy
             (2, COPY, 131072, {"FETCH_SIZE": kib / 2}),
             (3, COPY, 131072, {"FETCH_SIZE": kib / 2}),
             (4, COPY, 131072, {"FETCH_SIZE": kib / 2}),
             (5, K, 131072, {"FETCH_SIZE": 3.0e6}),
             (6, COPY, 131072, {"FETCH_SIZE": kib}),           # 2 GiB copies
             (7, COPY, 131072, {"FETCH_SIZE": kib})]
    write = [(d, n, g, {"WRITE_SIZE": {COPY: kib}.get(n, 1.0e6)})
             for d, n, g, _ in fetch]
    _write_counters(str(tmp_path / "f"), fetch)
    _write_counters(str(tmp_path / "w"), write)
    out = P.counters(str(tmp_path / "f"), str(tmp_path / "w"), "run", "cmd",
                     os.path.dirname(os.path.dirname(__file__)))
    assert "FETCH x2.0000, WRITE x1.0000" in out
    line = [l for l in out.splitlines() if l.startswith("pass16_s2_kernel")][0]
    read_gb, write_gb = (float(x) for x in line.split()[-3:-1])
    assert read_gb == pytest.approx(2 * 3.0e6 * 1024 / 1e9, rel=1e-4)
    assert write_gb == pytest.approx(1.0e6 * 1024 / 1e9, rel=1e-4)


def test_request_counts_to_bytes(tmp_path):
    """Reads: 32, 64 or 128 bytes per request; writes: 64 bytes, else 32."""
    rd = [(1, COPY, 131072, {"TCC_EA0_RDREQ_32B_sum": 0,
                             "TCC_EA0_RDREQ_64B_sum": 0,
                             "TCC_EA0_RDREQ_128B_sum": GIB // 128,
                             "TCC_EA0_RDREQ_sum": GIB // 128}),
          (2, K, 131072, {"TCC_EA0_RDREQ_32B_sum": 1000000,
                          "TCC_EA0_RDREQ_64B_sum": 2000000,
                          "TCC_EA0_RDREQ_128B_sum": 10000000,
                          "TCC_EA0_RDREQ_sum": 13000000})]
    wr = [(1, COPY, 131072, {"TCC_EA0_WRREQ_64B_sum": GIB // 64,
                             "TCC_EA0_WRREQ_sum": GIB // 64}),
          (2, K, 131072, {"TCC_EA0_WRREQ_64B_sum": 10000000,
                          "TCC_EA0_WRREQ_sum": 15000000})]
    _write_counters(str(tmp_path / "r"), rd)
    _write_counters(str(tmp_path / "w"), wr)
    out = P.requests(str(tmp_path / "r"), str(tmp_path / "w"), "cmd")
    assert "copy: read 1.0000 GiB, written 1.0000 GiB" in out
    line = [l for l in out.splitlines() if l.startswith("pass16_s2_kernel")][0]
    f = line.split()
    # 32 * 1e6 + 64 * 2e6 + 128 * 1e7 bytes read; 64 * 1e7 + 32 * 5e6 written
    assert float(f[-4]) == pytest.approx(1.44, abs=1e-4)
    assert float(f[-3]) == pytest.approx(0.80, abs=1e-4)
    assert float(f[-1]) == pytest.approx(10 / 13, abs=1e-3)


def test_library_kernels_have_short_names():
    """Every kernel of the built library maps to a short name of the form
    the profile summaries and the bench's launch records use."""
    names = library_kernel_names()
    assert any(n.startswith("pass16_s2_kernel<double, 16, 2, 256,")
               for n in names), sorted(names)[:20]
    assert "gram_reduce_kernel" in names
    assert "epilogue_kernel<16>" in names
    assert "tsqr_wave_apply_path_kernel<double, 16>" in names
    assert "tsqr_wave_tree_kernel<16>" in names
    assert all("(" not in n and "::" not in n for n in names)
