"""The names the library gives its profiled launches are exactly the
kernel names rocprofv3 reports (the demangled symbols of the library's
code objects, shortened as the profile summaries shorten them), for the
s <= 16 pass in both copy forms and binary32, the general pass, both TSQR
forms, the epilogue and the reduction."""

import pytest

from kernel_names import library_kernel_names
from parity import log, to_device
from paper_2507_21791_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m,n,s,variant,precision", [
    (20000, 64, 16, "p-1s", "fp64"), (20001, 64, 16, "bcgsi+", "fp64"),
    (3000, 128, 32, "p-2s", "fp64"), (5000, 64, 16, "p-1s", "fp32-bulk")])
def test_profiled_names_are_kernel_symbols(m, n, s, variant, precision):
    import torch
    from paper_2507_21791_amd import bcgs
    log(f"[gpu] launch names m={m} n={n} s={s} {variant} {precision}")
    X = to_device(W.conditioned_host(m, n, 2, seed=m + s),
                  torch.float64 if precision == "fp64" else torch.float32)
    stream = torch.cuda.current_stream()
    bcgs.profile_start(stream)
    bcgs.qr(X, s, variant, precision)
    recs = bcgs.profile_stop(stream)
    names = {r["name"] for r in recs}
    known = library_kernel_names()
    assert names and "" not in names
    assert names <= known, sorted(names - known)
