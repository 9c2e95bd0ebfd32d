"""bcgs_qr_noalloc (workspace in the library's fixed device array) against
bcgs_qr_ex (caller workspace) on the GPU: two calls in a row, the second on
a smaller problem, each bitwise equal to bcgs_qr_ex on the same input (the
same kernels in the same order) and within the oracle's tolerances."""

import sys

import numpy as np
import pytest

from paper_2507_21791_amd import bcgs, workloads as W

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _device_input(m, n, c, seed):
    Xh = W.conditioned_host(m, n, c, seed=seed)
    X = bcgs.empty_fortran(m, n, torch.float64, "cuda")
    X.copy_(torch.from_numpy(Xh))
    return Xh, X


def _info(buf):
    raw = buf[:bcgs.INFO_BYTES].cpu().numpy().tobytes()
    return bcgs.Info.from_buffer_copy(raw)


@pytest.mark.parametrize("variant", ["p-1s", "bcgsi+"])
def test_noalloc_equals_ex_twice_then_smaller(variant):
    from parity import compare
    cases = [(120001, 256, 16, 6, 31), (3001, 48, 8, 4, 32)]
    for m, n, s, c, seed in cases:
        assert bcgs.workspace_size(m, n, s, variant) <= \
            bcgs.NOALLOC_SCRATCH_BYTES
        print(f"noalloc case {variant} m={m} n={n} s={s}", flush=True)
        Xh, X = _device_input(m, n, c, seed)
        # reference: the caller-workspace entry point
        Qe, Re, ws = bcgs.qr(X, s, variant)
        # the no-allocation entry point, its outputs pre-filled with NaN so
        # that anything it fails to write shows
        Qn = bcgs.empty_fortran(m, n, torch.float64, "cuda")
        Rn = bcgs.empty_fortran(n, n, torch.float64, "cuda")
        Qn.fill_(float("nan"))
        Rn.fill_(float("nan"))
        info = torch.zeros(64, dtype=torch.uint8, device="cuda")
        bcgs.qr_noalloc(X, s, variant, "fp64", Qn, Rn, info)
        torch.cuda.synchronize()
        ie, inn = ws.info(), _info(info)
        assert inn.as_dict() == ie.as_dict()
        assert inn.status == 0
        assert torch.equal(Qn, Qe) and torch.equal(Rn, Re)
        compare(Xh, s, variant, Qn.cpu().numpy(), Rn.cpu().numpy(),
                       inn, kappa=10.0 ** c)
        sys.stdout.flush()
