"""FP32-bulk form on the GPU against the FP64 oracle, through the C ABI.

X and Q are binary32 in HBM and the per-row products accumulate in
binary32; reductions, Cholesky, the Pythagorean subtraction and R are
binary64.  Every case prints its name before touching the GPU.  Bounds:
see compare_bulk32 in tests/parity.py.
"""

import numpy as np
import pytest

from paper_2507_21791_amd import workloads as W

from parity import compare_bulk32, host, log, run_gpu

pytestmark = pytest.mark.gpu
VARIANTS = ["bcgsi+", "p-2s", "p-1s"]


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    from paper_2507_21791_amd import bcgs
    assert torch.cuda.is_available()
    bcgs.lib()
    yield
    bcgs.lib().bcgs_release()


def _fp32_input(m, n, decades, seed):
    """Seeded conditioned X rounded to binary32 (both sides see this X)."""
    X = W.conditioned_host(m, n, decades, seed=seed)
    return np.asfortranarray(X.astype(np.float32).astype(np.float64))


SHAPES = [  # (m, n, s, decades): ragged tails, several tiles, every s path
    (64, 8, 4, 1), (65, 12, 4, 1), (300, 48, 16, 2), (1000, 64, 16, 2),
    (257, 48, 2, 1), (513, 60, 5, 2), (2000, 128, 32, 2), (3000, 128, 64, 2),
    (4099, 96, 16, 2), (10000, 24, 8, 1), (33000, 48, 16, 2),
    (200000, 64, 16, 2),
]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("m,n,s,dec", SHAPES)
def test_bulk32_shapes(m, n, s, dec, variant):
    log(f"[gpu] fp32-bulk m={m} n={n} s={s} kappa=1e{dec} {variant}")
    X = _fp32_input(m, n, dec, seed=7 * m + n + s)
    Qg, Rg, info = run_gpu(X, s, variant, precision="fp32-bulk")
    out = compare_bulk32(X, s, variant, host(Qg), host(Rg), info,
                         kappa=10.0 ** dec)
    log("   ", out)


@pytest.mark.parametrize("variant", VARIANTS)
def test_bulk32_exact_case_bitwise(variant):
    """Scaled-identity columns at distinct rows: every product, square root
    and Householder step is exact in binary32 too, so R = diag(2^e) and
    Q = X diag(2^-e) bitwise."""
    n = 64
    e = np.random.default_rng(13).integers(-20, 20, size=n)
    X = W.scaled_permuted_identity(3000, n, e, seed=13)
    log(f"[gpu] fp32-bulk exact scaled permuted identity {variant}")
    Qg, Rg, info = run_gpu(X, 16, variant, precision="fp32-bulk")
    assert info.status == 0
    assert np.array_equal(host(Rg), np.diag(np.ldexp(1.0, e)))
    assert np.array_equal(host(Qg), X * np.ldexp(1.0, -e)[None, :])


@pytest.mark.parametrize("variant", VARIANTS)
def test_bulk32_bitwise_repeatable(variant):
    X = _fp32_input(20000, 64, 2, seed=5)
    log(f"[gpu] fp32-bulk repeat {variant}")
    Q1, R1, _ = run_gpu(X, 16, variant, precision="fp32-bulk")
    Q2, R2, _ = run_gpu(X, 16, variant, precision="fp32-bulk")
    assert np.array_equal(host(R1), host(R2))
    assert np.array_equal(host(Q1), host(Q2))


@pytest.mark.parametrize("m,n", [(40000, 128), (40001, 256), (30000, 512)])
def test_bulk32_fast_pass(m, n):
    """s = 16 in binary32 runs the binary32 form of the s <= 16 pass (tag
    digit W P with P >= 4), direct copies for aligned columns and register
    staging for odd m; the result meets the FP32-bulk bounds."""
    import torch
    from paper_2507_21791_amd import bcgs
    log(f"[gpu] fp32-bulk fast pass m={m} n={n}")
    X = _fp32_input(m, n, 2, seed=m + n)
    Xd = torch.empty((n, m), dtype=torch.float32, device="cuda").t()
    Xd.copy_(torch.from_numpy(np.asfortranarray(X)).float())
    ws = bcgs.Workspace(m, n, 16, "p-1s", "fp32-bulk")
    stream = torch.cuda.current_stream()
    bcgs.profile_start(stream)
    Q, R, _ = bcgs.qr(Xd, 16, "p-1s", "fp32-bulk", ws=ws)
    recs = bcgs.profile_stop(stream)
    tags = [r["tag"] for r in recs if r["kind"] == "pass"]
    assert tags and all(t >= 10 ** 9 and (t // 10 ** 7) % 10 >= 4
                        for t in tags), tags
    if m % 4:
        assert all((t // 10 ** 6) % 10 >= 5 for t in tags), tags
    out = compare_bulk32(X, 16, "p-1s", host(Q), host(R), ws.info(),
                         kappa=1e2)
    log("   ", out)
