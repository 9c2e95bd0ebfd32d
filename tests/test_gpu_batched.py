"""Batched launch and autotuner on the GPU, through the C ABI.

A problem in a batch must give exactly the bits it gives alone through
bcgs_qr_ex (same kernels, same order, same tuned choices), and the FP64
results must meet the oracle's tolerances.  Graph replays are checked
after eager work on the same stream and after the inputs change in place.
Every case prints its name before touching the GPU.
"""

import numpy as np
import pytest

from paper_2507_21791_amd import workloads as W

from parity import compare, compare_bulk32, host, log, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    from paper_2507_21791_amd import bcgs
    assert torch.cuda.is_available()
    bcgs.lib()
    bcgs.tuning_clear()
    yield
    bcgs.tuning_clear()
    bcgs.lib().bcgs_release()


# (m, n, s, decades, variant, precision): uneven sizes, every variant, both
# precisions, s on both pass kernels, a single-block-column problem
MIX = [
    (3000, 64, 16, 3, "p-1s", "fp64"),
    (20000, 128, 16, 4, "bcgsi+", "fp64"),
    (777, 32, 8, 2, "p-2s", "fp64"),
    (12000, 96, 32, 3, "p-2s", "fp64"),
    (5000, 48, 4, 2, "p-1s", "fp64"),
    (40000, 64, 16, 2, "p-1s", "fp32-bulk"),
    (9000, 32, 8, 1, "bcgsi+", "fp32-bulk"),
    (1000, 16, 16, 2, "p-1s", "fp64"),
    (65000, 256, 16, 3, "p-1s", "fp64"),
]


def _inputs(mix, seed0=0):
    import torch
    out = []
    for i, (m, n, s, dec, v, p) in enumerate(mix):
        X = W.conditioned_host(m, n, dec, seed=seed0 + 31 * i + m)
        if p == "fp32-bulk":
            X = np.asfortranarray(X.astype(np.float32).astype(np.float64))
        dt = torch.float64 if p == "fp64" else torch.float32
        out.append((X, to_device(X, dt)))
    return out


def _alone(Xd, s, variant, precision):
    import torch
    from paper_2507_21791_amd import bcgs
    Q, R, ws = bcgs.qr(Xd, s, variant, precision)
    torch.cuda.synchronize()
    return host(Q), host(R), ws.info()


def _check_batch_vs_alone(mix, inputs, batch):
    for (m, n, s, dec, v, p), (Xh, Xd), (Q, R, info) in zip(
            mix, inputs, batch.results()):
        Qa, Ra, ia = _alone(Xd, s, v, p)
        assert info.status == ia.status == 0, (info.as_dict(), ia.as_dict())
        assert np.array_equal(host(R), Ra), (m, n, s, v, p)
        assert np.array_equal(host(Q), Qa), (m, n, s, v, p)


def test_batch_equals_alone_and_oracle():
    import torch
    from paper_2507_21791_amd import bcgs
    log("[gpu] batched mix of", len(MIX), "problems")
    inputs = _inputs(MIX)
    batch = bcgs.Batch([(Xd, s, v, p) for (m, n, s, d, v, p), (Xh, Xd)
                        in zip(MIX, inputs)])
    bcgs.qr_batched(batch)
    torch.cuda.synchronize()
    _check_batch_vs_alone(MIX, inputs, batch)
    for (m, n, s, dec, v, p), (Xh, Xd), (Q, R, info) in zip(
            MIX, inputs, batch.results()):
        if m * n > 3_000_000:
            continue                      # oracle time; bitwise check covers it
        if p == "fp64":
            compare(Xh, s, v, host(Q), host(R), info, kappa=10.0 ** dec)
        else:
            compare_bulk32(Xh, s, v, host(Q), host(R), info, kappa=10.0 ** dec)


def test_graph_replays_after_eager_work_and_new_inputs():
    """Replay the cached graph several times with eager work between, and
    after rewriting X in place (same pointers): every replay must match the
    lone runs on the current inputs."""
    import torch
    from paper_2507_21791_amd import bcgs
    mix = MIX[:5]
    inputs = _inputs(mix, seed0=100)
    batch = bcgs.Batch([(Xd, s, v, p) for (m, n, s, d, v, p), (Xh, Xd)
                        in zip(mix, inputs)])
    for rep in range(3):
        log(f"[gpu] batched replay {rep}")
        bcgs.qr_batched(batch)
        junk = torch.randn(1 << 20, device="cuda").sum()   # eager work
        torch.cuda.synchronize()
        del junk
        _check_batch_vs_alone(mix, inputs, batch)
    fresh = _inputs(mix, seed0=200)
    for (_, Xd), (Xh2, Xd2) in zip(inputs, fresh):
        Xd.copy_(Xd2)
    log("[gpu] batched replay on rewritten inputs")
    bcgs.qr_batched(batch)
    torch.cuda.synchronize()
    _check_batch_vs_alone(mix, inputs, batch)


def test_streams_mode_matches_graph(monkeypatch):
    import torch
    from paper_2507_21791_amd import bcgs
    mix = MIX[:4]
    inputs = _inputs(mix, seed0=300)
    items = [(Xd, s, v, p) for (m, n, s, d, v, p), (Xh, Xd)
             in zip(mix, inputs)]
    log("[gpu] batched without graph")
    b1 = bcgs.qr_batched(bcgs.Batch(items))
    monkeypatch.setenv("BCGS_BATCH_MODE", "streams")
    b2 = bcgs.qr_batched(bcgs.Batch(items))
    torch.cuda.synchronize()
    for (Q1, R1, i1), (Q2, R2, i2) in zip(b1.results(), b2.results()):
        assert i1.status == i2.status == 0
        assert np.array_equal(host(R1), host(R2))
        assert np.array_equal(host(Q1), host(Q2))


def test_autotune_then_batch_equals_alone():
    """After tuning, lone and batched runs read the same table entry, so the
    bits still agree; the tuned choices stay within the tolerances."""
    import torch
    from paper_2507_21791_amd import bcgs
    mix = [MIX[0], MIX[1], MIX[5], MIX[8]]
    inputs = _inputs(mix, seed0=400)
    batch = bcgs.Batch([(Xd, s, v, p) for (m, n, s, d, v, p), (Xh, Xd)
                        in zip(mix, inputs)])
    log("[gpu] autotune")
    bcgs.autotune(batch)
    for (m, n, s, d, v, p) in mix:
        wg, shape, tuned = bcgs.tuning_get(m, n, s, v, p)
        log(f"    m={m} n={n} s={s} {v} {p}: max_wg={wg} shape={shape}")
        assert tuned
    bcgs.qr_batched(batch)
    torch.cuda.synchronize()
    _check_batch_vs_alone(mix, inputs, batch)
    (m, n, s, dec, v, p), (Xh, Xd) = mix[0], inputs[0]
    Q, R, info = batch.results()[0]
    compare(Xh, s, v, host(Q), host(R), info, kappa=10.0 ** dec)
    bcgs.tuning_clear()


def test_empty_batch():
    from paper_2507_21791_amd import bcgs
    log("[gpu] empty batch")
    bcgs.qr_batched(bcgs.Batch([]))
