"""The batched persistent launch on the GPU, through the C ABI.

bcgs_qr_batched runs binary64 batches whose block width is 4, 8 or 16 as
one persistent kernel whose workgroups pull (problem, step, row-chunk) work
items.  Forced here (BCGS_BATCH_MODE=persistent, which refuses batches the
persistent kernel cannot run), every problem must give the bits it gives
alone through bcgs_qr_ex, for every variant, odd and even row counts,
single-block-column problems and a breakdown, over replays with other
work in between, and the results must meet the oracle's tolerances.
Every case prints its name before touching the GPU."""

import numpy as np
import pytest

from paper_2507_21791_amd import workloads as W

from parity import compare, host, log, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _persistent(monkeypatch):
    import torch
    from paper_2507_21791_amd import bcgs
    assert torch.cuda.is_available()
    bcgs.lib()
    bcgs.tuning_clear()
    monkeypatch.setenv("BCGS_BATCH_MODE", "persistent")
    yield
    bcgs.tuning_clear()


# (m, n, s, decades, variant): every variant, s = 4, 8, 16, odd and even m,
# one block column only (n = s), the widest pass (n = 256)
MIX = [
    (3000, 64, 16, 3, "p-1s"),
    (20001, 128, 16, 4, "bcgsi+"),
    (777, 32, 8, 2, "p-2s"),
    (5000, 48, 4, 2, "p-1s"),
    (1000, 16, 16, 2, "p-1s"),
    (9001, 96, 8, 3, "pipi+"),
    (4096, 64, 16, 3, "bcgsi+1s"),
    (65001, 256, 16, 3, "p-1s"),
    (12000, 160, 16, 5, "p-2s"),
    (50, 8, 8, 1, "bcgsi+"),
]


def _inputs(mix, seed0=0):
    import torch
    return [(X, to_device(X, torch.float64)) for X in
            (W.conditioned_host(m, n, dec, seed=seed0 + 13 * i + m)
             for i, (m, n, s, dec, v) in enumerate(mix))]


def _alone(Xd, s, variant):
    import torch
    from paper_2507_21791_amd import bcgs
    Q, R, ws = bcgs.qr(Xd, s, variant)
    torch.cuda.synchronize()
    return host(Q), host(R), ws.info()


def _same_info(a, b):
    """Info records equal field by field, a NaN pivot value equal to NaN."""
    a, b = a.as_dict(), b.as_dict()
    return a.keys() == b.keys() and all(
        a[k] == b[k] or (isinstance(a[k], float) and np.isnan(a[k])
                         and np.isnan(b[k])) for k in a)


def _check(mix, inputs, batch):
    for (m, n, s, dec, v), (Xh, Xd), (Q, R, info) in zip(
            mix, inputs, batch.results()):
        Qa, Ra, ia = _alone(Xd, s, v)
        assert _same_info(info, ia), (m, n, s, v, info.as_dict(),
                                      ia.as_dict())
        if ia.status == 0:
            assert np.array_equal(host(R), Ra), (m, n, s, v)
            assert np.array_equal(host(Q), Qa), (m, n, s, v)


def _batch(mix, inputs):
    from paper_2507_21791_amd import bcgs
    return bcgs.Batch([(Xd, s, v, "fp64") for (m, n, s, d, v), (Xh, Xd)
                       in zip(mix, inputs)])


def test_persistent_equals_alone_and_oracle():
    import torch
    from paper_2507_21791_amd import bcgs
    log("[gpu] persistent batch of", len(MIX), "problems")
    inputs = _inputs(MIX)
    batch = _batch(MIX, inputs)
    bcgs.qr_batched(batch)
    torch.cuda.synchronize()
    _check(MIX, inputs, batch)
    for (m, n, s, dec, v), (Xh, Xd), (Q, R, info) in zip(
            MIX, inputs, batch.results()):
        if m * n <= 3_000_000:
            compare(Xh, s, v, host(Q), host(R), info, kappa=10.0 ** dec)


def test_persistent_replays_and_rewritten_inputs():
    import torch
    from paper_2507_21791_amd import bcgs
    mix = MIX[:6]
    inputs = _inputs(mix, seed0=100)
    batch = _batch(mix, inputs)
    for rep in range(3):
        log(f"[gpu] persistent replay {rep}")
        bcgs.qr_batched(batch)
        junk = torch.randn(1 << 20, device="cuda").sum()   # eager work
        torch.cuda.synchronize()
        del junk
        _check(mix, inputs, batch)
    for (_, Xd), (_, Xd2) in zip(inputs, _inputs(mix, seed0=200)):
        Xd.copy_(Xd2)
    log("[gpu] persistent replay on rewritten inputs")
    bcgs.qr_batched(batch)
    torch.cuda.synchronize()
    _check(mix, inputs, batch)


def test_persistent_many_uneven_problems():
    """48 problems drawn like the batched workload (smaller m): every one
    bitwise equal to its lone run."""
    import torch
    from paper_2507_21791_amd import bcgs
    rng = np.random.default_rng(77)
    mix = []
    for i in range(48):
        s = int(rng.choice([8, 16]))
        n = int(rng.choice([32, 64, 128, 256]))
        m = int(rng.integers(max(n, 2000), 30000))
        mix.append((m, n, s, float(rng.uniform(2, 6)),
                    ["p-1s", "p-2s", "bcgsi+"][i % 3]))
    log("[gpu] persistent batch of 48 uneven problems")
    inputs = _inputs(mix, seed0=300)
    batch = _batch(mix, inputs)
    bcgs.qr_batched(batch)
    torch.cuda.synchronize()
    _check(mix, inputs, batch)


def test_persistent_breakdown_matches_alone():
    """A problem with a non-finite entry breaks down in the batch exactly as
    alone (same info record: block and pivot of the first non-finite
    Cholesky pivot) and leaves its neighbours untouched."""
    import torch
    from paper_2507_21791_amd import bcgs
    log("[gpu] persistent batch with a breakdown")
    mix = [MIX[0], (4000, 64, 16, 3, "p-1s"), MIX[2]]
    inputs = _inputs(mix, seed0=400)
    Xh, Xd = inputs[1]
    Xh = np.array(Xh, order="F")
    Xh[7, 40] = np.nan
    inputs[1] = (Xh, to_device(Xh, torch.float64))
    batch = _batch(mix, inputs)
    bcgs.qr_batched(batch)
    torch.cuda.synchronize()
    _check(mix, inputs, batch)
    assert batch.results()[1][2].status == 2


def test_persistent_refuses_what_it_cannot_run():
    """Forced persistent mode refuses (status unsupported, nothing run) a
    batch with a binary32 problem or a block width above 16."""
    import torch
    from paper_2507_21791_amd import bcgs
    log("[gpu] persistent mode refuses unsupported problems")
    X = to_device(W.conditioned_host(3000, 64, 2, seed=5), torch.float32)
    with pytest.raises(bcgs.BcgsError) as e:
        bcgs.qr_batched(bcgs.Batch([(X, 16, "p-1s", "fp32-bulk")]))
    assert e.value.status == 7
    X = to_device(W.conditioned_host(3000, 64, 2, seed=6), torch.float64)
    with pytest.raises(bcgs.BcgsError) as e:
        bcgs.qr_batched(bcgs.Batch([(X, 32, "p-1s", "fp64")]))
    assert e.value.status == 7
