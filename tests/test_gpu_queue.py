"""Request queue with continuous batching on the GPU, through the C ABI.

Each request must give the bits it gives alone through bcgs_qr_ex, whatever
else runs beside it; requests must overlap on the device when slots and
memory allow, and never exceed the memory budget when they do not; one
request's breakdown must not touch the others.  Every case prints its name
before touching the GPU.
"""

import threading

import numpy as np
import pytest

import oracle as O
from paper_2507_21791_amd import workloads as W

from parity import compare, host, log, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    from paper_2507_21791_amd import bcgs
    assert torch.cuda.is_available()
    bcgs.lib()
    yield
    bcgs.lib().bcgs_release()


MIX = [  # (m, n, s, decades, variant, precision)
    (3000, 64, 16, 3, "p-1s", "fp64"),
    (60000, 128, 16, 4, "p-1s", "fp64"),
    (777, 32, 8, 2, "p-2s", "fp64"),
    (20000, 96, 32, 3, "bcgsi+", "fp64"),
    (40000, 64, 16, 2, "p-1s", "fp32-bulk"),
    (5000, 48, 4, 2, "p-1s", "fp64"),
    (150000, 256, 16, 3, "p-1s", "fp64"),
    (9000, 32, 8, 1, "p-2s", "fp32-bulk"),
]


def _inputs(mix, seed0=0):
    import torch
    out = []
    for i, (m, n, s, dec, v, p) in enumerate(mix):
        X = W.conditioned_host(m, n, dec, seed=seed0 + 17 * i + m)
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


def _overlaps(res):
    iv = sorted((r["t_start"], r["t_done"]) for r in res)
    return any(b[0] < a[1] for a, b in zip(iv, iv[1:]))


def test_queue_mix_equals_alone_and_overlaps():
    from paper_2507_21791_amd import bcgs
    log("[gpu] queue mix, 4 slots")
    mix = MIX * 2
    inputs = _inputs(mix)
    q = bcgs.Queue(hbm_budget_bytes=64 << 30, max_inflight=4)
    try:
        tickets = [q.submit(Xd, s, v, p) for (m, n, s, d, v, p), (_, Xd)
                   in zip(mix, inputs)]
        res = [q.wait(t) for t in tickets]
    finally:
        q.close()
    for r in res:
        assert r["status"] == 0
        assert r["t_submit"] <= r["t_start"] <= r["t_done"]
    assert _overlaps(res), "no two requests ever ran together"
    for (m, n, s, dec, v, p), (Xh, Xd), r in zip(mix, inputs, res):
        Qa, Ra, ia = _alone(Xd, s, v, p)
        assert np.array_equal(host(r["R"]), Ra), (m, n, s, v, p)
        assert np.array_equal(host(r["Q"]), Qa), (m, n, s, v, p)
    (m, n, s, dec, v, p), (Xh, Xd), r = mix[0], inputs[0], res[0]
    compare(Xh, s, v, host(r["Q"]), host(r["R"]), r["info"],
            kappa=10.0 ** dec)


def test_queue_budget_admits_one_at_a_time():
    """Budget just above one request's footprint: requests never overlap."""
    from paper_2507_21791_amd import bcgs
    log("[gpu] queue tight budget")
    mix = [(60000, 128, 16, 3, "p-1s", "fp64")] * 4
    inputs = _inputs(mix, seed0=50)
    m, n, s = 60000, 128, 16
    ws = bcgs.workspace_size(m, n, s, "p-1s")
    one = 2 * m * n * 8 + n * n * 8 + ws
    q = bcgs.Queue(hbm_budget_bytes=int(one * 1.5), max_inflight=4)
    try:
        tickets = [q.submit(Xd, s, "p-1s") for _, Xd in inputs]
        res = [q.wait(t) for t in tickets]
    finally:
        q.close()
    assert all(r["status"] == 0 for r in res)
    assert not _overlaps(res)
    # admitted in arrival order
    starts = [r["t_start"] for r in res]
    assert starts == sorted(starts)


def test_queue_breakdown_is_isolated():
    """A P-1S request with a non-finite entry breaks down (a non-finite
    Cholesky pivot in the block holding it); the others finish with the
    bits they give alone."""
    import torch
    from paper_2507_21791_amd import bcgs
    log("[gpu] queue breakdown isolation")
    mix = MIX[:3]
    inputs = _inputs(mix, seed0=70)
    Xbad = W.conditioned_host(4000, 64, 2, seed=9)
    Xbad[7, 40] = np.nan
    Xbad_d = to_device(Xbad, torch.float64)
    q = bcgs.Queue(hbm_budget_bytes=64 << 30, max_inflight=3)
    try:
        tb = q.submit(Xbad_d, 16, "p-1s")
        tickets = [q.submit(Xd, s, v, p) for (m, n, s, d, v, p), (_, Xd)
                   in zip(mix, inputs)]
        rb = q.wait(tb)
        res = [q.wait(t) for t in tickets]
    finally:
        q.close()
    assert rb["status"] == bcgs.BCGS_ERR_BREAKDOWN
    want = O.qr(Xbad, 16, "p-1s").breakdown
    assert want is not None
    assert (rb["info"].block, rb["info"].pivot) == (want.block, want.pivot)
    for (m, n, s, dec, v, p), (Xh, Xd), r in zip(mix, inputs, res):
        assert r["status"] == 0
        Qa, Ra, _ = _alone(Xd, s, v, p)
        assert np.array_equal(host(r["R"]), Ra)
        assert np.array_equal(host(r["Q"]), Qa)


def test_queue_poll_and_threads():
    """Submissions from several threads; poll until done; a collected
    ticket is forgotten."""
    import time
    from paper_2507_21791_amd import bcgs
    log("[gpu] queue threads + poll")
    inputs = _inputs(MIX[:6], seed0=90)
    q = bcgs.Queue(hbm_budget_bytes=64 << 30, max_inflight=8)
    tickets = [None] * len(inputs)

    def sub(i):
        (m, n, s, d, v, p), (_, Xd) = MIX[i], inputs[i]
        tickets[i] = q.submit(Xd, s, v, p)

    try:
        th = [threading.Thread(target=sub, args=(i,))
              for i in range(len(inputs))]
        for t in th:
            t.start()
        for t in th:
            t.join()
        assert len(set(tickets)) == len(tickets)
        res = {}
        deadline = time.time() + 60
        while len(res) < len(tickets) and time.time() < deadline:
            for t in tickets:
                if t not in res:
                    r = q.poll(t)
                    if r is not None:
                        res[t] = r
            time.sleep(0.001)
        assert len(res) == len(tickets)
        assert all(r["status"] == 0 for r in res.values())
        with pytest.raises(bcgs.BcgsError):
            q.poll(tickets[0])
    finally:
        q.close()


def _copy_out(ptr, m, n, dtype):
    """Column-major m x n device buffer at `ptr` -> host float64 array."""
    import ctypes
    import torch
    torch.cuda.synchronize()
    hip = ctypes.CDLL("libamdhip64.so")
    buf = np.empty((n, m), dtype=dtype)
    rc = hip.hipMemcpy(ctypes.c_void_p(buf.ctypes.data), ctypes.c_void_p(ptr),
                       ctypes.c_size_t(buf.nbytes), 2)   # device to host
    assert rc == 0, rc
    return np.asfortranarray(buf.T.astype(np.float64))


def test_queue_owned_outputs_equal_alone():
    """Q and R left to the queue (allocated at admission from the
    stream-ordered pool): same bits as a lone run; released afterwards."""
    from paper_2507_21791_amd import bcgs
    log("[gpu] queue-owned outputs")
    mix = MIX[:5]
    inputs = _inputs(mix, seed0=110)
    q = bcgs.Queue(hbm_budget_bytes=64 << 30, max_inflight=4,
                   output_arena_bytes=1 << 30)
    try:
        tickets = [q.submit(Xd, s, v, p, outputs="queue")
                   for (m, n, s, d, v, p), (_, Xd) in zip(mix, inputs)]
        res = [q.wait(t) for t in tickets]
        for (m, n, s, dec, v, p), (Xh, Xd), r in zip(mix, inputs, res):
            assert r["status"] == 0 and r["Q_ptr"] and r["R_ptr"]
            Qa, Ra, _ = _alone(Xd, s, v, p)
            dt = np.float64 if p == "fp64" else np.float32
            assert np.array_equal(_copy_out(r["R_ptr"], n, n, np.float64), Ra)
            assert np.array_equal(_copy_out(r["Q_ptr"], m, n, dt), Qa)
            q.free(r["Q_ptr"])
            q.free(r["R_ptr"])
    finally:
        q.close()


def test_queue_arena_space_gates_admission():
    """An arena that holds the outputs of one request at a time: requests
    wait for space (never overlap), every output is correct, and a request
    whose outputs can never fit is refused at submission."""
    import torch
    from paper_2507_21791_amd import bcgs
    log("[gpu] queue arena admission")
    m, n, s = 30001, 64, 16
    mix = [(m, n, s, 2, "p-1s", "fp64")] * 4
    inputs = _inputs(mix, seed0=130)
    one = m * n * 8 + n * n * 8 + 512
    q = bcgs.Queue(hbm_budget_bytes=64 << 30, max_inflight=4,
                   output_arena_bytes=int(one * 1.5))
    try:
        big = to_device(W.conditioned_host(2 * m, n, 1, seed=1),
                        torch.float64)
        with pytest.raises(bcgs.BcgsError):
            q.submit(big, s, "p-1s", outputs="queue")
        tickets = [q.submit(Xd, s, "p-1s", outputs="queue")
                   for _, Xd in inputs]
        res = []
        for t, (Xh, Xd) in zip(tickets, inputs):
            r = q.wait(t)
            assert r["status"] == 0
            Qa, Ra, _ = _alone(Xd, s, "p-1s", "fp64")
            assert np.array_equal(_copy_out(r["Q_ptr"], m, n, np.float64), Qa)
            q.free(r["Q_ptr"])
            q.free(r["R_ptr"])
            res.append(r)
    finally:
        q.close()
    assert not _overlaps(res)


def test_queue_retries_breakdown_with_stable_variant():
    """kappa = 1e12: BCGSI+P-1S breaks down (u kappa^2 >> 1) while
    BCGSI+P-2S holds O(u) orthogonality (u kappa <= 1, Table 1).  With
    retry enabled the request is rerun once as P-2S into the same outputs:
    status ok, variant p-2s, two attempts, the bits of a lone P-2S run and
    the oracle's P-2S tolerances; without retry it reports the breakdown."""
    import torch
    from paper_2507_21791_amd import bcgs
    log("[gpu] queue retry on breakdown")
    X = W.conditioned_host(3000, 64, 12, seed=1)
    Xd = to_device(X, torch.float64)
    want = O.qr(X, 16, "p-1s").breakdown
    assert want is not None
    q = bcgs.Queue(hbm_budget_bytes=8 << 30, max_inflight=2,
                   output_arena_bytes=64 << 20, retry_variant="p-2s")
    q0 = bcgs.Queue(hbm_budget_bytes=8 << 30, max_inflight=2)
    try:
        t = q.submit(Xd, 16, "p-1s")
        r = q.wait(t)
        tq = q.submit(Xd, 16, "p-1s", outputs="queue")
        rq = q.wait(tq)
        r0 = q0.wait(q0.submit(Xd, 16, "p-1s"))
        assert rq["status"] == 0 and rq["attempts"] == 2
        Qq = _copy_out(rq["Q_ptr"], 3000, 64, np.float64)
        q.free(rq["Q_ptr"])
        q.free(rq["R_ptr"])
    finally:
        q.close()
        q0.close()
    assert r0["status"] == bcgs.BCGS_ERR_BREAKDOWN and r0["attempts"] == 1
    # far past Table 1's assumption the failing pivot is a rounding-order
    # matter; the failing block is the parity criterion
    assert r0["info"].block == want.block, (r0["info"].as_dict(), want)
    assert r["status"] == 0 and r["variant"] == "p-2s" and r["attempts"] == 2
    Qa, Ra, _ = _alone(Xd, 16, "p-2s", "fp64")
    assert np.array_equal(host(r["R"]), Ra)
    assert np.array_equal(host(r["Q"]), Qa)
    assert np.array_equal(Qq, Qa)
    compare(X, 16, "p-2s", host(r["Q"]), host(r["R"]), r["info"], kappa=1e12)


def test_queue_orders_after_async_write_of_x():
    """X written asynchronously on the caller's stream (a large device copy
    from a second buffer and a scaling kernel, no synchronization) and
    submitted straight away: every request reads the finished X, so its
    result equals the one computed on X after a synchronization."""
    import torch
    from paper_2507_21791_amd import bcgs
    log("[gpu] queue: submit right after an asynchronous write of X")
    m, n, s = 200000, 128, 16
    src = to_device(W.conditioned_host(m, n, 3, seed=91), torch.float64)
    q = bcgs.Queue(hbm_budget_bytes=8 << 30, max_inflight=4)
    outs = []
    try:
        for k in range(4):
            X = bcgs.empty_fortran(m, n, torch.float64, "cuda")
            X.fill_(float("nan"))          # what a too-early read would see
            X.copy_(src)                   # enqueued, not waited for
            X.mul_(2.0 ** k)               # exact scaling, still pending
            t = q.submit(X, s, "p-1s")
            outs.append((k, X, q.wait(t)))
    finally:
        q.close()
    torch.cuda.synchronize()
    for k, X, r in outs:
        assert r["status"] == 0, r
        Qa, Ra, ws = bcgs.qr(X, s, "p-1s")
        torch.cuda.synchronize()
        assert torch.equal(r["Q"], Qa) and torch.equal(r["R"], Ra), k
