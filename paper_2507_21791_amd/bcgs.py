"""Python binding of the C ABI in include/bcgs.h (argument marshalling only).

Every step of the factorization runs in the gfx950 library
``_lib/libbcgs.so``; PyTorch supplies device memory and the stream.  If the
library is missing this module raises: there is no fallback path.

Matrices are torch tensors in column-major order: shape (m, n) with
strides (1, ld) -- e.g. ``torch.empty(n, m).t()``.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libbcgs.so")

VARIANTS = {"bcgsi+": 0, "p-2s": 1, "p-1s": 2, "pipi+": 3, "bcgsi+1s": 4}
PRECISIONS = {"fp64": 0, "fp32-bulk": 1}
STATUS = {0: "ok", 1: "invalid argument", 2: "Cholesky breakdown",
          3: "out of device memory", 4: "HIP runtime error", 5: "queue full",
          6: "pending", 7: "unsupported"}
BCGS_OK, BCGS_ERR_ARG, BCGS_ERR_BREAKDOWN = 0, 1, 2


class Info(ctypes.Structure):
    """Mirror of bcgs_info."""
    _fields_ = [("status", ctypes.c_int32), ("block", ctypes.c_int32),
                ("pivot", ctypes.c_int32), ("stage", ctypes.c_int32),
                ("syncs", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("value", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


INFO_BYTES = ctypes.sizeof(Info)

KERNEL_KINDS = {0: "pass", 1: "reduce", 2: "epilogue", 3: "tsqr_leaf",
                4: "tsqr_node", 5: "tsqr_down", 6: "tsqr_apply", 7: "other"}


class LaunchRecord(ctypes.Structure):
    """Mirror of bcgs_launch_record."""
    _fields_ = [("kind", ctypes.c_int32), ("tag", ctypes.c_int32),
                ("ms", ctypes.c_double), ("bytes", ctypes.c_double),
                ("flops", ctypes.c_double), ("name", ctypes.c_char * 112)]


class Problem(ctypes.Structure):
    """Mirror of bcgs_problem."""
    _fields_ = [("X", ctypes.c_void_p), ("Q", ctypes.c_void_p),
                ("R", ctypes.c_void_p), ("m", ctypes.c_int64),
                ("n", ctypes.c_int64), ("s", ctypes.c_int64),
                ("ldx", ctypes.c_int64), ("ldq", ctypes.c_int64),
                ("ldr", ctypes.c_int64), ("variant", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("d_info", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    """Mirror of bcgs_tuning."""
    _fields_ = [("max_wg", ctypes.c_int32), ("shape", ctypes.c_int32)]


class QueueConfig(ctypes.Structure):
    """Mirror of bcgs_queue_config."""
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t),
                ("max_inflight", ctypes.c_int32), ("device", ctypes.c_int32),
                ("output_arena_bytes", ctypes.c_size_t),
                ("retry_on_breakdown", ctypes.c_int32),
                ("retry_variant", ctypes.c_int32),
                ("admission", ctypes.c_int32), ("reserved", ctypes.c_int32)]


ADMISSION = {"arrival": 0, "shortest": 1}


class RequestStats(ctypes.Structure):
    """Mirror of bcgs_request_stats."""
    _fields_ = [("status", ctypes.c_int), ("info", Info),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double), ("Q", ctypes.c_void_p),
                ("R", ctypes.c_void_p), ("variant", ctypes.c_int32),
                ("attempts", ctypes.c_int32)]


_lib = None

_PROTOS = {
    "bcgs_qr": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64,
                               ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                               ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p]),
    "bcgs_qr_ex": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64,
                                  ctypes.c_int64, ctypes.c_int64,
                                  ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_void_p, ctypes.c_int64,
                                  ctypes.c_void_p, ctypes.c_int64,
                                  ctypes.c_void_p, ctypes.c_size_t,
                                  ctypes.c_void_p, ctypes.c_void_p]),
    "bcgs_qr_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_int64, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_void_p,
                                       ctypes.c_int64, ctypes.c_void_p,
                                       ctypes.c_int64, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "bcgs_workspace_size": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int64,
                                              ctypes.c_int64, ctypes.c_int,
                                              ctypes.c_int]),
    "bcgs_sync_count": (ctypes.c_int32, [ctypes.c_int64, ctypes.c_int64,
                                         ctypes.c_int64, ctypes.c_int]),
    "bcgs_get_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Info)]),
    "bcgs_release": (None, []),
    "bcgs_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "bcgs_qr_batched": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.c_void_p]),
    "bcgs_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.c_void_p]),
    "bcgs_tuning_get": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_int64, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_void_p]),
    "bcgs_tuning_set": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_int64, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_void_p]),
    "bcgs_tuning_clear": (None, []),
    "bcgs_queue_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "bcgs_queue_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "bcgs_queue_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64,
                                       ctypes.c_void_p]),
    "bcgs_queue_wait": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64,
                                       ctypes.c_void_p]),
    "bcgs_queue_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "bcgs_queue_free_output": (ctypes.c_int, [ctypes.c_void_p,
                                              ctypes.c_void_p,
                                              ctypes.c_void_p]),
    "bcgs_check_workspace_size": (ctypes.c_size_t, [ctypes.c_int64,
                                                    ctypes.c_int64]),
    "bcgs_check": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int64,
                                  ctypes.c_void_p, ctypes.c_int64,
                                  ctypes.c_void_p, ctypes.c_int64,
                                  ctypes.c_int64, ctypes.c_int64,
                                  ctypes.c_int, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_int64, ctypes.c_void_p,
                                  ctypes.c_size_t, ctypes.c_void_p]),
    "bcgs_profile_start": (ctypes.c_int, [ctypes.c_void_p]),
    "bcgs_profile_stop": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_int32]),
}


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2507_21791_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class BcgsError(RuntimeError):
    def __init__(self, status, what=""):
        super().__init__(f"{what}: {STATUS.get(status, status)}")
        self.status = status


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _col_major(t, name):
    if t.dim() != 2 or t.stride(0) != 1 or t.stride(1) < max(1, t.shape[0]):
        raise ValueError(f"{name} must be a column-major (m, n) tensor with "
                         f"strides (1, ld >= m); got strides {t.stride()}")
    return t.stride(1)


def workspace_size(m, n, s, variant="p-1s", precision="fp64"):
    return lib().bcgs_workspace_size(m, n, s, VARIANTS[variant],
                                     PRECISIONS[precision])


def sync_count(m, n, s, variant):
    return lib().bcgs_sync_count(m, n, s, VARIANTS[variant])


def empty_fortran(m, n, dtype, device, ld=None):
    """Uninitialised m x n column-major tensor with leading dimension ld
    (default m): strides (1, ld)."""
    import torch
    ld = m if ld is None else ld
    if ld < m:
        raise ValueError(f"leading dimension {ld} < rows {m}")
    return torch.empty((n, ld), dtype=dtype, device=device)[:, :m].t()


class Workspace:
    """Device workspace + info record for repeated factorizations."""

    def __init__(self, m, n, s, variant="p-1s", precision="fp64",
                 device="cuda"):
        import torch
        nbytes = workspace_size(m, n, s, variant, precision)
        if nbytes == 0:
            raise BcgsError(BCGS_ERR_ARG, "workspace_size")
        self.nbytes = nbytes
        self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.buf.data_ptr()) % 256
        self.ptr = self.buf.data_ptr() + off
        self.info_buf = torch.zeros(64, dtype=torch.uint8, device=device)

    def info(self):
        """Copy the info record to the host (synchronizes on the copy)."""
        raw = self.info_buf[:INFO_BYTES].cpu().numpy().tobytes()
        return Info.from_buffer_copy(raw)


def qr(X, s, variant="p-1s", precision="fp64", Q=None, R=None, ws=None,
       stream=None):
    """Enqueue X = Q R on the current stream; returns (Q, R, ws).

    ``ws.info()`` reads the breakdown record after the work has finished."""
    import torch
    m, n = X.shape
    ldx = _col_major(X, "X")
    want = torch.float64 if precision == "fp64" else torch.float32
    if X.dtype != want:
        raise ValueError(f"X must be {want} for precision {precision}")
    if Q is None:
        Q = empty_fortran(m, n, want, X.device)
    ldq = _col_major(Q, "Q")
    if R is None:
        R = empty_fortran(n, n, torch.float64, X.device)
    ldr = _col_major(R, "R")
    if ws is None:
        ws = Workspace(m, n, s, variant, precision, X.device)
    st = lib().bcgs_qr_ex(
        ctypes.c_void_p(X.data_ptr()), ldx, m, n, s, VARIANTS[variant],
        PRECISIONS[precision], ctypes.c_void_p(Q.data_ptr()), ldq,
        ctypes.c_void_p(R.data_ptr()), ldr, ctypes.c_void_p(ws.ptr),
        ws.nbytes, ctypes.c_void_p(ws.info_buf.data_ptr()),
        _stream_handle(stream))
    if st != BCGS_OK:
        raise BcgsError(st, "bcgs_qr_ex")
    return Q, R, ws


NOALLOC_SCRATCH_BYTES = 64 << 20    # BCGS_NOALLOC_SCRATCH_BYTES


def qr_noalloc(X, s, variant, precision, Q, R, info_buf, stream=None):
    """bcgs_qr_noalloc: the factorization with the library's fixed device
    scratch array as workspace (the caller passes every output: Q, R and a
    device buffer of at least INFO_BYTES for the info record)."""
    m, n = X.shape
    st = lib().bcgs_qr_noalloc(
        ctypes.c_void_p(X.data_ptr()), _col_major(X, "X"), m, n, s,
        VARIANTS[variant], PRECISIONS[precision],
        ctypes.c_void_p(Q.data_ptr()), _col_major(Q, "Q"),
        ctypes.c_void_p(R.data_ptr()), _col_major(R, "R"),
        ctypes.c_void_p(info_buf.data_ptr()), _stream_handle(stream))
    if st != BCGS_OK:
        raise BcgsError(st, "bcgs_qr_noalloc")
    return Q, R


def qr_simple(X, s, variant, Q, R, stream=None):
    """The library-owned-workspace entry point bcgs_qr (ld = m, n)."""
    m, n = X.shape
    st = lib().bcgs_qr(ctypes.c_void_p(X.data_ptr()), m, n, s,
                       VARIANTS[variant], ctypes.c_void_p(Q.data_ptr()),
                       ctypes.c_void_p(R.data_ptr()), _stream_handle(stream))
    if st != BCGS_OK:
        raise BcgsError(st, "bcgs_qr")
    return Q, R


def profile_start(stream=None):
    lib().bcgs_profile_start(_stream_handle(stream))


def profile_stop(stream=None, capacity=1 << 16):
    """Stop profiling the stream; returns a list of launch dicts
    (kind, tag, name, ms, bytes, flops) in launch order."""
    recs = (LaunchRecord * capacity)()
    n = lib().bcgs_profile_stop(_stream_handle(stream), recs, capacity)
    if n < 0:
        raise BcgsError(BCGS_ERR_ARG, "bcgs_profile_stop")
    return [{"kind": KERNEL_KINDS.get(r.kind, r.kind), "tag": r.tag,
             "name": r.name.decode(), "ms": r.ms, "bytes": r.bytes,
             "flops": r.flops}
            for r in recs[:min(n, capacity)]]


def get_info(stream=None):
    info = Info()
    st = lib().bcgs_get_info(_stream_handle(stream), ctypes.byref(info))
    if st != BCGS_OK:
        raise BcgsError(st, "bcgs_get_info")
    return info


class Checker:
    """bcgs_check with a reusable device workspace and Gram buffers.

    ``grams`` enqueues the three n x n Gram matrices (Q^T Q, E^T E with
    E = X - Q R, X^T X) on the stream and returns them as device tensors;
    ``measures`` turns them into the loss of orthogonality and the relative
    residual: largest absolute eigenvalues of the small symmetric matrices,
    taken on the host."""

    def __init__(self, device="cuda"):
        self.device = device
        self.ws = None
        self.nbytes = 0
        self.G = None

    def grams(self, X, Q, R, precision="fp64", stream=None):
        import torch
        m, n = X.shape
        need = lib().bcgs_check_workspace_size(m, n)
        if need == 0:
            raise BcgsError(BCGS_ERR_ARG, "bcgs_check_workspace_size")
        if need > self.nbytes:
            self.ws = torch.empty(need + 256, dtype=torch.uint8,
                                  device=self.device)
            self.nbytes = need
        ptr = self.ws.data_ptr() + (-self.ws.data_ptr()) % 256
        G = torch.empty((3, n, n), dtype=torch.float64, device=self.device)
        st = lib().bcgs_check(
            ctypes.c_void_p(X.data_ptr()), _col_major(X, "X"),
            ctypes.c_void_p(Q.data_ptr()), _col_major(Q, "Q"),
            ctypes.c_void_p(R.data_ptr()), _col_major(R, "R"), m, n,
            PRECISIONS[precision], ctypes.c_void_p(G[0].data_ptr()),
            ctypes.c_void_p(G[1].data_ptr()), ctypes.c_void_p(G[2].data_ptr()),
            n, ctypes.c_void_p(ptr), self.nbytes, _stream_handle(stream))
        if st != BCGS_OK:
            raise BcgsError(st, "bcgs_check")
        return G

    @staticmethod
    def measures(G):
        import numpy as np
        g = G.cpu().numpy()

        def norm2(M):
            M = 0.5 * (M + M.T)
            return float(np.max(np.abs(np.linalg.eigvalsh(M))))
        n = g.shape[1]
        loo = norm2(g[0] - np.eye(n))
        res = max(norm2(g[1]), 0.0) ** 0.5 / norm2(g[2]) ** 0.5
        return loo, res

    def __call__(self, X, Q, R, precision="fp64", stream=None):
        """(loss of orthogonality, relative residual); synchronizes."""
        return self.measures(self.grams(X, Q, R, precision, stream))


class Batch:
    """A list of problems with device outputs and one info record each, in
    the layout bcgs_qr_batched takes.  Keeps the tensors alive."""

    INFO_STRIDE = 128

    def __init__(self, items, device="cuda"):
        """items: iterable of (X, s, variant, precision) with X a column-major
        device tensor (float64 for fp64, float32 for fp32-bulk)."""
        import torch
        self.items = []
        arr = []
        self.info_buf = None
        items = list(items)
        # one 128-byte cache line per info record: no two problems write
        # the same line
        self.info_buf = torch.zeros(max(1, len(items)) * self.INFO_STRIDE,
                                    dtype=torch.uint8, device=device)
        for i, (X, s, variant, precision) in enumerate(items):
            m, n = X.shape
            ldx = _col_major(X, "X")
            want = torch.float64 if precision == "fp64" else torch.float32
            if X.dtype != want:
                raise ValueError(f"X must be {want} for precision {precision}")
            Q = empty_fortran(m, n, want, X.device)
            R = empty_fortran(n, n, torch.float64, X.device)
            self.items.append((X, Q, R, s, variant, precision))
            arr.append(Problem(X.data_ptr(), Q.data_ptr(), R.data_ptr(), m, n,
                               s, ldx, Q.stride(1), R.stride(1),
                               VARIANTS[variant], PRECISIONS[precision],
                               self.info_buf.data_ptr() +
                               i * self.INFO_STRIDE))
        self.array = (Problem * max(1, len(arr)))(*arr)
        self.count = len(arr)

    def results(self):
        """[(Q, R, Info)] in input order (synchronizes on the info copy)."""
        raw = self.info_buf.cpu().numpy().tobytes()
        k = self.INFO_STRIDE
        return [(Q, R, Info.from_buffer_copy(raw[i * k:i * k + INFO_BYTES]))
                for i, (_, Q, R, *_r) in enumerate(self.items)]


def qr_batched(batch, stream=None):
    """Enqueue every problem of `batch` (a Batch) as one graph launch."""
    st = lib().bcgs_qr_batched(ctypes.byref(batch.array), batch.count,
                               _stream_handle(stream))
    if st != BCGS_OK:
        raise BcgsError(st, "bcgs_qr_batched")
    return batch


def autotune(batch, stream=None):
    """Tune every problem class of `batch` that has no entry yet."""
    st = lib().bcgs_autotune(ctypes.byref(batch.array), batch.count,
                             _stream_handle(stream))
    if st != BCGS_OK:
        raise BcgsError(st, "bcgs_autotune")


def tuning_get(m, n, s, variant, precision="fp64"):
    """(max_wg, shape, tuned) of a problem class."""
    t = Tuning()
    st = lib().bcgs_tuning_get(m, n, s, VARIANTS[variant],
                               PRECISIONS[precision], ctypes.byref(t))
    if st not in (BCGS_OK, 6):
        raise BcgsError(st, "bcgs_tuning_get")
    return t.max_wg, t.shape, st == BCGS_OK


def tuning_set(m, n, s, variant, precision="fp64", max_wg=None, shape=-1):
    """Set the entry of a class (max_wg None erases it)."""
    ptr = None
    if max_wg is not None:
        ptr = ctypes.byref(Tuning(max_wg, shape))
    st = lib().bcgs_tuning_set(m, n, s, VARIANTS[variant],
                               PRECISIONS[precision], ptr)
    if st != BCGS_OK:
        raise BcgsError(st, "bcgs_tuning_set")


def tuning_clear():
    lib().bcgs_tuning_clear()


BCGS_PENDING = 6


class Queue:
    """Request queue with continuous batching (bcgs_queue_*).  Holds the
    tensors of every request until it is collected."""

    def __init__(self, hbm_budget_bytes, max_inflight=8, device=0,
                 output_arena_bytes=0, retry_variant=None,
                 admission="arrival"):
        """retry_variant: variant name a request that breaks down is rerun
        with once (e.g. "p-2s"), or None.  admission: "arrival" (oldest
        first) or "shortest" (least estimated work net of waiting time)."""
        self.handle = ctypes.c_void_p()
        cfg = QueueConfig(int(hbm_budget_bytes), int(max_inflight),
                          int(device), int(output_arena_bytes),
                          0 if retry_variant is None else 1,
                          0 if retry_variant is None
                          else VARIANTS[retry_variant],
                          ADMISSION[admission], 0)
        st = lib().bcgs_queue_create(ctypes.byref(cfg),
                                     ctypes.byref(self.handle))
        if st != BCGS_OK:
            raise BcgsError(st, "bcgs_queue_create")
        self.live = {}

    def submit(self, X, s, variant="p-1s", precision="fp64", Q=None, R=None,
               outputs="caller", stream=None):
        """Submit X = QR; returns the ticket.  outputs="caller": Q and R are
        torch tensors (allocated here when not given); outputs="queue": the
        queue carves them out of its output arena at admission and the
        result carries their device pointers (return them with free()).
        The tensors and a device info record stay alive until the request
        is collected.  The request runs after everything enqueued so far on
        `stream` (the current stream by default), which may still be
        writing X."""
        import torch
        m, n = X.shape
        ldx = _col_major(X, "X")
        want = torch.float64 if precision == "fp64" else torch.float32
        if X.dtype != want:
            raise ValueError(f"X must be {want} for precision {precision}")
        if outputs == "queue":
            Q = R = None
            qp = rp = None
            ldq, ldr = m, n
        else:
            if Q is None:
                Q = empty_fortran(m, n, want, X.device)
            if R is None:
                R = empty_fortran(n, n, torch.float64, X.device)
            qp, rp = Q.data_ptr(), R.data_ptr()
            ldq, ldr = _col_major(Q, "Q"), _col_major(R, "R")
        # no kernel here: the request's own first kernel initializes the
        # record, on the queue's stream
        info = torch.empty(INFO_BYTES, dtype=torch.uint8, device=X.device)
        prob = Problem(X.data_ptr(), qp, rp, m, n, s, ldx, ldq, ldr,
                       VARIANTS[variant], PRECISIONS[precision],
                       info.data_ptr())
        t = ctypes.c_uint64()
        st = lib().bcgs_queue_submit(self.handle, ctypes.byref(prob),
                                     _stream_handle(stream), ctypes.byref(t))
        if st != BCGS_OK:
            raise BcgsError(st, "bcgs_queue_submit")
        self.live[t.value] = (X, Q, R, info)
        return t.value

    def _finish(self, fn, ticket):
        out = RequestStats()
        st = fn(self.handle, ticket, ctypes.byref(out))
        if st == BCGS_PENDING:
            return None
        if st == BCGS_ERR_ARG and ticket not in self.live:
            raise BcgsError(st, "unknown ticket")
        X, Q, R, info = self.live.pop(ticket)
        return {"status": st, "info": out.info, "t_submit": out.t_submit,
                "t_start": out.t_start, "t_done": out.t_done, "Q": Q, "R": R,
                "Q_ptr": out.Q, "R_ptr": out.R,
                "variant": {v: k for k, v in VARIANTS.items()}[out.variant],
                "attempts": out.attempts}

    def free(self, ptr, stream=None):
        """Return a queue-allocated Q or R to the arena once the work on
        `stream` (the current stream by default) so far has finished."""
        if ptr:
            st = lib().bcgs_queue_free_output(self.handle, ctypes.c_void_p(ptr),
                                              _stream_handle(stream))
            if st != BCGS_OK:
                raise BcgsError(st, "bcgs_queue_free_output")

    def poll(self, ticket):
        """None while pending, else a dict (status, info, times, Q, R)."""
        return self._finish(lib().bcgs_queue_poll, ticket)

    def wait(self, ticket):
        return self._finish(lib().bcgs_queue_wait, ticket)

    def close(self):
        if self.handle:
            st = lib().bcgs_queue_destroy(self.handle)
            self.handle = ctypes.c_void_p()
            self.live.clear()
            if st != BCGS_OK:
                raise BcgsError(st, "bcgs_queue_destroy")
