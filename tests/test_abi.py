"""The C ABI on the CPU: the library loads, exports every function bcgs.h
declares, sizes workspaces, reports sync counts, and rejects bad arguments
synchronously (before any device work)."""

import ctypes
import os
import re

import pytest

from paper_2507_21791_amd import bcgs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", fn)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(bcgs_\w+)\s*\(", src,
                             flags=re.M):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    L = bcgs.lib()
    names = _declared_functions()
    assert {"bcgs_qr", "bcgs_qr_ex", "bcgs_workspace_size",
            "bcgs_sync_count", "bcgs_get_info"} <= names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_info_struct_layout():
    assert ctypes.sizeof(bcgs.Info) == 32
    assert bcgs.Info.value.offset == 24


@pytest.mark.parametrize("variant,q,want", [
    ("p-1s", 16, 17), ("p-2s", 16, 32), ("bcgsi+", 16, 61),
    ("p-1s", 1, 1), ("p-2s", 1, 1), ("bcgsi+", 1, 1), ("p-1s", 2, 3),
    ("pipi+", 16, 31), ("bcgsi+1s", 16, 17), ("pipi+", 1, 1)])
def test_sync_counts(variant, q, want):
    assert bcgs.sync_count(1000, 4 * q, 4, variant) == want


def test_workspace_size_is_modest():
    ws = bcgs.workspace_size(1 << 22, 256, 16, "p-1s")
    assert 0 < ws < 256 << 20          # partial Grams + TSQR tree, not m*n
    assert bcgs.workspace_size(100, 7, 2, "p-1s") == 0     # s does not divide n
    assert bcgs.workspace_size(5, 8, 4, "p-1s") == 0       # m < n
    assert bcgs.workspace_size(100, 128, 128, "p-1s") == 0  # s > 64


FAKE = ctypes.c_void_p(0x10000)   # never dereferenced: the checks fail first


@pytest.mark.parametrize("m,n,s,ldx,ldq,ldr,variant,prec", [
    (100, 8, 3, 100, 100, 8, 2, 0),     # s does not divide n
    (7, 8, 4, 7, 7, 8, 2, 0),           # m < n
    (100, 8, 0, 100, 100, 8, 2, 0),     # s < 1
    (100, 8, 4, 99, 100, 8, 2, 0),      # ldx < m
    (100, 8, 4, 100, 50, 8, 2, 0),      # ldq < m
    (100, 8, 4, 100, 100, 7, 2, 0),     # ldr < n
    (100, 8, 4, 100, 100, 8, 9, 0),     # unknown variant
    (100, 8, 4, 100, 100, 8, 2, 5),     # unknown precision
])
def test_bad_arguments_rejected_synchronously(m, n, s, ldx, ldq, ldr,
                                              variant, prec):
    L = bcgs.lib()
    st = L.bcgs_qr_ex(FAKE, ldx, m, n, s, variant, prec,
                      ctypes.c_void_p(0x9000000), ldq,
                      ctypes.c_void_p(0x20000000), ldr,
                      ctypes.c_void_p(0x40000000), 1 << 40,
                      ctypes.c_void_p(0x80000000), None)
    assert st == bcgs.BCGS_ERR_ARG


def test_null_and_aliasing_rejected():
    L = bcgs.lib()
    args = dict(m=100, n=8, s=4)
    # null workspace
    assert L.bcgs_qr_ex(FAKE, 100, 100, 8, 4, 2, 0, ctypes.c_void_p(0x900000),
                        100, ctypes.c_void_p(0x2000000), 8, None, 1 << 30,
                        ctypes.c_void_p(0x8000000), None) == bcgs.BCGS_ERR_ARG
    # Q overlapping X
    assert L.bcgs_qr_ex(ctypes.c_void_p(0x100000), 100, 100, 8, 4, 2, 0,
                        ctypes.c_void_p(0x100000 + 800), 100,
                        ctypes.c_void_p(0x2000000), 8,
                        ctypes.c_void_p(0x4000000), 1 << 30,
                        ctypes.c_void_p(0x8000000), None) == bcgs.BCGS_ERR_ARG
    # workspace too small
    assert L.bcgs_qr_ex(FAKE, 100, 100, 8, 4, 2, 0, ctypes.c_void_p(0x900000),
                        100, ctypes.c_void_p(0x2000000), 8,
                        ctypes.c_void_p(0x4000000), 16,
                        ctypes.c_void_p(0x8000000), None) == bcgs.BCGS_ERR_ARG
    # misaligned workspace
    assert L.bcgs_qr_ex(FAKE, 100, 100, 8, 4, 2, 0, ctypes.c_void_p(0x900000),
                        100, ctypes.c_void_p(0x2000000), 8,
                        ctypes.c_void_p(0x4000008), 1 << 30,
                        ctypes.c_void_p(0x8000000), None) == bcgs.BCGS_ERR_ARG
    assert L.bcgs_qr(None, 100, 8, 4, 2, FAKE, FAKE, None) == bcgs.BCGS_ERR_ARG
    del args


def test_noalloc_rejects_oversize_before_enqueue():
    """bcgs_qr_noalloc refuses a problem whose workspace exceeds its fixed
    array, before any device call (fake pointers are never touched)."""
    m, n, s = 1 << 22, 256, 16
    assert bcgs.workspace_size(m, n, s, "p-1s") > bcgs.NOALLOC_SCRATCH_BYTES
    fake = ctypes.c_void_p
    st = bcgs.lib().bcgs_qr_noalloc(
        fake(0x1000000000), m, m, n, s, 2, 0, fake(0x3000000000), m,
        fake(0x5000000000), n, fake(0x6000000000), None)
    assert st == 3      # BCGS_ERR_NOMEM: the problem does not fit the array
    # and the usual argument checks come first
    st = bcgs.lib().bcgs_qr_noalloc(
        fake(0x1000000000), 10, 100, 8, 4, 2, 0, fake(0x3000000000), 100,
        fake(0x5000000000), 8, fake(0x6000000000), None)
    assert st == bcgs.BCGS_ERR_ARG      # ldx < m


def test_status_strings():
    L = bcgs.lib()
    assert L.bcgs_status_string(0) == b"ok"
    assert L.bcgs_status_string(2) == b"Cholesky breakdown"


def _problem(m=100, n=8, s=4, ldx=100, ldq=100, ldr=8, variant=2, prec=0,
             X=0x100000, Q=0x9000000, R=0x20000000, info=0x80000000):
    return bcgs.Problem(X, Q, R, m, n, s, ldx, ldq, ldr, variant, prec, info)


def test_problem_struct_layout():
    assert ctypes.sizeof(bcgs.Problem) == 88
    assert bcgs.Problem.d_info.offset == 80
    assert ctypes.sizeof(bcgs.Tuning) == 8


@pytest.mark.parametrize("bad", [
    dict(s=3), dict(m=7), dict(ldx=99), dict(ldq=50), dict(ldr=7),
    dict(variant=9), dict(prec=5), dict(X=0), dict(info=0),
    dict(Q=0x100000 + 800),             # Q overlaps X
])
def test_batched_rejects_any_bad_problem_synchronously(bad):
    """One bad problem among good ones: BCGS_ERR_ARG before any device
    call (the good problems use fake pointers that are never touched)."""
    L = bcgs.lib()
    good = _problem(X=0x200000, Q=0x300000, R=0x400000, info=0x500000)
    arr = (bcgs.Problem * 2)(good, _problem(**bad))
    assert L.bcgs_qr_batched(ctypes.byref(arr), 2, None) == bcgs.BCGS_ERR_ARG
    assert L.bcgs_autotune(ctypes.byref(arr), 2, None) == bcgs.BCGS_ERR_ARG


def test_batched_count_checks():
    L = bcgs.lib()
    assert L.bcgs_qr_batched(None, -1, None) == bcgs.BCGS_ERR_ARG
    assert L.bcgs_qr_batched(None, 3, None) == bcgs.BCGS_ERR_ARG
    assert L.bcgs_qr_batched(None, 0, None) == bcgs.BCGS_OK


def test_tuning_table():
    bcgs.tuning_clear()
    assert bcgs.tuning_get(100000, 256, 16, "p-1s") == (512, -1, False)
    bcgs.tuning_set(100000, 256, 16, "p-1s", max_wg=64, shape=2)
    # the class is floor(log2 m): 65536 <= m < 131072
    assert bcgs.tuning_get(70000, 256, 16, "p-1s") == (64, 2, True)
    assert bcgs.tuning_get(131072, 256, 16, "p-1s")[2] is False
    assert bcgs.tuning_get(100000, 256, 16, "p-2s")[2] is False
    assert bcgs.tuning_get(100000, 256, 16, "p-1s", "fp32-bulk")[2] is False
    with pytest.raises(bcgs.BcgsError):
        bcgs.tuning_set(100000, 256, 16, "p-1s", max_wg=0)
    with pytest.raises(bcgs.BcgsError):
        bcgs.tuning_set(100000, 256, 16, "p-1s", max_wg=64, shape=99)
    bcgs.tuning_set(100000, 256, 16, "p-1s")          # erase
    assert bcgs.tuning_get(100000, 256, 16, "p-1s")[2] is False
    bcgs.tuning_set(100000, 256, 16, "p-1s", max_wg=32)
    bcgs.tuning_clear()
    assert bcgs.tuning_get(100000, 256, 16, "p-1s")[2] is False


@pytest.mark.parametrize("variant", ["bcgsi+", "p-2s", "p-1s", "pipi+",
                                     "bcgsi+1s"])
def test_tuning_set_every_variant(variant):
    """Every variant the entry points accept can be tuned by hand too."""
    bcgs.tuning_clear()
    bcgs.tuning_set(50000, 64, 8, variant, max_wg=128, shape=3)
    assert bcgs.tuning_get(50000, 64, 8, variant) == (128, 3, True)
    bcgs.tuning_set(50000, 64, 8, variant)            # erase
    assert bcgs.tuning_get(50000, 64, 8, variant)[2] is False
    bcgs.tuning_clear()


def test_queue_struct_layouts():
    assert ctypes.sizeof(bcgs.QueueConfig) == 40
    assert bcgs.QueueConfig.output_arena_bytes.offset == 16
    assert bcgs.QueueConfig.retry_variant.offset == 28
    assert bcgs.QueueConfig.admission.offset == 32
    assert ctypes.sizeof(bcgs.RequestStats) == 88
    assert bcgs.RequestStats.info.offset == 8
    assert bcgs.RequestStats.t_done.offset == 56
    assert bcgs.RequestStats.R.offset == 72
    assert bcgs.RequestStats.attempts.offset == 84


@pytest.mark.parametrize("budget,inflight,retry,admission", [
    (0, 4, (0, 0), 0), (1 << 30, 0, (0, 0), 0), (1 << 30, 17, (0, 0), 0),
    (1 << 30, 4, (1, 9), 0), (1 << 30, 4, (0, 0), 2),
    (1 << 30, 4, (0, 0), -1)])
def test_queue_bad_config_rejected(budget, inflight, retry, admission):
    L = bcgs.lib()
    cfg = bcgs.QueueConfig(budget, inflight, 0, 0, *retry, admission, 0)
    h = ctypes.c_void_p()
    assert L.bcgs_queue_create(ctypes.byref(cfg), ctypes.byref(h)) == \
        bcgs.BCGS_ERR_ARG
    assert L.bcgs_queue_create(None, ctypes.byref(h)) == bcgs.BCGS_ERR_ARG


def test_queue_null_handles_rejected():
    L = bcgs.lib()
    p = _problem()
    t = ctypes.c_uint64()
    out = bcgs.RequestStats()
    assert L.bcgs_queue_submit(None, ctypes.byref(p), None,
                               ctypes.byref(t)) == \
        bcgs.BCGS_ERR_ARG
    assert L.bcgs_queue_poll(None, 1, ctypes.byref(out)) == bcgs.BCGS_ERR_ARG
    assert L.bcgs_queue_wait(None, 1, ctypes.byref(out)) == bcgs.BCGS_ERR_ARG
    assert L.bcgs_queue_destroy(None) == bcgs.BCGS_ERR_ARG
    assert L.bcgs_queue_free_output(None, FAKE, None) == bcgs.BCGS_ERR_ARG


def test_check_rejects_bad_arguments_before_enqueue():
    """bcgs_check validates shapes, leading dimensions, precision and the
    workspace before any device call (fake pointers are never touched)."""
    L = bcgs.lib()
    f = ctypes.c_void_p
    m, n = 5000, 64
    need = L.bcgs_check_workspace_size(m, n)
    assert need >= m * n * 8
    assert L.bcgs_check_workspace_size(10, 20) == 0      # m < n
    assert L.bcgs_check_workspace_size(10, 0) == 0

    def call(m=m, n=n, ldx=m, ldq=m, ldr=n, prec=0, ldg=n, ws=0x7000000000,
             nbytes=need, X=0x1000000000):
        return L.bcgs_check(f(X), ldx, f(0x2000000000), ldq, f(0x3000000000),
                            ldr, m, n, prec, f(0x4000000000), f(0x5000000000),
                            f(0x6000000000), ldg, f(ws), nbytes, None)
    assert call(X=0) == bcgs.BCGS_ERR_ARG
    assert call(ldx=m - 1) == bcgs.BCGS_ERR_ARG
    assert call(ldq=m - 1) == bcgs.BCGS_ERR_ARG
    assert call(ldr=n - 1) == bcgs.BCGS_ERR_ARG
    assert call(ldg=n - 1) == bcgs.BCGS_ERR_ARG
    assert call(prec=5) == bcgs.BCGS_ERR_ARG
    assert call(nbytes=need - 1) == bcgs.BCGS_ERR_ARG
    assert call(ws=0x7000000008) == bcgs.BCGS_ERR_ARG
    assert call(m=n - 1, ldx=n, ldq=n) == bcgs.BCGS_ERR_ARG
