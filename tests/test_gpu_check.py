"""The device accuracy checker (bcgs_check) on the GPU, through the C ABI.

Two kinds of cases:
  * factorizations computed by the library: the checker's loss of
    orthogonality and relative residual agree with the oracle's measures
    within 4 n u absolute (both sides round their Gram sums; the measures
    themselves are O(u) here) plus 1e-9 relative;
  * planted departures of known size: a Householder Q with one column
    scaled by 1 + d has ||Q^T Q - I||_2 = 2d + d^2 up to O(u), and adding
    a rank-one sigma a b^T (unit a, b) to X = Q R gives a residual of
    sigma / ||X'||_2 up to O(u) ||X|| / ||X'||, with ||X'||_2 taken by
    numpy's SVD; these values do not come from the oracle's checker.
Ragged row counts (not multiples of 64 or of the 4096-row chunk), column
counts that leave a partial 64 x 64 block, m = n, several row ranges and
the binary32 element type are covered.  Every case prints its name before
touching the GPU."""

import numpy as np
import pytest

import oracle as O
from paper_2507_21791_amd import workloads as W

from parity import U64, host, log, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def checker():
    import torch
    from paper_2507_21791_amd import bcgs
    assert torch.cuda.is_available()
    bcgs.lib()
    return bcgs.Checker()


CASES = [
    (5000, 64, 16, 3, "p-1s", "fp64"),
    (20001, 96, 8, 5, "bcgsi+", "fp64"),
    (9000, 48, 16, 2, "p-2s", "fp32-bulk"),
    (300001, 256, 16, 8, "p-1s", "fp64"),
    (100, 100, 4, 2, "bcgsi+", "fp64"),
    (65, 64, 16, 1, "p-1s", "fp64"),
    (123457, 160, 16, 6, "pipi+", "fp64"),
]


@pytest.mark.parametrize("m,n,s,dec,variant,prec", CASES)
def test_checker_matches_oracle_measures(checker, m, n, s, dec, variant,
                                         prec):
    import torch
    from paper_2507_21791_amd import bcgs
    log(f"[gpu] check m={m} n={n} s={s} {variant} {prec}")
    Xh = W.conditioned_host(m, n, dec, seed=m + n)
    dt = torch.float64 if prec == "fp64" else torch.float32
    Xd = to_device(Xh, dt)
    Q, R, ws = bcgs.qr(Xd, s, variant, prec)
    loo, res = checker(Xd, Q, R, prec)
    assert ws.info().status == 0
    Xw, Qw, Rw = host(Xd), host(Q), host(R)
    want_loo = O.loss_of_orthogonality(Qw)
    want_res = O.relative_residual(Xw, Qw, np.triu(Rw))
    tol = 4 * n * U64
    assert abs(loo - want_loo) <= tol + 1e-9 * want_loo, (loo, want_loo)
    assert abs(res - want_res) <= tol + 1e-9 * want_res, (res, want_res)


@pytest.mark.parametrize("m,n", [(30001, 96), (4096 * 3 + 7, 64)])
def test_checker_planted_departures(checker, m, n):
    import torch
    log(f"[gpu] check planted m={m} n={n}")
    rng = np.random.default_rng(m)
    Xh = np.asfortranarray(rng.standard_normal((m, n)))
    Qh, Rh = np.linalg.qr(Xh)
    d = 1e-7
    Qp = np.asfortranarray(Qh.copy())
    Qp[:, 5] *= 1.0 + d
    a = rng.standard_normal(m)
    a /= np.linalg.norm(a)
    b = rng.standard_normal(n)
    b /= np.linalg.norm(b)
    sigma = 1e-5 * np.linalg.norm(Xh, 2)
    Xp = np.asfortranarray(Qh @ Rh + sigma * np.outer(a, b))
    loo, _ = checker(to_device(Qh @ Rh), to_device(Qp), to_device(Rh))
    assert abs(loo - (2 * d + d * d)) <= 64 * n * U64, loo
    torch.cuda.synchronize()
    _, res = checker(to_device(Xp), to_device(Qh), to_device(Rh))
    want = sigma / np.linalg.norm(Xp, 2)
    assert abs(res - want) <= 1e-9 * want + 64 * n * U64, (res, want)


def test_checker_reads_only_upper_triangle(checker):
    """Garbage below R's diagonal does not change the residual."""
    import torch
    from paper_2507_21791_amd import bcgs
    log("[gpu] check ignores the strictly lower part of R")
    Xh = W.conditioned_host(7000, 64, 3, seed=11)
    Xd = to_device(Xh)
    Q, R, ws = bcgs.qr(Xd, 16, "p-1s")
    G1 = checker.grams(Xd, Q, R).cpu()
    R2 = R.clone()
    R2 += torch.tril(torch.full_like(R, 1e3), -1)
    G2 = checker.grams(Xd, Q, R2).cpu()
    assert torch.equal(G1, G2)
