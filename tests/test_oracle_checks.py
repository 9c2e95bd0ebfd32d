"""Pins of the oracle's accuracy checkers (CPU only).

Every GPU parity verdict goes through ``chunked_gram``,
``loss_of_orthogonality`` and ``relative_residual``, so each is pinned here
against a value fixed by construction, not by re-running its own formula:

- chunked_gram: small-integer matrices, whose Gram entries are exact in
  binary64, against the int64 product, on row counts that span several
  4096-row chunks, an odd number of chunks and a ragged last chunk;
- loss_of_orthogonality (section 1: ||Q^T Q - I|| in the 2-norm): an
  orthonormal Q with planted column scalings, where Q^T Q - I is diagonal
  with known entries, and with a planted rank-one departure I +- eps w w^T,
  whose 2-norm is eps while its largest entry is smaller; the two together
  separate the 2-norm from both the largest-entry and the Frobenius norm;
- relative_residual (||X - QR|| / ||X||, 2-norms): X = QR + E with E of two
  known singular values, orthogonal to range(Q), placed in the last rows.

The mutation tests at the bottom plant a plausible mistake in each checker
(largest-entry or Frobenius norm, the largest eigenvalue instead of the
largest absolute one, a dropped last chunk, a missing square root) and
check that a pin above catches it.
"""

import numpy as np
import pytest

from oracle import checks as C

U64 = 2.0 ** -53


# ----------------------------------------------------------- constructions

def _int_matrix(m, n, seed):
    return np.random.default_rng(seed).integers(-8, 9, size=(m, n))


def _orthonormal(m, n, seed):
    G = np.random.default_rng(seed).standard_normal((m, n))
    Q, _ = np.linalg.qr(G)
    return Q


def _spread_unit_vector(n, seed):
    w = np.random.default_rng(seed).standard_normal(n)
    return w / np.linalg.norm(w)


# ------------------------------------------------------------------- pins

def pin_chunked_gram():
    """Exact integer Grams over several chunks (4096 rows each) with a
    ragged tail: binary64 holds every partial sum exactly (|sum| <=
    64 m < 2^53), so the chunked pairwise sum must equal the int64
    product bit for bit."""
    for m, chunk in [(3 * 4096 + 17, 4096), (5 * 4096, 4096), (1000, 96),
                     (4096, 4096), (1, 4096)]:
        A = _int_matrix(m, 7, seed=m)
        B = _int_matrix(m, 5, seed=m + 1)
        exact_ab = A.T @ B                       # int64 arithmetic
        exact_aa = A.T @ A
        got_ab = C.chunked_gram(A.astype(np.float64), B.astype(np.float64),
                                chunk=chunk)
        got_aa = C.chunked_gram(A.astype(np.float64), chunk=chunk)
        assert np.array_equal(got_ab, exact_ab.astype(np.float64)), (m, chunk)
        assert np.array_equal(got_aa, exact_aa.astype(np.float64)), (m, chunk)


def pin_loo_diagonal():
    """Q diag(1 + d): Q^T Q - I = diag((1 + d_i)^2 - 1), 2-norm
    max_i |(1 + d_i)^2 - 1| (the largest absolute entry, not the
    Frobenius norm, which is larger here)."""
    m, n = 3 * 4096 + 17, 12
    Q = _orthonormal(m, n, seed=1)
    d = np.linspace(-3e-6, 2e-6, n)              # the largest |.| is negative
    Qs = Q * (1.0 + d)[None, :]
    want = np.max(np.abs((1.0 + d) ** 2 - 1.0))
    fro = np.linalg.norm((1.0 + d) ** 2 - 1.0)
    got = C.loss_of_orthogonality(Qs)
    assert abs(got - want) <= 1e-6 * want + 100 * n * U64, (got, want)
    assert fro > 1.5 * want                      # the pin separates them


def pin_loo_rank_one():
    """Q (I + c w w^T) with (1 + c)^2 = 1 + eps: Q'^T Q' - I = eps w w^T,
    2-norm |eps|, largest entry |eps| max_i w_i^2 < |eps|.  Both signs of
    eps, so the largest eigenvalue alone does not pass."""
    m, n = 2 * 4096 + 3, 16
    Q = _orthonormal(m, n, seed=2)
    w = _spread_unit_vector(n, seed=3)
    for eps in (4e-7, -4e-7):
        c = np.sqrt(1.0 + eps) - 1.0
        Qp = Q + c * np.outer(Q @ w, w)
        got = C.loss_of_orthogonality(Qp)
        assert abs(got - abs(eps)) <= 1e-6 * abs(eps) + 100 * n * U64, (
            eps, got)
        assert abs(eps) * np.max(w ** 2) < 0.5 * abs(eps)


def pin_loo_exact_orthonormal():
    """Columns of the identity: Q^T Q = I exactly, LOO exactly 0."""
    Q = np.eye(9000)[:, :20]
    assert C.loss_of_orthogonality(Q) == 0.0


def pin_residual():
    """X = Q R + E with R = diag(r), r_1 = 1 the largest, and
    E = e1 a1 e_n^T + e2 a2 e_{n-1}^T where a1, a2 are orthonormal, orthogonal
    to range(Q), and nonzero only in the last rows (past every full
    chunk).  Then ||X - QR||_2 = max(e1, e2) and ||X||_2 = 1 (e1, e2 small
    against r_1), so the relative residual is max(e1, e2), which is neither
    the Frobenius norm of E nor its largest entry."""
    m, n = (1 << 16) + 2 * 4096 + 37, 8
    rng = np.random.default_rng(4)
    Q = np.zeros((m, n))
    Q[: m - 64] = _orthonormal(m - 64, n, seed=5)
    A = np.zeros((m, 2))
    A[m - 64:] = np.linalg.qr(rng.standard_normal((64, 2)))[0]
    r = np.concatenate([[1.0], np.linspace(0.9, 0.5, n - 1)])
    R = np.diag(r)
    e1, e2 = 3e-9, 2e-9
    E = e1 * np.outer(A[:, 0], np.eye(n)[n - 1]) + \
        e2 * np.outer(A[:, 1], np.eye(n)[n - 2])
    X = Q @ R + E
    got = C.relative_residual(X, Q, R)
    want = max(e1, e2)
    assert abs(got - want) <= 1e-6 * want, (got, want)
    assert np.linalg.norm(E) > 1.1 * want
    assert np.max(np.abs(E)) < 0.9 * want
    # no residual at all: exactly zero
    assert C.relative_residual(Q @ R, Q, R) == 0.0


PINS = [pin_chunked_gram, pin_loo_diagonal, pin_loo_rank_one,
        pin_loo_exact_orthonormal, pin_residual]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_checker_pin(pin):
    pin()


# -------------------------------------------------------------- mutations

def _caught(monkeypatch, name, bad):
    """True when some pin fails with C.<name> replaced by `bad`."""
    monkeypatch.setattr(C, name, bad)
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            return True
    return False


def test_mutation_largest_entry_norm(monkeypatch):
    def bad(M):
        return float(np.max(np.abs(0.5 * (M + M.T))))
    assert _caught(monkeypatch, "_sym_norm2", bad)


def test_mutation_frobenius_norm(monkeypatch):
    def bad(M):
        return float(np.linalg.norm(0.5 * (M + M.T)))
    assert _caught(monkeypatch, "_sym_norm2", bad)


def test_mutation_largest_eigenvalue_not_absolute(monkeypatch):
    def bad(M):
        return float(np.max(np.linalg.eigvalsh(0.5 * (M + M.T))))
    assert _caught(monkeypatch, "_sym_norm2", bad)


def test_mutation_dropped_last_chunk(monkeypatch):
    def bad(A, B=None, chunk=4096):
        B = A if B is None else B
        m = A.shape[0]
        stop = max(chunk, m - m % chunk) if m > chunk else m
        parts = [A[i:i + chunk].T @ B[i:i + chunk]
                 for i in range(0, stop, chunk)]
        out = parts[0]
        for p in parts[1:]:
            out = out + p
        return out
    assert _caught(monkeypatch, "chunked_gram", bad)


def test_mutation_pairwise_sum_drops_odd_part(monkeypatch):
    def bad(A, B=None, chunk=4096):
        B = A if B is None else B
        m = A.shape[0]
        parts = [A[i:i + chunk].T @ B[i:i + chunk] for i in range(0, m, chunk)]
        while len(parts) > 1:            # the odd last part is lost
            parts = [parts[i] + parts[i + 1]
                     for i in range(0, len(parts) - 1, 2)]
        return parts[0]
    assert _caught(monkeypatch, "chunked_gram", bad)


def test_mutation_missing_square_root(monkeypatch):
    orig = C.relative_residual

    def bad(X, Q, R, chunk=1 << 16):
        return orig(X, Q, R, chunk) ** 2
    assert _caught(monkeypatch, "relative_residual", bad)


def test_mutation_residual_drops_last_row_chunk(monkeypatch):
    orig = C.relative_residual

    def bad(X, Q, R, chunk=1 << 16):
        keep = (X.shape[0] // chunk) * chunk or X.shape[0]
        return orig(X[:keep], Q[:keep], R, chunk)
    assert _caught(monkeypatch, "relative_residual", bad)
