"""Accuracy measures and the Householder reference.

TEST INFRASTRUCTURE (see the package docstring).

Section 1 of the paper defines the loss of orthogonality as ||Q^T Q - I||
and the condition number kappa(X) = ||X|| / sigma_min(X), both in the
2-norm.  For an n x n symmetric matrix the 2-norm is the largest absolute
eigenvalue, which is what these functions compute.

For tall inputs (millions of rows) a straight FP64 Q^T Q accumulates an
error that grows with the row count; ``chunked_gram`` sums per-chunk Gram
matrices pairwise so the checker's own error stays well below u*n.
"""

import numpy as np

from .linalg import FP64


def chunked_gram(A, B=None, chunk=4096):
    """A^T B (FP64) as a pairwise sum of per-chunk products over the rows."""
    B = A if B is None else B
    m = A.shape[0]
    parts = [A[i:i + chunk].T @ B[i:i + chunk] for i in range(0, m, chunk)]
    if not parts:
        return np.zeros((A.shape[1], B.shape[1]))
    while len(parts) > 1:
        nxt = [parts[i] + parts[i + 1] for i in range(0, len(parts) - 1, 2)]
        if len(parts) % 2:
            nxt.append(parts[-1])
        parts = nxt
    return parts[0]


def _sym_norm2(M):
    M = 0.5 * (M + M.T)
    return float(np.max(np.abs(np.linalg.eigvalsh(M))))


def loss_of_orthogonality(Q):
    """||Q^T Q - I||_2 (section 1)."""
    Q = np.asarray(Q, dtype=np.float64)
    G = chunked_gram(Q)
    return _sym_norm2(G - np.eye(G.shape[0]))


def relative_residual(X, Q, R, chunk=1 << 16):
    """||X - Q R||_2 / ||X||_2, from the eigenvalues of the n x n Gram
    matrices of X - QR and of X (residual rows formed chunk by chunk)."""
    X = np.asarray(X, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    m, n = X.shape
    parts = []
    for i in range(0, m, chunk):
        E = X[i:i + chunk] - Q[i:i + chunk] @ R
        parts.append(chunked_gram(E))
    GE = parts[0]
    for p in parts[1:]:
        GE = GE + p
    GX = chunked_gram(X)
    num = max(_sym_norm2(GE), 0.0) ** 0.5
    den = _sym_norm2(GX) ** 0.5
    return num / den


def householder_reference(X):
    """The unique economic QR with diag(R) >= 0 (section 1's problem), by
    LAPACK Householder QR and a sign fix."""
    return FP64.qr_pos(np.asarray(X, dtype=np.float64))
