"""Dense primitives used by the oracle variants, in two number systems.

TEST INFRASTRUCTURE (see the package docstring): never imported by the
product path.

Conventions (section 1 of the paper: MATLAB-style indexing, 2-norm;
``chol`` returns the upper-triangular factor):
  * ``chol(A)``            upper R with R^T R = A.  Breakdown when a pivot is
                           not strictly positive or is not finite (the
                           criterion LAPACK's potrf uses); the caller learns
                           the block index and pivot through ``Breakdown``.
  * ``right_solve(B, T)``  B T^{-1} for upper-triangular T (a right solve, as
                           in "(X - QS) S^{-1}" of Alg. 1 and Alg. 2).
  * ``left_solve_t(T, B)`` T^{-T} B for upper-triangular T (the Y_kk^{-T}
                           solve of eq. (1)).
  * ``qr_pos(V)``          the economic QR of V with a non-negative diagonal
                           of R: the unique factorization that TSQR, the
                           paper's unconditionally stable intra-
                           orthogonalization (section 1), produces in exact
                           arithmetic whatever its reduction tree.

The substitution and Cholesky loops are written once and run unchanged on
numpy float64 arrays and on numpy object arrays holding mpmath numbers.
"""

import math

import numpy as np


class Breakdown(Exception):
    """Cholesky of an intra-block Gram matrix failed (a pivot <= 0 or
    non-finite).  ``block`` is the 0-based block column whose factor was being
    formed, ``pivot`` the 0-based pivot index and ``value`` the failing
    pivot value."""

    def __init__(self, block, pivot, value, where=""):
        super().__init__(f"Cholesky breakdown at block {block}, pivot {pivot}"
                         f" (value {value!r}) {where}")
        self.block = block
        self.pivot = pivot
        self.value = value
        self.where = where


class _Backend:
    """Shared plain-loop algorithms; subclasses provide the scalar field."""

    name = "?"

    # -- scalar field -------------------------------------------------
    def asarray(self, a):
        raise NotImplementedError

    def zeros(self, shape):
        raise NotImplementedError

    def sqrt(self, x):
        raise NotImplementedError

    def isfinite(self, x):
        raise NotImplementedError

    def qr_raw(self, V):
        """Householder QR (reduced) from a library; signs unspecified."""
        raise NotImplementedError

    # -- plain algorithms --------------------------------------------
    def eye(self, n):
        """n x n identity in this number system."""
        out = self.zeros((n, n))
        for i in range(n):
            out[i, i] = out[i, i] + 1
        return out

    def matmul(self, A, B):
        return A @ B

    def chol(self, A, block=-1):
        """Upper Cholesky factor R of the symmetric matrix A (R^T R = A).

        Row-by-row (Cholesky-Banachiewicz) order.  Raises ``Breakdown`` at
        the first pivot d_j = A_jj - sum_i R_ij^2 that is <= 0 or not
        finite."""
        s = A.shape[0]
        R = self.zeros((s, s))
        for j in range(s):
            d = A[j, j] - (R[:j, j] @ R[:j, j] if j else 0)
            if not (self.isfinite(d) and d > 0):
                raise Breakdown(block, j, d)
            r = self.sqrt(d)
            R[j, j] = r
            for l in range(j + 1, s):
                R[j, l] = (A[j, l] - (R[:j, j] @ R[:j, l] if j else 0)) / r
        return R

    def right_solve(self, B, T):
        """X = B T^{-1} for upper-triangular T: column j of X T = B reads
        X[:, j] T_jj + X[:, :j] T[:j, j] = B[:, j]."""
        s = T.shape[0]
        X = self.zeros(B.shape)
        for j in range(s):
            acc = B[:, j] - (X[:, :j] @ T[:j, j] if j else 0)
            X[:, j] = acc / T[j, j]
        return X

    def left_solve_t(self, T, B):
        """X = T^{-T} B for upper-triangular T (T^T is lower triangular):
        row i of T^T X = B reads T_ii X[i, :] + T[:i, i]^T X[:i, :] = B[i, :]."""
        s = T.shape[0]
        X = self.zeros(B.shape)
        for i in range(s):
            acc = B[i, :] - (T[:i, i] @ X[:i, :] if i else 0)
            X[i, :] = acc / T[i, i]
        return X

    def qr_pos(self, V):
        """Economic QR with diag(R) >= 0: Householder QR, then
        Q <- Q D, R <- D R with D = sign(diag R) and sign(0) := +1."""
        Q, R = self.qr_raw(V)
        d = np.array([(-1 if R[i, i] < 0 else 1) for i in range(R.shape[0])],
                     dtype=object if R.dtype == object else float)
        return Q * d[None, :], R * d[:, None]


class _FP64(_Backend):
    name = "fp64"
    eps = 2.0 ** -53   # unit roundoff u of binary64

    def asarray(self, a):
        return np.array(a, dtype=np.float64)

    def zeros(self, shape):
        return np.zeros(shape, dtype=np.float64)

    def sqrt(self, x):
        return math.sqrt(x)

    def isfinite(self, x):
        return math.isfinite(x)

    def qr_raw(self, V):
        # LAPACK dgeqrf + dorgqr
        return np.linalg.qr(np.asarray(V, dtype=np.float64), mode="reduced")


class _MP(_Backend):
    """mpmath arithmetic at ``dps`` decimal digits, on numpy object arrays."""

    def __init__(self, dps=50):
        import mpmath
        self.mpmath = mpmath
        self.ctx = mpmath.MPContext()
        self.ctx.dps = dps
        self.dps = dps
        self.name = f"mp{dps}"
        self.eps = self.ctx.mpf(10) ** (-dps)

    def asarray(self, a):
        a = np.asarray(a)
        out = np.empty(a.shape, dtype=object)
        for idx in np.ndindex(a.shape):
            out[idx] = self.ctx.mpf(a[idx])
        return out

    def zeros(self, shape):
        out = np.empty(shape, dtype=object)
        z = self.ctx.mpf(0)
        for idx in np.ndindex(shape):
            out[idx] = z
        return out

    def sqrt(self, x):
        return self.ctx.sqrt(x)

    def isfinite(self, x):
        return self.ctx.isfinite(x)

    def qr_raw(self, V):
        A = self.ctx.matrix(V.tolist())
        Q, R = self.ctx.qr(A, mode="skinny")
        m, n = V.shape
        Qa = self.zeros((m, n))
        Ra = self.zeros((n, n))
        for i in range(m):
            for j in range(n):
                Qa[i, j] = Q[i, j]
        for i in range(n):
            for j in range(n):
                Ra[i, j] = R[i, j] if j >= i else self.ctx.mpf(0)
        return Qa, Ra

    def to_float(self, A):
        return np.array([[float(x) for x in row] for row in np.atleast_2d(A)])


FP64 = _FP64()
_MP_CACHE = {}


def make_mp(dps=50):
    if dps not in _MP_CACHE:
        _MP_CACHE[dps] = _MP(dps)
    return _MP_CACHE[dps]


MP = None  # created lazily through make_mp(); kept for the package export
