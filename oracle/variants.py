"""The block Gram-Schmidt variants, written out step by step.

TEST INFRASTRUCTURE (see the package docstring).

Notation follows the paper with its m and n swapped to the convention of
this repository: X is m x n (m rows, n = q*s columns), X_k is the k-th block
column of width s, Q_{1:k} the first k block columns of Q, and R, S, Y are
n x n block upper-triangular with s x s blocks.  Comments use the paper's
1-based block indices; the code uses 0-based Python slices.

Each "sync" below is one global reduction in the paper's distributed
setting (section 3: the tall-skinny products, and TSQR's reduction tree);
``Stats.syncs`` counts them so that Table 1's synchronization counts can be
checked.

Readings of passages the paper leaves implicit:
  * BCGSI+ is only named (section 1; Table 1).  It is BCGS run twice per
    block column, each pass with its own TSQR intra-orthogonalization, with
    R assembled as in Alg. 1: four syncs per block column.
  * BCGSI+P-2S is given in prose only (section 2.3): Alg. 2 with TSQR in
    place of the Cholesky factorizations that form S_22 and S_{k+1,k+1};
    T is then not needed and S_12 = Q_1^T X_2 is its own product.
  * Alg. 2 is written for q >= 3.  For q = 1 only TSQR(X_1) runs; for q = 2
    the first product after U_2 is [Q_1 U_2]^T U_2, the form Alg. 2 itself
    uses in its last iteration.
  * BCGSI+1s is described (section 2.2) as Alg. 2 without its first
    intra-orthogonalization (the chol that forms S_{k+1,k+1}): U_{k+1} =
    X_{k+1} - Q_{1:k} S is not scaled, i.e. S_{k+1,k+1} = I, so R_{1:k,k+1}
    = S + Y and R_{k+1,k+1} = Y_{k+1,k+1}.  The same holds for the first
    block (S_12 = Q_1^T X_2, U_2 = X_2 - Q_1 S_12), and T is never formed.
"""

from dataclasses import dataclass, field

from .linalg import FP64, Breakdown


@dataclass
class Stats:
    syncs: int = 0
    log: list = field(default_factory=list)

    def sync(self, what):
        self.syncs += 1
        self.log.append(what)


def _blk(A, k, s):
    """Block column k (1-based, as in the paper) of A."""
    return A[:, (k - 1) * s:k * s]


def _first(A, k, s):
    """Q_{1:k}: the first k block columns of A."""
    return A[:, :k * s]


def tsqr_slot(bk, V, stats, what="TSQR"):
    """[Q, R] = TSQR(V) (section 1; Alg. 1 and Alg. 2 apply it to X_1).

    In exact arithmetic TSQR returns the economic QR of V with positive
    diag(R), whatever its reduction tree; the oracle computes that unique
    factorization by Householder QR with a sign fix (``bk.qr_pos``).  One
    global reduction."""
    stats.sync(what)
    return bk.qr_pos(V)


def _r_assemble(bk, R, k, s, S_col, Y_col, S_diag, Y_diag):
    """R_{1:k,k+1} = S_{1:k,k+1} + Y_{1:k,k+1} S_{k+1,k+1} and
    R_{k+1,k+1} = Y_{k+1,k+1} S_{k+1,k+1} (Alg. 1 last step; Alg. 2 last
    step of each iteration)."""
    R[:k * s, k * s:(k + 1) * s] = S_col + bk.matmul(Y_col, S_diag)
    R[k * s:(k + 1) * s, k * s:(k + 1) * s] = bk.matmul(Y_diag, S_diag)


def _chol(bk, A, block, where):
    try:
        return bk.chol(A, block=block)
    except Breakdown as e:
        raise Breakdown(block, e.pivot, e.value, where) from None


def bcgs_i_plus(X, s, bk=FP64, stats=None):
    """BCGSI+: reorthogonalized BCGS, four syncs per block column
    (section 1; Table 1).  Both intra-orthogonalizations are TSQR."""
    stats = stats if stats is not None else Stats()
    m, n = X.shape
    q = n // s
    Q = bk.zeros((m, n))
    R = bk.zeros((n, n))
    Q1, R11 = tsqr_slot(bk, _blk(X, 1, s), stats, "TSQR(X_1)")
    Q[:, :s] = Q1
    R[:s, :s] = R11
    for k in range(1, q):
        Qk = _first(Q, k, s)
        Xk1 = _blk(X, k + 1, s)
        # first BCGS pass: project, then intra-orthogonalize
        stats.sync(f"S = Q_1:{k}^T X_{k+1}")
        S = bk.matmul(Qk.T, Xk1)
        U, S_diag = tsqr_slot(bk, Xk1 - bk.matmul(Qk, S), stats,
                              f"TSQR(V_{k+1})")
        # second pass (reorthogonalization)
        stats.sync(f"Y = Q_1:{k}^T U_{k+1}")
        Y = bk.matmul(Qk.T, U)
        Qn, Y_diag = tsqr_slot(bk, U - bk.matmul(Qk, Y), stats,
                               f"TSQR(W_{k+1})")
        Q[:, k * s:(k + 1) * s] = Qn
        _r_assemble(bk, R, k, s, S, Y, S_diag, Y_diag)
    return Q, R


def bcgs_pipi_plus(X, s, bk=FP64, stats=None):
    """BCGS-PIPI+ (Alg. 1): two syncs per block column, Pythagorean
    Cholesky for both intra-orthogonalizations."""
    stats = stats if stats is not None else Stats()
    m, n = X.shape
    q = n // s
    Q = bk.zeros((m, n))
    R = bk.zeros((n, n))
    Q1, R11 = tsqr_slot(bk, _blk(X, 1, s), stats, "TSQR(X_1)")
    Q[:, :s] = Q1
    R[:s, :s] = R11
    for k in range(1, q):
        Qk = _first(Q, k, s)
        Xk1 = _blk(X, k + 1, s)
        # [S_{1:k,k+1}; T_{k+1}] = [Q_k X_{k+1}]^T X_{k+1}   (first sync)
        stats.sync(f"[S;T] = [Q_1:{k} X_{k+1}]^T X_{k+1}")
        G = bk.matmul(_concat(bk, Qk, Xk1).T, Xk1)
        S, T = G[:k * s], G[k * s:]
        S_diag = _chol(bk, T - bk.matmul(S.T, S), k, "S_{k+1,k+1}")
        U = bk.right_solve(Xk1 - bk.matmul(Qk, S), S_diag)
        # [Y_{1:k,k+1}; Omega_{k+1}] = [Q_k U_{k+1}]^T U_{k+1}   (second sync)
        stats.sync(f"[Y;Om] = [Q_1:{k} U_{k+1}]^T U_{k+1}")
        G = bk.matmul(_concat(bk, Qk, U).T, U)
        Y, Om = G[:k * s], G[k * s:]
        Y_diag = _chol(bk, Om - bk.matmul(Y.T, Y), k, "Y_{k+1,k+1}")
        Q[:, k * s:(k + 1) * s] = bk.right_solve(U - bk.matmul(Qk, Y), Y_diag)
        _r_assemble(bk, R, k, s, S, Y, S_diag, Y_diag)
    return Q, R


def _concat(bk, *blocks):
    import numpy as np
    return np.concatenate(blocks, axis=1)


def _delayed_s(bk, Z_prev, P_k, Y_prev, Y_kk):
    """Eq. (1): S_{1:k,k+1} = [Z_{k-1}; Y_kk^{-T}(P_k - Y_{1:k-1,k}^T Z_{k-1})],
    the projection coefficients of X_{k+1} on Q_{1:k} obtained without a
    new product with Q_k (delayed normalization)."""
    import numpy as np
    lower = bk.left_solve_t(Y_kk, P_k - bk.matmul(Y_prev.T, Z_prev))
    return np.concatenate([Z_prev, lower], axis=0)


def _one_or_two_sync(X, s, bk, stats, first_intra):
    """Alg. 2 and its siblings, which differ only in the first
    intra-orthogonalization of each block column (``first_intra`` is
    "chol" for BCGSI+P-1S, "tsqr" for BCGSI+P-2S (section 2.3), "none" for
    BCGSI+1s (section 2.2, S_{k+1,k+1} = I))."""
    m, n = X.shape
    q = n // s
    Q = bk.zeros((m, n))
    R = bk.zeros((n, n))
    # [Q_1, R_11] = TSQR(X_1)
    Q1, R11 = tsqr_slot(bk, _blk(X, 1, s), stats, "TSQR(X_1)")
    Q[:, :s] = Q1
    R[:s, :s] = R11
    if q == 1:
        return Q, R
    X2 = _blk(X, 2, s)
    if first_intra == "chol":
        # [S_12; T_2] = [Q_1 X_2]^T X_2 ; S_22 = chol(T_2 - S_12^T S_12)
        stats.sync("[S_12;T_2] = [Q_1 X_2]^T X_2")
        G = bk.matmul(_concat(bk, Q1, X2).T, X2)
        S12, T2 = G[:s], G[s:]
        S22 = _chol(bk, T2 - bk.matmul(S12.T, S12), 1, "S_22")
        # U_2 = (X_2 - Q_1 S_12) S_22^{-1}
        U = bk.right_solve(X2 - bk.matmul(Q1, S12), S22)
    elif first_intra == "tsqr":
        # S_12 = Q_1^T X_2 ; [U_2, S_22] = TSQR(X_2 - Q_1 S_12)
        stats.sync("S_12 = Q_1^T X_2")
        S12 = bk.matmul(Q1.T, X2)
        U, S22 = tsqr_slot(bk, X2 - bk.matmul(Q1, S12), stats, "TSQR(V_2)")
    else:
        # S_12 = Q_1^T X_2 ; U_2 = X_2 - Q_1 S_12 (no intra-orthogonalization)
        stats.sync("S_12 = Q_1^T X_2")
        S12 = bk.matmul(Q1.T, X2)
        U = X2 - bk.matmul(Q1, S12)
        S22 = bk.eye(s)
    S_col, S_diag = S12, S22
    # the loop below handles block columns k+1 = 2..q; for k = 1 the S
    # coefficients come from the set-up above, afterwards from eq. (1)
    Z = P = T = None
    Y_col = Y_diag = None
    for k in range(1, q):
        Qk = _first(Q, k, s)
        Xk1 = _blk(X, k + 1, s)
        if k >= 2:
            S_col = _delayed_s(bk, Z, P, Y_col, Y_diag)
            if first_intra == "chol":
                # S_{k+1,k+1} = chol(T_{k+1} - S^T S) ;
                # U_{k+1} = (X_{k+1} - Q_k S) S_{k+1,k+1}^{-1}
                S_diag = _chol(bk, T - bk.matmul(S_col.T, S_col), k,
                               "S_{k+1,k+1}")
                U = bk.right_solve(Xk1 - bk.matmul(Qk, S_col), S_diag)
            elif first_intra == "tsqr":
                # [U_{k+1}, S_{k+1,k+1}] = TSQR(X_{k+1} - Q_k S)
                U, S_diag = tsqr_slot(bk, Xk1 - bk.matmul(Qk, S_col), stats,
                                      f"TSQR(V_{k+1})")
            else:
                # U_{k+1} = X_{k+1} - Q_k S, S_{k+1,k+1} = I
                U = Xk1 - bk.matmul(Qk, S_col)
                S_diag = bk.eye(s)
        if k < q - 1:
            # [Y Z_k; Omega P_{k+1}] = [Q_k U_{k+1}]^T [U_{k+1} X_{k+2}]
            # (and T_{k+2} = X_{k+2}^T X_{k+2} in the same sync, P-1S only)
            Xk2 = _blk(X, k + 2, s)
            stats.sync(f"[Y Z;Om P] = [Q_1:{k} U_{k+1}]^T [U_{k+1} X_{k+2}]")
            G = bk.matmul(_concat(bk, Qk, U).T, _concat(bk, U, Xk2))
            Y, Z = G[:k * s, :s], G[:k * s, s:]
            Om, P = G[k * s:, :s], G[k * s:, s:]
            T = bk.matmul(Xk2.T, Xk2) if first_intra == "chol" else None
        else:
            # [Y; Omega] = [Q_k U_{k+1}]^T U_{k+1}
            stats.sync(f"[Y;Om] = [Q_1:{k} U_{k+1}]^T U_{k+1}")
            G = bk.matmul(_concat(bk, Qk, U).T, U)
            Y, Om = G[:k * s], G[k * s:]
        # Y_{k+1,k+1} = chol(Omega - Y^T Y) ;
        # Q_{k+1} = (U_{k+1} - Q_k Y) Y_{k+1,k+1}^{-1}
        Y_d = _chol(bk, Om - bk.matmul(Y.T, Y), k, "Y_{k+1,k+1}")
        Q[:, k * s:(k + 1) * s] = bk.right_solve(U - bk.matmul(Qk, Y), Y_d)
        _r_assemble(bk, R, k, s, S_col, Y, S_diag, Y_d)
        Y_col, Y_diag = Y, Y_d
    return Q, R


def bcgs_p_1s(X, s, bk=FP64, stats=None):
    """BCGSI+P-1S (Alg. 2): one sync per block column (section 2.2)."""
    stats = stats if stats is not None else Stats()
    return _one_or_two_sync(X, s, bk, stats, "chol")


def bcgs_p_2s(X, s, bk=FP64, stats=None):
    """BCGSI+P-2S (section 2.3): Alg. 2 with TSQR as the first
    intra-orthogonalization of every block column; two syncs per block
    column."""
    stats = stats if stats is not None else Stats()
    return _one_or_two_sync(X, s, bk, stats, "tsqr")


def bcgs_i_plus_1s(X, s, bk=FP64, stats=None):
    """BCGSI+1s (section 2.2; Table 1): Alg. 2 without the Cholesky factor
    of the first intra-orthogonalization; one sync per block column, LOO
    O(u) kappa^2 under O(u) kappa^3 <= 1."""
    stats = stats if stats is not None else Stats()
    return _one_or_two_sync(X, s, bk, stats, "none")


VARIANTS = {
    "bcgsi+": bcgs_i_plus,
    "bcgsi+1s": bcgs_i_plus_1s,
    "p-2s": bcgs_p_2s,
    "p-1s": bcgs_p_1s,
    "pipi+": bcgs_pipi_plus,
}


@dataclass
class Result:
    Q: object
    R: object
    syncs: int
    breakdown: object = None   # a Breakdown, or None


def qr(X, s, variant, bk=FP64):
    """Run one variant on X (m x n, m >= n, s | n).  On a Cholesky breakdown
    the result carries the ``Breakdown`` (first failing block and pivot)
    and Q, R are None."""
    m, n = X.shape
    if s < 1 or n % s != 0 or m < n:
        raise ValueError(f"need s | n and m >= n (m={m}, n={n}, s={s})")
    stats = Stats()
    Xb = bk.asarray(X) if bk is not FP64 else X
    try:
        Q, R = VARIANTS[variant](Xb, s, bk, stats)
    except Breakdown as e:
        return Result(None, None, stats.syncs, e)
    return Result(Q, R, stats.syncs, None)
