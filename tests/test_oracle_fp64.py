"""Pins of the FP64 oracle (CPU only): library routines, closed forms,
invariants of Table 1, and the regimes Table 1 predicts.

u = 2^-53.  "O(u)" is read as <= 10 n u (with n the column count), applied
only where Table 1's assumption holds with margin.
"""

import math

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
from paper_2507_21791_amd import workloads as W

U64 = 2.0 ** -53
ALL = ["bcgsi+", "p-2s", "p-1s", "pipi+"]
# BCGSI+1s: LOO O(u) kappa^2 (Table 1), so it joins only the tests whose
# bound does not assume O(u) LOO at large kappa
ALL5 = ALL + ["bcgsi+1s"]


# -------------------------------------------------- primitives vs LAPACK ---

def test_chol_matches_lapack():
    rng = np.random.default_rng(0)
    for s in [1, 2, 5, 16, 33]:
        A = rng.standard_normal((3 * s, s))
        G = A.T @ A
        R = O.FP64.chol(G)
        Rl = sla.cholesky(G, lower=False)
        assert np.allclose(R, Rl, rtol=1e-13, atol=1e-13 * np.abs(Rl).max())
        assert np.all(np.tril(R, -1) == 0)


def test_chol_breakdown_reports_first_bad_pivot():
    A = np.diag([4.0, 1.0, -1.0, 2.0])
    with pytest.raises(O.Breakdown) as e:
        O.FP64.chol(A, block=7)
    assert e.value.block == 7 and e.value.pivot == 2
    with pytest.raises(O.Breakdown) as e:
        O.FP64.chol(np.array([[1.0, 0], [0, np.nan]]))
    assert e.value.pivot == 1


def test_triangular_solves_match_lapack():
    rng = np.random.default_rng(1)
    T = np.triu(rng.standard_normal((7, 7))) + 4 * np.eye(7)
    B = rng.standard_normal((50, 7))
    X = O.FP64.right_solve(B, T)
    assert np.allclose(X, sla.solve_triangular(T, B.T, trans="T").T,
                       rtol=1e-13)
    C = rng.standard_normal((7, 9))
    Y = O.FP64.left_solve_t(T, C)
    assert np.allclose(Y, sla.solve_triangular(T, C, trans="T"), rtol=1e-13)


def test_qr_pos_unique_sign():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((40, 6))
    Q, R = O.FP64.qr_pos(X)
    assert np.all(np.diag(R) > 0)
    assert np.allclose(Q @ R, X, atol=1e-14)
    # R equals the Cholesky factor of X^T X (uniqueness)
    assert np.allclose(R, sla.cholesky(X.T @ X), rtol=1e-10)


# ----------------------------------------------------- accuracy, Table 1 ---

@pytest.mark.parametrize("variant", ALL)
def test_small_workload_accuracy(variant):
    """The 2000 x 80, s = 8, kappa = 1e6 workload: every variant's
    assumption holds (u kappa^2 = 1.1e-4), so LOO and residual are O(u)
    and R agrees with Householder to u*kappa."""
    w = W.WORKLOADS["small"]
    X = W.make_host("small")
    n = w["n"]
    r = O.qr(X, w["s"], variant)
    assert r.breakdown is None
    assert O.loss_of_orthogonality(r.Q) <= 10 * n * U64
    assert O.relative_residual(X, r.Q, r.R) <= 10 * n * U64
    Qh, Rh = O.householder_reference(X)
    kappa = 1e6
    assert np.linalg.norm(r.R - Rh) / np.linalg.norm(Rh) <= 10 * n * U64 * kappa
    assert np.all(np.tril(r.R, -1) == 0) and np.all(np.diag(r.R) > 0)


@pytest.mark.parametrize("variant", ALL5)
@pytest.mark.parametrize("s", [1, 2, 4, 8])
def test_block_sizes_and_tails(variant, s):
    X = W.conditioned_host(257, 48, 3, seed=11 + s)
    r = O.qr(X, s, variant)
    assert r.breakdown is None
    grow = 1e6 if variant == "bcgsi+1s" else 1.0      # kappa^2, kappa = 1e3
    assert O.loss_of_orthogonality(r.Q) <= 10 * 48 * U64 * grow
    assert O.relative_residual(X, r.Q, r.R) <= 10 * 48 * U64


@pytest.mark.parametrize("q", [1, 2, 3])
@pytest.mark.parametrize("variant", ALL5)
def test_few_block_columns(variant, q):
    """q = 1 and q = 2 need the short forms of Alg. 2 (see the oracle)."""
    X = W.conditioned_host(64, 4 * q, 2, seed=q)
    r = O.qr(X, 4, variant)
    Qh, Rh = O.householder_reference(X)
    assert np.allclose(r.R, Rh, rtol=1e-12, atol=1e-13)


def test_p1s_and_pipi_plus_agree_in_fp64():
    """Same algorithm reorganized (section 2.2): same R up to rounding."""
    X = W.conditioned_host(600, 64, 4, seed=4)
    a = O.qr(X, 8, "p-1s")
    b = O.qr(X, 8, "pipi+")
    assert np.linalg.norm(a.R - b.R) / np.linalg.norm(b.R) < 1e-11


def test_regimes_of_table1():
    """Table 1: BCGSI+ and BCGSI+P-2S keep O(u) LOO while u*kappa <= 1;
    BCGSI+P-1S needs u*kappa^2 <= 1 and fails (breakdown or LOO >> u) well
    beyond it."""
    X = W.conditioned_host(1000, 40, 12, seed=5)       # kappa = 1e12
    for v in ["bcgsi+", "p-2s"]:
        r = O.qr(X, 4, v)
        assert r.breakdown is None
        assert O.loss_of_orthogonality(r.Q) <= 10 * 40 * U64
    r = O.qr(X, 4, "p-1s")
    assert (r.breakdown is not None
            or O.loss_of_orthogonality(r.Q) > 1e3 * U64)


def test_bcgsi_1s_loses_orthogonality_like_kappa_squared():
    """Table 1: BCGSI+1s has LOO O(u) kappa^2 under O(u) kappa^3 <= 1 and
    no better: it drops the first Cholesky factor of Alg. 2, so its LOO
    grows with kappa where BCGSI+P-1S stays O(u).  Its residual stays
    O(u) and its R agrees with Householder to u kappa."""
    n = 80
    for dec in (2, 4):
        X = W.conditioned_host(2000, n, dec, seed=5)
        r = O.qr(X, 8, "bcgsi+1s")
        assert r.breakdown is None
        assert O.loss_of_orthogonality(r.Q) <= 10 * n * U64 * 10.0 ** (2 * dec)
        assert O.relative_residual(X, r.Q, r.R) <= 10 * n * U64
        Qh, Rh = O.householder_reference(X)
        assert (np.linalg.norm(r.R - Rh) / np.linalg.norm(Rh)
                <= 10 * n * U64 * 10.0 ** dec)
    X = W.conditioned_host(2000, n, 6, seed=5)
    loo_1s = O.loss_of_orthogonality(O.qr(X, 8, "bcgsi+1s").Q)
    loo_p1s = O.loss_of_orthogonality(O.qr(X, 8, "p-1s").Q)
    assert loo_p1s <= 10 * n * U64
    assert loo_1s >= 10 * loo_p1s


def test_rank_deficient_breaks_down_in_cholesky_variants():
    X = W.conditioned_host(100, 12, 2, seed=6)
    X[:, 7] = X[:, 2]
    for v in ["p-1s", "pipi+"]:
        r = O.qr(X, 4, v)
        assert r.breakdown is not None and r.breakdown.block == 1


# ------------------------------------------------------- closed forms ---

@pytest.mark.parametrize("variant", ALL5)
def test_scaled_permuted_identity_is_exact(variant):
    """One nonzero 2^e per column, distinct rows: every product is exact, so
    R = diag(2^e) and Q = X diag(2^-e) bit for bit."""
    n = 24
    e = np.random.default_rng(3).integers(-20, 20, size=n)
    X = W.scaled_permuted_identity(300, n, e, seed=3)
    r = O.qr(X, 4, variant)
    assert np.array_equal(r.R, np.diag(np.ldexp(1.0, e)))
    assert np.array_equal(r.Q, X * np.ldexp(1.0, -e)[None, :])


@pytest.mark.parametrize("variant", ALL5)
def test_hadamard_closed_form(variant):
    """Sylvester-Hadamard columns scaled by 2^e: R = sqrt(m) diag(2^e)."""
    m, n = 256, 16
    e = np.arange(n) % 5 - 2
    X = W.hadamard_columns(m, n, e)
    r = O.qr(X, 4, variant)
    Rex = math.sqrt(m) * np.diag(np.ldexp(1.0, e))
    kappa = 2.0 ** (e.max() - e.min())
    assert np.linalg.norm(r.R - Rex) / np.linalg.norm(Rex) <= 10 * n * U64 * kappa
    assert O.loss_of_orthogonality(r.Q) <= 10 * n * U64


def test_pythagorean_identity_exact_q():
    """With Q exactly orthonormal (columns of I), T - S^T S equals
    (X - QS)^T (X - QS) exactly: the subtraction the Pythagorean Cholesky
    (Alg. 1, Alg. 2) relies on."""
    rng = np.random.default_rng(8)
    m, k, s = 64, 6, 4
    Q = np.eye(m)[:, :k]
    Xb = np.ldexp(rng.integers(-8, 8, size=(m, s)).astype(float), -3)
    S = Q.T @ Xb
    T = Xb.T @ Xb
    V = Xb - Q @ S
    assert np.array_equal(T - S.T @ S, V.T @ V)


def test_input_generator_conditioning():
    X = W.conditioned_host(500, 40, 6, seed=9)
    sv = np.linalg.svd(X, compute_uv=False)
    assert abs(sv[0] - 1) < 1e-12
    assert abs(sv[0] / sv[-1] / 1e6 - 1) < 1e-6
