"""Helpers for GPU-vs-oracle parity tests (imported by the GPU tests).

Tolerances (binary64, u = 2^-53, n columns, kappa = kappa(X)):
  syncs      the device's count of completed synchronization points equals
             the oracle's count of the same variant
  status     identical; a breakdown on one side only is accepted when the
             other side's failing pivot is within 64 s u ||A|| of zero
             (a rounding-level tie at the breakdown threshold)
  structure  R strictly lower == 0, diag(R) > 0 (when no breakdown)
  LOO        if the oracle's ||Q^T Q - I|| <= 10 n u then the GPU's too;
             otherwise within a factor 10 of the oracle's
  residual   ||X - QR|| / ||X|| <= 10 n u
  R          ||R_gpu - R_oracle||_F / ||R_oracle||_F <= 10 n u kappa, and
             the same ratio for every block column of s columns
  Q          ||Q_gpu - Q_oracle||_F / sqrt(n) <= 10 n u kappa
The factor 10 n u is the reading of Table 1's O(u); the kappa factor is
the first-order perturbation bound of the QR factors.
"""

import math
import sys

import numpy as np

import oracle as O

U64 = 2.0 ** -53


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_device(Xh, dtype=None):
    import torch
    Xh = np.asfortranarray(Xh)
    t = torch.from_numpy(Xh)
    if dtype is not None:
        t = t.to(dtype)
    out = torch.empty((Xh.shape[1], Xh.shape[0]), dtype=t.dtype,
                      device="cuda").t()
    out.copy_(t)
    return out


def run_gpu(X, s, variant, precision="fp64"):
    """X: host array or device tensor.  Returns host Q, R and the info."""
    import torch
    from paper_2507_21791_amd import bcgs
    Xd = X if hasattr(X, "is_cuda") else to_device(
        X, torch.float64 if precision == "fp64" else torch.float32)
    Q, R, ws = bcgs.qr(Xd, s, variant, precision)
    torch.cuda.synchronize()
    info = ws.info()
    return Q, R, info


def host(t):
    return np.asfortranarray(t.double().cpu().numpy())


def kappa_of(X):
    sv = np.linalg.svd(X, compute_uv=False)
    return sv[0] / sv[-1]


def compare(X, s, variant, Qg, Rg, info, kappa=None, oracle_result=None):
    """Assert C5 parity of (Qg, Rg, info) with the oracle on X (host)."""
    m, n = X.shape
    r = oracle_result or O.qr(X, s, variant)
    kappa = kappa if kappa is not None else kappa_of(X)
    tol_pert = 10 * n * U64 * kappa
    if r.breakdown is not None or info.status != 0:
        assert r.breakdown is not None and info.status == 2, (
            f"breakdown mismatch: oracle {r.breakdown}, gpu {info.as_dict()}")
        assert info.block == r.breakdown.block, (info.as_dict(), r.breakdown)
        return {"breakdown": info.block}
    Rg = np.asarray(Rg)
    Qg = np.asarray(Qg)
    # synchronization points counted on the device as they completed
    assert info.syncs == r.syncs, (info.syncs, r.syncs)
    assert np.all(np.tril(Rg, -1) == 0.0), "R not upper triangular"
    assert np.all(np.diag(Rg) > 0), "diag(R) not positive"
    loo_o = O.loss_of_orthogonality(r.Q)
    loo_g = O.loss_of_orthogonality(Qg)
    if loo_o <= 10 * n * U64:
        assert loo_g <= 10 * n * U64, (loo_g, loo_o)
    else:
        assert abs(math.log10(loo_g / loo_o)) <= 1, (loo_g, loo_o)
    res = O.relative_residual(X, Qg, Rg)
    assert res <= 10 * n * U64, res
    rerr = np.linalg.norm(Rg - r.R) / np.linalg.norm(r.R)
    assert rerr <= tol_pert, (rerr, tol_pert)
    rcol = block_column_errors(Rg, r.R, s)
    worst = int(np.argmax(rcol))
    assert rcol[worst] <= tol_pert, (worst, rcol[worst], tol_pert)
    qerr = np.linalg.norm(Qg - r.Q) / math.sqrt(n)
    assert qerr <= tol_pert, (qerr, tol_pert)
    return {"loo_gpu": loo_g, "loo_oracle": loo_o, "res": res,
            "r_err": rerr, "r_col_err": float(rcol[worst]), "q_err": qerr}


def block_column_errors(Rg, Ro, s):
    """||R_gpu[:, K] - R_or[:, K]||_F / ||R_or[:, K]||_F for every block
    column K (s columns): a whole-matrix ratio would hide errors in block
    columns whose norm is far below ||R||."""
    n = Ro.shape[1]
    out = np.empty(n // s)
    for k in range(n // s):
        c = slice(k * s, (k + 1) * s)
        out[k] = np.linalg.norm(Rg[:, c] - Ro[:, c]) / np.linalg.norm(Ro[:, c])
    return out


U32 = 2.0 ** -24


def compare_bulk32(X, s, variant, Qg, Rg, info, kappa):
    """FP32-bulk result (Qg binary32 promoted, Rg binary64) against the FP64
    oracle on the same X (X holds binary32-representable values).

    The inputs are chosen inside Table 1's assumptions with u = u32 and a
    margin (u32 kappa <= 1e-3 for BCGSI+ and P-2S, u32 kappa^2 <= 1e-2 for
    P-1S), so no breakdown is allowed and the O(u) bounds apply with
    u = u32:  LOO <= 10 n u32, residual <= 10 n u32, R and Q within
    10 n u32 kappa of the FP64 oracle."""
    m, n = X.shape
    r = O.qr(X, s, variant)
    assert r.breakdown is None, r.breakdown
    assert info.status == 0, info.as_dict()
    assert info.syncs == r.syncs, (info.syncs, r.syncs)
    Rg = np.asarray(Rg)
    Qg = np.asarray(Qg)
    assert np.all(np.tril(Rg, -1) == 0.0), "R not upper triangular"
    assert np.all(np.diag(Rg) > 0), "diag(R) not positive"
    tol = 10 * n * U32
    loo_g = O.loss_of_orthogonality(Qg)
    assert loo_g <= tol, (loo_g, tol)
    res = O.relative_residual(X, Qg, Rg)
    assert res <= tol, (res, tol)
    rerr = np.linalg.norm(Rg - r.R) / np.linalg.norm(r.R)
    assert rerr <= tol * kappa, (rerr, tol * kappa)
    rcol = block_column_errors(Rg, r.R, s)
    assert rcol.max() <= tol * kappa, (int(np.argmax(rcol)), rcol.max())
    qerr = np.linalg.norm(Qg - r.Q) / math.sqrt(n)
    assert qerr <= tol * kappa, (qerr, tol * kappa)
    return {"loo_gpu": loo_g, "loo_oracle": O.loss_of_orthogonality(r.Q),
            "res": res, "r_err": rerr, "q_err": qerr}
