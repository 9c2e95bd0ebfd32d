"""Seeded synthetic inputs for the BCGS QR kernels and for their checks.

The paper tests on random matrices (section 4).  The workloads here follow
its shape (tall-skinny, rows >> columns) with a prescribed singular-value
profile so that the condition number kappa(X) is known by construction:

    X = U diag(sigma) V^T,   U (m x n) and V (n x n) orthonormal,
    sigma = logspace(0, -c, n)   =>  ||X||_2 = 1,  kappa(X) = 10^c.

U and V are the Q factors of seeded standard-normal matrices, obtained with
the library Householder QR (numpy/LAPACK on the host, torch on the device).
Nothing in this module uses the code under test or the oracle; both sides
receive the same arrays.

All matrices are returned in column-major (Fortran) order: a host array
with ``flags.f_contiguous``, or a torch tensor of shape (m, n) with strides
(1, m).
"""

import math

import numpy as np

# ---------------------------------------------------------------- host ---


def sigma_profile(n, decades):
    """sigma_i = 10^(-decades * i / (n-1)), i = 0..n-1 (n points)."""
    if n == 1:
        return np.ones(1)
    return np.logspace(0.0, -float(decades), n)


def orthonormal_host(rng, m, n):
    """Q factor of an m x n standard-normal matrix (LAPACK Householder)."""
    G = rng.standard_normal((m, n))
    Q, _ = np.linalg.qr(G, mode="reduced")
    return Q


def conditioned_host(m, n, decades, seed):
    """X = U diag(logspace(0, -decades, n)) V^T on the host, kappa = 10^decades."""
    rng = np.random.default_rng(seed)
    U = orthonormal_host(rng, m, n)
    V = orthonormal_host(rng, n, n)
    sig = sigma_profile(n, decades)
    return np.asfortranarray((U * sig[None, :]) @ V.T)


def gaussian_plus_structured_host(m, n, decades, scale, seed):
    """X = G + scale * U diag(logspace(0, -decades, n)) V^T with G i.i.d.
    N(0,1): the block-size sweep workload (kappa close to 1)."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((m, n))
    U = orthonormal_host(rng, m, n)
    V = orthonormal_host(rng, n, n)
    sig = sigma_profile(n, decades)
    return np.asfortranarray(G + scale * ((U * sig[None, :]) @ V.T))


# -------------------------------------------------------------- device ---


def _torch():
    import torch
    return torch


def fortran_empty(m, n, dtype, device):
    """Uninitialised m x n tensor in column-major order (strides (1, m))."""
    torch = _torch()
    return torch.empty((n, m), dtype=dtype, device=device).t()


def to_fortran(T):
    """Copy of a 2-D tensor in column-major order."""
    return T.t().contiguous().t()


def conditioned_device(m, n, decades, seed, device="cuda"):
    """Device twin of ``conditioned_host`` (torch generator, torch QR).

    Used for inputs too large to build on the host (millions of rows).
    X^T = (V diag(sigma)) U^T is formed as one n x m row-major product, which
    is X in column-major order."""
    torch = _torch()
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    G = torch.randn((n, m), generator=g, device=device, dtype=torch.float64).t()
    U, _ = torch.linalg.qr(G, mode="reduced")
    del G
    H = torch.randn((n, n), generator=g, device=device, dtype=torch.float64)
    V, _ = torch.linalg.qr(H, mode="reduced")
    sig = torch.from_numpy(sigma_profile(n, decades)).to(device)
    Xt = torch.mm(V * sig[None, :], U.t())
    del U
    return Xt.t()


def gaussian_plus_structured_device(m, n, decades, scale, seed, device="cuda"):
    """Device twin of ``gaussian_plus_structured_host``."""
    torch = _torch()
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    Xt = torch.randn((n, m), generator=g, device=device, dtype=torch.float64)
    G = torch.randn((n, m), generator=g, device=device, dtype=torch.float64).t()
    U, _ = torch.linalg.qr(G, mode="reduced")
    del G
    H = torch.randn((n, n), generator=g, device=device, dtype=torch.float64)
    V, _ = torch.linalg.qr(H, mode="reduced")
    sig = torch.from_numpy(sigma_profile(n, decades)).to(device)
    Xt.addmm_(V * (scale * sig)[None, :], U.t())
    return Xt.t()


# ------------------------------------------------------------ workloads ---

# The five workloads the benchmarks and tests are built around.  Each entry
# gives the shape, block size, singular-value decay (decades) and seed.
WORKLOADS = {
    # accuracy case: kappa = 1e6, 10 block columns
    "small": dict(m=2000, n=80, s=8, decades=6, seed=1),
    # the headline streaming case: 4M x 256, s = 16, kappa = 1e8 (about
    # 8.6 GB of FP64 input); "tall-k6" is its kappa = 1e6 twin
    "tall": dict(m=1 << 22, n=256, s=16, decades=8, seed=2),
    "tall-k6": dict(m=1 << 22, n=256, s=16, decades=6, seed=2),
    # block-size sweep: 1M x 512, N(0,1) plus a 1e-2 scaled structured part
    "sweep": dict(m=1 << 20, n=512, s=16, decades=10, seed=3, scale=1e-2),
}


def make_host(name, m=None, **over):
    w = dict(WORKLOADS[name])
    w.update(over)
    if m is not None:
        w["m"] = m
    if "scale" in w:
        return gaussian_plus_structured_host(w["m"], w["n"], w["decades"],
                                             w["scale"], w["seed"])
    return conditioned_host(w["m"], w["n"], w["decades"], w["seed"])


def make_device(name, m=None, device="cuda", **over):
    w = dict(WORKLOADS[name])
    w.update(over)
    if m is not None:
        w["m"] = m
    if "scale" in w:
        return gaussian_plus_structured_device(w["m"], w["n"], w["decades"],
                                               w["scale"], w["seed"], device)
    return conditioned_device(w["m"], w["n"], w["decades"], w["seed"], device)


# ------------------------------------------------- special structured X ---


def scaled_permuted_identity(m, n, exponents, seed):
    """Each column has one nonzero 2^e_j, in distinct rows (a random row
    permutation).  Every Gram matrix, Cholesky factor and Householder step on
    it is exact in binary floating point, so every variant must return
    R = diag(2^e) and Q = X diag(2^-e) exactly."""
    rng = np.random.default_rng(seed)
    rows = rng.permutation(m)[:n]
    X = np.zeros((m, n), order="F")
    for j in range(n):
        X[rows[j], j] = math.ldexp(1.0, int(exponents[j]))
    return X


def hadamard_columns(m, n, exponents):
    """First n columns of the Sylvester-Hadamard matrix of order m (a power
    of two), column j scaled by 2^e_j.  Its exact QR has
    R = sqrt(m) diag(2^e) and Q = H[:, :n] / sqrt(m)."""
    assert m & (m - 1) == 0 and m >= n
    H = np.ones((1, 1))
    while H.shape[0] < m:
        H = np.block([[H, H], [H, -H]])
    X = H[:, :n] * np.ldexp(1.0, np.asarray(exponents, dtype=int))[None, :]
    return np.asfortranarray(X)


# ------------------------------------------------ batched and served mixes ---


def batched_specs(count=256, seed=4):
    """Shapes of the batched workload: `count` independent problems with m
    uniform in [10000, 200000], n in {32, 64, 128, 256}, s in {8, 16} and
    singular values logspace(0, -c, n), c uniform in [2, 10].  Returns a
    list of dicts (m, n, s, decades, seed); problem i is generated from
    seed + i."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        out.append(dict(m=int(rng.integers(10000, 200001)),
                        n=int(rng.choice([32, 64, 128, 256])),
                        s=int(rng.choice([8, 16])),
                        decades=float(rng.uniform(2.0, 10.0)),
                        seed=seed + i))
    return out


def served_pool_specs(count, seed=5):
    """Inputs of the served stream, drawn once into a device pool: m
    log-uniform in [4096, 2^21], n in {16, 32, ..., 512}, s = 16 and
    kappa log-uniform in [1e2, 1e8] (singular values logspace(0, -c, n))."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        m = int(round(math.exp(rng.uniform(math.log(4096),
                                           math.log(1 << 21)))))
        n = int(16 * rng.integers(1, 33))
        out.append(dict(m=max(m, n), n=n, s=16,
                        decades=float(rng.uniform(2.0, 8.0)),
                        seed=1000 * seed + i))
    return out


def served_trace(nreq, rate, pool_size, seed=5):
    """Poisson arrivals at `rate` requests/s: (arrival time in s, pool index
    drawn uniformly with replacement) for each of `nreq` requests."""
    rng = np.random.default_rng(seed + 7919)
    t = np.cumsum(rng.exponential(1.0 / rate, size=nreq))
    idx = rng.integers(0, pool_size, size=nreq)
    return [(float(a), int(b)) for a, b in zip(t, idx)]
