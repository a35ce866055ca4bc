"""Seeded synthetic inputs shaped like the paper's workloads.

Shared by the tests, the benchmark and the smoke check, and by both sides of
every parity comparison (GPU library and CPU oracle).  It only *constructs*
matrices; it holds none of the factorisation arithmetic of the method: no
Householder QR, Cholesky, eigensolver or Gram kernel.

Constructions
  * ``orthonormal_columns``: Q0 = H_1 ... H_p [I; 0] with H_i = I - 2 v v^T / (v^T v),
    v iid N(0, 1) -- a dense m x n matrix with orthonormal columns.
  * ``triangular_with_singular_values``: an upper-triangular R0 with
    prescribed singular values, built from diag(sigma) by two-sided plane
    rotations (a random rotation of two adjacent rows, then the column
    rotation that restores the zero below the diagonal).  Orthogonal
    transformations on both sides keep the singular values, so
    kappa(R0) = sigma_max / sigma_min exactly up to rounding.
  * ``known_r``: X = Q0 R0, whose sign-normalised R factor is R0.

The paper uses synthetic matrices with m*n held fixed, n in {1, 8, 16, 32, 64}
and kappa below eps^{-1/2} (Sec. 4.1).  The seeds and shapes below follow the
five workload definitions this project benchmarks (see ``CONFIGS``).
"""
from __future__ import annotations

import math

import numpy as np

# ------------------------------------------------------------ random streams


def rng(seed: int) -> np.random.Generator:
    """numpy PCG64 stream for a seed (host-side inputs)."""
    return np.random.Generator(np.random.PCG64(seed))


def gaussian(m: int, n: int, seed: int) -> np.ndarray:
    """m x n row-major matrix with iid N(0, 1) entries."""
    return rng(seed).standard_normal((m, n))


def dyadic(m: int, n: int, seed: int, lo: int = -16, hi: int = 16) -> np.ndarray:
    """Entries k/8 with integer k in [lo, hi]: exactly representable, and
    their products and sums are exact in binary64 for tiny sizes, so exact
    rational arithmetic can reproduce every input bit."""
    return rng(seed).integers(lo, hi + 1, size=(m, n)).astype(np.float64) / 8.0


# -------------------------------------------------------------- structures


def orthonormal_columns(m: int, n: int, g: np.random.Generator, p: int | None = None) -> np.ndarray:
    """Q0 = H_1 ... H_p [I_n; 0] (m x n, m >= n) with dense random reflectors."""
    if m < n:
        raise ValueError("orthonormal_columns needs m >= n")
    p = n if p is None else p
    E = np.zeros((m, n))
    E[np.arange(n), np.arange(n)] = 1.0
    vs = [g.standard_normal(m) for _ in range(p)]
    for v in reversed(vs):                       # E <- H_i E, innermost first
        w = v @ E
        E -= np.outer(v, w * (2.0 / (v @ v)))
    return E


def triangular_with_singular_values(sigma, g: np.random.Generator, sweeps: int | None = None) -> np.ndarray:
    """Upper-triangular n x n R0 with singular values ``sigma`` and a
    non-negative diagonal, by random two-sided adjacent plane rotations."""
    sigma = np.asarray(sigma, dtype=np.float64)
    n = sigma.size
    T = np.diag(sigma).copy()
    sweeps = max(2 * n, 4) if sweeps is None else sweeps
    for _ in range(sweeps):
        for i in range(n - 1):
            th = g.uniform(0.0, 2.0 * math.pi)
            c, s = math.cos(th), math.sin(th)
            ri, rj = T[i].copy(), T[i + 1].copy()
            T[i] = c * ri - s * rj
            T[i + 1] = s * ri + c * rj          # fills T[i+1, i]
            a, b = T[i + 1, i], T[i + 1, i + 1]
            r = math.hypot(a, b)
            if r == 0.0:
                continue
            cc, ss = b / r, a / r
            ci, cj = T[: i + 2, i].copy(), T[: i + 2, i + 1].copy()
            T[: i + 2, i] = cc * ci - ss * cj
            T[: i + 2, i + 1] = ss * ci + cc * cj
            T[i + 1, i] = 0.0                    # zero by construction
    T = np.triu(T)
    neg = np.diag(T) < 0
    T[neg] *= -1.0
    return T + 0.0


def logspace_sigma(n: int, k: float) -> np.ndarray:
    """sigma_i = 10^{-k (i-1)/(n-1)}, i = 1..n (n = 1: sigma = 1)."""
    if n == 1:
        return np.ones(1)
    return 10.0 ** (-k * np.arange(n) / (n - 1))


def loguniform_sigma(n: int, smin: float, g: np.random.Generator) -> np.ndarray:
    """sigma_1 = 1, sigma_n = smin, the rest log-uniform on [smin, 1]."""
    if n == 1:
        return np.ones(1)
    mid = np.exp(g.uniform(math.log(smin), 0.0, size=max(n - 2, 0)))
    return np.concatenate([[1.0], np.sort(mid)[::-1], [smin]])


def known_r(m: int, n: int, sigma, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """(X, R0) with X = Q0 R0, Q0 orthonormal columns, R0 upper triangular with
    singular values sigma and diag(R0) >= 0, so R(X) = R0."""
    g = rng(seed)
    R0 = triangular_with_singular_values(sigma, g)
    Q0 = orthonormal_columns(m, n, g)
    return Q0 @ R0, R0


def svd_form(m: int, n: int, sigma, seed: int) -> np.ndarray:
    """X = U diag(sigma) V^T with U (m x n) and V (n x n) orthonormal, each a
    product of dense random reflectors: singular values sigma, and the
    ill-conditioning spread over all columns rather than graded along them."""
    g = rng(seed)
    U = orthonormal_columns(m, n, g)
    V = orthonormal_columns(n, n, g)
    return (U * np.asarray(sigma, dtype=np.float64)) @ V.T


# ------------------------------------------------- device-side construction


def known_r_torch(m: int, n: int, sigma, seed: int, device="cuda"):
    """Same construction as ``known_r`` for sizes where host generation is too
    slow: R0 on the host (numpy, seed), Q0 from reflectors drawn with torch's
    generator on ``device`` (seed + 1).  Returns (X tensor, R0 ndarray)."""
    import torch
    g = rng(seed)
    R0 = triangular_with_singular_values(sigma, g)
    tg = torch.Generator(device=device)
    tg.manual_seed(seed + 1)
    E = torch.zeros((m, n), dtype=torch.float64, device=device)
    E[torch.arange(n), torch.arange(n)] = 1.0
    vs = [torch.randn(m, dtype=torch.float64, device=device, generator=tg) for _ in range(n)]
    for v in reversed(vs):
        w = v @ E
        E.addr_(v, w, alpha=-2.0 / float(v @ v))
    del vs
    X = E @ torch.from_numpy(R0).to(device)
    del E
    return X.contiguous(), R0


def gaussian_torch(m: int, n: int, seed: int, device="cuda"):
    """m x n iid N(0, 1) drawn with torch's generator on ``device``."""
    import torch
    tg = torch.Generator(device=device)
    tg.manual_seed(seed)
    return torch.randn((m, n), dtype=torch.float64, device=device, generator=tg)


# ---------------------------------------------------------------- workloads

CONFIGS = {
    1: "single 100000 x 4, iid N(0,1), seed 1",
    2: "single 5e7 x 8, X = Q0 R0, sigma(R0) log-uniform in [1e-4, 1] with both ends, seed 2",
    3: "m = 2^25, n in {1,2,4,8,16,32,64}, sigma_i = 10^{-k(i-1)/(n-1)}, k in {0,4,8}, seed 3000+100k+n",
    4: "512 matrices, m log-uniform [1e4, 1e7], n uniform {4,8,16,32}, iid N(0,1), seed 4",
    5: "Poisson least-squares requests [A b], m log-uniform [1e4, 5e7], n uniform 3..47, seed 5",
}


def config1() -> np.ndarray:
    return gaussian(100_000, 4, seed=1)


def config2_sigma(n: int = 8) -> np.ndarray:
    return loguniform_sigma(n, 1e-4, rng(2))


def config2(m: int = 50_000_000, n: int = 8, device=None):
    """X = Q0 R0 with kappa = 1e4.  ``device`` None: numpy on the host."""
    sig = config2_sigma(n)
    if device is None:
        return known_r(m, n, sig, seed=2)
    return known_r_torch(m, n, sig, seed=2, device=device)


def config3_seed(n: int, k: int) -> int:
    return 3000 + 100 * k + n


def config3(n: int, k: int, m: int = 2 ** 25, device=None):
    sig = logspace_sigma(n, k)
    if device is None:
        return known_r(m, n, sig, seed=config3_seed(n, k))
    return known_r_torch(m, n, sig, seed=config3_seed(n, k), device=device)


def batched_shapes(count: int = 512, seed: int = 4, mlo: float = 1e4, mhi: float = 1e7,
                   ns=(4, 8, 16, 32)) -> list[tuple[int, int]]:
    """(m_i, n_i) for the batched workload: m log-uniform, n uniform over ns."""
    g = rng(seed)
    ms = np.floor(np.exp(g.uniform(math.log(mlo), math.log(mhi), size=count))).astype(np.int64)
    nn = g.choice(np.asarray(ns), size=count)
    return [(int(a), int(b)) for a, b in zip(ms, nn)]


def server_requests(count: int, rate_per_s: float, seed: int = 5, mlo: float = 1e4, mhi: float = 5e7,
                    nlo: int = 3, nhi: int = 47) -> list[dict]:
    """Poisson arrivals (exponential gaps at ``rate_per_s``) of least-squares
    requests.  Each gets m (log-uniform), n (uniform nlo..nhi) and its own
    data seed; the data itself is drawn by ``ls_request_data``."""
    g = rng(seed)
    t = np.cumsum(g.exponential(1.0 / rate_per_s, size=count))
    ms = np.floor(np.exp(g.uniform(math.log(mlo), math.log(mhi), size=count))).astype(np.int64)
    ns = g.integers(nlo, nhi + 1, size=count)
    return [{"id": i, "arrival_s": float(t[i]), "m": int(ms[i]), "n": int(ns[i]),
             "seed": int(seed * 1_000_003 + i)} for i in range(count)]


def ls_request_data(m: int, n: int, seed: int, noise: float = 1e-6, device=None):
    """[A b] (m x (n+1), row-major) and x0 with b = A x0 + noise * N(0, 1)."""
    if device is None:
        g = rng(seed)
        A = g.standard_normal((m, n))
        x0 = g.standard_normal(n)
        Ab = np.empty((m, n + 1))
        Ab[:, :n] = A
        Ab[:, n] = A @ x0 + noise * g.standard_normal(m)
        return Ab, x0
    import torch
    tg = torch.Generator(device=device)
    tg.manual_seed(seed)
    Ab = torch.randn((m, n + 1), dtype=torch.float64, device=device, generator=tg)
    x0 = torch.randn(n, dtype=torch.float64, device=device, generator=tg)
    e = torch.randn(m, dtype=torch.float64, device=device, generator=tg)
    Ab[:, n] = Ab[:, :n] @ x0 + noise * e
    return Ab, x0.cpu().numpy()


def two_phase_data(m: int, p: int, n: int, k: float, seed: int):
    """(Y, X, B0, R0) for the two-phase problem: [Y W] = H_1 ... H_{p+n} [I; 0]
    with orthonormal columns (m x (p+n)), B0 iid N(0,1) (p x n), R0 upper
    triangular with singular values 1 .. 10^-k, X = Y B0 + W R0 -- so that
    Y^T X = B0 and R((I - Y Y^T) X) = R0."""
    g = rng(seed)
    U = orthonormal_columns(m, p + n, g)
    Y, W = np.ascontiguousarray(U[:, :p]), U[:, p:]
    B0 = g.standard_normal((p, n))
    R0 = triangular_with_singular_values(logspace_sigma(n, k), g)
    return Y, np.ascontiguousarray(Y @ B0 + W @ R0), B0, R0

