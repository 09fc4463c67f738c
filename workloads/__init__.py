"""Seeded synthetic inputs for the randomized LU hot path.

This module only draws random matrices with prescribed shapes and spectra.
It contains none of the factorization's arithmetic and is shared by the
tests, the benchmark and the oracle alike.

Recipes (shapes and spectra follow the paper's experiments in Section 5.1:
square matrices with exponentially decaying singular values, l = k + small
oversampling; and Section 5.2: slowly decaying spectra):

  * ``low_rank_plus_noise``  A = X Y^T + eps * N(0,1), X (m x r), Y (n x r)
  * ``spectral_matrix``      A = U diag(sigma) V^T with U, V Haar-distributed
    (Q factor of a Gaussian matrix with the signs of diag(R) folded in,
    Mezzadri 2007) -- on the host with NumPy, or on a device with torch
    (``spectral_matrix_torch``) when the sizes make a host QR too slow.
  * ``gaussian``             i.i.d. N(0,1) test matrices (explicit G).

All host draws use NumPy's PCG64 with the given seed.
"""
from __future__ import annotations

import math

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gaussian(shape, seed: int) -> np.ndarray:
    return rng(seed).standard_normal(shape)


def low_rank_plus_noise(m: int, n: int, r: int, eps: float, seed: int) -> np.ndarray:
    """X Y^T + eps * N(0, 1) with X (m x r), Y (n x r) standard normal."""
    g = rng(seed)
    X = g.standard_normal((m, r))
    Y = g.standard_normal((n, r))
    A = X @ Y.T
    if eps:
        A += eps * g.standard_normal((m, n))
    return A


def haar(n: int, g: np.random.Generator, cols: int | None = None) -> np.ndarray:
    """First ``cols`` columns of a Haar-distributed n x n orthogonal matrix."""
    cols = n if cols is None else cols
    Z = g.standard_normal((n, cols))
    Q, R = np.linalg.qr(Z, mode="reduced")
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s


def exp_decay(count: int, rate: float) -> np.ndarray:
    """sigma_i = exp(-i / rate), i = 1..count."""
    return np.exp(-np.arange(1, count + 1) / rate)


def inv_square(count: int) -> np.ndarray:
    """sigma_i = i^-2, i = 1..count."""
    i = np.arange(1, count + 1, dtype=np.float64)
    return 1.0 / (i * i)


def slow_decay(count: int) -> np.ndarray:
    """sigma_i = 100 / (9 + i)^2 (Section 5.2's slowly decaying spectrum)."""
    i = np.arange(1, count + 1, dtype=np.float64)
    return 100.0 / (9.0 + i) ** 2


def synthetic_factors(m: int, n: int, k: int, seed: int):
    """Seeded stand-ins for the outputs of a rank-k randomized LU, as inputs
    of the least-squares solve: L (m x k) unit lower trapezoidal with
    entries U(-1, 1) below the diagonal, U (k x n) upper trapezoidal with
    N(0, 1) entries and a diagonal of magnitude in [2, 3], and random
    permutations p (length m) and q (length n)."""
    g = rng(seed)
    L = np.tril(g.uniform(-1.0, 1.0, (m, k)), -1)
    L[np.arange(k), np.arange(k)] = 1.0
    U = np.triu(g.standard_normal((k, n)))
    U[np.arange(k), np.arange(k)] = g.choice([-1.0, 1.0], k) * g.uniform(2.0, 3.0, k)
    return L, U, g.permutation(m), g.permutation(n)


def spectral_matrix(m: int, n: int, sigma: np.ndarray, seed: int) -> np.ndarray:
    """U diag(sigma) V^T with Haar U (m x r), V (n x r), r = len(sigma)."""
    r = len(sigma)
    if r > min(m, n):
        raise ValueError("len(sigma) must be <= min(m, n)")
    g = rng(seed)
    U = haar(m, g, r)
    V = haar(n, g, r)
    return (U * sigma) @ V.T


def spectral_matrix_torch(m: int, n: int, sigma: np.ndarray, seed: int,
                          device: str = "cuda", dtype=None):
    """Device-side variant of ``spectral_matrix`` (same recipe, torch RNG):
    used where a host QR of the full Haar factors would take minutes."""
    import torch

    dtype = torch.float64 if dtype is None else dtype
    r = len(sigma)
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)

    def _haar(rows):
        Z = torch.randn(rows, r, generator=gen, device=device, dtype=torch.float64)
        Q, R = torch.linalg.qr(Z, mode="reduced")
        s = torch.sign(torch.diagonal(R))
        s[s == 0] = 1.0
        return Q * s

    U = _haar(m)
    V = _haar(n)
    sig = torch.as_tensor(np.asarray(sigma, dtype=np.float64), device=device)
    A = (U * sig) @ V.T.contiguous()
    return A.to(dtype)


# ---------------------------------------------------------------------------
# Named workloads (the five configurations the project measures)
# ---------------------------------------------------------------------------

def config_small(seed: int = 101):
    """512 x 512, A = X Y^T + 1e-9 N(0,1) with X, Y of 512 x 10, k=10, l=15."""
    A = low_rank_plus_noise(512, 512, 10, 1e-9, seed)
    return A, 10, 15


def config_exp_spectrum(size: int = 8192, seed: int = 102, device=None):
    """size^2 Haar U, V, sigma_i = exp(-i/50), k=200, l=210."""
    sigma = exp_decay(size, 50.0)
    if device is None:
        A = spectral_matrix(size, size, sigma, seed)
    else:
        A = spectral_matrix_torch(size, size, sigma, seed, device=device)
    return A, 200, 210


def batch_problems(count: int = 256, seed: int = 104, mn_lo: int = 256,
                   mn_hi: int = 4096, r_lo: int = 8, r_hi: int = 64,
                   eps: float = 1e-6):
    """Uneven batch: m, n ~ U[mn_lo, mn_hi], rank r ~ U[r_lo, r_hi];
    A = X Y^T + eps N(0,1) stored FP32; k = r, l = r + 8."""
    g = rng(seed)
    out = []
    for _ in range(count):
        m = int(g.integers(mn_lo, mn_hi + 1))
        n = int(g.integers(mn_lo, mn_hi + 1))
        r = int(g.integers(r_lo, r_hi + 1))
        s = int(g.integers(0, 2 ** 62))
        A = low_rank_plus_noise(m, n, r, eps, s).astype(np.float32)
        out.append((A, r, min(r + 8, m, n)))
    return out


def batch_shapes(count: int = 256, seed: int = 104, mn_lo: int = 256, mn_hi: int = 4096,
                 r_lo: int = 8, r_hi: int = 64):
    """Shapes of the uneven batch (same draws as ``batch_problems``):
    (m, n, r, data seed) with k = r and l = r + 8."""
    g = rng(seed)
    out = []
    for _ in range(count):
        m = int(g.integers(mn_lo, mn_hi + 1))
        n = int(g.integers(mn_lo, mn_hi + 1))
        r = int(g.integers(r_lo, r_hi + 1))
        s = int(g.integers(0, 2 ** 62))
        out.append((m, n, r, s))
    return out


def low_rank_plus_noise_torch(m: int, n: int, r: int, eps: float, seed: int,
                              device: str = "cuda", dtype=None):
    """Device-side ``low_rank_plus_noise`` (same recipe, torch RNG), returned
    column-major (stride (1, m)) in ``dtype``."""
    import torch

    dtype = torch.float32 if dtype is None else dtype
    gen = torch.Generator(device=device)
    gen.manual_seed(seed % (2 ** 63))
    X = torch.randn(m, r, generator=gen, device=device, dtype=torch.float64)
    Y = torch.randn(n, r, generator=gen, device=device, dtype=torch.float64)
    At = Y @ X.t()                       # n x m = A^T, contiguous -> A column-major
    if eps:
        At += eps * torch.randn(n, m, generator=gen, device=device, dtype=torch.float64)
    return At.to(dtype).t()


def serve_stream(count: int, seed: int = 105, m_lo: int = 512, m_hi: int = 32768,
                 n_lo: int = 512, n_hi: int = 8192, k_lo: int = 16, k_hi: int = 256):
    """Request shapes for the serving stream: m, n log-uniform, k uniform,
    l = k + 10, sigma_i = exp(-i/k) truncated at R = min(m, n, 24 k)."""
    g = rng(seed)
    shapes = []
    for _ in range(count):
        m = int(round(math.exp(g.uniform(math.log(m_lo), math.log(m_hi)))))
        n = int(round(math.exp(g.uniform(math.log(n_lo), math.log(n_hi)))))
        k = int(g.integers(k_lo, k_hi + 1))
        l = min(k + 10, m, n)
        k = min(k, l)
        shapes.append((m, n, k, l, int(g.integers(0, 2 ** 62))))
    return shapes
