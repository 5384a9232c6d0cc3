"""Seeded synthetic input matrices for the randomized QRCP workloads.

This module only *generates inputs*: it holds none of the factorization's
arithmetic and is shared by the oracle tests, the GPU parity tests and the
benchmark, so that both sides of every comparison read identical bytes.

Matrix families (all from the paper's experimental setting, Section V, which
uses random full-rank matrices and matrices with decaying spectra):

* ``lowrank(m, n, sigma, seed)`` -- ``U diag(sigma) V^T`` with ``U``, ``V``
  Haar-distributed (QR of a Gaussian matrix with the signs of ``diag(R)``
  folded into ``Q``, Mezzadri 2007).
* ``gaussian(m, n, seed)`` -- i.i.d. N(0, 1) entries.
* ``kahan(n, c, s2)`` -- the Kahan matrix ``diag(s^(i-1)) (I - c N)`` of the
  paper's pathological-matrix experiment (Section V-B), where ``N`` is the
  strictly upper triangular matrix of ones and ``s2 = s^2``.
* ``kahan_embedded(m, n, nk, ...)`` -- a Kahan block in the top-left corner
  next to graded Gaussian columns: QRCP keeps the Kahan columns first, so the
  swaps of Alg. 3 have many trailing candidates to choose from.
* ``integer_matrix`` -- small integer matrices for exact rational tests.
* ``rbf_kernel(n, d, seed, gamma)`` -- an n x n Gaussian (RBF) kernel matrix
  exp(-gamma ||x_i - x_j||^2) of n seeded points in d dimensions: a stand-in
  for the kernel matrix of the CUR/CX experiment (Section V-D, 4177 points of
  8 features), whose data set is not used here.

Random streams are ``numpy.random.default_rng([family_seed, stream])``.
The large matrices of the benchmark can also be generated on the GPU with
torch (``lowrank_torch``), with the same recipe and a torch generator.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "rng", "haar_columns", "lowrank", "gaussian", "kahan", "integer_matrix",
    "sigma_exp", "sigma_pow", "separated_lowrank", "lowrank_torch",
    "gaussian_torch", "batch_shapes", "kahan_embedded", "rbf_kernel",
]


def rng(seed: int, stream: int = 0) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(stream)])


def haar_columns(m: int, r: int, gen: np.random.Generator) -> np.ndarray:
    """First ``r`` columns of a Haar-distributed ``m x m`` orthogonal matrix."""
    g = gen.standard_normal((m, r))
    q, rr = np.linalg.qr(g)
    d = np.sign(np.diag(rr))
    d[d == 0] = 1.0
    return q * d


def sigma_exp(r: int, scale: float) -> np.ndarray:
    """sigma_j = exp(-j / scale), j = 1..r."""
    return np.exp(-np.arange(1, r + 1, dtype=np.float64) / scale)


def sigma_pow(r: int, power: float) -> np.ndarray:
    """sigma_j = j^(-power), j = 1..r."""
    return np.arange(1, r + 1, dtype=np.float64) ** (-power)


def lowrank(m: int, n: int, sigma: np.ndarray, seed: int,
            noise_std: float = 0.0) -> np.ndarray:
    """``U diag(sigma) V^T`` (Fortran order, float64), plus optional N(0, noise_std^2)."""
    r = len(sigma)
    assert r <= min(m, n)
    u = haar_columns(m, r, rng(seed, 1))
    v = haar_columns(n, r, rng(seed, 2))
    a = (u * sigma) @ v.T
    if noise_std:
        a = a + noise_std * rng(seed, 3).standard_normal((m, n))
    return np.asfortranarray(a)


def gaussian(m: int, n: int, seed: int) -> np.ndarray:
    return np.asfortranarray(rng(seed, 4).standard_normal((m, n)))


def kahan(n: int, c: float = 0.285, s2: float | None = None) -> np.ndarray:
    """Kahan matrix ``diag(1, s, s^2, ...) (I - c N)``, ``s^2 = s2``.

    The default ``s2 = 0.9998 - c^2`` is the value for which the Kahan
    residuals of the paper's first table are reproduced.
    """
    if s2 is None:
        s2 = 0.9998 - c * c
    s = math.sqrt(s2)
    k = np.eye(n) - c * np.triu(np.ones((n, n)), 1)
    return np.asfortranarray(np.diag(s ** np.arange(n)) @ k)


def kahan_embedded(m: int, n: int, nk: int, seed: int, c: float = 0.285,
                   scale: float = 0.03, decay: float = 30.0) -> np.ndarray:
    """``kahan(nk, c)`` in rows/columns 0..nk-1; columns nk..n-1 are N(0, 1)
    scaled by ``scale * exp(-j / decay)`` (j = 0, 1, ...) over all m rows."""
    a = np.zeros((m, n))
    a[:nk, :nk] = kahan(nk, c)
    a[:, nk:] = (scale * rng(seed, 7).standard_normal((m, n - nk))
                 * np.exp(-np.arange(n - nk) / decay))
    return np.asfortranarray(a)


def rbf_kernel(n: int, d: int, seed: int, gamma: float = 1.0) -> np.ndarray:
    """exp(-gamma ||x_i - x_j||^2) for n points x_i: d features, each feature an
    N(0,1) draw scaled by a per-feature spread in [0.1, 1] (clustered, unevenly
    scaled data rather than an isotropic cloud)."""
    g = rng(seed, 8)
    spread = np.linspace(0.1, 1.0, d)
    centers = g.standard_normal((8, d)) * spread
    x = centers[g.integers(0, 8, size=n)] + 0.3 * g.standard_normal((n, d)) * spread
    sq = np.sum(x * x, axis=1)
    d2 = np.maximum(sq[:, None] + sq[None, :] - 2.0 * x @ x.T, 0.0)
    return np.asfortranarray(np.exp(-gamma * d2))


def integer_matrix(m: int, n: int, seed: int, lo: int = -9, hi: int = 9) -> np.ndarray:
    return np.asfortranarray(rng(seed, 5).integers(lo, hi + 1, size=(m, n)).astype(np.float64))


def separated_lowrank(m: int, n: int, seed: int, decay: float = 40.0) -> np.ndarray:
    """Low-rank-ish test matrix with ``sigma_j = exp(-j/decay)`` and rank min(m, n)."""
    r = min(m, n)
    return lowrank(m, n, sigma_exp(r, decay), seed)


# ---------------------------------------------------------------------------
# Large inputs, generated on a GPU with torch (same recipe, torch generator).
# ---------------------------------------------------------------------------

def _torch_haar_columns(m, r, gen, device, dtype):
    import torch
    g = torch.randn(m, r, generator=gen, device=device, dtype=torch.float64)
    q, rr = torch.linalg.qr(g)
    d = torch.sign(torch.diagonal(rr))
    d[d == 0] = 1.0
    return (q * d).to(dtype)


def lowrank_torch(m, n, sigma, seed, device="cuda", dtype=None, noise_std=0.0):
    """Column-major ``U diag(sigma) V^T`` on ``device``; returns a tensor whose
    storage is column-major (a transposed view of a row-major ``n x m``)."""
    import torch
    dtype = dtype or torch.float64
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) * 1000003 + 17)
    sig = torch.as_tensor(np.asarray(sigma), device=device, dtype=torch.float64)
    r = sig.numel()
    u = _torch_haar_columns(m, r, gen, device, torch.float64)
    v = _torch_haar_columns(n, r, gen, device, torch.float64)
    # build A^T (n x m, row-major) so that the storage is A in column-major
    at = (v * sig) @ u.T.contiguous()
    del u, v
    if noise_std:
        at += noise_std * torch.randn(n, m, generator=gen, device=device, dtype=torch.float64)
    return at.to(dtype).t()


def gaussian_torch(m, n, seed, device="cuda", dtype=None):
    import torch
    dtype = dtype or torch.float64
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed) * 1000003 + 29)
    return torch.randn(n, m, generator=gen, device=device, dtype=torch.float64).to(dtype).t()


def batch_shapes(count: int, seed: int, m_range=(64, 1024), n_range=(64, 512)):
    """Uneven batch: m ~ U{m_range}, n ~ U{n_range}, k = n // 8."""
    g = rng(seed, 6)
    ms = g.integers(m_range[0], m_range[1] + 1, size=count)
    ns = g.integers(n_range[0], n_range[1] + 1, size=count)
    return [(int(m), int(n), int(n) // 8) for m, n in zip(ms, ns)]
