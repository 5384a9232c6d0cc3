"""Gaussian sketching matrix Omega from a counter-based generator.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper only asks for an i.i.d. N(0, 1) matrix Omega of size (b+p) x m
(the Gaussian sketching matrix of Alg. 2; Alg. 3 draws a second one of size
d x (l+1)).  To let the oracle and the GPU library draw the *same* Omega from
a seed without sharing any code, both implement one published generator:

* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As Easy
  as 1, 2, 3", SC'11): 256-bit counter, 128-bit key, 10 rounds of
  ``(c0, c1, c2, c3) -> (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0))``
  with the key bumped by the Weyl constants between rounds.
* key = (seed, stream); normal number q uses counter (q // 4 + 1, 0, 0, 0) and
  output word q % 4 (the "+1" matches NumPy's Philox, which increments its
  counter before producing a block).
* uniform u = ((x >> 12) + 1/2) * 2^-52: the top 52 bits plus one half, which is
  exact in double precision and lies in [2^-53, 1 - 2^-53], strictly inside (0, 1)
  (with 53 bits the largest word would round to exactly 1).
* Box-Muller on the word pairs (0, 1) and (2, 3):
  ``z_even = sqrt(-2 ln u_even) cos(2 pi u_odd)``, ``z_odd = sqrt(-2 ln u_even) sin(2 pi u_odd)``.
* Omega[r, c] (column-major, leading dimension = rows) is normal number
  ``q = c * rows + r``.
"""
from __future__ import annotations

import math

import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
MASK64 = (1 << 64) - 1
TWO_PI = 6.283185307179586  # the double nearest to 2*pi

# Stream ids: the sketch of the factorization uses stream 0, problem i of a
# batch uses stream i + 1, and the j-th probe matrix of the SRQR g2 estimator
# uses stream 2^32 + j.
SRQR_STREAM_BASE = 1 << 32


def philox4x64_10(counter, key):
    """One Philox4x64-10 block, on plain Python integers (the readable definition)."""
    c0, c1, c2, c3 = (int(x) & MASK64 for x in counter)
    k0, k1 = (int(x) & MASK64 for x in key)
    for _ in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        c0, c1, c2, c3 = ((p1 >> 64) ^ c1 ^ k0, p1 & MASK64,
                          (p0 >> 64) ^ c3 ^ k1, p0 & MASK64)
        k0 = (k0 + W0) & MASK64
        k1 = (k1 + W1) & MASK64
    return c0, c1, c2, c3


def _mulhilo64(a: np.ndarray, b: int):
    """(hi, lo) 64-bit halves of a * b for uint64 arrays, via 32-bit limbs."""
    m32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    a0, a1 = a & m32, a >> s32
    b0, b1 = np.uint64(b & 0xFFFFFFFF), np.uint64(b >> 32)
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> s32) + (p01 & m32) + (p10 & m32)
    hi = p11 + (p01 >> s32) + (p10 >> s32) + (mid >> s32)
    lo = (mid << s32) | (p00 & m32)
    return hi, lo


def philox_blocks(first_block: int, nblocks: int, key) -> np.ndarray:
    """Vectorized Philox4x64-10 over counters (first_block .. first_block+nblocks-1, 0, 0, 0).

    Returns a (nblocks, 4) uint64 array.  Same arithmetic as ``philox4x64_10``.
    """
    with np.errstate(over="ignore"):
        c0 = np.arange(first_block, first_block + nblocks, dtype=np.uint64)
        c1 = np.zeros(nblocks, np.uint64)
        c2 = np.zeros(nblocks, np.uint64)
        c3 = np.zeros(nblocks, np.uint64)
        k0 = int(key[0]) & MASK64
        k1 = int(key[1]) & MASK64
        for _ in range(10):
            hi0, lo0 = _mulhilo64(c0, M0)
            hi1, lo1 = _mulhilo64(c2, M1)
            c0, c1, c2, c3 = hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0
            k0 = (k0 + W0) & MASK64
            k1 = (k1 + W1) & MASK64
    return np.stack([c0, c1, c2, c3], axis=1)


def raw_words(count: int, seed: int, stream: int) -> np.ndarray:
    """The first ``count`` 64-bit words of stream (seed, stream)."""
    nb = (count + 3) // 4
    return philox_blocks(1, nb, (seed, stream)).reshape(-1)[:count]


def uniforms(words: np.ndarray) -> np.ndarray:
    return ((words >> np.uint64(12)).astype(np.float64) + 0.5) * (2.0 ** -52)


def normals(count: int, seed: int, stream: int) -> np.ndarray:
    """Normal numbers q = 0 .. count-1 of stream (seed, stream)."""
    nb = (count + 3) // 4
    u = uniforms(philox_blocks(1, nb, (seed, stream)))  # (nb, 4)
    r01 = np.sqrt(-2.0 * np.log(u[:, 0]))
    r23 = np.sqrt(-2.0 * np.log(u[:, 2]))
    t01 = TWO_PI * u[:, 1]
    t23 = TWO_PI * u[:, 3]
    z = np.stack([r01 * np.cos(t01), r01 * np.sin(t01),
                  r23 * np.cos(t23), r23 * np.sin(t23)], axis=1)
    return z.reshape(-1)[:count]


def normal_scalar(q: int, seed: int, stream: int) -> float:
    """Normal number q, computed with plain Python integers and ``math``."""
    x = philox4x64_10((q // 4 + 1, 0, 0, 0), (seed, stream))
    u = [((w >> 12) + 0.5) * 2.0 ** -52 for w in x]
    lane = q % 4
    rad = math.sqrt(-2.0 * math.log(u[0 if lane < 2 else 2]))
    ang = TWO_PI * u[1 if lane < 2 else 3]
    return rad * (math.cos(ang) if lane % 2 == 0 else math.sin(ang))


def gauss(rows: int, cols: int, seed: int, stream: int = 0) -> np.ndarray:
    """The rows x cols Gaussian matrix Omega (Fortran order): Omega[r, c] = normal(c*rows + r)."""
    z = normals(rows * cols, seed, stream)
    return np.asfortranarray(z.reshape(cols, rows).T)
