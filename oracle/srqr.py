"""Spectrum-revealing QR (Alg. 3), plain FP64 reference.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Alg. 3 takes the l-step RQRCP of Alg. 2, estimates the trailing column norms
from the final sketch B (r_i = ||B(:, i)||^2 / (b+p)), brings the largest one to
position l (0-based; the paper's l+1), does one more QR step on the trailing
block, and estimates g2 = |alpha| ||R^-T||_{1,2} (definition of g1, g2 in
Section IV-C) with a d x (l+1) Gaussian probe:
g2 ~ |alpha|/sqrt(d) ||Omega R^-T||_{1,2}.  While g2 > g it rotates the column
with the largest probed column norm to position l (round robin), restores the
triangular form with Givens rotations, repivots the trailing candidates and
repeats the QR step.

Readings of points the paper leaves open:

* "Round Robin rotation": a cyclic shift; column i moves to position l and
  columns i+1..l move one position to the left.  The rows i..l of R are then
  upper Hessenberg; adjacent-row Givens rotations G(j, j+1), j = i..l-1, with
  r = sign(f) hypot(f, g), c = f/r, s = g/r (sign(0) = +), zero the
  subdiagonal, acting on all columns j..n-1.
* r_i bookkeeping uses the current row l after the rotations; estimates are
  clamped at 0; at most ``max_swaps`` swaps.
* ``exact=True`` replaces the probe by the exact norm: g2 = |alpha| * (largest
  row norm of R^-1), and the column choice uses the exact row norms.
* The j-th probe matrix uses the Philox stream 2^32 + j.
* Alg. 3 does not track Q through the rotations; after any swap the
  factorization is recomputed with the final pivots frozen so that
  (V, tau, R) again satisfy A Pi = Q R.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.linalg import solve_triangular

from .philox import SRQR_STREAM_BASE, gauss
from .rqrcp import apply_reflector, factor_frozen, householder, rqrcp


def givens(f: float, g: float):
    """(c, s, r) with [c s; -s c] [f; g] = [r; 0], r = sign(f) hypot(f, g)."""
    if g == 0.0:
        return 1.0, 0.0, f
    r = float(np.hypot(f, g))
    if f < 0.0:
        r = -r
    return f / r, g / r, r


@dataclass
class SRQRResult:
    r: np.ndarray               # m x n: R rows 0..l (upper trapezoidal) and trailing block below
    jpvt: np.ndarray
    alpha: float                # |R[l, l]| after the last QR step
    g2: float                   # last g2 value (estimate, or exact in exact mode)
    nswaps: int
    history: list = field(default_factory=list)   # (g2, alpha) before each swap decision
    a_refactored: np.ndarray | None = None
    tau_refactored: np.ndarray | None = None


def _g2(rhat: np.ndarray, alpha: float, exact: bool, d: int, seed: int, it: int):
    """(g2, per-column norms used for the swap choice)."""
    lp1 = rhat.shape[0]
    if exact:
        inv = solve_triangular(rhat, np.eye(lp1), lower=False)   # R^-1
        cn = np.sqrt(np.sum(inv ** 2, axis=1))                   # column norms of R^-T
        return alpha * float(cn.max()), cn
    om = gauss(d, lp1, seed, SRQR_STREAM_BASE + it)              # d x (l+1)
    y = solve_triangular(rhat, om.T, lower=False)                # R^-1 Omega^T = (Omega R^-T)^T
    cn = np.sqrt(np.sum(y ** 2, axis=1))                         # column norms of Omega R^-T
    return alpha / np.sqrt(d) * float(cn.max()), cn


def srqr(a, l: int, b: int, p: int, g: float, seed: int = 0, *, d: int = 16,
         exact: bool = False, max_swaps: int | None = None, omega=None,
         refactor: bool = True, trace: list | None = None) -> SRQRResult:
    """Alg. 3 with an l-step RQRCP (block size b, oversampling p) and tolerance g > 1.

    ``trace``: if a list, one dict per bookkeeping point is appended:
    ``stage`` ("start", "pick", "qr", "rotate"), ``top`` (first row of the
    trailing block the estimates refer to), copies of ``est`` and ``rw``, and
    for "pick" the position brought to l.
    """
    a = np.asarray(a, dtype=np.float64)
    m, n = a.shape
    if not (1 <= l < min(m, n)):
        raise ValueError("need 1 <= l < min(m, n)")
    f = rqrcp(a, l, b, p, seed, omega=omega)
    max_swaps = 2 * n if max_swaps is None else max_swaps
    rw = np.zeros((m, n))
    rw[:l, :] = np.triu(f.a[:l, :])
    rw[l:, l:] = f.a[l:, l:]
    jpvt = f.jpvt.copy()
    lsk = f.b.shape[0]
    # est[i], i >= l, estimates the squared norm of the part of column i that
    # lies in the trailing block of rw: rows l..m-1 before the one-step QR,
    # rows l+1..m-1 after it.  It starts from the final sketch (Section IV-E:
    # ||B(:, i)||^2 / (b+p) estimates ||R22(:, i)||^2) and then follows the
    # block exactly as rows leave it (the QR step removes row l) or rejoin it
    # (a swap's rotations put a new row l in front of it).  Squared norms are
    # never negative, so a downdate that would undershoot stops at 0.
    est = np.zeros(n)
    est[l:] = np.sum(f.b[:, l:] ** 2, axis=0) / lsk

    def record(stage, top, pick=None):
        if trace is not None:
            trace.append({"stage": stage, "top": top, "est": est.copy(),
                          "rw": rw.copy(), "pick": pick})

    def swap(i, j):
        if i != j:
            rw[:, [i, j]] = rw[:, [j, i]]
            jpvt[[i, j]] = jpvt[[j, i]]
            est[[i, j]] = est[[j, i]]

    def bring_largest_to_l():
        j = l + int(np.argmax(est[l:]))
        record("pick", l, j)
        swap(j, l)

    def qr_step():
        """One-step QR of rw[l:, l:]; row l then leaves the trailing block.
        Returns |alpha|."""
        beta, tau, v = householder(rw[l, l], rw[l + 1:, l])
        rw[l, l] = beta
        rw[l + 1:, l] = 0.0
        apply_reflector(np.concatenate(([1.0], v)), tau, rw[l:, l + 1:])
        est[l + 1:] = np.maximum(est[l + 1:] - rw[l, l + 1:] ** 2, 0.0)
        record("qr", l + 1)
        return abs(beta)

    record("start", l)
    bring_largest_to_l()
    alpha = qr_step()
    it = 0
    g2, cn = _g2(rw[:l + 1, :l + 1], alpha, exact, d, seed, it)
    history = [(g2, alpha)]
    nswaps = 0
    while g2 > g and nswaps < max_swaps:
        ii = int(np.argmax(cn))
        # round robin: column ii -> position l, columns ii+1..l shift left
        order = list(range(ii)) + list(range(ii + 1, l + 1)) + [ii] + list(range(l + 1, n))
        rw[:, :] = rw[:, order]
        jpvt[:] = jpvt[order]
        for j in range(ii, l):                                   # restore upper triangular R
            c, s, r = givens(rw[j, j], rw[j + 1, j])
            top = rw[j, j:].copy()
            bot = rw[j + 1, j:].copy()
            rw[j, j:] = c * top + s * bot
            rw[j + 1, j:] = -s * top + c * bot
            rw[j, j] = r
            rw[j + 1, j] = 0.0
        # the rotated row l rejoins the trailing block; column l (formerly
        # column ii) has no entries below row l, so its estimate is exact
        est[:l + 1] = 0.0
        est[l] = rw[l, l] ** 2
        est[l + 1:] += rw[l, l + 1:] ** 2
        record("rotate", l)
        bring_largest_to_l()
        alpha = qr_step()
        nswaps += 1
        it += 1
        g2, cn = _g2(rw[:l + 1, :l + 1], alpha, exact, d, seed, it)
        history.append((g2, alpha))
    res = SRQRResult(rw, jpvt, alpha, g2, nswaps, history)
    if refactor:
        res.a_refactored, res.tau_refactored = factor_frozen(a, jpvt, l + 1, b)
    return res


def g1_g2_exact(r: np.ndarray, l: int):
    """Exact g1 = ||R22||_{1,2}/|alpha| and g2 = |alpha| ||R^-T||_{1,2} (Section IV-C)
    for an m x n array whose rows 0..l are upper trapezoidal and whose block
    r[l+1:, l+1:] is the trailing matrix after l+1 QR steps."""
    alpha = abs(r[l, l])
    rhat = np.triu(r[:l + 1, :l + 1])
    inv = solve_triangular(rhat, np.eye(l + 1), lower=False)
    g2 = alpha * float(np.sqrt(np.sum(inv ** 2, axis=1)).max())
    r22 = r[l:, l:].copy()           # trailing block at the time of the (l+1)-st step
    r22[0, :] = r[l, l:]
    g1 = float(np.sqrt(np.sum(r22 ** 2, axis=0)).max()) / alpha if alpha else np.inf
    return g1, g2
