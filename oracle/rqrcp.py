"""Plain FP64 reference of randomized QR with column pivoting (RQRCP).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Follows the paper step by step:

* Alg. 1 (QRCP): greedy pivot = largest trailing column norm, swap, Householder
  reflection, norm update.  Here the norms are *recomputed* from the trailing
  rows at every step, which is the literal definition of r_s in Alg. 1.
* Alg. 2 (RQRCP): Gaussian Omega ((b+p) x m), sketch B = Omega A, then per block
  of b columns: partial QRCP on B(:, i:n) picks b pivots, the same swaps are
  applied to A and Pi, unpivoted Householder QR of the pivoted panel, the
  transposed block reflector is applied to the trailing columns of A, and the
  first b rows of B's trailing columns are refreshed with update formula (1)
  of Section III-B:  B12 <- B12 - B11 R11^{-1} R12  (B11, B12 are the top b rows
  of the QRCP-transformed sketch; rows b..b+p-1 keep R^hat_22).
* Update formula (2) of Section III-B (B2 - Omega Q1 R12), for the equivalence
  check stated there (both formulas give the same permutations).

Readings of points the paper leaves open:

* Householder convention (the reflector step of Alg. 1): LAPACK dlarfg,
  beta = -sign(alpha) ||(alpha, x)||, sign(0) = +, tau = (beta - alpha)/beta,
  v = x/(alpha - beta); tau = 0 and no sign flip when x = 0.
* Swaps are LAPACK-style sequential transpositions of whole columns (all rows of
  A, all rows of B, and the permutation vector).
* argmax ties go to the lowest current column position.
* The garbled index "B(1:b, i:j+b-1)" of Alg. 2 / Alg. 4 is read as B(1:b, i:i+b-1).
* The last block has bb = k - i columns; Omega and B keep b + p rows throughout.
* Exact rank deficiency (R11 assumed invertible in Section III-C): if the
  largest trailing sketch norm at global step s is exactly 0, info = s + 1;
  from then on no column is moved (the remaining steps take the columns in
  their current order) and the sketch is no longer updated (formula (1)
  needs R11^{-1}), while the Householder factorization of A is completed.
  On exactly zero trailing columns this is the same as stopping at step s:
  their reflectors are the identity (tau = 0).

Storage is LAPACK's: on exit ``a`` holds R in its upper trapezoid (rows 0..k-1),
the Householder vectors v (unit leading entry implied) below the diagonal of
columns 0..k-1, and the updated trailing block R22 in ``a[k:, k:]``.
``jpvt[j]`` is the original index of the column placed at position j.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.linalg import solve_triangular

from .philox import gauss


# ---------------------------------------------------------------------------
# Householder reflections (the reflector step of Alg. 1)
# ---------------------------------------------------------------------------

def householder(alpha: float, x: np.ndarray):
    """Reflector H = I - tau [1; v][1; v]^T with H [alpha; x] = [beta; 0].

    Returns (beta, tau, v).  LAPACK dlarfg sign convention (no underflow
    rescaling).
    """
    xnorm = float(np.linalg.norm(x))
    if xnorm == 0.0:
        return float(alpha), 0.0, np.zeros_like(x)
    norm = float(np.hypot(alpha, xnorm))
    beta = -norm if alpha >= 0.0 else norm
    tau = (beta - alpha) / beta
    v = x / (alpha - beta)
    return beta, tau, v


def apply_reflector(v_full: np.ndarray, tau: float, c: np.ndarray) -> None:
    """c <- (I - tau v v^T) c, in place (v_full includes the leading 1)."""
    if tau == 0.0 or c.size == 0:
        return
    w = v_full @ c
    c -= tau * np.outer(v_full, w)


# ---------------------------------------------------------------------------
# Alg. 1 on the sketch: partial QRCP
# ---------------------------------------------------------------------------

@dataclass
class StepTrace:
    """Per pivot step: the largest and second-largest squared trailing norm."""
    top2: list = field(default_factory=list)

    def min_rel_gap(self) -> float:
        gaps = [(a - b) / a for a, b in self.top2 if a > 0]
        return min(gaps) if gaps else float("inf")


def partial_qrcp(w: np.ndarray, nsteps: int, trace: StepTrace | None = None):
    """``nsteps`` steps of Alg. 1 on the sketch block ``w`` (in place).

    Returns (pivots, rank_stop): pivots[t] is the position (within w) that was
    swapped into position t; rank_stop is the first step at which every
    trailing norm was exactly zero (that step and the later ones then keep the
    current column order), or None.
    """
    rows, ncols = w.shape
    pivots = []
    rank_stop = None
    for t in range(nsteps):
        # r_s = ||w(t:rows, s)||, recomputed for every trailing column s >= t
        norms = np.sqrt(np.sum(w[t:, t:] ** 2, axis=0))
        j = t + int(np.argmax(norms))          # first maximum = lowest position
        if norms[j - t] == 0.0:
            if rank_stop is None:
                rank_stop = t
        elif trace is not None:
            sq = np.sort(norms ** 2)[::-1]
            trace.top2.append((sq[0], sq[1] if sq.size > 1 else 0.0))
        if j != t:
            w[:, [t, j]] = w[:, [j, t]]
        beta, tau, v = householder(w[t, t], w[t + 1:, t])
        w[t, t] = beta
        w[t + 1:, t] = 0.0
        apply_reflector(np.concatenate(([1.0], v)), tau, w[t:, t + 1:])
        pivots.append(j)
    return pivots, rank_stop


# ---------------------------------------------------------------------------
# Tournament pivoting on the sketch (the first future-work item of Section V-C:
# QR with tournament pivoting in place of the partial QRCP of B)
# ---------------------------------------------------------------------------

def _qrcp_choose(w: np.ndarray, nsteps: int, trace: StepTrace | None = None) -> list:
    """Positions (within w) chosen by nsteps greedy steps of Alg. 1 on a copy of
    w (norms recomputed, ties to the lowest position), in the order chosen.
    Stops early when every remaining norm is exactly zero."""
    w = np.array(w, dtype=np.float64, copy=True)
    rows, ncols = w.shape
    order = list(range(ncols))
    chosen = []
    for t in range(min(nsteps, ncols)):
        norms = np.sqrt(np.sum(w[t:, t:] ** 2, axis=0)) if t < rows else np.zeros(ncols - t)
        j = t + int(np.argmax(norms))
        if norms[j - t] == 0.0:
            break
        if trace is not None:
            sq = np.sort(norms ** 2)[::-1]
            trace.top2.append((sq[0], sq[1] if sq.size > 1 else 0.0))
        if j != t:
            w[:, [t, j]] = w[:, [j, t]]
            order[t], order[j] = order[j], order[t]
        chosen.append(order[t])
        if t < rows:
            beta, tau, v = householder(w[t, t], w[t + 1:, t])
            w[t, t] = beta
            w[t + 1:, t] = 0.0
            apply_reflector(np.concatenate(([1.0], v)), tau, w[t:, t + 1:])
    return chosen


def tournament_choose(w: np.ndarray, nsteps: int, group: int,
                      trace: StepTrace | None = None, fanout: int = 2) -> list:
    """QR with tournament pivoting (Demmel, Grigori, Gu and Xiang, 2015) on the
    columns of w: the columns are split into consecutive groups of ``group``;
    each group nominates up to nsteps columns by Alg. 1; nominations are then
    merged ``fanout`` sets at a time (sets fanout*i .. fanout*i + fanout - 1,
    concatenated in order; a last chunk holding a single set passes to the
    next round unchanged), each merged set again reduced to nsteps columns by
    Alg. 1, until one set is left.  Returns its columns (positions within w)
    in the order the last Alg. 1 run chose them."""
    ncols = w.shape[1]
    sets = [list(range(s, min(s + group, ncols))) for s in range(0, ncols, group)]
    # every selection decision (leaves and merges) is recorded in the trace
    sets = [[c[j] for j in _qrcp_choose(w[:, c], nsteps, trace)] for c in sets]
    while len(sets) > 1:
        merged = []
        for g in range(0, len(sets), fanout):
            chunk = sets[g:g + fanout]
            if len(chunk) == 1:
                merged.append(chunk[0])
                continue
            u = [c for st in chunk for c in st]
            merged.append([u[j] for j in _qrcp_choose(w[:, u], nsteps, trace)])
        sets = merged
    return sets[0]


def transpositions(winners: list) -> list:
    """LAPACK-style transpositions (t, p_t), t = 0, 1, ..., that bring the
    columns at positions winners[0], winners[1], ... to positions 0, 1, ...,
    applied in order."""
    pos = list(range(max(winners + [len(winners) - 1]) + 1))   # position -> column
    where = {c: c for c in pos}                                  # column -> position
    out = []
    for t, c in enumerate(winners):
        p = where[c]
        out.append((t, p))
        if p != t:
            ct = pos[t]
            pos[t], pos[p] = c, ct
            where[c], where[ct] = t, p
    return out


def partial_qr_fixed(w: np.ndarray, pivots_tp: list) -> None:
    """Apply the transpositions to the columns of w, then Householder steps on
    the first len(pivots_tp) columns (no further pivoting), in place."""
    rows = w.shape[0]
    for t, p in pivots_tp:
        if p != t:
            w[:, [t, p]] = w[:, [p, t]]
    for t in range(len(pivots_tp)):
        if t >= rows:
            break
        beta, tau, v = householder(w[t, t], w[t + 1:, t])
        w[t, t] = beta
        w[t + 1:, t] = 0.0
        apply_reflector(np.concatenate(([1.0], v)), tau, w[t:, t + 1:])


def qrcp(a: np.ndarray, k: int, trace: StepTrace | None = None):
    """Alg. 1 (deterministic QRCP) to k steps on a copy of ``a``.

    Returns (a_factored, tau, jpvt) in LAPACK storage.
    """
    a = np.array(a, dtype=np.float64, order="F", copy=True)
    m, n = a.shape
    jpvt = np.arange(n)
    tau = np.zeros(k)
    for t in range(k):
        norms = np.sqrt(np.sum(a[t:, t:] ** 2, axis=0))
        j = t + int(np.argmax(norms))
        if trace is not None:
            sq = np.sort(norms ** 2)[::-1]
            trace.top2.append((sq[0], sq[1] if sq.size > 1 else 0.0))
        if j != t:
            a[:, [t, j]] = a[:, [j, t]]
            jpvt[[t, j]] = jpvt[[j, t]]
        beta, tau[t], v = householder(a[t, t], a[t + 1:, t])
        a[t, t] = beta
        a[t + 1:, t] = v
        apply_reflector(np.concatenate(([1.0], v)), tau[t], a[t:, t + 1:])
    return a, tau, jpvt


# ---------------------------------------------------------------------------
# Panel QR, compact WY, trailing update (Alg. 2 body; PDGEQRF / PDLARFT / PDLARFB
# in Alg. 4)
# ---------------------------------------------------------------------------

def panel_qr(a: np.ndarray, i: int, bb: int, tau: np.ndarray) -> None:
    """Unpivoted Householder QR of a[i:, i:i+bb], reflectors applied inside the panel only."""
    for t in range(bb):
        c = i + t
        beta, tau[c], v = householder(a[c, c], a[c + 1:, c])
        a[c, c] = beta
        a[c + 1:, c] = v
        apply_reflector(np.concatenate(([1.0], v)), tau[c], a[c:, c + 1:i + bb])


def reflector_block(a: np.ndarray, i: int, bb: int) -> np.ndarray:
    """V = unit lower trapezoidal (m-i) x bb matrix of the panel's Householder vectors."""
    v = np.tril(a[i:, i:i + bb], -1)
    v[np.arange(bb), np.arange(bb)] = 1.0
    return v


def compact_wy_t(v: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """Upper triangular T with H_0 H_1 ... H_{bb-1} = I - V T V^T (forward, columnwise)."""
    bb = v.shape[1]
    t = np.zeros((bb, bb))
    for j in range(bb):
        t[j, j] = tau[j]
        if j:
            t[:j, j] = -tau[j] * (t[:j, :j] @ (v[:, :j].T @ v[:, j]))
    return t


def apply_block_reflector_t(v: np.ndarray, t: np.ndarray, c: np.ndarray) -> None:
    """c <- (I - V T V^T)^T c = c - V (T^T (V^T c)), in place."""
    if c.size == 0:
        return
    c -= v @ (t.T @ (v.T @ c))


# ---------------------------------------------------------------------------
# Alg. 2
# ---------------------------------------------------------------------------

@dataclass
class Factorization:
    a: np.ndarray          # R, V and R22 in LAPACK storage
    tau: np.ndarray        # k reflector scalars
    jpvt: np.ndarray       # jpvt[j] = original column at position j
    b: np.ndarray | None   # final sketch (rows b+p, n columns); trailing part used by SRQR
    info: int              # 0, or s+1 when the sketch pivot at step s was exactly 0
    omega: np.ndarray | None
    trace: StepTrace
    k: int = 0             # rank reached (the requested k, or where stop_tol stopped)
    est_ratio: float = 0.0  # stop_tol: sketch estimate of ||R22||_F / ||A||_F at k


def rqrcp(a, k: int, b: int, p: int, seed: int = 0, *, omega=None,
          mode: str = "plain", update: str = "formula1",
          stop_tol: float | None = None, tournament: int | None = None,
          fanout: int = 2) -> Factorization:
    """Alg. 2 on a copy of ``a`` (m x n), target rank k, block size b, oversampling p.

    mode = "plain": the reflectors of each panel are applied one at a time to
    every column to their right (sequential rank-1 updates).
    mode = "blocked": panel QR, then the compact WY block reflector on the
    trailing matrix (same result up to rounding).
    update = "formula1" (Section III-B, eq. updating_1) or "formula2"
    (Section III-B, eq. updating_2).
    omega: optional explicit (b+p) x m sketching matrix (otherwise
    Philox Omega with key (seed, 0)).
    stop_tol: error-tolerance form (Section III-A: the loop can stop on a
    tolerance instead of a rank).  After the sample update of each block the
    trailing sketch B(:, i+bb:n) is Omega-hat_2 R22 (formula (1)), whose
    Frobenius norm over sqrt(l) estimates ||R22||_F, as the first sketch's
    estimates ||A||_F; the loop stops after the first block where the ratio
    of the two is <= stop_tol, and k is then the rank reached.
    tournament: group size of QR with tournament pivoting used in place of
    the partial QRCP of the sketch (``tournament_choose``, merging ``fanout``
    sets at a time); the chosen columns
    are brought to the front in order and the sketch block is then factored
    by Householder steps without further pivoting.
    """
    a0 = np.asarray(a, dtype=np.float64)
    a = np.array(a0, order="F", copy=True)
    m, n = a.shape
    if not 1 <= k <= min(m, n):
        raise ValueError("need 1 <= k <= min(m, n)")
    l = b + p
    om = gauss(l, m, seed, 0) if omega is None else np.asarray(omega, dtype=np.float64)
    if om.shape != (l, m) and omega is not None:
        l = om.shape[0]
    bsk = om @ a                                   # B = Omega A
    b_orig = bsk.copy() if update == "formula2" else None
    norm_a_est = np.linalg.norm(bsk) / np.sqrt(l)
    ratio = 0.0
    jpvt = np.arange(n)
    tau = np.zeros(k)
    info = 0
    trace = StepTrace()
    i = 0
    while i < k:
        bb = min(b, k - i)
        w = bsk[:, i:]                             # view: partial QRCP acts on B(:, i:n)
        if info == 0 and tournament is not None:
            win = tournament_choose(w, bb, tournament, trace, fanout)
            tp = transpositions(win)
            partial_qr_fixed(w, tp)
            for t, j in tp:                        # same transpositions on A and Pi
                if j != t:
                    a[:, [i + t, i + j]] = a[:, [i + j, i + t]]
                    jpvt[[i + t, i + j]] = jpvt[[i + j, i + t]]
            if len(win) < bb:                      # every remaining sketch column was zero
                info = i + len(win) + 1
        elif info == 0:
            pivots, rank_stop = partial_qrcp(w, bb, trace)
            for t, j in enumerate(pivots):         # same transpositions on A and Pi
                if j != t:
                    a[:, [i + t, i + j]] = a[:, [i + j, i + t]]
                    jpvt[[i + t, i + j]] = jpvt[[i + j, i + t]]
            if rank_stop is not None:
                info = i + rank_stop + 1
        if mode == "plain":
            for t in range(bb):
                c = i + t
                beta, tau[c], v = householder(a[c, c], a[c + 1:, c])
                a[c, c] = beta
                a[c + 1:, c] = v
                apply_reflector(np.concatenate(([1.0], v)), tau[c], a[c:, c + 1:])
        elif mode == "blocked":
            panel_qr(a, i, bb, tau)
            v = reflector_block(a, i, bb)
            apply_block_reflector_t(v, compact_wy_t(v, tau[i:i + bb]), a[i:, i + bb:])
        else:
            raise ValueError(mode)
        if i + bb < n and info == 0:
            if update == "formula1":
                r11 = np.triu(a[i:i + bb, i:i + bb])
                r12 = a[i:i + bb, i + bb:]
                x = solve_triangular(r11, r12, lower=False)        # R11^{-1} R12
                w[:bb, bb:] -= np.triu(w[:bb, :bb]) @ x              # B11 R11^{-1} R12
            else:
                s = i + bb
                q1 = form_q(a[:, :s], tau[:s])                        # m x s
                w[:, bb:] = b_orig[:, jpvt[s:]] - (om @ q1) @ a[:s, s:]
        i += bb
        if stop_tol is not None and i < n:
            est = np.linalg.norm(bsk[:, i:]) / np.sqrt(l)
            ratio = est / norm_a_est if norm_a_est > 0 else 0.0
            if ratio <= stop_tol:
                break
    if stop_tol is not None:
        tau = tau[:i]
    return Factorization(a, tau, jpvt, bsk, info, om, trace, min(i, k), ratio)


def factor_frozen(a, jpvt, k: int, b: int, mode: str = "blocked"):
    """Unpivoted blocked Householder QR of a[:, jpvt] to k steps (pivots frozen).

    Returns (a_factored, tau).  This is the Alg. 2 loop with the QRCP step
    replaced by a given permutation.
    """
    a = np.array(np.asarray(a, dtype=np.float64)[:, np.asarray(jpvt)], order="F", copy=True)
    m, n = a.shape
    tau = np.zeros(k)
    i = 0
    while i < k:
        bb = min(b, k - i)
        if mode == "plain":
            for t in range(bb):
                c = i + t
                beta, tau[c], v = householder(a[c, c], a[c + 1:, c])
                a[c, c] = beta
                a[c + 1:, c] = v
                apply_reflector(np.concatenate(([1.0], v)), tau[c], a[c:, c + 1:])
        else:
            panel_qr(a, i, bb, tau)
            v = reflector_block(a, i, bb)
            apply_block_reflector_t(v, compact_wy_t(v, tau[i:i + bb]), a[i:, i + bb:])
        i += bb
    return a, tau


# ---------------------------------------------------------------------------
# Q and the factorization's pieces
# ---------------------------------------------------------------------------

def form_q(a_fact: np.ndarray, tau: np.ndarray, ncols: int | None = None) -> np.ndarray:
    """Explicit Q[:, :ncols] = H_0 H_1 ... H_{k-1} [I; 0] from LAPACK storage (k = len(tau))."""
    m = a_fact.shape[0]
    k = len(tau)
    ncols = k if ncols is None else ncols
    q = np.zeros((m, ncols))
    q[np.arange(min(m, ncols)), np.arange(min(m, ncols))] = 1.0
    for c in range(k - 1, -1, -1):
        v = np.concatenate(([1.0], a_fact[c + 1:, c]))
        apply_reflector(v, tau[c], q[c:, :])
    return q


def apply_qt(a_fact: np.ndarray, tau: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Q^T c for Q = H_0 ... H_{k-1} (returns a new array)."""
    c = np.array(c, dtype=np.float64, copy=True)
    for j in range(len(tau)):
        v = np.concatenate(([1.0], a_fact[j + 1:, j]))
        apply_reflector(v, tau[j], c[j:, :])
    return c


def r_factor(a_fact: np.ndarray, k: int) -> np.ndarray:
    """The full m x n R of the k-step factorization: [R11 R12; 0 R22]."""
    r = np.array(a_fact, copy=True)
    r[:, :k] = np.triu(r[:, :k])
    return r


def pieces(f: Factorization, k: int):
    """(Q1, R11, R12, R22) of the truncated factorization A Pi = Q [R11 R12; 0 R22]."""
    q1 = form_q(f.a, f.tau[:k])
    r = r_factor(f.a, k)
    return q1, r[:k, :k], r[:k, k:], r[k:, k:]


# ---------------------------------------------------------------------------
# Theory helper: Theorem 1's oversampling bound
# ---------------------------------------------------------------------------

def oversampling_bound(n: int, k: int, eps: float, delta: float) -> int:
    """Smallest p of Theorem 1: p >= ceil(4/(eps^2 - eps^3) * ln(2nk/delta)) - 1."""
    return int(np.ceil(4.0 / (eps ** 2 - eps ** 3) * np.log(2.0 * n * k / delta))) - 1

