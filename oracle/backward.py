"""Reference gradients of the truncated factorization with frozen pivots (FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper's low-rank approximation is A ~ Q1 [R11 R12] Pi^T (Section I-A, block
form of eq. (1)).  With the permutation Pi held fixed, Q1 spans the first k
pivoted columns A_S = (A Pi)(:, 0:k), so Q1 [R11 R12] Pi^T = P A with the
orthogonal projector P = Q1 Q1^T.  The paper does not differentiate anything;
these are two independent FP64 references for the adjoint map
(dL/dQ1, dL/dR) -> dL/dA, and for the gradient of L = sum(W * Q1 [R11 R12] Pi^T):

(i)  closed form (derivative of an orthogonal projector, Golub & Pereyra 1973):
     dL/dA = P W + scatter_S( P_perp (W A^T Q1 + A W^T Q1) R11^-T ),
     P_perp = I - P, scatter_S placing the k columns at jpvt[0:k].
(ii) the chain of the factorization's own steps: R12 = Q1^T A2 and the QR of
     A1 = Q1 R11 (adjoint of the Householder QR of the panel):
       A2_bar  = Q1 R12_bar
       Q1_bar' = Q1_bar + A2 R12_bar^T
       M       = R11 R11_bar^T - Q1_bar'^T Q1
       A1_bar  = (Q1_bar' + Q1 copyltu(M)) R11^-T,   copyltu(M) = tril(M) + tril(M, -1)^T
     then [A1_bar A2_bar] Pi^T.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular

from .rqrcp import factor_frozen, form_q


def factor_pieces(a, jpvt, k: int, b: int = 64):
    """(Q1, R11, R12) of the frozen-pivot factorization A Pi = Q R."""
    af, tau = factor_frozen(a, jpvt, k, b)
    q1 = form_q(af, tau)
    r = np.triu(af[:k, :])
    return q1, r[:, :k], r[:, k:]


def loss(a, jpvt, k: int, w, b: int = 64) -> float:
    """L = sum(W * Q1 [R11 R12] Pi^T)."""
    q1, r11, r12 = factor_pieces(a, jpvt, k, b)
    approx_pi = q1 @ np.hstack([r11, r12])
    approx = np.empty_like(approx_pi)
    approx[:, np.asarray(jpvt)] = approx_pi
    return float(np.sum(np.asarray(w) * approx))


def loss_cotangents(a, jpvt, k: int, w, b: int = 64):
    """(Q1_bar, R_bar) of L = <W Pi, Q1 R~> with R~ = [R11 R12] (pivot order)."""
    q1, r11, r12 = factor_pieces(a, jpvt, k, b)
    wpi = np.asarray(w)[:, np.asarray(jpvt)]
    rt = np.hstack([r11, r12])
    return wpi @ rt.T, q1.T @ wpi


def grad_closed_form(a, jpvt, k: int, w, b: int = 64) -> np.ndarray:
    a = np.asarray(a, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    jpvt = np.asarray(jpvt)
    q1, r11, _ = factor_pieces(a, jpvt, k, b)
    pw = q1 @ (q1.T @ w)
    inner = w @ (a.T @ q1) + a @ (w.T @ q1)                  # m x k
    inner = inner - q1 @ (q1.T @ inner)                      # P_perp
    gs = solve_triangular(r11, inner.T, lower=False).T   # X R11^-T = (R11^-1 X^T)^T
    g = pw.copy()
    g[:, jpvt[:k]] += gs
    return g


def adjoint_chain(a, jpvt, k: int, q1_bar, r_bar, b: int = 64) -> np.ndarray:
    """dL/dA from (Q1_bar, R_bar) through R12 = Q1^T A2 and the panel QR A1 = Q1 R11."""
    a = np.asarray(a, dtype=np.float64)
    jpvt = np.asarray(jpvt)
    q1, r11, _ = factor_pieces(a, jpvt, k, b)
    api = a[:, jpvt]
    a2 = api[:, k:]
    r11_bar = np.asarray(r_bar)[:, :k]
    r12_bar = np.asarray(r_bar)[:, k:]
    a2_bar = q1 @ r12_bar
    q1b = np.asarray(q1_bar) + a2 @ r12_bar.T
    mm = r11 @ r11_bar.T - q1b.T @ q1
    copyltu = np.tril(mm) + np.tril(mm, -1).T
    a1_bar = solve_triangular(r11, (q1b + q1 @ copyltu).T, lower=False).T   # X R11^-T = (R11^-1 X^T)^T
    g = np.empty_like(a)
    g[:, jpvt] = np.hstack([a1_bar, a2_bar])
    return g


def grad_chain(a, jpvt, k: int, w, b: int = 64) -> np.ndarray:
    q1_bar, r_bar = loss_cotangents(a, jpvt, k, w, b)
    return adjoint_chain(a, jpvt, k, q1_bar, r_bar, b)


def grad_fd(a, jpvt, k: int, w, h: float = 1e-3, b: int = 64) -> np.ndarray:
    """Central finite differences of ``loss`` with the pivots frozen."""
    a = np.array(a, dtype=np.float64, copy=True)
    g = np.zeros_like(a)
    for i in range(a.shape[0]):
        for j in range(a.shape[1]):
            old = a[i, j]
            a[i, j] = old + h
            lp = loss(a, jpvt, k, w, b)
            a[i, j] = old - h
            lm = loss(a, jpvt, k, w, b)
            a[i, j] = old
            g[i, j] = (lp - lm) / (2.0 * h)
    return g
