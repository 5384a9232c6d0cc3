"""CX and CUR decompositions from spectrum-revealing QR (Section V-D), and the
SVD compression of an l-step factorization to rank k (Section IV-E), plain
FP64 reference.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Definitions (Section V-D):
* CX: C = A(:, J) for k selected columns J, X = C^+ A, the minimizer of
  ||C X - A||_F.
* CUR: C as above, R = A(I, :) for k selected rows I, U = C^+ A R^+, the
  minimizer of ||C U R - A||_F.
The columns are the first k pivots of SRQR (Alg. 3) on A, the rows the first
k pivots of SRQR on A^T.  X and U are computed here from their definitions
with a library pseudo-inverse (numpy's SVD-based pinv).

SVD compression (the remark after Alg. 3): with the l-step factorization
A Pi ~ Q_l R_l (R_l = first l rows of R, l x n), the rank-k approximation is
Q_l U_k U_k^T R_l, U_k the k leading left singular vectors of R_l; returned
as the factors Q_l U_k (m x k) and U_k^T R_l Pi^T (k x n).
"""
from __future__ import annotations

import numpy as np

from .rqrcp import form_q
from .srqr import srqr


def select(a, k: int, b: int, p: int, g: float, seed: int = 0, **kw):
    """The k columns SRQR (Alg. 3 with l = k, as the CUR/CX experiment sets
    it) leaves in front, and the SRQR result."""
    res = srqr(a, k, b, p, g, seed, **kw)
    return res.jpvt[:k].copy(), res


def cx(a, cols):
    c = a[:, cols]
    return c, np.linalg.pinv(c) @ a


def cur(a, cols, rows):
    c = a[:, cols]
    r = a[rows, :]
    u = np.linalg.pinv(c) @ a @ np.linalg.pinv(r)
    return c, u, r


def svd_compress(a_fact: np.ndarray, tau: np.ndarray, jpvt: np.ndarray, l: int, k: int):
    """(X, Y) with A ~ X Y: X = Q_l U_k (m x k), Y = (U_k^T R_l) Pi^T (k x n), from an
    l-step factorization in LAPACK storage (l = len(tau) >= k)."""
    m, n = a_fact.shape
    rl = np.triu(a_fact[:l, :])
    u, _, _ = np.linalg.svd(rl, full_matrices=False)
    uk = u[:, :k]
    x = form_q(a_fact, tau[:l], l) @ uk
    y = np.zeros((k, n))
    y[:, jpvt] = uk.T @ rl
    return x, y
