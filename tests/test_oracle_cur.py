"""Pins of the CX / CUR decompositions (Section V-D) and of the SVD compression
of an l-step factorization to rank k (Section IV-E).

* X = C^+ A satisfies the normal equations C^T (C X - A) = 0, has the identity
  in the selected columns, and its residual equals ||R22||_F of the QR
  factorization that puts the selected columns first (closed form).
* U = C^+ A R^+ satisfies C^T (C U R - A) R^T = 0, and equals X Q_r1 T11^-T
  built from the two QR factorizations (an independent route).
* The compressed factors reproduce Q_l (U_k U_k^T) R_l, and by orthogonality
  ||A - X Y||_F^2 = ||R22||_F^2 + sum_{j > k} sigma_j(R_l)^2; with k = l the
  compression is the plain truncated factorization.
"""
import numpy as np
from scipy.linalg import solve_triangular

from oracle import cur as C
from oracle import rqrcp as R
from workloads import lowrank, rbf_kernel, sigma_exp


def _setup(n=300, k=40):
    a = rbf_kernel(n, 8, 3, 1.0)
    cols, res = C.select(a, k, 16, 8, 5.0, seed=1)
    rows, rres = C.select(np.asfortranarray(a.T), k, 16, 8, 5.0, seed=2)
    return a, k, cols, rows, res, rres


def test_cx_definition_and_closed_form_residual():
    a, k, cols, _, res, _ = _setup()
    c, x = C.cx(a, cols)
    assert np.linalg.norm(c.T @ (c @ x - a)) <= 1e-10 * np.linalg.norm(c) * np.linalg.norm(a)
    assert np.allclose(x[:, cols], np.eye(k), atol=1e-10)
    af, _ = R.factor_frozen(a, res.jpvt, k, 16)
    r22 = np.linalg.norm(af[k:, k:])
    assert abs(np.linalg.norm(a - c @ x) - r22) <= 1e-10 * np.linalg.norm(a)


def test_cur_definition_and_factorization_route():
    a, k, cols, rows, res, rres = _setup()
    c, u, r = C.cur(a, cols, rows)
    lhs = c.T @ (c @ u @ r - a) @ r.T
    assert np.linalg.norm(lhs) <= 1e-12 * np.linalg.norm(c) ** 2 * np.linalg.norm(r) ** 2 * np.linalg.norm(u)
    # the route through the two factorizations: U = X Q_r1 T11^-T
    _, x = C.cx(a, cols)
    afr, taur = R.factor_frozen(np.asfortranarray(a.T), rres.jpvt, k, 16)
    qr1 = R.form_q(afr, taur, k)
    t11 = np.triu(afr[:k, :k])
    u2 = solve_triangular(t11, (x @ qr1).T, lower=False).T       # (X Q_r1) T11^-T
    assert np.linalg.norm(u2 - u) <= 1e-9 * np.linalg.norm(u)


def test_svd_compression_residual_identity():
    m, n, l, k = 200, 150, 40, 25
    a = lowrank(m, n, sigma_exp(150, 10.0), 4)
    f = R.rqrcp(a, l, 8, 8, seed=3, mode="blocked")
    x, y = C.svd_compress(f.a, f.tau, f.jpvt, l, k)
    rl = np.triu(f.a[:l, :])
    s = np.linalg.svd(rl, compute_uv=False)
    lhs = np.linalg.norm(a - x @ y) ** 2
    rhs = np.linalg.norm(f.a[l:, l:]) ** 2 + np.sum(s[k:] ** 2)
    assert abs(lhs - rhs) <= 1e-10 * np.linalg.norm(a) ** 2
    # never better than the best rank-k approximation of A
    sa = np.linalg.svd(a, compute_uv=False)
    assert lhs >= np.sum(sa[k:] ** 2) * (1 - 1e-12)
    # k = l: the plain truncated factorization Q1 [R11 R12] Pi^T (up to the
    # orthogonal U_l, which cancels)
    x2, y2 = C.svd_compress(f.a, f.tau, f.jpvt, l, l)
    q1 = R.form_q(f.a, f.tau, l)
    ref = np.zeros_like(a)
    ref[:, f.jpvt] = q1 @ rl
    assert np.linalg.norm(x2 @ y2 - ref) <= 1e-12 * np.linalg.norm(a)
