"""Element-level comparison of a factorization with the oracle's.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): used by the GPU parity
tests and the benchmark's parity check of its CPU-baseline sample.

A normwise difference of a whole output array can hide a wrong column that is
small next to the array's norm, so every output is also compared column by
column, each column against the scale its rounding errors live on:

* R (rows 0..k-1) and R22 (rows k..m-1) of column j: the norm of the input
  column it came from, ||A(:, jpvt[j])||.  R(:, j) and R22(:, j) are that
  column after orthogonal transformations, so a backward-stable computation
  errs by a small multiple of u ||A(:, jpvt[j])|| in each of them.
* V (column j < k, rows below the diagonal): the norm of the whole reflector
  vector [1; v_j] times the column's cancellation factor
  ||A(:, jpvt[j])|| / |R_jj| (>= 1).  The reflector is built from what is left
  of the column after j eliminations, whose entries carry absolute errors of
  about u ||A(:, jpvt[j])|| while its norm is |R_jj|; on graded inputs any two
  backward-stable computations of v_j differ by u times that factor.
* tau: elementwise, relative to max(1, |tau_j|) times the same factor (tau
  lies in [0, 2]).
* The trailing sketch B(:, j), j >= k: the norm of the original sketch column
  (Omega A)(:, jpvt[j]), which it is computed from by orthogonal
  transformations and the update formula.

The bar is max over columns of (max |difference| / scale) <= tol; the
normwise figures are reported beside it.
"""
from __future__ import annotations

import numpy as np


def colwise(x, y, scale):
    """max_j max_i |x - y|(i, j) / scale[j] (scale > 0)."""
    if x.size == 0:
        return 0.0
    d = np.abs(np.asarray(x) - np.asarray(y)).max(axis=0)
    return float((d / np.maximum(scale, np.finfo(float).tiny)).max())


def normwise(x, y, scale=None):
    s = np.linalg.norm(y) if scale is None else scale
    return float(np.linalg.norm(np.asarray(x) - np.asarray(y)) / (s if s > 0 else 1.0))


def factor_errors(a, k, jp, af_g, tau_g, af_o, tau_o, b_g=None, b_o=None, omega=None):
    """Columnwise (key) and normwise (key + "_F") errors of a k-step factorization
    (af, tau, final sketch b) of ``a`` with pivots ``jp`` against the oracle's."""
    a = np.asarray(a, dtype=np.float64)
    m, n = a.shape
    cola = np.linalg.norm(a[:, jp], axis=0)
    r_g, r_o = np.triu(af_g[:k, :]), np.triu(af_o[:k, :])
    v_g, v_o = np.tril(af_g[:, :k], -1), np.tril(af_o[:, :k], -1)
    rjj = np.abs(np.diag(af_o[:k, :k]))
    cancel = np.where(rjj > 0, cola[:k] / np.maximum(rjj, np.finfo(float).tiny), 1.0)
    cancel = np.maximum(cancel, 1.0)
    vscale = np.sqrt(1.0 + np.sum(v_o ** 2, axis=0)) * cancel
    errs = {
        "R": colwise(r_g, r_o, cola),
        "V": colwise(v_g, v_o, vscale),
        "tau": float((np.abs(tau_g - tau_o) / (np.maximum(1.0, np.abs(tau_o)) * cancel)).max()),
        "R_F": normwise(r_g, r_o),
        "V_F": normwise(v_g, v_o),
    }
    if k < min(m, n):
        errs["R22"] = colwise(af_g[k:, k:], af_o[k:, k:], cola[k:])
        errs["R22_F"] = normwise(af_g[k:, k:], af_o[k:, k:], np.linalg.norm(a))
    if b_g is not None and b_o is not None and omega is not None and k < n:
        sk = np.asarray(omega) @ a[:, jp[k:]]
        errs["B"] = colwise(b_g[:, k:], b_o[:, k:], np.linalg.norm(sk, axis=0))
        errs["B_F"] = normwise(b_g[:, k:], b_o[:, k:], np.linalg.norm(np.asarray(omega) @ a))
    return errs


def assert_within(errs, tol, label=""):
    print(label, {kk: float("%.3g" % v) for kk, v in errs.items()})
    for name, e in errs.items():
        if name.endswith("_F"):
            continue
        assert e <= tol, f"{label} {name}: columnwise error {e:.3e} > {tol:.1e}"
