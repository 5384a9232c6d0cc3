"""Pins of the tolerance-driven form of Alg. 2 (Section III-A: the loop may stop
on an error tolerance instead of a target rank).

The oracle stops after the first block whose trailing sketch estimate
||B(:, i:n)||_F / sqrt(l) is at most tol times the initial sketch's estimate
of ||A||_F.  Pins:
* Omega = sqrt(m) I (l = m rows): the sketch norms are exact, so the stop
  rank is the smallest multiple of b at which LAPACK's QRCP (dgeqp3, the
  same pivots) has ||R22||_F <= tol ||A||_F, and the reported ratio equals
  ||R22||_F / ||A||_F;
* an input of exact rank r stops at the first block boundary at or past r
  with R22 = 0 to rounding;
* with a Gaussian sketch the estimate is within a factor 2 of the true ratio.
"""
import numpy as np
import scipy.linalg as sl

from oracle import rqrcp as R
from workloads import gaussian, lowrank, sigma_exp


def _true_ratio(a, f):
    r22 = f.a[f.k:, f.k:]
    return np.linalg.norm(r22) / np.linalg.norm(a)


def test_exact_sketch_stops_where_qrcp_residual_drops_below_tol():
    m, n, b = 120, 100, 8
    a = lowrank(m, n, sigma_exp(100, 6.0), 5)
    _, rr, piv = sl.qr(a, pivoting=True, mode="economic")
    na = np.linalg.norm(a)
    for tol in (1e-1, 1e-2, 1e-3, 1e-5):
        f = R.rqrcp(a, n, b, m - b, omega=np.sqrt(m) * np.eye(m), mode="blocked", stop_tol=tol)
        ks = [k for k in range(b, n + 1, b) if np.linalg.norm(rr[k:, k:]) <= tol * na]
        assert f.k == ks[0], (tol, f.k, ks[0])
        assert np.array_equal(f.jpvt[:f.k], piv[:f.k])
        assert abs(f.est_ratio - np.linalg.norm(rr[f.k:, f.k:]) / na) <= 1e-12
        assert abs(f.est_ratio - _true_ratio(a, f)) <= 1e-12
        assert len(f.tau) == f.k


def test_exact_rank_stops_at_the_next_block_boundary():
    m, n, r, b = 150, 90, 37, 8
    a = gaussian(m, r, 1) @ gaussian(r, n, 2)
    f = R.rqrcp(a, n, b, 8, seed=3, mode="blocked", stop_tol=1e-10)
    assert f.k == 40
    assert _true_ratio(a, f) <= 1e-13
    assert f.est_ratio <= 1e-13


def test_gaussian_sketch_estimate_within_factor_two():
    m, n, b, p = 400, 300, 16, 56
    a = lowrank(m, n, sigma_exp(300, 20.0), 7)
    for tol in (1e-1, 1e-2, 1e-3):
        f = R.rqrcp(a, n, b, p, seed=11, mode="blocked", stop_tol=tol)
        true = _true_ratio(a, f)
        assert 0.5 <= f.est_ratio / true <= 2.0, (tol, f.est_ratio, true)
        assert f.est_ratio <= tol


def test_no_stop_when_tolerance_not_met():
    a = gaussian(80, 60, 4)
    f = R.rqrcp(a, 24, 8, 8, seed=1, mode="blocked", stop_tol=1e-8)
    assert f.k == 24 and len(f.tau) == 24
    g = R.rqrcp(a, 24, 8, 8, seed=1, mode="blocked")
    assert np.array_equal(f.a, g.a) and np.array_equal(f.jpvt, g.jpvt)
