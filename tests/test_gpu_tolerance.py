"""Tolerance-driven RQRCP on the GPU (rqrcp_factor_tol) against the oracle's
stop_tol form of Alg. 2: the same stopping rank, identical pivots, results
within 1e-12 column by column, and the same estimate ratio."""
import numpy as np
import pytest

from oracle import rqrcp as R
from oracle.compare import assert_within, factor_errors
from workloads import gaussian, lowrank, sigma_exp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1804_05138_amd as lib
    lib.load_library()
    return lib


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x).T)).cuda().t()


def _np(t):
    return t.detach().cpu().numpy()


def _check(f, est, f_or, a, label):
    print(label, "k", f.k, "oracle k", f_or.k, "estimate %.6e oracle %.6e" % (est, f_or.est_ratio))
    assert f.k == f_or.k
    # formula (1) leaves the trailing sketch with rounding errors of order
    # u ||B||, so the ratio carries an absolute error of order u besides the
    # relative one
    assert abs(est - f_or.est_ratio) <= 1e-10 * f_or.est_ratio + 1e-14
    jp = _np(f.jpvt)
    assert np.array_equal(jp, f_or.jpvt)
    errs = factor_errors(a, f.k, jp, _np(f.a), _np(f.tau), f_or.a, f_or.tau, _np(f.b), f_or.b,
                         f_or.omega)
    assert_within(errs, 1e-12, label)


@pytest.mark.parametrize("tol", [1e-1, 1e-3, 1e-6])
def test_gaussian_sketch(rq, tol):
    m, n, b, p = 600, 400, 32, 8
    a = lowrank(m, n, sigma_exp(400, 15.0), 3)
    f_or = R.rqrcp(a, 300, b, p, seed=4, mode="blocked", stop_tol=tol)
    assert f_or.trace.min_rel_gap() >= 1e-8
    f, est = rq.factor_tol(_dev(a), tol, 300, b, p, seed=4)
    _check(f, est, f_or, a, f"tol {tol:g}")


def test_exact_sketch(rq):
    """Omega = sqrt(m) I passed as the sketch: the estimate is the true ratio."""
    m, n, b = 120, 100, 8
    a = lowrank(m, n, sigma_exp(100, 6.0), 5)
    om = np.sqrt(m) * np.eye(m)
    f_or = R.rqrcp(a, n, b, m - b, omega=om, mode="blocked", stop_tol=1e-3)
    f, est = rq.factor_tol(_dev(a), 1e-3, n, b, m - b, sketch_b=_dev(om @ a))
    _check(f, est, f_or, a, "exact sketch")


def test_exact_rank(rq):
    m, n, r, b = 150, 90, 37, 8
    a = gaussian(m, r, 1) @ gaussian(r, n, 2)
    f, est = rq.factor_tol(_dev(a), 1e-10, n, b, 8, seed=3)
    assert f.k == 40
    assert est <= 1e-13
    r22 = _np(f.a)[40:, 40:]
    assert np.linalg.norm(r22) <= 1e-13 * np.linalg.norm(a)


def test_kmax_reached(rq):
    a = gaussian(200, 150, 4)
    f, est = rq.factor_tol(_dev(a), 1e-8, 48, 16, 8, seed=1)
    f_or = R.rqrcp(a, 48, 16, 8, seed=1, mode="blocked", stop_tol=1e-8)
    _check(f, est, f_or, a, "kmax")


def test_early_stop_left_looking(rq):
    """kmax <= n/2 (the left-looking schedule) and a tolerance met before kmax:
    the deferred trailing update must be applied at the stopping rank."""
    m, n, b, p = 600, 400, 32, 8
    a = lowrank(m, n, sigma_exp(400, 15.0), 3)
    f_or = R.rqrcp(a, 200, b, p, seed=4, mode="blocked", stop_tol=1e-3)
    assert f_or.k < 200
    assert f_or.trace.min_rel_gap() >= 1e-8
    f, est = rq.factor_tol(_dev(a), 1e-3, 200, b, p, seed=4)
    _check(f, est, f_or, a, "tol 1e-3, kmax 200")
