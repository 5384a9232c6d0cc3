"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Bar: identical pivots on inputs whose trailing sketch norms are separated
(relative gap of the two largest >= 1e-8 at every step, measured by the
oracle), and FP64 results within 1e-12 relative (normwise per output array:
R and V in the factored A, tau; R22 relative to ||A||_F and the trailing
sketch relative to ||Omega A||_F, the scales their rounding errors live on --
both can be zero in exact arithmetic, e.g. the sketch when k = m).
"""
import numpy as np
import pytest

from oracle import philox as P
from oracle import rqrcp as R
from workloads import gaussian, lowrank, separated_lowrank, sigma_exp, sigma_pow

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def rq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1804_05138_amd as lib
    lib.load_library()
    return lib


def _dev(x):
    """Column-major device copy of a NumPy matrix."""
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x).T)).cuda().t()


def _np(t):
    return t.detach().cpu().numpy()


def _rel(x, y, scale=None):
    s = np.linalg.norm(y) if scale is None else scale
    return np.linalg.norm(x - y) / (s if s > 0 else 1.0)


def _compare(f_gpu, f_or, a, k, label=""):
    af = _np(f_gpu.a)
    jp = _np(f_gpu.jpvt)
    assert np.array_equal(jp, f_or.jpvt), f"{label} pivots differ"
    na = np.linalg.norm(a)
    r_g = np.triu(af[:k, :])
    r_o = np.triu(f_or.a[:k, :])
    v_g = np.tril(af[:, :k], -1)
    v_o = np.tril(f_or.a[:, :k], -1)
    errs = {
        "R": _rel(r_g, r_o),
        "V": _rel(v_g, v_o),
        "tau": _rel(_np(f_gpu.tau), f_or.tau),
        "R22": _rel(af[k:, k:], f_or.a[k:, k:], na),
    }
    if f_gpu.b is not None and k < a.shape[1]:
        nb = np.linalg.norm(f_or.omega @ a) if f_or.omega is not None else None
        errs["B"] = _rel(_np(f_gpu.b)[:, k:], f_or.b[:, k:], nb)
    print(label, {kk: float("%.3g" % v) for kk, v in errs.items()})
    if errs.get("B", 0.0) > TOL:
        bd = np.abs(_np(f_gpu.b)[:, k:] - f_or.b[:, k:])
        print("B max error per row:", np.array2string(bd.max(axis=1), precision=2))
        print("B max error per column:", np.array2string(bd.max(axis=0), precision=2))
    for name, e in errs.items():
        assert e <= TOL, f"{label} {name} rel err {e:.3e}"


def test_gaussian_matches_oracle(rq):
    for rows, cols, seed, stream in [(40, 1024, 1, 0), (7, 13, 5, 3), (72, 333, 0, 1 << 32)]:
        om = _np(rq.gaussian(rows, cols, seed, stream))
        ref = P.gauss(rows, cols, seed, stream)
        err = np.abs(om - ref) / np.maximum(1.0, np.abs(ref))
        assert err.max() <= 16 * 2.0 ** -52, (rows, cols, err.max())


def test_sketch_is_omega_a(rq):
    for m, n, l in [(1024, 1024, 40), (333, 517, 72), (3000, 700, 24), (64, 5, 9)]:
        a = gaussian(m, n, 1)
        b = _np(rq.sketch(_dev(a), l, seed=7))
        ref = P.gauss(l, m, 7, 0) @ a
        assert _rel(b, ref) <= 1e-14, (m, n, l)


def test_sketch_with_user_omega(rq):
    m, n, l = 500, 300, 20
    a = gaussian(m, n, 2)
    om = np.random.default_rng(0).standard_normal((l, m))
    b = _np(rq.sketch(_dev(a), l, omega=_dev(om)))
    assert _rel(b, om @ a) <= 1e-14


@pytest.mark.parametrize("m,n,k,b,p", [
    (64, 48, 16, 8, 4),        # single small blocks
    (200, 150, 40, 16, 8),     # several blocks
    (333, 271, 77, 16, 8),     # ragged tiles and a short last block
    (130, 257, 64, 32, 8),     # wide
    (700, 300, 96, 32, 8),     # tall, several row tiles
    (256, 256, 256, 64, 8),    # k = n: full factorization
    (97, 131, 97, 13, 5),      # k = m < n, odd block size
    (500, 400, 160, 80, 16),   # tall sketch (l = 96): four columns per thread, several workgroups
    (400, 300, 150, 128, 8),   # a 128-wide panel in two halves, then a narrow one after it
    (600, 500, 256, 128, 16),  # 128-wide panels after 128-wide blocks
    (256, 16384, 192, 64, 8),  # sketch QRCP over the full-width grid: 64 workgroups exchange candidates
    (160, 32768, 128, 64, 8),  # 128 workgroups; candidate headers read first, then the winner's column
])
def test_factor_parity(rq, m, n, k, b, p):
    a = separated_lowrank(m, n, 11)
    f_or = R.rqrcp(a, k, b, p, seed=5, mode="blocked")
    assert f_or.trace.min_rel_gap() >= 1e-8
    f = rq.factor(_dev(a), k, b, p, seed=5)
    assert int(_np(f.info)[0]) == 0
    _compare(f, f_or, a, k, f"{m}x{n} k={k} b={b} p={p}")


def test_factor_c1_configuration(rq):
    """1024 x 1024, sigma_j = exp(-j/40), Haar U, V; k=64, b=32, p=8."""
    a = lowrank(1024, 1024, sigma_exp(1024, 40.0), 1)
    f_or = R.rqrcp(a, 64, 32, 8, seed=1, mode="blocked")
    assert f_or.trace.min_rel_gap() >= 1e-8
    f = rq.factor(_dev(a), 64, 32, 8, seed=1)
    _compare(f, f_or, a, 64, "C1")


def test_factor_invariants(rq):
    import torch
    m, n, k = 900, 700, 128
    a = lowrank(m, n, sigma_pow(700, 1.5), 3)
    f = rq.factor(_dev(a), k, 64, 8, seed=2)
    q1 = rq.form_q(f.a, f.tau, k, 64)
    qq = _np(q1)
    assert np.linalg.norm(qq.T @ qq - np.eye(k)) <= 1e-13
    af = _np(f.a)
    jp = _np(f.jpvt)
    qf = R.form_q(af, _np(f.tau), m)          # full Q from the GPU's reflectors
    assert np.allclose(qf[:, :k], qq, atol=1e-13)
    res = np.linalg.norm(a[:, jp] - qf @ R.r_factor(af, k)) / np.linalg.norm(a)
    assert res <= 1e-13


def test_frozen_pivots_equal_dgeqrf(rq):
    import scipy.linalg as sl
    m, n, k, b = 300, 200, 70, 32
    a = gaussian(m, n, 4)
    jp = np.random.default_rng(1).permutation(n)
    f = rq.factor(_dev(a), k, b, 8, jpvt=jp)
    (qr, tau), _ = sl.qr(a[:, jp], mode="raw")
    af = _np(f.a)
    assert np.array_equal(_np(f.jpvt), jp)
    assert _rel(np.triu(af[:k]), np.triu(qr[:k])) <= TOL
    assert _rel(np.tril(af[:, :k], -1), np.tril(qr[:, :k], -1)) <= TOL
    assert _rel(_np(f.tau), tau[:k]) <= TOL


def test_user_sketch_identity_reduces_to_qrcp(rq):
    """Omega = I (l = m): the sketch QRCP is QRCP on A itself."""
    import scipy.linalg as sl
    m, n, k, b = 96, 120, 40, 8
    a = gaussian(m, n, 6)
    f_or = R.rqrcp(a, k, b, m - b, omega=np.eye(m))
    if f_or.trace.min_rel_gap() < 1e-8:
        pytest.skip("near tie")
    f = rq.factor(_dev(a), k, b, m - b, sketch_b=_dev(a.copy()))
    _, _, piv = sl.qr(a, pivoting=True)
    assert list(_np(f.jpvt)[:k]) == list(piv[:k])
    _compare(f, f_or, a, k, "omega=I")


def test_rank_deficient_info(rq):
    a = np.zeros((120, 90))
    a[:, :13] = gaussian(120, 13, 9)
    f_or = R.rqrcp(a, 40, 8, 8, seed=3)
    f = rq.factor(_dev(a), 40, 8, 8, seed=3)
    assert int(_np(f.info)[0]) == f_or.info == 14
    assert np.array_equal(_np(f.jpvt), f_or.jpvt)
    assert np.all(_np(f.tau)[13:] == 0.0)


def test_repeatable_bitwise(rq):
    a = separated_lowrank(400, 300, 2)
    f1 = rq.factor(_dev(a), 100, 32, 8, seed=9)
    f2 = rq.factor(_dev(a), 100, 32, 8, seed=9)
    assert np.array_equal(_np(f1.a), _np(f2.a))
    assert np.array_equal(_np(f1.b), _np(f2.b))


def test_form_q_zero_tau_and_wide_block(rq):
    """Explicit Q1 from the GPU's reflectors against the oracle's product of
    reflectors: a rank-deficient input (tau = 0 past the rank, whose reflectors
    are the identity) with 16-wide blocks, and a 128-wide block."""
    a = np.zeros((120, 90))
    a[:, :13] = gaussian(120, 13, 9)
    f = rq.factor(_dev(a), 40, 8, 8, seed=3)
    assert np.all(_np(f.tau)[13:] == 0.0)
    q = _np(rq.form_q(f.a, f.tau, 40, 16))
    qf = R.form_q(_np(f.a), _np(f.tau), 120)[:, :40]
    assert np.abs(q - qf).max() <= 1e-13
    a2 = gaussian(300, 200, 4)
    f2 = rq.factor(_dev(a2), 150, 128, 8, seed=1)
    q2 = _np(rq.form_q(f2.a, f2.tau, 150, 128))
    qf2 = R.form_q(_np(f2.a), _np(f2.tau), 300)[:, :150]
    assert np.abs(q2 - qf2).max() <= 1e-13
