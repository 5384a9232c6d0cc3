"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Bar: identical pivots on inputs whose trailing sketch norms are separated
(relative gap of the two largest >= 1e-8 at every step, measured by the
oracle), and FP64 results within 1e-12 column by column (``oracle/compare.py``):
each column of R, V, R22 and the trailing sketch against the scale its
rounding errors live on (the norm of the input column it came from, of the
reflector, of the original sketch column), tau elementwise.
"""
import numpy as np
import pytest

from oracle import philox as P
from oracle import rqrcp as R
from oracle.compare import assert_within, factor_errors
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
    jp = _np(f_gpu.jpvt)
    assert np.array_equal(jp, f_or.jpvt), f"{label} pivots differ"
    b_g = _np(f_gpu.b) if f_gpu.b is not None else None
    errs = factor_errors(a, k, jp, _np(f_gpu.a), _np(f_gpu.tau), f_or.a, f_or.tau,
                         b_g, f_or.b, f_or.omega)
    assert_within(errs, TOL, label)


def test_gaussian_matches_oracle(rq):
    for rows, cols, seed, stream in [(40, 1024, 1, 0), (7, 13, 5, 3), (72, 333, 0, 1 << 32)]:
        om = _np(rq.gaussian(rows, cols, seed, stream))
        ref = P.gauss(rows, cols, seed, stream)
        err = np.abs(om - ref) / np.maximum(1.0, np.abs(ref))
        print("Omega", (rows, cols), "max error in units of 2^-52: %.2f" % (err.max() / 2.0 ** -52))
        assert err.max() <= 4 * 2.0 ** -52, (rows, cols, err.max())


def test_sketch_is_omega_a(rq):
    # even m with l divisible by 4 takes the transposed-Omega product (row tiles of
    # 16: l <= 64, 80 or 128); odd m or other l the direct kernel
    for m, n, l in [(1024, 1024, 40), (333, 517, 72), (3000, 700, 24), (64, 5, 9),
                    (2048, 600, 72), (1000, 300, 96), (4096, 1000, 128), (258, 77, 76)]:
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
    (1100, 900, 700, 48, 8),   # k > n/2 and above one outer block: A2 -= V W' mid-way (at column 480)
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
    errs = factor_errors(a, k, jp, af, _np(f.tau), qr, tau[:k])
    # LAPACK's R22 is that of the full factorization, not of k steps
    errs = {kk: v for kk, v in errs.items() if not kk.startswith("R22")}
    assert_within(errs, TOL, "frozen vs dgeqrf")


@pytest.mark.parametrize("case", ["out_of_range", "negative", "duplicate"])
def test_frozen_pivots_invalid_permutation(rq, case):
    """A caller's jpvt that is not a permutation is rejected on the device:
    info = -8 and rqrcp_check reports RQRCP_ERR_PIVOTS (every index the
    kernels use is clamped, so nothing outside the matrices is touched)."""
    import torch
    m, n, k, b = 200, 150, 40, 16
    a = gaussian(m, n, 4)
    jp = np.arange(n)
    if case == "out_of_range":
        jp[7] = n + 1000
    elif case == "negative":
        jp[n - 1] = -5
    else:
        jp[3] = jp[90]
    with pytest.raises(RuntimeError, match="1008"):
        rq.factor(_dev(a), k, b, 8, jpvt=jp)
    # the same handle and a valid permutation work afterwards
    f = rq.factor(_dev(a), k, b, 8, jpvt=np.arange(n))
    assert int(_np(f.info)[0]) == 0
    # the backward rejects it too
    fb = rq.factor(_dev(a), k, b, 8, seed=1)
    fb.jpvt.copy_(torch.as_tensor(jp, dtype=torch.int32, device=fb.jpvt.device))
    with pytest.raises(RuntimeError, match="1008"):
        rq.backward(_dev(a), fb, dr=_dev(np.ones((k, n))))


def _graded(m, n, decades, seed):
    """sigma_j = 10^(-decades (j-1)/63) for j <= 64, then 10^-decades e^(-(j-64)/30):
    the first 64 pivoted columns form a panel with condition number near
    10^decades inside one block."""
    j = np.arange(1, n + 1, dtype=float)
    sig = np.where(j <= 64, 10.0 ** (-decades * (j - 1) / 63.0),
                   10.0 ** (-decades) * np.exp(-(j - 64) / 30.0))
    return lowrank(m, n, sig, seed)


@pytest.mark.parametrize("decades", [3, 5, 6])
def test_graded_panel(rq, decades):
    """A panel graded inside one 64-column block: the Cholesky-QR2 panel (taken
    while diag(R1) spreads less than its trust bound, else the stepwise
    kernel) and the stepwise Householder panel both against the oracle."""
    m, n, k, b, p = 2048, 256, 128, 64, 8
    a = _graded(m, n, decades, 7)
    f_or = R.rqrcp(a, k, b, p, seed=3, mode="blocked")
    assert f_or.trace.min_rel_gap() >= 1e-8
    r11 = np.abs(np.diag(f_or.a[:64, :64]))
    print(f"graded 1e{decades}: diag(R11) of block 0 spreads {r11.max() / r11.min():.2e}")
    for hh in (False, True):
        f = rq.factor(_dev(a), k, b, p, seed=3, householder_panel=hh)
        _compare(f, f_or, a, k, f"graded 1e{decades} {'stepwise' if hh else 'default'} panel")


def test_factor_c2a_matrix_k256(rq):
    """The benchmark's 16384 x 16384 matrix (sigma_j = j^-1.5, Haar U, V,
    generated on the GPU) at k = 256, b = 64, p = 8 against the blocked oracle:
    128-row Gram chunks of the panel, four row splits of the trailing update and
    64 workgroups in the sketch QRCP, all at the full size."""
    import torch
    from workloads import lowrank_torch
    m = n = 16384
    k, b, p, seed = 256, 64, 8, 2
    a_dev = lowrank_torch(m, n, sigma_pow(n, 1.5), seed, device="cuda")
    a = np.asfortranarray(_np(a_dev))
    f = rq.factor(a_dev, k, b, p, seed=seed)
    assert int(_np(f.info)[0]) == 0
    af, tau_g, jp, b_g = _np(f.a), _np(f.tau), _np(f.jpvt), _np(f.b)
    del f, a_dev
    torch.cuda.empty_cache()
    f_or = R.rqrcp(a, k, b, p, seed=seed, mode="blocked")
    gap = f_or.trace.min_rel_gap()
    print("C2a k=256: smallest relative gap of the top two sketch norms", gap)
    assert gap >= 1e-8
    assert np.array_equal(jp, f_or.jpvt)
    errs = factor_errors(a, k, jp, af, tau_g, f_or.a, f_or.tau, b_g, f_or.b, f_or.omega)
    assert_within(errs, TOL, "C2a k=256")


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
