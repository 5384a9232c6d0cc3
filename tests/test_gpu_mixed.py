"""The mixed-precision form on the GPU (FP32 storage and trailing update, BF16
or FP8 sketch, FP64 reflectors) through the C ABI.

The paper computes in FP64 only, so these results have no FP64 oracle to be
bit-compared with; what is checked:

* the low-precision sketches equal an emulation built from torch's own
  casts (``to(bfloat16)``, ``to(float8_e4m3fn)`` with the per-column power-of-two
  scales) followed by an FP64 product, up to FP32 accumulation error -- this
  pins the rounding mode, the e4m3 encoding and the MFMA operand layouts;
* the FP32 factorization equals the FP64 oracle run on the same FP32-rounded
  matrix to FP32 accuracy, with identical pivots on well-separated inputs;
* the FP32 explicit Q1 is orthonormal to FP32 accuracy;
* the low-rank residual ||A Pi - Q1 [R11 R12]||_F / ||A||_F of the mixed form is
  within 1.01x of the FP64 run on the same matrix (the target stated for
  the mixed form), evaluated in FP64.
"""
import numpy as np
import pytest

from oracle import philox as P
from oracle import rqrcp as R
from workloads import gaussian, lowrank, separated_lowrank, sigma_pow

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1804_05138_amd as lib
    lib.load_library()
    return lib


def _dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(np.asarray(x).T)).cuda().t()
    return t if dtype is None else t.to(dtype)


def _np(t):
    return t.detach().double().cpu().numpy()


def _rel(x, y):
    s = np.linalg.norm(y)
    return np.linalg.norm(x - y) / (s if s > 0 else 1.0)


def _fp8_scales(a32):
    mx = np.abs(a32).max(axis=0)
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(448.0 / np.where(mx > 0, mx, 1.0)))
    return np.where(mx > 0, 2.0 ** e, 1.0)


@pytest.mark.parametrize("stype", ["bf16", "fp8"])
@pytest.mark.parametrize("m,n,l", [(1000, 700, 72), (4096, 300, 144), (257, 129, 24)])
def test_low_precision_sketch_matches_emulation(rq, stype, m, n, l):
    import torch
    a = gaussian(m, n, 5) * np.linspace(0.01, 30.0, n)     # columns of very different scale
    a32 = a.astype(np.float32)
    om = P.gauss(l, m, 7, 0)
    if stype == "bf16":
        oq = torch.from_numpy(om).to(torch.bfloat16).double().numpy()
        aq = torch.from_numpy(a32).to(torch.bfloat16).double().numpy()
        ref = oq @ aq
    else:
        s = _fp8_scales(a32)
        oq = torch.from_numpy(om).to(torch.float8_e4m3fn).double().numpy()
        aq = torch.from_numpy((a32 * s).astype(np.float32)).to(torch.float8_e4m3fn).double().numpy()
        ref = (oq @ aq) / s
    b = _np(rq.sketch(_dev(a32), l, seed=7, sketch_type=stype))
    err = _rel(b, ref)
    exact = _rel(b, om @ a)
    print(stype, (m, n, l), "vs emulation %.2e" % err, "vs exact FP64 %.2e" % exact)
    # FP32 accumulation of m products: a few ulps of FP32 times sqrt(m).  For
    # e4m3 the hardware conversion may also treat the format's subnormal range
    # (|x| < 2^-6, reached by about 1% of the unscaled Omega entries)
    # differently from torch's cast; that shows up at the 1e-5 level, three
    # orders of magnitude below the format's own rounding error.
    bound = 4e-7 * np.sqrt(m) if stype == "bf16" else 1e-4
    assert err <= bound
    assert exact <= (0.02 if stype == "bf16" else 0.2)


def test_fp32_sketch_f64_arithmetic(rq):
    a32 = gaussian(900, 400, 3).astype(np.float32)
    b = _np(rq.sketch(_dev(a32), 40, seed=1))
    assert _rel(b, P.gauss(40, 900, 1, 0) @ a32.astype(np.float64)) <= 1e-14


@pytest.mark.parametrize("m,n,k,b,p", [(400, 300, 96, 32, 8), (333, 271, 77, 16, 8),
                                        (600, 500, 128, 64, 8), (300, 260, 200, 128, 16)])
def test_fp32_factor_matches_oracle(rq, m, n, k, b, p):
    import torch
    a32 = separated_lowrank(m, n, 11).astype(np.float32)
    a = a32.astype(np.float64)
    f_or = R.rqrcp(a, k, b, p, seed=5, mode="blocked")
    f = rq.factor(_dev(a32), k, b, p, seed=5)
    assert f.a.dtype == torch.float32
    af = _np(f.a)
    gap = f_or.trace.min_rel_gap()
    same = np.array_equal(_np(f.jpvt).astype(int), f_or.jpvt)
    errs = {"R": _rel(np.triu(af[:k]), np.triu(f_or.a[:k])),
            "V": _rel(np.tril(af[:, :k], -1), np.tril(f_or.a[:, :k], -1)),
            "tau": _rel(_np(f.tau), f_or.tau)}
    # the factorization's own invariants hold whatever the pivots: A Pi = Q R and
    # orthonormal Q1, to FP32 accuracy
    jp = _np(f.jpvt).astype(int)
    q = R.form_q(af.astype(np.float64), _np(f.tau), m)
    res = np.linalg.norm(a[:, jp] - q @ R.r_factor(af.astype(np.float64), k)) / np.linalg.norm(a)
    orth = np.linalg.norm(q[:, :k].T @ q[:, :k] - np.eye(k))
    print((m, n, k, b, p), "min gap %.1e" % gap, "pivots equal", same,
          {kk: "%.2e" % v for kk, v in errs.items()}, "residual %.1e orth %.1e" % (res, orth))
    assert res <= 2e-5 and orth <= 2e-5
    # FP32 storage perturbs a trailing sketch norm by about eps32 times the ratio
    # of the column's first norm to its trailing norm; every decision the oracle
    # takes with a relative gap of 1e-5 or more must agree (the smallest gap on
    # these inputs is 1.1e-4)
    if gap >= 1e-5:
        assert same
    if same:
        for name, e in errs.items():
            assert e <= 2e-5, name


def test_fp32_frozen_equals_dgeqrf_and_q_is_orthonormal(rq):
    import scipy.linalg as sl
    m, n, k, b = 700, 300, 150, 64
    a32 = gaussian(m, n, 4).astype(np.float32)
    jp = np.random.default_rng(1).permutation(n)
    f = rq.factor(_dev(a32), k, b, 8, jpvt=jp)
    (qr, tau), _ = sl.qr(a32.astype(np.float64)[:, jp], mode="raw")
    af = _np(f.a)
    assert _rel(np.triu(af[:k]), np.triu(qr[:k])) <= 1e-5
    assert _rel(np.tril(af[:, :k], -1), np.tril(qr[:, :k], -1)) <= 1e-5
    q = _np(rq.form_q(f.a, f.tau, k, b))
    assert np.linalg.norm(q.T @ q - np.eye(k)) <= 1e-5


def _residual(rq, a_dev, f, k, b):
    """||A Pi - Q1 [R11 R12]||_F / ||A||_F in FP64."""
    import torch
    q = rq.form_q(f.a, f.tau, k, b).double()
    r = torch.triu(f.a[:k].double())
    api = a_dev.double()[:, f.jpvt.long()]
    return float(torch.linalg.norm(api - q @ r) / torch.linalg.norm(a_dev.double()))


@pytest.mark.parametrize("stype", ["f64", "bf16", "fp8"])
def test_mixed_residual_within_one_percent(rq, stype):
    """A = U diag(j^-2) V^T + N(0, s^2), 2048 x 2048, k = 256, b = 128, p = 16.

    Rounding A to the sketch format perturbs every sketch column by about
    u_fmt ||A(:, j)||, and the sample update carries that perturbation along, so
    it competes with the trailing columns' own content in the late blocks.  At
    the 32768 x 32768 configuration (noise std 1e-6) the noise in a column,
    1e-6 sqrt(32768) = 1.8e-4, is 7.5 times the BF16 rounding of a column; at
    2048 x 2048 the same ratio needs s = 2e-5, which this test uses.  FP8's
    rounding (2^-4) is larger than the noise at either size, yet its residual
    stays within the same 1% (measured ratio 1.0014).
    """
    import torch
    m = n = 2048
    k, b, p = 256, 128, 16
    a = lowrank(m, n, sigma_pow(n, 2.0), 3) + 2e-5 * gaussian(m, n, 4)
    a64 = _dev(a)
    f64 = rq.factor(a64, k, b, p, seed=2)
    res64 = _residual(rq, a64, f64, k, b)
    a32 = a64.to(torch.float32)
    fm = rq.factor(a32, k, b, p, seed=2, sketch_type=stype)
    resm = _residual(rq, a64, fm, k, b)
    print(stype, "residual FP64 %.6e  mixed %.6e  ratio %.5f" % (res64, resm, resm / res64))
    assert resm <= 1.01 * res64
