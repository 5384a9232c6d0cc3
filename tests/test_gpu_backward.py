"""GPU backward (rqrcp_backward behind torch.autograd) against the FP64 oracle.

The loss is L = sum(W * Q1 [R11 R12] Pi^T) with the pivots frozen at the GPU
forward's choice.  References (oracle/backward.py): the projector closed form
and the QR-adjoint chain (FP64), and central finite differences on a 64 x 32
case.  The FP32 backward at 8192 x 4096 is compared with the FP64 one on the
same pivots and its error stated.
"""
import numpy as np
import pytest

from oracle import backward as BW
from workloads import gaussian, lowrank

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
    return t.detach().double().cpu().numpy()


def _rel(x, y):
    return np.linalg.norm(x - y) / np.linalg.norm(y)


def _loss_grad(rq, a_dev, w_dev, k, b, p, seed=0, jpvt=None):
    """(dL/dA, jpvt) through the autograd Function."""
    import torch
    a = a_dev.detach().clone().requires_grad_(True)
    q1, r, jp = rq.rqrcp(a, k, b, p, seed, jpvt=jpvt)
    approx = torch.empty_like(q1 @ r)
    approx[:, jp.long()] = q1 @ r
    loss = (w_dev * approx).sum()
    loss.backward()
    return a.grad, jp


def test_fp64_gradient_matches_closed_form_and_chain(rq):
    m, n, k, b, p = 300, 200, 40, 16, 8
    a = lowrank(m, n, 1.0 / np.arange(1, n + 1), 1)
    w = gaussian(m, n, 2)
    g, jp = _loss_grad(rq, _dev(a), _dev(w), k, b, p, seed=3)
    jp = _np(jp).astype(int)
    g_cf = BW.grad_closed_form(a, jp, k, w, b)
    g_ch = BW.grad_chain(a, jp, k, w, b)
    e_cf, e_ch = _rel(_np(g), g_cf), _rel(_np(g), g_ch)
    print("FP64 300x200: vs closed form %.2e, vs chain %.2e" % (e_cf, e_ch))
    assert e_cf <= 1e-10 and e_ch <= 1e-10


def test_fp64_gradient_matches_finite_differences(rq):
    """The 64 x 32 sub-case: k = 8, b = 4, p = 8, h = 1e-3 central differences."""
    m, n, k, b, p = 64, 32, 8, 4, 8
    a = gaussian(m, n, 5)
    w = gaussian(m, n, 6)
    g, jp = _loss_grad(rq, _dev(a), _dev(w), k, b, p, seed=1)
    jp = _np(jp).astype(int)
    fd = BW.grad_fd(a, jp, k, w, h=1e-3, b=b)
    err = _rel(_np(g), fd)
    print("FP64 64x32 vs central differences %.2e" % err)
    assert err <= 1e-6


def test_partial_cotangents(rq):
    """Only Q1_bar, or only R_bar, against the adjoint chain."""
    import torch
    m, n, k, b, p = 150, 120, 30, 8, 8
    a = gaussian(m, n, 7)
    f = rq.factor(_dev(a), k, b, p, seed=2)
    jp = _np(f.jpvt).astype(int)
    rng = np.random.default_rng(3)
    q1b = rng.standard_normal((m, k))
    rb = rng.standard_normal((k, n))
    for dq1, dr in ((q1b, None), (None, rb), (q1b, rb)):
        g = rq.backward(_dev(a), f, _dev(dq1) if dq1 is not None else None,
                        _dev(dr) if dr is not None else None)
        ref = BW.adjoint_chain(a, jp, k, q1b if dq1 is not None else np.zeros((m, k)),
                               rb if dr is not None else np.zeros((k, n)), b)
        assert _rel(_np(g), ref) <= 1e-10
    assert torch.isfinite(g).all()


def test_fp32_backward_8192x4096(rq):
    """8192 x 4096, sigma_j = 1/j (Haar U, V), k = 256, b = 64, p = 8: FP32 vs FP64."""
    import torch
    from workloads import lowrank_torch
    m, n, k, b, p = 8192, 4096, 256, 64, 8
    a64 = lowrank_torch(m, n, 1.0 / np.arange(1, n + 1), 5, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    w = torch.randn(n, m, generator=gen, device="cuda", dtype=torch.float64).t()
    g64, jp = _loss_grad(rq, a64, w, k, b, p, seed=4)
    g32, _ = _loss_grad(rq, a64.float(), w.float(), k, b, p, jpvt=_np(jp).astype(np.int64))
    err = float(torch.linalg.norm(g32.double() - g64) / torch.linalg.norm(g64))
    print("FP32 vs FP64 backward at 8192x4096: %.2e" % err)
    assert err <= 1e-3
    # the FP64 GPU gradient against the oracle's closed form at full size
    g_cf = BW.grad_closed_form(_np(a64), _np(jp).astype(int), k, _np(w), b)
    e = _rel(_np(g64), g_cf)
    print("FP64 backward at 8192x4096 vs closed form: %.2e" % e)
    assert e <= 1e-9
