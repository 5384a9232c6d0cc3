"""CX, CUR (Section V-D) and the SVD compression of an l-step factorization
(Section IV-E) on the GPU, through the C ABI, against the oracle's plain
definitions (X = C^+ A, U = C^+ A R^+ with a library pseudo-inverse; the SVD
of R_l).  Inputs: a seeded RBF kernel matrix (the shape of the CUR/CX
experiment, scaled down for the oracle) and a decaying low-rank matrix."""
import numpy as np
import pytest

from oracle import cur as C
from oracle import rqrcp as R
from workloads import lowrank, rbf_kernel, sigma_exp

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


def _srqr_fact(rq, a, k, seed):
    """SRQR with l = k (the experiment's setting) on the GPU; the result as a
    Factorization with k = l (its first l columns are the selection)."""
    res = rq.srqr(_dev(a), k, 16, 8, 5.0, seed=seed)
    return rq.Factorization(res.a, res.jpvt, res.tau, None, None, k, 16)


def test_cx_and_cur_on_kernel_matrix(rq):
    n, k = 700, 60
    a = rbf_kernel(n, 8, 3, 1.0)
    fc = _srqr_fact(rq, a, k, 1)
    fr = _srqr_fact(rq, np.asfortranarray(a.T), k, 2)
    cols, rows = _np(fc.jpvt)[:k], _np(fr.jpvt)[:k]
    # the oracle's SRQR makes the same selections
    ocols, _ = C.select(a, k, 16, 8, 5.0, seed=1)
    orows, _ = C.select(np.asfortranarray(a.T), k, 16, 8, 5.0, seed=2)
    assert np.array_equal(cols, ocols) and np.array_equal(rows, orows)
    x = _np(rq.cx_from(fc, k))
    c, x_ref = C.cx(a, cols)
    ex = np.abs(x - x_ref).max() / np.abs(x_ref).max()
    u = _np(rq.cur_from(fc, fr, k))
    _, u_ref, r = C.cur(a, cols, rows)
    eu = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
    res_cx = np.linalg.norm(a - c @ x) / np.linalg.norm(a)
    res_cur = np.linalg.norm(a - c @ u @ r) / np.linalg.norm(a)
    print(f"CX: X err {ex:.2e} residual {res_cx:.4e}; CUR: U err {eu:.2e} residual {res_cur:.4e}; "
          f"kappa(C) {np.linalg.cond(c):.1e} kappa(R) {np.linalg.cond(r):.1e}")
    # the factorization route and the pseudo-inverse route agree to the
    # conditioning of C (and R) times the FP64 unit
    assert ex <= 1e-10
    assert eu <= 1e-9
    assert abs(res_cx - np.linalg.norm(a - c @ x_ref) / np.linalg.norm(a)) <= 1e-12


@pytest.mark.parametrize("l,k", [(40, 25), (64, 64), (100, 30)])
def test_svd_compression(rq, l, k):
    m, n = 500, 400
    a = lowrank(m, n, sigma_exp(400, 12.0), 4)
    f = rq.factor(_dev(a), l, 16, 8, seed=3)
    x, y, sig = rq.compress(f, l, k)
    x, y, sig = _np(x), _np(y), _np(sig)
    f_or = R.rqrcp(a, l, 16, 8, seed=3, mode="blocked")
    assert np.array_equal(_np(f.jpvt), f_or.jpvt)
    xo, yo = C.svd_compress(f_or.a, f_or.tau, f_or.jpvt, l, k)
    so = np.linalg.svd(np.triu(f_or.a[:l, :]), compute_uv=False)[:k]
    exy = np.abs(x @ y - xo @ yo).max(axis=0) / np.linalg.norm(a, axis=0)
    es = np.abs(sig - so) / so[0]
    print(f"l={l} k={k}: XY columnwise err {exy.max():.2e}, sigma err {es.max():.2e}")
    assert exy.max() <= 1e-12
    assert es.max() <= 1e-13
    assert np.linalg.norm(x.T @ x - np.eye(k)) <= 1e-12
