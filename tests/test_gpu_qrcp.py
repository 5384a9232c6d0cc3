"""GPU QR with column pivoting of the whole matrix (Alg. 1, the comparator of
RQRCP) through the C ABI, against the oracle's Alg. 1 (trailing norms
recomputed at every step, pinned to LAPACK dgeqp3 by the CPU tests).

The GPU downdates the norms (recomputing them when a downdate has lost half
the digits), so pivots are asserted equal where the oracle's pivot decisions
are separated (relative gap of the two largest squared norms >= 1e-6 at every
step); results within 1e-12 column by column (``oracle/compare.py``).
"""
import numpy as np
import pytest

from oracle import rqrcp as R
from oracle.compare import assert_within, factor_errors
from workloads import gaussian, lowrank, separated_lowrank, sigma_exp

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
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x).T)).cuda().t()


def _np(t):
    return t.detach().cpu().numpy()


def _check(rq, a, k, nb, label):
    tr = R.StepTrace()
    af_o, tau_o, jp_o = R.qrcp(a, k, trace=tr)
    gap = tr.min_rel_gap()
    f = rq.qrcp(_dev(a), k, nb)
    jp = _np(f.jpvt)
    print(label, "oracle min gap %.2e" % gap)
    assert np.array_equal(np.sort(jp), np.arange(a.shape[1]))
    assert gap >= 1e-6, "input not separated"
    assert np.array_equal(jp, jp_o), f"{label}: pivots differ"
    errs = factor_errors(a, k, jp, _np(f.a), _np(f.tau), af_o, tau_o)
    assert_within(errs, TOL, label)


@pytest.mark.parametrize("m,n,k,nb", [
    (64, 48, 16, 8),         # one small block
    (300, 200, 60, 16),      # several blocks, ragged last one
    (500, 400, 160, 64),     # 64-wide blocks, block update by the GEMM
    (256, 1000, 200, 64),    # wide
    (1500, 300, 300, 64),    # k = n: the whole factorization
    (333, 271, 100, 128),    # the widest block
])
def test_qrcp_matches_oracle(rq, m, n, k, nb):
    a = separated_lowrank(m, n, 4)
    _check(rq, a, k, nb, f"qrcp {m}x{n} k={k} nb={nb}")


def test_qrcp_norm_recomputation(rq):
    """sigma_j = exp(-j/4): the trailing norms fall by far more than 1e-4 of the
    starting ones within a block, so most downdates trigger the exact recompute."""
    m, n, k = 400, 300, 120
    a = lowrank(m, n, sigma_exp(300, 4.0), 2)
    _check(rq, a, k, 64, "qrcp fast decay")


def test_qrcp_equals_dgeqp3(rq):
    import scipy.linalg as sl
    a = gaussian(600, 250, 3)
    f = rq.qrcp(_dev(a), 250, 64)
    _, _, piv = sl.qr(a, pivoting=True, mode="economic")
    assert list(_np(f.jpvt)) == list(piv)


def test_qrcp_rank_deficient(rq):
    """Exactly zero trailing columns: tau = 0 past the rank, pivots still a
    permutation, the factorization reproduces A Pi."""
    a = np.zeros((200, 120))
    a[:, :17] = gaussian(200, 17, 9)
    f = rq.qrcp(_dev(a), 60, 16)
    tau = _np(f.tau)
    assert np.all(tau[17:] == 0.0)
    af, jp = _np(f.a), _np(f.jpvt)
    q = R.form_q(af, tau, 200)
    assert np.linalg.norm(a[:, jp] - q @ R.r_factor(af, 60)) <= 1e-13 * np.linalg.norm(a)
