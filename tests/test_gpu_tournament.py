"""RQRCP with QR with tournament pivoting on the sketch (RQRCP_TOURNAMENT)
against the oracle's tournament form of Alg. 2 (groups of 256 columns,
four-way merges): identical pivots where every selection decision of the tree
is separated, results within 1e-12 column by column."""
import numpy as np
import pytest

from oracle import rqrcp as R
from oracle.compare import assert_within, factor_errors
from workloads import gaussian, separated_lowrank

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


@pytest.mark.parametrize("m,n,k,b,p", [
    (300, 200, 64, 16, 8),      # one group: the tournament is the partial QRCP
    (400, 1000, 96, 32, 8),     # four leaves, one merge
    (300, 5000, 128, 64, 8),    # 20 leaves: 4-way merges with a lone set passing through
    (256, 16384, 192, 64, 8),   # 64 leaves, three merge levels
])
def test_tournament_matches_oracle(rq, m, n, k, b, p):
    a = separated_lowrank(m, n, 7)
    f_or = R.rqrcp(a, k, b, p, seed=3, mode="blocked", tournament=rq.TOURNAMENT_GROUP,
                   fanout=rq.TOURNAMENT_FANOUT)
    gap = f_or.trace.min_rel_gap()
    print(f"{m}x{n}: oracle min gap {gap:.2e}")
    assert gap >= 1e-8
    f = rq.factor(_dev(a), k, b, p, seed=3, tournament=True)
    assert int(_np(f.info)[0]) == 0
    jp = _np(f.jpvt)
    assert np.array_equal(jp, f_or.jpvt)
    errs = factor_errors(a, k, jp, _np(f.a), _np(f.tau), f_or.a, f_or.tau, _np(f.b), f_or.b,
                         f_or.omega)
    assert_within(errs, 1e-12, f"tournament {m}x{n}")


def test_tournament_rank_deficient(rq):
    a = np.zeros((120, 600))
    a[:, :13] = gaussian(120, 13, 9)
    f_or = R.rqrcp(a, 40, 8, 8, seed=3, tournament=256, fanout=4)
    f = rq.factor(_dev(a), 40, 8, 8, seed=3, tournament=True)
    assert int(_np(f.info)[0]) == f_or.info == 14
    assert np.array_equal(_np(f.jpvt), f_or.jpvt)
    assert np.all(_np(f.tau)[13:] == 0.0)
