"""The allocation-free entry point rqrcp_factor_noalloc against rqrcp_factor.

Both run the same kernels; only the workspace differs (the library's static
device scratch instead of a caller's buffer), so the outputs must be
identical bit for bit.  Two calls in a row, the second smaller, check that
the shared scratch is reset between calls; sizes beyond the scratch are
rejected before anything is enqueued."""
import numpy as np
import pytest

from workloads import lowrank, separated_lowrank, sigma_exp

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


def _run(rq, a, k, b, p, seed, noalloc, flags=0, jpvt=None):
    import torch
    m, n = a.shape
    at = _dev(a).t().clone().t()
    jp = torch.empty(n, dtype=torch.int32, device="cuda")
    if jpvt is not None:
        jp.copy_(torch.as_tensor(jpvt, dtype=torch.int32))
    tau = torch.empty(k, dtype=torch.float64, device="cuda")
    bs = None if flags & rq.FROZEN_PIVOTS else torch.empty((n, b + p), dtype=torch.float64,
                                                           device="cuda").t()
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    if noalloc:
        assert rq.workspace_bytes(m, n, k, b, p, flags) <= rq.NOALLOC_MAX_BYTES
        rq.factor_noalloc_into(at, k, b, p, seed, jp, tau, bs, info, flags)
        rq.check(None)
    else:
        ws = rq.workspace(rq.workspace_bytes(m, n, k, b, p, flags), "cuda")
        rq.factor_into(at, k, b, p, seed, jp, tau, bs, info, ws, flags)
        rq.check(ws)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (at, jp, tau, info) + ((bs,) if bs is not None else ())]


CASES = [(1024, 1024, 64, 32, 8, 1), (300, 220, 64, 32, 8, 2)]   # the second is smaller


def _input(m, n, seed):
    return lowrank(m, n, sigma_exp(min(m, n), 40.0), seed) if m == 1024 else separated_lowrank(m, n, seed)


def test_noalloc_matches_factor(rq):
    refs = [_run(rq, _input(m, n, s), k, b, p, s, False) for (m, n, k, b, p, s) in CASES]
    # two no-alloc calls in a row on the same static scratch, the second smaller
    got = [_run(rq, _input(m, n, s), k, b, p, s, True) for (m, n, k, b, p, s) in CASES]
    for case, ref, out in zip(CASES, refs, got):
        assert int(out[3][0]) == 0
        for x, y in zip(ref, out):
            assert np.array_equal(x, y), case


def test_noalloc_frozen_pivots(rq):
    a = separated_lowrank(500, 400, 3)
    jp = np.random.default_rng(4).permutation(400)
    ref = _run(rq, a, 96, 32, 8, 0, False, flags=rq.FROZEN_PIVOTS, jpvt=jp)
    got = _run(rq, a, 96, 32, 8, 0, True, flags=rq.FROZEN_PIVOTS, jpvt=jp)
    for x, y in zip(ref, got):
        assert np.array_equal(x, y)


def test_noalloc_rejects_sizes_beyond_the_scratch(rq):
    import torch
    m = n = 4096
    k, b, p = 512, 64, 8
    assert rq.workspace_bytes(m, n, k, b, p) > rq.NOALLOC_MAX_BYTES
    a = torch.zeros((n, m), dtype=torch.float64, device="cuda").t()
    jp = torch.empty(n, dtype=torch.int32, device="cuda")
    tau = torch.empty(k, dtype=torch.float64, device="cuda")
    bs = torch.empty((n, b + p), dtype=torch.float64, device="cuda").t()
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(RuntimeError, match="1009"):
        rq.factor_noalloc_into(a, k, b, p, 0, jp, tau, bs, info)
