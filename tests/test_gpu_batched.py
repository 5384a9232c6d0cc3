"""Batched RQRCP (one persistent launch, work queue) against the FP64 oracle.

Every problem j is the single-matrix Alg. 2 with Omega from Philox stream
j + 1, run by the oracle on the same FP32-rounded matrix in FP64.  The batched
kernel keeps A in FP32 (trailing update in FP32, reflectors and sketch in
FP64), so results agree to FP32 accuracy and pivots agree exactly on every
problem whose pivot decisions are separated by more than the FP32 rounding
can move them (GAP below); every problem, separated or not, must satisfy the
factorization's invariants to FP32 accuracy.
"""
import numpy as np
import pytest

from oracle import philox as P
from oracle import rqrcp as R
from workloads import batch_shapes, lowrank

pytestmark = pytest.mark.gpu

B, PP = 16, 8
L = B + PP


@pytest.fixture(scope="module")
def rq():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1804_05138_amd as lib
    lib.load_library()
    return lib


def _problem(m, n, seed):
    """A = U diag(exp(-j / (n / 10))) V^T, Haar U, V (rank min(m, n)), FP32."""
    r = min(m, n)
    sig = np.exp(-np.arange(1, r + 1) / (n / 10.0))
    return lowrank(m, n, sig, seed).astype(np.float32)


def _fill(rq, shapes, seed0):
    import torch
    bt = rq.make_batch(shapes, L)
    mats = []
    host = np.zeros(bt.a.numel(), dtype=np.float32)
    for j, (m, n, k) in enumerate(shapes):
        a = _problem(m, n, seed0 + j)
        mats.append(a)
        off = int(bt.offsets[j]["a_off"])
        host[off:off + m * n] = a.T.reshape(-1)      # column-major
    bt.a.copy_(torch.from_numpy(host))
    return bt, mats


def _unpack(bt, j):
    rec = bt.offsets[j]
    m, n, k = int(rec["m"]), int(rec["n"]), int(rec["k"])
    a = bt.a.cpu().numpy()
    af = a[rec["a_off"]:rec["a_off"] + m * n].reshape(n, m).T.astype(np.float64)
    jp = bt.jpvt.cpu().numpy()[rec["jpvt_off"]:rec["jpvt_off"] + n]
    tau = bt.tau.cpu().numpy()[rec["tau_off"]:rec["tau_off"] + k]
    bs = bt.b.cpu().numpy()[rec["b_off"]:rec["b_off"] + L * n].reshape(n, L).T
    return af, jp, tau, bs


def _rel(x, y, s=None):
    s = np.linalg.norm(y) if s is None else s
    return np.linalg.norm(x - y) / (s if s > 0 else 1.0)


# FP32 storage and trailing update perturb the trailing sketch norms by a few
# FP32 ulps of the original column norms, amplified by at most ||A(:, j)|| over
# the trailing norm (below 4 at k = n/8 with sigma_j = exp(-j/(n/10))): a
# relative gap of 1e-5 between the two largest squared norms is far above that.
GAP = 1e-5


def test_batched_matches_oracle(rq):
    """256 uneven problems (plus the largest and smallest allowed shapes) against
    the single-matrix oracle: identical pivots on every problem whose pivot
    decisions are separated by more than GAP; FP32-level agreement of R, V, tau
    and the final sketch where the pivots agree; on every problem the
    factorization's own invariants (A Pi = Q R and orthonormal Q) to FP32
    accuracy."""
    import torch
    nb = 256
    shapes = list(batch_shapes(nb, 3))
    shapes[0] = (1024, 512, 64)       # the largest problem the kernel takes
    shapes[1] = (64, 64, 8)           # the smallest
    shapes[2] = (100, 300, 37)        # wide, ragged last block
    bt, mats = _fill(rq, shapes, 100)
    rq.factor_batched(bt, B, PP, seed=9)
    torch.cuda.synchronize()
    info = bt.info.cpu().numpy()
    assert np.all(info == 0), info
    worst = {"R": 0.0, "V": 0.0, "tau": 0.0, "B": 0.0, "res": 0.0, "orth": 0.0}
    nsep = nsame = 0
    for j, (m, n, k) in enumerate(shapes):
        a = mats[j].astype(np.float64)
        om = P.gauss(L, m, 9, j + 1)
        f = R.rqrcp(a, k, B, PP, omega=om, mode="blocked")
        af, jp, tau, bs = _unpack(bt, j)
        assert np.array_equal(np.sort(jp), np.arange(n)), f"problem {j}: not a permutation"
        same = np.array_equal(jp, f.jpvt)
        gap = f.trace.min_rel_gap()
        if gap >= GAP:
            nsep += 1
            assert same, f"problem {j} {shapes[j]}: pivots differ (gap {gap:.1e})"
        q = R.form_q(af, tau, m)
        res = np.linalg.norm(a[:, jp] - q @ R.r_factor(af, k)) / np.linalg.norm(a)
        orth = np.linalg.norm(q[:, :k].T @ q[:, :k] - np.eye(k))
        worst["res"] = max(worst["res"], res)
        worst["orth"] = max(worst["orth"], orth)
        if not same:
            continue
        nsame += 1
        e = {"R": _rel(np.triu(af[:k]), np.triu(f.a[:k])),
             "V": _rel(np.tril(af[:, :k], -1), np.tril(f.a[:, :k], -1)),
             "tau": _rel(tau, f.tau),
             "B": _rel(bs[:, k:], f.b[:, k:], np.linalg.norm(om @ a))}
        for kk, v in e.items():
            worst[kk] = max(worst[kk], v)
    print("separated problems", nsep, "equal pivots", nsame, "of", nb, "worst", worst)
    assert nsep >= nb // 2
    for kk, v in worst.items():
        assert v <= 2e-5, kk


def test_invalid_descriptor_is_skipped(rq):
    import torch
    shapes = [(200, 100, 12), (1100, 100, 12), (300, 200, 25)]   # m = 1100 is over the limit
    bt, mats = _fill(rq, shapes, 7)
    rq.factor_batched(bt, B, PP, seed=1)
    torch.cuda.synchronize()
    info = bt.info.cpu().numpy()
    assert info[1] == -1 and info[0] == 0 and info[2] == 0
    f = R.rqrcp(mats[2].astype(np.float64), 25, B, PP, omega=P.gauss(L, 300, 1, 3), mode="blocked")
    af, jp, _, _ = _unpack(bt, 2)
    assert np.array_equal(jp, f.jpvt)


def test_graph_replay_matches_eager(rq):
    """Capture [restore A; factor_batched] in a HIP graph; replay three times with
    eager work in between; every replay equals the eager run bitwise."""
    import torch
    shapes = list(batch_shapes(40, 5))
    bt, _ = _fill(rq, shapes, 50)
    a0 = bt.a.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bt.a.copy_(a0)
        rq.factor_batched(bt, B, PP, seed=4)     # eager, on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    ref = [x.clone() for x in (bt.a, bt.jpvt, bt.tau, bt.b, bt.info)]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
        bt.a.copy_(a0)
        rq.factor_batched(bt, B, PP, seed=4)
    for rep in range(3):
        bt.a.fill_(7.0)
        bt.b.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for x, y in zip((bt.a, bt.jpvt, bt.tau, bt.b, bt.info), ref):
            assert torch.equal(x, y), f"replay {rep} differs"


def test_autotuner_picks_a_variant(rq):
    import torch
    shapes = list(batch_shapes(64, 8))
    bt, mats = _fill(rq, shapes, 300)
    a0 = bt.a.clone()
    best, ms_v = rq.autotune_batched(bt, a0, B, PP, seed=2)
    print("autotuner: best variant", best, "ms per variant", ms_v)
    assert best in (0, 1) and all(t > 0 for t in ms_v)
    torch.cuda.synchronize()
    assert np.all(bt.info.cpu().numpy() == 0)
    # the tuned variant is used from now on and gives a valid factorization
    bt.a.copy_(a0)
    rq.factor_batched(bt, B, PP, seed=2)
    torch.cuda.synchronize()
    m, n, k = shapes[0]
    f = R.rqrcp(mats[0].astype(np.float64), k, B, PP, omega=P.gauss(L, m, 2, 1), mode="blocked")
    af, jp, _, _ = _unpack(bt, 0)
    if np.array_equal(jp, f.jpvt):
        assert _rel(np.triu(af[:k]), np.triu(f.a[:k])) <= 2e-5
