"""Pins of QR with tournament pivoting on the sketch (Section V-C's proposed
replacement of the partial QRCP of B; Demmel, Grigori, Gu and Xiang 2015).

* One group holding every column reduces to the partial QRCP of Alg. 1,
  bit for bit.
* A two-level tournament on a small integer matrix, worked out node by node
  in exact rational arithmetic (each node: greedy largest-residual-norm
  selection by Gram-Schmidt), gives the oracle's winners.
* The transpositions bring the winners to the front in order.
* Exact rank r <= b: the chosen columns span the sketch, so the trailing
  sketch block vanishes; the factorization's invariants hold.
* On a decaying spectrum the tournament's choice is about as good as QRCP's
  (the smallest singular value of the chosen sketch columns).
"""
from fractions import Fraction

import numpy as np

from oracle import rqrcp as R
from workloads import gaussian, integer_matrix, lowrank, sigma_exp


def _exact_choose(cols, nsteps):
    """Greedy selection (Alg. 1 in exact arithmetic): at each step the column
    with the largest squared residual after projecting out the chosen ones
    (ties to the lowest position).  cols: list of exact column vectors."""
    basis, chosen = [], []
    for _ in range(min(nsteps, len(cols))):
        best, bq = None, None
        for q, c in enumerate(cols):
            if q in chosen:
                continue
            r = list(c)
            for u in basis:
                uu = sum(x * x for x in u)
                if uu:
                    f = sum(x * y for x, y in zip(r, u)) / uu
                    r = [x - f * y for x, y in zip(r, u)]
            v = sum(x * x for x in r)
            if best is None or v > best:
                best, bq, br = v, q, r
        if best == 0:
            break
        chosen.append(bq)
        basis.append(br)
    return chosen


def test_single_group_is_qrcp_bitwise():
    a = lowrank(300, 200, sigma_exp(200, 30.0), 2)
    f1 = R.rqrcp(a, 64, 16, 8, seed=4, mode="blocked")
    f2 = R.rqrcp(a, 64, 16, 8, seed=4, mode="blocked", tournament=10 ** 6)
    assert np.array_equal(f1.jpvt, f2.jpvt)
    assert np.array_equal(f1.a, f2.a) and np.array_equal(f1.b, f2.b)


def test_two_level_tournament_in_exact_arithmetic():
    checked = 0
    for seed in range(40):
        w = integer_matrix(5, 12, seed).astype(float)
        exact = [[Fraction(int(x)) for x in w[:, c]] for c in range(12)]
        # leaves {0,1,2}, {3,4,5}, {6,7,8}, {9,10,11}; merges (L0, L1), (L2, L3); final
        leaves = []
        for g in range(4):
            idx = [3 * g, 3 * g + 1, 3 * g + 2]
            leaves.append([idx[j] for j in _exact_choose([exact[c] for c in idx], 2)])
        mids = []
        for h in range(2):
            u = leaves[2 * h] + leaves[2 * h + 1]
            mids.append([u[j] for j in _exact_choose([exact[c] for c in u], 2)])
        u = mids[0] + mids[1]
        final = [u[j] for j in _exact_choose([exact[c] for c in u], 2)]
        tr = R.StepTrace()
        got = R.tournament_choose(w, 2, 3, tr)
        if tr.min_rel_gap() < 1e-9:
            continue                      # a near tie: either answer is correct
        assert got == final, seed
        checked += 1
    assert checked >= 30


def test_transpositions_bring_winners_forward():
    rng = np.random.default_rng(0)
    for _ in range(50):
        n = int(rng.integers(5, 40))
        k = int(rng.integers(1, n))
        win = list(rng.choice(n, size=k, replace=False))
        order = list(range(n))
        for t, p in R.transpositions(win):
            order[t], order[p] = order[p], order[t]
        assert order[:k] == win
        assert sorted(order) == list(range(n))


def test_exact_rank_sketch_block_vanishes():
    m, n, r, b = 120, 300, 11, 16
    a = gaussian(m, r, 1) @ gaussian(r, n, 2)
    f = R.rqrcp(a, 32, b, 8, seed=3, mode="blocked", tournament=40)
    q = R.form_q(f.a, f.tau, m)
    assert np.linalg.norm(a[:, f.jpvt] - q @ R.r_factor(f.a, 32)) <= 1e-13 * np.linalg.norm(a)
    assert np.linalg.norm(R.r_factor(f.a, 32)[r:, r:]) <= 1e-12 * np.linalg.norm(a)


def test_tournament_quality_close_to_qrcp():
    worst = np.inf
    for seed in range(5):
        w = lowrank(72, 2000, sigma_exp(72, 10.0), seed) + 1e-3 * gaussian(72, 2000, seed + 10)
        k = 32
        win_t = R.tournament_choose(w, k, 128)
        win_q = R._qrcp_choose(w, k)
        st = np.linalg.svd(w[:, win_t], compute_uv=False)[-1]
        sq = np.linalg.svd(w[:, win_q], compute_uv=False)[-1]
        worst = min(worst, st / sq)
    assert worst >= 0.2


def test_odd_number_of_groups_in_exact_arithmetic():
    """Three leaves: (L0, L1) merge, L2 passes through, then the final merge."""
    checked = 0
    for seed in range(40):
        w = integer_matrix(4, 9, 100 + seed).astype(float)
        exact = [[Fraction(int(x)) for x in w[:, c]] for c in range(9)]
        leaves = []
        for g in range(3):
            idx = [3 * g, 3 * g + 1, 3 * g + 2]
            leaves.append([idx[j] for j in _exact_choose([exact[c] for c in idx], 2)])
        u = leaves[0] + leaves[1]
        mid = [u[j] for j in _exact_choose([exact[c] for c in u], 2)]
        u = mid + leaves[2]
        final = [u[j] for j in _exact_choose([exact[c] for c in u], 2)]
        tr = R.StepTrace()
        got = R.tournament_choose(w, 2, 3, tr)
        if tr.min_rel_gap() < 1e-9:
            continue
        assert got == final, seed
        checked += 1
    assert checked >= 30


def test_exact_ties_go_to_the_lowest_position():
    """Duplicated columns tie exactly at every level: the lowest positions win."""
    base = gaussian(6, 4, 3)
    w = np.concatenate([base, base, base], axis=1)       # columns j, j + 4, j + 8 equal
    win = R.tournament_choose(w, 3, 4)
    q = R._qrcp_choose(base, 3)
    assert win == q                                       # the copies in group 0 win


def test_four_way_merges_in_exact_arithmetic():
    """Five leaves, fanout 4: (L0..L3) merge, L4 passes through, then the final
    merge of the two."""
    checked = 0
    for seed in range(30):
        w = integer_matrix(4, 15, 200 + seed).astype(float)
        exact = [[Fraction(int(x)) for x in w[:, c]] for c in range(15)]
        leaves = []
        for g in range(5):
            idx = [3 * g, 3 * g + 1, 3 * g + 2]
            leaves.append([idx[j] for j in _exact_choose([exact[c] for c in idx], 2)])
        u = leaves[0] + leaves[1] + leaves[2] + leaves[3]
        mid = [u[j] for j in _exact_choose([exact[c] for c in u], 2)]
        u = mid + leaves[4]
        final = [u[j] for j in _exact_choose([exact[c] for c in u], 2)]
        tr = R.StepTrace()
        got = R.tournament_choose(w, 2, 3, tr, fanout=4)
        if tr.min_rel_gap() < 1e-9:
            continue
        assert got == final, seed
        checked += 1
    assert checked >= 20
