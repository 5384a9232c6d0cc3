"""Pins of the RQRCP oracle (Alg. 1, Alg. 2, update formulas (1) and (2)).

Each test checks the oracle against something other than itself:
* exact rational brute force of the greedy sketch selection (Section III-B/C:
  every pivot is the largest column of a Gaussian matrix times the trailing
  matrix, i.e. of Omega P_perp A),
* LAPACK special cases (Omega = I reduces RQRCP to QRCP = dgeqp3; frozen pivots
  reduce it to dgeqrf),
* the equivalence of the two update formulas (Section III-B),
* the invariants and singular-value inequalities of Lemma 1, Lemma 3 and
  Section IV-B,
* the worked example of Theorem 1.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sl

from oracle import rqrcp as R
from workloads import (gaussian, integer_matrix, lowrank, rng, separated_lowrank,
                       sigma_exp)


# ---------------------------------------------------------------------------
# exact brute force
# ---------------------------------------------------------------------------

def _dot(x, y):
    return sum(a * b for a, b in zip(x, y))


def _proj_out(x, basis):
    """x minus its projection on span(basis); basis is mutually orthogonal."""
    x = list(x)
    for u in basis:
        uu = _dot(u, u)
        if uu == 0:
            continue
        c = _dot(x, u) / uu
        x = [a - c * b for a, b in zip(x, u)]
    return x


def exact_rqrcp(a_int, om_int, k, b):
    """Greedy selection of Alg. 2 in exact rational arithmetic.

    At a block start with chosen set S the sketch is C = Omega P_perp_S A
    (update formula (2)); within the block the greedy steps are Gram-Schmidt
    in sketch space.  Ties go to the lowest position.  Returns the position
    order, the exact |r_ii|^2, the exact squared trailing sketch norms and the
    smallest relative gap between the two largest candidates over all steps.
    """
    m, n = a_int.shape
    cols = [[Fraction(int(a_int[r, c])) for r in range(m)] for c in range(n)]
    om = [[Fraction(int(x)) for x in row] for row in om_int]
    pos = list(range(n))
    a_basis = []
    rdiag = []
    min_gap = None
    i = 0
    while i < k:
        bb = min(b, k - i)
        sk = {}
        for q in range(i, n):
            y = _proj_out(cols[pos[q]], a_basis)
            sk[pos[q]] = [_dot(row, y) for row in om]
        s_basis = []
        for t in range(bb):
            vals = []
            for q in range(i + t, n):
                r = _proj_out(sk[pos[q]], s_basis)
                vals.append((_dot(r, r), q))
            best = max(v for v, _ in vals)
            q = min(qq for v, qq in vals if v == best)
            others = sorted((v for v, qq in vals if qq != q), reverse=True)
            if best > 0 and others:
                gap = (best - others[0]) / best
                min_gap = gap if min_gap is None else min(min_gap, gap)
            pos[i + t], pos[q] = pos[q], pos[i + t]
            s_basis.append(_proj_out(sk[pos[i + t]], s_basis))
            u = _proj_out(cols[pos[i + t]], a_basis)
            rdiag.append(_dot(u, u))
            a_basis.append(u)
        i += bb
    trailing = []
    for q in range(k, n):
        y = _proj_out(cols[pos[q]], a_basis)
        z = [_dot(row, y) for row in om]
        trailing.append(_dot(z, z))
    return pos, rdiag, trailing, min_gap


@pytest.mark.parametrize("case", range(40))
def test_exact_bruteforce_pivots_diagonal_and_sketch(case):
    g = rng(900 + case)
    m = int(g.integers(6, 13))
    n = int(g.integers(5, 11))
    k = int(g.integers(2, min(m, n) + 1))
    b = int(g.integers(1, 4))
    p = int(g.integers(1, 4))
    l = b + p
    a = integer_matrix(m, n, 1000 + case)
    om = g.integers(-3, 4, size=(l, m)).astype(np.float64)
    pos, rdiag, trailing, gap = exact_rqrcp(a, om, k, b)
    if gap is not None and float(gap) < 1e-9:
        pytest.skip("exact tie between candidates")
    if min(rdiag) == 0:
        pytest.skip("exactly rank deficient")
    f = R.rqrcp(a, k, b, p, omega=om)
    assert f.info == 0
    assert list(f.jpvt) == pos
    d = np.diag(f.a[:k, :k]) ** 2
    ex = np.array([float(x) for x in rdiag])
    assert np.allclose(d, ex, rtol=1e-11, atol=0)
    if k < n:
        bn = np.sum(f.b[:, k:] ** 2, axis=0)
        ext = np.array([float(x) for x in trailing])
        assert np.allclose(bn, ext, rtol=1e-9, atol=1e-9 * max(1.0, ext.max()))


# ---------------------------------------------------------------------------
# LAPACK special cases
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_identity_sketch_reduces_to_qrcp_dgeqp3(seed):
    m, n, k, b = 48, 36, 20, 6
    a = gaussian(m, n, seed)
    f = R.rqrcp(a, k, b, m - b, omega=np.eye(m))
    if f.trace.min_rel_gap() < 1e-8:
        pytest.skip("near tie")
    _, _, piv = sl.qr(a, pivoting=True)
    assert list(f.jpvt[:k]) == list(piv[:k])
    af, tau, jp = R.qrcp(a, k)
    assert list(jp[:k]) == list(piv[:k])
    assert np.allclose(np.abs(np.diag(af[:k, :k])), np.abs(np.diag(f.a[:k, :k])), rtol=1e-12)


def test_lemma1_pseudo_diagonal_dominance_of_qrcp():
    a = gaussian(60, 45, 3)
    af, tau, _ = R.qrcp(a, 30)
    r = np.triu(af)
    r[30:, 30:] = af[30:, 30:]
    for i in range(30):
        tail = np.sqrt(np.sum(r[i:, i + 1:] ** 2, axis=0))
        assert abs(r[i, i]) >= tail.max() * (1 - 1e-12)


@pytest.mark.parametrize("k,b", [(20, 7), (36, 36), (1, 1), (33, 16)])
def test_frozen_pivots_equal_dgeqrf(k, b):
    a = gaussian(70, 36, 4)
    jp = rng(5).permutation(36)
    af, tau = R.factor_frozen(a, jp, k, b)
    (qr, tau_l), _ = sl.qr(a[:, jp], mode="raw")
    assert np.allclose(af[:, :k], qr[:, :k], rtol=0, atol=1e-13)
    assert np.allclose(tau, tau_l[:k], rtol=0, atol=1e-14)
    qt = R.apply_qt(af, tau, a[:, jp])
    assert np.allclose(af[k:, k:], qt[k:, k:], atol=1e-13)
    assert np.allclose(np.triu(af[:k]), np.triu(qt[:k]), atol=1e-13)


def test_householder_matches_dlarfg_signs():
    for alpha, x in [(3.0, [4.0]), (-3.0, [4.0]), (0.0, [1.0, 2.0]), (2.0, [0.0, 0.0]), (-2.0, [0.0])]:
        beta, tau, v = R.householder(alpha, np.array(x))
        if not np.any(x):
            assert tau == 0.0 and beta == alpha
            continue
        (qr, tl), _ = sl.qr(np.array([[alpha] + list(x)]).T, mode="raw")
        assert np.isclose(beta, qr[0, 0]) and np.isclose(tau, tl[0])
        assert np.allclose(v, qr[1:, 0])


# ---------------------------------------------------------------------------
# modes and update formulas
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("m,n,k,b,p", [(200, 150, 40, 16, 8), (97, 131, 50, 13, 5), (64, 64, 64, 8, 4)])
def test_plain_blocked_and_formula2_agree(m, n, k, b, p):
    a = separated_lowrank(m, n, 7)
    f1 = R.rqrcp(a, k, b, p, seed=3, mode="plain")
    f2 = R.rqrcp(a, k, b, p, seed=3, mode="blocked")
    f3 = R.rqrcp(a, k, b, p, seed=3, update="formula2")
    assert f1.trace.min_rel_gap() > 1e-8
    assert np.array_equal(f1.jpvt, f2.jpvt)
    assert np.array_equal(f1.jpvt, f3.jpvt)       # Section III-B: identical permutations
    scale = np.abs(f1.a).max()
    assert np.abs(f1.a - f2.a).max() < 1e-13 * scale
    if k < n:
        n1 = np.linalg.norm(f1.b[:, k:], axis=0)
        n3 = np.linalg.norm(f3.b[:, k:], axis=0)
        assert np.abs(n1 - n3).max() < 1e-12 * n1.max()


def test_sketch_is_omega_times_a():
    a = gaussian(30, 20, 1)
    f = R.rqrcp(a, 1, 4, 4, seed=9)
    from oracle.philox import gauss
    om = gauss(8, 30, 9, 0)
    assert np.array_equal(f.omega, om)
    # the first column of the final B was the first pivot; the rest of B is the
    # formula-(1) update of Omega A, whose norms equal those of Omega P_perp A
    q = R.form_q(f.a, f.tau)
    proj = a[:, f.jpvt[1:]] - q @ (q.T @ a[:, f.jpvt[1:]])
    assert np.allclose(np.linalg.norm(f.b[:, 1:], axis=0), np.linalg.norm(om @ proj, axis=0), rtol=1e-12)


# ---------------------------------------------------------------------------
# invariants and bounds
# ---------------------------------------------------------------------------

def test_invariants_c1_shape():
    """The small configuration: 1024 x 1024, sigma_j = exp(-j/40), k=64, b=32, p=8."""
    a = lowrank(1024, 1024, sigma_exp(1024, 40.0), 1)
    k = 64
    f = R.rqrcp(a, k, 32, 8, seed=1, mode="blocked")
    q1, r11, r12, r22 = R.pieces(f, k)
    assert np.linalg.norm(q1.T @ q1 - np.eye(k)) <= 1e-13
    qf = R.form_q(f.a, f.tau, 1024)
    res = np.linalg.norm(a[:, f.jpvt] - qf @ R.r_factor(f.a, k)) / np.linalg.norm(a)
    assert res <= 1e-13


def test_exact_rank_leaves_zero_trailing_block():
    k = 24
    a = lowrank(150, 120, sigma_exp(k, 10.0), 2)
    f = R.rqrcp(a, k, 8, 8, seed=2)
    _, _, _, r22 = R.pieces(f, k)
    assert np.linalg.norm(r22) / np.linalg.norm(a) <= 1e-13


def test_prescribed_spectrum_inequalities():
    """Interlacing (Section IV-B), Lemma 3 (both parts) and R22 >= sigma_{k+1}."""
    m, n, k = 180, 140, 30
    sig = np.arange(1, 141, dtype=float) ** -1.5
    a = lowrank(m, n, sig, 3)
    f = R.rqrcp(a, k, 8, 8, seed=5)
    q1, r11, r12, r22 = R.pieces(f, k)
    rt = np.hstack([r11, r12])
    s11 = np.linalg.svd(r11, compute_uv=False)
    srt = np.linalg.svd(rt, compute_uv=False)
    n22 = np.linalg.norm(r22, 2)
    tol = 1e-12
    assert np.all(s11 <= srt * (1 + tol))
    assert np.all(srt <= sig[:k] * (1 + tol))
    assert n22 >= sig[k] * (1 - tol)
    assert np.all(sig[:k] ** 2 <= srt ** 2 + n22 ** 2 + tol)
    u, s, vt = np.linalg.svd(rt, full_matrices=False)
    rk = (u[:, :k] * s[:k]) @ vt[:k]
    qf = R.form_q(f.a, f.tau, m)
    approx = qf[:, :k] @ rk
    lhs = np.linalg.norm(a[:, f.jpvt] - approx, 2)
    rhs = sig[k] * np.sqrt(1 + (n22 / sig[k]) ** 2)
    assert lhs <= rhs * (1 + tol)
    ratio = s11 / sig[:k]
    assert ratio.max() <= 1 + tol and ratio.min() > 0.1


def test_theorem1_dominance_holds_for_moderate_eps():
    """Theorem 1's dominance with eps = 0.9 on a random matrix (p = 10)."""
    a = gaussian(300, 200, 8)
    k = 60
    f = R.rqrcp(a, k, 16, 10, seed=4)
    r = R.r_factor(f.a, k)
    c = np.sqrt((1 - 0.9) / (1 + 0.9))
    for i in range(k):
        tail = np.sqrt(np.sum(r[i:, i + 1:] ** 2, axis=0))
        assert abs(r[i, i]) >= c * tail.max()


def test_rank_deficiency_sets_info():
    a = np.zeros((40, 30))
    a[:, :7] = gaussian(40, 7, 11)
    f = R.rqrcp(a, 20, 5, 4, seed=1)
    assert f.info == 8
    assert np.all(f.tau[7:] == 0.0)
    assert sorted(f.jpvt[:7]) == list(range(7))
    q1 = R.form_q(f.a, f.tau[:7])
    res = a[:, f.jpvt] - q1 @ np.triu(f.a[:7, :])
    assert np.linalg.norm(res) <= 1e-13 * np.linalg.norm(a)


def test_argument_errors():
    with pytest.raises(ValueError):
        R.rqrcp(np.ones((4, 3)), 4, 2, 2)
    with pytest.raises(ValueError):
        R.rqrcp(np.ones((4, 3)), 0, 2, 2)


def test_oversampling_worked_example(golden_dir):
    with open(os.path.join(golden_dir, "oversampling_example.json")) as fh:
        ex = json.load(fh)
    assert R.oversampling_bound(ex["n"], ex["k"], ex["eps"], ex["delta"]) == ex["p_min"]
