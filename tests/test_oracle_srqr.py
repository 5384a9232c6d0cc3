"""Pins of the SRQR oracle (Alg. 3) and its definitions (Section IV).

* The paper's Kahan tables (Table I, Table II), stored under tests/golden.
* Closed form of the best achievable last diagonal: placing column j last
  gives |R[n-1, n-1]| = 1 / ||e_j^T A^-1||, so the optimum is
  1 / max_j ||e_j^T A^-1||.
* QRCP bounds on g1, g2 (Section IV-D) and the tau bound of Section IV-C.
* The factorization recomputed after swaps satisfies A Pi = Q R.
"""
import json
import os

import numpy as np
import pytest

from oracle import rqrcp as R
from oracle import srqr as S
from workloads import gaussian, kahan, kahan_embedded, lowrank


@pytest.fixture(scope="module")
def tables(golden_dir):
    with open(os.path.join(golden_dir, "kahan_tables.json")) as fh:
        return json.load(fh)


def _best_last_diag(a):
    inv = np.linalg.inv(a)
    return 1.0 / np.sqrt(np.sum(inv ** 2, axis=1)).max()


@pytest.mark.parametrize("row", [0, 1, 2])
def test_kahan_table1(tables, row):
    ent = tables["table1_residual_RF_over_AF"][row]
    n, k = ent["n"], ent["k"]
    kk = kahan(n, tables["setting"]["c"])
    nk = np.linalg.norm(kk)
    # QRCP makes no interchanges on the Kahan matrix (Section V-B)
    af, _, jp = R.qrcp(kk, k)
    assert np.array_equal(jp, np.arange(n))
    assert abs(abs(af[k, k]) / nk - ent["qrcp"]) <= 5e-4 * ent["qrcp"]
    # SRQR, starting from QRCP (Omega = I makes Alg. 2 equal Alg. 1), exact g2
    res = S.srqr(kk, k, 64, n - 64, tables["setting"]["g"], exact=True, omega=np.eye(n))
    assert res.nswaps >= 1
    assert res.g2 <= tables["setting"]["g"]
    assert abs(res.alpha / nk - ent["srqr"]) <= 5e-4 * ent["srqr"]
    assert abs(res.alpha - _best_last_diag(kk)) <= 1e-9 * res.alpha


def test_kahan_table2(tables):
    n, k = 192, 191
    kk = kahan(n, tables["setting"]["c"])
    sa = np.linalg.svd(kk, compute_uv=False)
    af, _, _ = R.qrcp(kk, k)
    sq = np.linalg.svd(np.triu(af[:k, :k]), compute_uv=False)
    res = S.srqr(kk, k, 64, n - 64, 5.0, exact=True, omega=np.eye(n))
    ss = np.linalg.svd(np.triu(res.a_refactored[:k, :k]), compute_uv=False)
    for ent in tables["table2_sigma_ratio_n192"]:
        j = ent["j"] - 1
        assert abs(ss[j] / sa[j] - ent["srqr"]) < 5e-4
        if ent["j"] < 191:
            assert abs(sq[j] / sa[j] - ent["qrcp"]) < 5e-5
        else:
            assert sq[j] / sa[j] < 1e-15


@pytest.mark.parametrize("n", [96, 192])
def test_kahan_randomized_probe(n):
    """d = 16 probes: exits with the estimate below g and a residual within g*sqrt(3) of the best."""
    kk = kahan(n)
    best = _best_last_diag(kk)
    res = S.srqr(kk, n - 1, 64, n - 64, 5.0, seed=3, d=16, omega=np.eye(n))
    assert res.g2 <= 5.0
    assert res.alpha <= 5.0 * np.sqrt(3.0) * best


def test_kahan_from_rqrcp_start():
    n = 96
    kk = kahan(n)
    res = S.srqr(kk, n - 1, 64, 10, 5.0, seed=0, exact=True)
    assert res.g2 <= 5.0
    assert abs(res.alpha - _best_last_diag(kk)) <= 1e-9 * res.alpha


def test_refactored_factorization_is_consistent():
    n = 96
    kk = kahan(n)
    res = S.srqr(kk, n - 1, 64, n - 64, 5.0, exact=True, omega=np.eye(n))
    af, tau = res.a_refactored, res.tau_refactored
    q = R.form_q(af, tau, n)
    rr = R.r_factor(af, len(tau))
    assert np.linalg.norm(kk[:, res.jpvt] - q @ rr) <= 1e-13 * np.linalg.norm(kk)
    # the same permutation gives the same |R| as the Givens-updated R of Alg. 3
    assert np.allclose(np.abs(np.diag(rr)), np.abs(np.diag(res.r[:n, :n])), rtol=1e-8)


def test_qrcp_g1_g2_bounds():
    """Section IV-D: for QRCP g1 <= 1 and g2 <= 2^l."""
    a = gaussian(80, 60, 2)
    l = 20
    af, _, _ = R.qrcp(a, l + 1)
    r = np.triu(af)
    r[l + 1:, l + 1:] = af[l + 1:, l + 1:]
    g1, g2 = S.g1_g2_exact(r, l)
    assert g1 <= 1.0 + 1e-12
    assert g2 <= 2.0 ** l


def test_tau_bound_section_iv_c():
    m, n, l = 150, 120, 25
    sig = np.arange(1, 121, dtype=float) ** -1.0
    a = lowrank(m, n, sig, 4)
    res = S.srqr(a, l, 8, 8, 5.0, seed=1, exact=True, refactor=False)
    g1, g2 = S.g1_g2_exact(res.r, l)
    assert abs(g2 - res.g2) <= 1e-9 * g2
    r22 = res.r[l:, l:]
    n22 = np.linalg.norm(r22, 2)
    n12 = np.sqrt(np.sum(r22 ** 2, axis=0)).max()
    rhat = np.triu(res.r[:l + 1, :l + 1])
    inv = np.linalg.inv(rhat)
    n_inv12 = np.sqrt(np.sum(inv ** 2, axis=1)).max()
    tau = g1 * g2 * (n22 / n12) * (1.0 / n_inv12) / sig[l]
    assert abs(tau * sig[l] - n22) <= 1e-9 * n22           # eq. defining tau
    assert tau <= g1 * g2 * np.sqrt((l + 1) * (n - l))     # its upper bound


def test_random_matrix_needs_no_swaps():
    """Section IV-E: g2 stays modest on ordinary matrices, so no swaps."""
    a = lowrank(200, 160, np.exp(-np.arange(1, 161) / 20.0), 6)
    res = S.srqr(a, 30, 16, 8, 5.0, seed=2, d=16, refactor=False)
    assert res.nswaps == 0 and res.g2 <= 5.0


def test_max_swaps_cap():
    n = 96
    kk = kahan(n)
    res = S.srqr(kk, n - 1, 64, n - 64, 0.5, exact=True, omega=np.eye(n), max_swaps=3, refactor=False)
    assert res.nswaps == 3 and res.g2 > 0.5


def _trailing_sq_norms(rw, top, lo):
    return np.sum(rw[top:, lo:] ** 2, axis=0)


def test_trailing_estimates_track_exact_norms():
    """Alg. 3's trailing-norm estimates (Section IV-E) checked against their
    definition.  With Omega = sqrt(m) I_m (b + p = m sketch rows) the starting
    estimate ||B(:, i)||^2 / (b+p) is the exact squared norm of column i of the
    trailing block, so after every QR step and every round robin the estimates
    must equal the squared norms recomputed from the working array, and every
    column brought to position l must be the exact argmax."""
    m, n, nk = 80, 140, 40
    l = nk - 1
    a = kahan_embedded(m, n, nk, 8, c=0.4, scale=0.01)
    tr = []
    res = S.srqr(a, l, 8, m - 8, 1.1, exact=True, omega=np.sqrt(m) * np.eye(m),
                 refactor=False, max_swaps=50, trace=tr)
    assert res.nswaps >= 3
    assert n - l - 1 >= 50
    stages = [t["stage"] for t in tr]
    assert stages.count("rotate") == res.nswaps and stages.count("qr") == res.nswaps + 1
    for t in tr:
        top = t["top"]
        lo = top if t["stage"] != "qr" else l + 1
        exact = _trailing_sq_norms(t["rw"], top, lo)
        est = t["est"][lo:]
        assert np.all(est >= 0.0)
        assert np.max(np.abs(est - exact)) <= 1e-12 * exact.max(), t["stage"]
        if t["stage"] == "pick":
            srt = np.sort(exact)[::-1]
            assert (srt[0] - srt[1]) > 1e-8 * srt[0]     # separated: the argmax is unique
            assert t["pick"] == lo + int(np.argmax(exact))


def test_trailing_estimate_downdate_stops_at_zero():
    """A sketch-based estimate can be smaller than the squared entry of the row
    that leaves the trailing block; the downdate then gives 0 (a squared norm),
    never a negative estimate that would rank below exactly-zero columns."""
    m, n, nk = 80, 140, 40
    l = nk - 1
    a = kahan_embedded(m, n, nk, 8, c=0.4, scale=0.01)
    tr = []
    S.srqr(a, l, 8, 4, 1.1, seed=2, exact=True, refactor=False, max_swaps=50, trace=tr)
    undershoot = 0
    prev = None
    for t in tr:
        assert np.all(t["est"] >= 0.0)
        if t["stage"] == "qr" and prev is not None:
            row = t["rw"][l, l + 1:]
            before = prev["est"].copy()
            # the pick before this QR step swapped the estimates of l and pick
            j = prev["pick"]
            before[[l, j]] = before[[j, l]]
            raw = before[l + 1:] - row ** 2
            undershoot += int(np.sum(raw < 0.0))
            np.testing.assert_array_equal(t["est"][l + 1:], np.maximum(raw, 0.0))
        prev = t if t["stage"] == "pick" else prev
    assert undershoot >= 1
