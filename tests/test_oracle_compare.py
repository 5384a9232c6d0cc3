"""Pins of the column-by-column comparison used by the parity tests.

A wrong column that is small next to the whole array passes a normwise test
of the array; the columnwise measure must catch it, and must not flag
differences at the rounding level of each column's own scale."""
import numpy as np

from oracle import rqrcp as R
from oracle.compare import colwise, factor_errors, normwise
from workloads import separated_lowrank


def test_colwise_catches_a_small_wrong_column():
    rng = np.random.default_rng(0)
    y = rng.standard_normal((50, 40))
    y[:, 7] *= 1e-9                      # a column far below the array's norm
    x = y.copy()
    x[3, 7] += 1e-3 * np.linalg.norm(y[:, 7])   # an error of 1e-3 of that column's norm
    scale = np.linalg.norm(y, axis=0)
    assert normwise(x, y) < 1e-12        # invisible normwise
    assert abs(colwise(x, y, scale) - 1e-3) < 1e-9   # caught column by column


def test_factor_errors_of_identical_and_perturbed_factorizations():
    a = separated_lowrank(120, 90, 3)
    f = R.rqrcp(a, 30, 8, 8, seed=1, mode="blocked")
    g = R.rqrcp(a, 30, 8, 8, seed=1, mode="plain")
    assert np.array_equal(f.jpvt, g.jpvt)
    e = factor_errors(a, 30, f.jpvt, g.a, g.tau, f.a, f.tau, g.b, f.b, f.omega)
    assert max(v for kk, v in e.items() if not kk.endswith("_F")) < 1e-13
    # a wrong V column, a wrong R22 column and a wrong sketch column are each caught
    for which in ("V", "R22", "B"):
        ga, gb = g.a.copy(), g.b.copy()
        if which == "V":
            ga[50:, 29] *= 1.0 + 1e-9
        elif which == "R22":
            ga[30:, 80] += 1e-9 * np.linalg.norm(a[:, f.jpvt[80]])
        else:
            gb[:, 60] += 1e-9 * np.linalg.norm(f.omega @ a[:, f.jpvt[60]])
        e = factor_errors(a, 30, f.jpvt, ga, g.tau, f.a, f.tau, gb, f.b, f.omega)
        assert e[which] > 1e-11, which
