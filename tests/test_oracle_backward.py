"""Pins of the two reference gradients of A -> Q1 [R11 R12] Pi^T with frozen pivots.

* The closed-form projector derivative and the QR-adjoint chain agree (FP64).
* Both agree with central finite differences on the 64 x 32 sub-case
  (k = 8, b = 4, p = 8, h = 1e-3).
* Special case k = m = n: Q1 [R11 R12] Pi^T = A, so dL/dA = W exactly.
"""
import numpy as np
import pytest

from oracle import backward as BW
from oracle import rqrcp as R
from workloads import gaussian, lowrank, rng, sigma_pow


def _setup(m, n, k, b, p, seed):
    a = lowrank(m, n, sigma_pow(min(m, n), 1.0), seed)
    f = R.rqrcp(a, k, b, p, seed=seed)
    w = rng(seed, 10).standard_normal((m, n))
    return a, f.jpvt, w


@pytest.mark.parametrize("m,n,k,b", [(64, 32, 8, 4), (120, 90, 30, 16), (50, 50, 50, 8)])
def test_closed_form_equals_adjoint_chain(m, n, k, b):
    a, jp, w = _setup(m, n, k, b, 8, 3)
    g1 = BW.grad_closed_form(a, jp, k, w, b)
    g2 = BW.grad_chain(a, jp, k, w, b)
    assert np.abs(g1 - g2).max() <= 1e-12 * np.abs(g1).max() * max(1.0, np.linalg.cond(a[:, jp[:k]]))


def test_finite_differences_64x32():
    a, jp, w = _setup(64, 32, 8, 4, 8, 1)
    a = a * np.sqrt(a.size)          # O(1) entries, so h = 1e-3 is a small relative step
    g = BW.grad_chain(a, jp, 8, w, 4)
    gf = BW.grad_fd(a, jp, 8, w, h=1e-3, b=4)
    assert np.abs(g - gf).max() <= 1e-6 * np.abs(g).max()


def test_full_rank_square_gradient_is_w():
    a = gaussian(20, 20, 5)
    f = R.rqrcp(a, 20, 4, 4, seed=5)
    w = rng(5, 11).standard_normal((20, 20))
    for fn in (BW.grad_closed_form, BW.grad_chain):
        assert np.allclose(fn(a, f.jpvt, 20, w, 4), w, atol=1e-11)


def test_gradient_independent_of_block_size():
    a, jp, w = _setup(70, 40, 12, 4, 8, 2)
    g4 = BW.grad_chain(a, jp, 12, w, 4)
    g12 = BW.grad_chain(a, jp, 12, w, 12)
    assert np.allclose(g4, g12, atol=1e-12 * np.abs(g4).max())
