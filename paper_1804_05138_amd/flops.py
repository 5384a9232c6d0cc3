"""Algorithmic flop counts used to report RQRCP throughput.

``rqrcp_flops`` counts the arithmetic of Alg. 2 as the paper describes it
(the sketch B = Omega A, then per block of bb columns: the partial QRCP of the
l-row sketch, the Householder panel QR and its T factor, the block-reflector
update of the trailing matrix, and the sample update formula (1) of Section
III-B with its O(n k b) total cost), independent of how the kernels tile it:

    2 l m n
    + sum over blocks [ sum_{t<bb} 4 (l - t)(n_r - t)        QRCP of the sketch
                        + 2 m_r bb^2 + m_r bb^2              panel QR, T factor
                        + 4 m_r bb (n_r - bb)                trailing update
                        + bb^2 (n_r - bb) + 2 bb^2 (n_r - bb) ]   W' = T^T W, sample update

with m_r = m - i, n_r = n - i at block start i, bb = min(b, k - i), l = b + p.
``qr_equivalent_flops`` is the usual count of a k-step Householder QR.
"""
from __future__ import annotations


def rqrcp_flops(m: int, n: int, k: int, b: int, p: int) -> float:
    l = b + p
    total = 2.0 * l * m * n
    i = 0
    while i < k:
        bb = min(b, k - i)
        mr, nr = m - i, n - i
        total += sum(4.0 * (l - t) * (nr - t) for t in range(bb))
        total += 3.0 * mr * bb * bb
        total += 4.0 * mr * bb * (nr - bb)
        total += 3.0 * bb * bb * (nr - bb)
        i += bb
    return total


def qr_equivalent_flops(m: int, n: int, k: int) -> float:
    return 4.0 * m * n * k - 2.0 * (m + n) * k * k + 4.0 * k ** 3 / 3.0


def backward_flops(m: int, n: int, k: int, b: int) -> float:
    """Algorithmic flops of the frozen-pivot adjoint as the library computes it:
    Q1 from the reflectors (per block: V^T Q, T Y, Q -= V Z and the Gram V^T V),
    R11^-1, and the products A2 R12_bar^T, Q1 R12_bar, R11 R11_bar^T,
    Q1_bar'^T Q1, Q1 copyltu(M) and (.) R11^-T."""
    total = 0.0
    j = 0
    while j < k:
        bb = min(b, k - j)
        rows, nc = m - j, k - j
        total += 2.0 * rows * bb * bb + 4.0 * rows * bb * nc + 2.0 * bb * bb * nc
        j += bb
    n2 = n - k
    total += k ** 3 / 3.0
    total += 4.0 * m * k * n2 + 2.0 * k ** 3 + 6.0 * m * k * k
    return total
