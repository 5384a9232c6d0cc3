"""Pins of the oracle's Gaussian generator (Omega of Alg. 2 / Alg. 3).

* Bit-exact against the published Philox4x64-10 known-answer vectors.
* Bit-exact against NumPy's independent Philox implementation (its
  ``random_raw`` increments the counter before producing a block).
* The vectorized generator against the plain-integer definition.
* Distribution checks on the resulting normals.
"""
import math
import os

import numpy as np
import pytest

from oracle import philox


def _kat(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "philox4x64_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_known_answer_vectors(golden_dir):
    rows = _kat(golden_dir)
    assert len(rows) == 3
    for ctr, key, out in rows:
        assert list(philox.philox4x64_10(ctr, key)) == out


def test_known_answer_vectors_vectorized(golden_dir):
    for ctr, key, out in _kat(golden_dir):
        if ctr[1:] != [0, 0, 0]:
            continue
        got = philox.philox_blocks(ctr[0], 1, key)[0]
        assert [int(x) for x in got] == out


@pytest.mark.parametrize("seed,stream", [(0, 0), (1, 2), (12345, 7), (3, 1 << 32), (2**62 + 5, 99)])
def test_matches_numpy_philox(seed, stream):
    ref = np.random.Philox(key=[seed, stream]).random_raw(1001)
    assert np.array_equal(philox.raw_words(1001, seed, stream), ref)


def test_vectorized_equals_scalar_definition():
    blocks = philox.philox_blocks(1, 50, (77, 3))
    for i in range(50):
        assert tuple(int(x) for x in blocks[i]) == philox.philox4x64_10((i + 1, 0, 0, 0), (77, 3))


def test_uniform_stays_inside_open_interval():
    ext = np.array([0, 2**64 - 1, 2**12 - 1, 2**12], dtype=np.uint64)
    u = philox.uniforms(ext)
    assert np.all(u > 0.0) and np.all(u < 1.0)
    assert u[0] == 2.0 ** -53 and u[2] == 2.0 ** -53
    assert u[1] == 1.0 - 2.0 ** -53
    assert u[3] == 3 * 2.0 ** -53


def test_normals_vector_vs_scalar():
    z = philox.normals(40, 5, 0)
    zs = np.array([philox.normal_scalar(q, 5, 0) for q in range(40)])
    assert np.max(np.abs(z - zs) / np.maximum(np.abs(zs), 1e-300)) < 4 * 2.0 ** -52


def test_gauss_layout_is_column_major_counter_order():
    om = philox.gauss(7, 5, 11, 2)
    z = philox.normals(35, 11, 2)
    for c in range(5):
        for r in range(7):
            assert om[r, c] == z[c * 7 + r]


def test_normal_statistics():
    n = 1 << 20
    z = philox.normals(n, 2024, 0)
    mean = z.mean()
    var = z.var()
    kurt = np.mean((z - mean) ** 4) / var ** 2
    assert abs(mean) < 5.0 / math.sqrt(n)
    assert abs(var - 1.0) < 5.0 * math.sqrt(2.0 / n)
    assert abs(kurt - 3.0) < 5.0 * math.sqrt(24.0 / n)
    # the sin and cos halves of each Box-Muller pair are uncorrelated
    zz = z.reshape(-1, 2)
    assert abs(np.mean(zz[:, 0] * zz[:, 1])) < 5.0 / math.sqrt(n / 2)


def test_streams_are_independent():
    a = philox.normals(4096, 9, 0)
    b = philox.normals(4096, 9, 1)
    assert abs(np.corrcoef(a, b)[0, 1]) < 5.0 / math.sqrt(4096)
