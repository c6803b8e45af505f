"""Pins for the transform-coding oracle (Sec. III-C): what the paper's
description fixes about the two transform sets (additions, subtractions and
power-of-two scalings of the 8 bins; every transformed element a difference,
so a flat histogram maps to zero; together they keep all the shape of a
histogram, i.e. only the constant is lost), the checkerboard use of the two
sets on neighbouring cells, the ternary thresholds, and the code layout
(round trip, rate 2 bits per coded element)."""
import numpy as np
import pytest

from oracle import tq


def _matrix(f):
    return np.stack([f(np.eye(8, dtype=np.float32)[i]) for i in range(8)], axis=1).astype(np.float64)


@pytest.mark.parametrize("f,rank", [(tq.transform_a, 6), (tq.transform_b, 7)])
def test_transform_structure(f, rank):
    T = _matrix(f)                                   # T[k][bin]
    # every element is a difference: a flat histogram gives zero
    np.testing.assert_array_equal(T.sum(axis=1), 0.0)
    # rank: set B keeps all but the constant; in set A as printed, the
    # last element (even bins minus odd bins, over 8) is the sum of the
    # four neighbouring-pair differences v2..v5 over 4, so one more
    # direction is lost -- a property of the printed set that a dropped
    # term or a wrong index would change
    assert np.linalg.matrix_rank(T) == rank
    # additions, subtractions and shifts: coefficients 0 or +-2^-m, and one
    # magnitude per row (a difference of two equal-size groups, scaled)
    for row in T:
        nz = np.abs(row[row != 0])
        assert len(nz) in (2, 4, 8) and np.all(nz == nz[0]) and nz[0] in (0.5, 0.25, 0.125)
        assert (row > 0).sum() == (row < 0).sum()
    # every bin enters the set
    assert np.all(np.abs(T).sum(axis=0) > 0)
    # the two sets differ
    assert not np.array_equal(_matrix(tq.transform_a), _matrix(tq.transform_b))


def test_set_a_dependency():
    T = _matrix(tq.transform_a)
    np.testing.assert_array_equal(T[7], (T[2] + T[3] + T[4] + T[5]) / 4)


def test_transform_is_linear_and_cellwise():
    rng = np.random.default_rng(0)
    d = rng.uniform(0, 0.2, (5, 128)).astype(np.float32)
    v = tq.transform(d).astype(np.float64)
    for cell in range(16):
        T = _matrix(tq.transform_a if tq.cell_uses_a(cell) else tq.transform_b)
        np.testing.assert_allclose(v[:, 8 * cell:8 * cell + 8], d[:, 8 * cell:8 * cell + 8].astype(np.float64) @ T.T,
                                   atol=1e-7)


def test_checkerboard():
    a = np.array([[tq.cell_uses_a(4 * r + c) for c in range(4)] for r in range(4)])
    assert a.sum() == 8
    assert np.all(a[:, 1:] != a[:, :-1]) and np.all(a[1:, :] != a[:-1, :])


def test_quantise_thresholds():
    v = np.array([-1.0, -0.5, -0.49, 0.0, 0.3, 0.31, 2.0], dtype=np.float32)
    lo = np.full(7, -0.5, dtype=np.float32)
    hi = np.full(7, 0.3, dtype=np.float32)
    np.testing.assert_array_equal(tq.quantise(v, lo, hi), [-1, 0, 0, 0, 0, 1, 1])


@pytest.mark.parametrize("n", [128, 100, 16, 1])
def test_pack_round_trip_and_rate(n):
    rng = np.random.default_rng(n)
    q = rng.integers(-1, 2, (6, 128)).astype(np.int8)
    order = rng.permutation(128)
    w = tq.pack(q, order, n)
    assert w.shape == (6, 8) and w.dtype == np.uint32
    back = tq.unpack(w, order, n)
    coded = np.zeros(128, bool)
    coded[order[:n]] = True
    np.testing.assert_array_equal(back[:, coded], q[:, coded])
    assert not back[:, ~coded].any()
    # bits beyond 2n are zero, and no position holds the pattern 11
    bits = np.unpackbits(w.view(np.uint8), bitorder="little").reshape(6, 256)
    assert not bits[:, 2 * n:].any()
    assert not (bits[:, 0::2] & bits[:, 1::2]).any()
