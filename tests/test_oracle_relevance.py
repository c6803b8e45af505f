"""Pins for the relevance oracle (Sec. III-B, Eqs. (4)-(5)): bin lookup
against a library search, the product of table values on hand-built
tables, the centre distance's closed values, and the selection order."""
import numpy as np

from oracle import relevance

KP = np.dtype([("x", "f4"), ("y", "f4"), ("sigma", "f4"), ("p", "f4"), ("rho", "f4"), ("p_ss", "f4")])


def _kp(rows):
    a = np.zeros(len(rows), dtype=KP)
    for i, r in enumerate(rows):
        a[i] = r
    return a


def test_bins_match_searchsorted():
    rng = np.random.default_rng(0)
    edges = np.sort(rng.uniform(0, 10, (5, 15)), axis=1).astype(np.float32)
    F = rng.uniform(-1, 11, (200, 5)).astype(np.float32)
    F[:5, :] = edges[:, :5].T            # values exactly on edges fall into the upper bin
    b = relevance.bins(F, edges)
    for k in range(5):
        np.testing.assert_array_equal(b[:, k], np.searchsorted(edges[k], F[:, k], side="right"))


def test_score_is_product_of_tables():
    edges = np.tile(np.arange(1, 16, dtype=np.float32), (5, 1))
    values = np.ones((5, 16), dtype=np.float32)
    values[1] = np.arange(16, dtype=np.float32) / 16 + 0.5      # depends on |p| only
    m = {"edges": edges, "values": values}
    kp = _kp([(10, 10, 1.0, -3.5, 5.0, 0.1), (10, 10, 1.0, 7.0, 5.0, 0.1)])
    r = relevance.score(relevance.features(kp, 21, 21), m)
    np.testing.assert_array_equal(r, [values[1][3], values[1][7]])
    values[3] = 2.0                                              # scales every score
    r2 = relevance.score(relevance.features(kp, 21, 21), m)
    np.testing.assert_array_equal(r2, 2 * r)


def test_centre_distance():
    W, H = 641, 481
    kp = _kp([(320, 240, 2, 1, 1, 1), (0, 0, 2, 1, 1, 1), (640, 480, 2, 1, 1, 1), (640, 240, 2, 1, 1, 1)])
    d = relevance.features(kp, W, H)[:, 2]
    np.testing.assert_allclose(d, [0.0, 1.0, 1.0, 320 / np.hypot(320, 240)], rtol=1e-6)


def test_select_order_and_ties():
    edges = np.tile(np.arange(1, 16, dtype=np.float32), (5, 1))
    values = np.ones((5, 16), dtype=np.float32)
    values[0] = np.linspace(0.1, 0.9, 16).astype(np.float32)    # by sigma
    m = {"edges": edges, "values": values}
    kp = _kp([(5, 5, s, 1, 1, 1) for s in (2.0, 9.0, 2.0, 14.0, 9.0)])
    idx, r = relevance.select(kp, 11, 11, m, 4)
    np.testing.assert_array_equal(idx, [3, 1, 4, 0])
    idx, _ = relevance.select(kp, 11, 11, m, 10)
    assert len(idx) == 5
