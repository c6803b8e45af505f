"""Pins for the oracle's ALP detector (Eqs. (2)-(3); Algorithm 1 stages A-C)."""
import numpy as np
import pytest

import oracle


def _vandermonde(O):
    s = np.array([O.scale_sigma(k) for k in range(5)])
    return np.vander(s, 4, increasing=True), s


def test_beta_is_left_inverse_and_pinv(O64):
    V, _ = _vandermonde(O64)
    beta = O64.alp_beta()                      # beta[k, i]
    np.testing.assert_allclose(beta.T @ V, np.eye(4), atol=1e-9)
    np.testing.assert_allclose(beta.T, np.linalg.pinv(V), atol=1e-9)


@pytest.mark.parametrize("seed", range(5))
def test_fit_recovers_exact_cubic(O64, O32, seed):
    rng = np.random.default_rng(seed)
    c = rng.uniform(-20, 20, size=4)
    _, s = _vandermonde(O64)
    L = c[0] + c[1] * s + c[2] * s ** 2 + c[3] * s ** 3
    np.testing.assert_allclose(O64.alp_fit(L), c, atol=1e-9 * 20 * 50)
    np.testing.assert_allclose(O32.alp_fit(L), c, rtol=0, atol=2e-3 * np.abs(c).max())


def test_fit_is_least_squares(O64):
    rng = np.random.default_rng(7)
    V, _ = _vandermonde(O64)
    for _ in range(20):
        L = rng.normal(0, 10, size=5)
        ref, *_ = np.linalg.lstsq(V, L, rcond=None)
        np.testing.assert_allclose(O64.alp_fit(L), ref, atol=1e-9)


def _dense_argmax(alpha, lo, hi, n=20001):
    """Brute force: interior local maxima of |p| on a dense grid in [lo, hi)."""
    s = np.linspace(lo, hi, n, endpoint=False)
    p = alpha[0] + alpha[1] * s + alpha[2] * s ** 2 + alpha[3] * s ** 3
    a = np.abs(p)
    inner = (a[1:-1] > a[:-2]) & (a[1:-1] >= a[2:])
    idx = np.nonzero(inner)[0] + 1
    if len(idx) == 0:
        return None
    j = idx[np.argmax(a[idx])]
    return s[j], p[j]


def test_extremum_matches_dense_search(O64):
    rng = np.random.default_rng(1)
    lo, hi = O64.scale_sigma(0), O64.scale_sigma(4)
    found = 0
    for _ in range(3000):
        # random cubics with a stationary point somewhere near the octave
        r1, r2 = rng.uniform(0.5, 4.5, size=2)
        a3 = rng.uniform(-3, 3)
        # p'(s) = 3 a3 (s - r1)(s - r2)  ->  a2, a1 from the roots
        alpha = np.array([rng.uniform(-20, 20), 3 * a3 * r1 * r2, -1.5 * a3 * (r1 + r2), a3])
        ok, s, p, pss = O64.alp_extremum(alpha)
        ref = _dense_argmax(alpha, lo, hi)
        # a grid maximum on the boundary sample is not an interior extremum
        if ref is not None and (ref[0] - lo < 1e-3 or hi - ref[0] < 1e-3):
            continue
        assert ok == (ref is not None), (alpha, ok, ref)
        if ok:
            found += 1
            assert abs(s - ref[0]) < 2e-4
            assert abs(p - ref[1]) < 1e-6 * max(1, abs(p)) + 1e-6
            dp = alpha[1] + 2 * alpha[2] * s + 3 * alpha[3] * s * s
            assert abs(dp) < 1e-9 * (1 + np.abs(alpha).max())
            assert p * pss < 0
    assert found > 500


def test_extremum_degenerate_cases(O64):
    # quadratic p (a3 = 0): the single stationary point of a concave parabola
    ok, s, p, _ = O64.alp_extremum(np.array([0.0, 8.0, -2.0, 0.0]))   # p = 8s - 2s^2, max at 2
    assert ok and abs(s - 2.0) < 1e-12 and abs(p - 8.0) < 1e-12
    # monotone p in the octave: no extremum
    ok, *_ = O64.alp_extremum(np.array([1.0, 1.0, 0.0, 0.0]))
    assert not ok
    # |p| minimum, not maximum (p > 0 and p'' > 0): rejected
    ok, *_ = O64.alp_extremum(np.array([10.0, -8.0, 2.0, 0.0]))      # min of 2s^2-8s+10 at 2
    assert not ok
    # negative response with a minimum of p is a maximum of |p|: kept
    ok, s, p, _ = O64.alp_extremum(np.array([-10.0, 8.0, -2.0, 0.0]) * -1)
    assert not ok  # p = 2s^2 - 8s + 10 > 0 at its minimum -> |p| minimum
    ok, s, p, _ = O64.alp_extremum(np.array([-2.0, 8.0, -2.0, 0.0]) * -1)  # p = 2 - 8s + 2s^2
    assert ok and abs(s - 2.0) < 1e-12 and abs(p - (2 - 16 + 8)) < 1e-12
    # no real stationary point
    ok, *_ = O64.alp_extremum(np.array([0.0, 5.0, 0.0, 1.0]))        # p' = 3s^2 + 5 > 0
    assert not ok


def _quad_surface(ox, oy, a, b, c, peak):
    """v(i,j) = peak - a (i-ox)^2 - b (j-oy)^2 - c (i-ox)(j-oy) on the 3x3 grid."""
    v = np.empty((3, 3))
    for j in range(-1, 2):
        for i in range(-1, 2):
            dx, dy = i - ox, j - oy
            v[j + 1, i + 1] = peak - a * dx * dx - b * dy * dy - c * dx * dy
    return v


def test_refine_recovers_quadratic_offset(O64):
    for (ox, oy, a, b, c) in [(0.2, -0.3, 1.0, 1.3, 0.2), (-0.45, 0.1, 2.0, 1.5, -0.4),
                              (0.0, 0.0, 1.0, 1.0, 0.0)]:
        v = _quad_surface(ox, oy, a, b, c, 50.0)
        ok, rx, ry, pr, rho = O64.refine3x3(v)
        assert ok
        assert abs(rx - ox) < 1e-12 and abs(ry - oy) < 1e-12
        assert abs(pr - 50.0) < 1e-10          # the vertex value of the quadratic
        hxx, hyy, hxy = -2 * a, -2 * b, -c
        assert abs(rho - (hxx + hyy) ** 2 / (hxx * hyy - hxy * hxy)) < 1e-10


def test_refine_rejections(O64):
    # ridge: curvature ratio 30 -> tr^2/det = 31^2/30 > 12.1
    ok, *_ = O64.refine3x3(_quad_surface(0.1, 0.1, 30.0, 1.0, 0.0, 40.0))
    assert not ok
    # curvature ratio 8 -> 81/8 = 10.1 < 12.1: kept
    ok, *_ = O64.refine3x3(_quad_surface(0.1, 0.1, 8.0, 1.0, 0.0, 40.0))
    assert ok
    # offset beyond half a pixel
    ok, *_ = O64.refine3x3(_quad_surface(0.7, 0.0, 1.0, 1.0, 0.0, 40.0))
    assert not ok
    # saddle: det < 0
    ok, *_ = O64.refine3x3(_quad_surface(0.1, 0.1, 1.0, -1.0, 0.0, 40.0))
    assert not ok


def _alp_fields_numpy(planes, O):
    """Independent numpy ALP: own Laplacian (edge padding) and lstsq fit."""
    K, h, w = planes.shape
    s = np.array([O.scale_sigma(k) for k in range(K)])
    L = np.empty_like(planes)
    for k in range(K):
        g = np.pad(planes[k], 1, mode="edge")
        L[k] = s[k] ** 2 * (g[:-2, 1:-1] + g[2:, 1:-1] + g[1:-1, :-2] + g[1:-1, 2:] - 4 * g[1:-1, 1:-1])
    V = np.vander(s, 4, increasing=True)
    coef, *_ = np.linalg.lstsq(V, L.reshape(K, -1), rcond=None)
    return coef.reshape(4, h, w)


def test_detect_equals_bruteforce_nms(O64):
    """Stage A on random planes vs a brute-force 3x3 scan (refinement gates off)."""
    P = oracle.Oracle.default_params()
    P.contrast = 0.5
    P.edge_r = 1e30
    P.max_offset = 1e30
    O = oracle.Oracle("f64", P)
    rng = np.random.default_rng(5)
    h, w = 24, 28
    planes = np.cumsum(rng.normal(0, 1, size=(5, h, w)), axis=0) * 3.0
    flat = np.ascontiguousarray(planes.reshape(-1))
    cands = O.detect(flat, w, h)
    alpha = _alp_fields_numpy(planes, O)
    lo, hi = O.scale_sigma(0), O.scale_sigma(4)
    expect = set()
    for y in range(4, h - 4):
        for x in range(4, w - 4):
            a = alpha[:, y, x]
            # stationary points of the cubic by np.roots, keep |p| maxima in [lo, hi)
            best = None
            for r in np.roots([3 * a[3], 2 * a[2], a[1]]):
                if abs(r.imag) > 1e-9 or not (lo <= r.real < hi):
                    continue
                sr = r.real
                p = np.polyval(a[::-1], sr)
                if p * (6 * a[3] * sr + 2 * a[2]) >= 0:
                    continue
                if best is None or abs(p) > abs(best[1]):
                    best = (sr, p)
            if best is None or abs(best[1]) < P.contrast:
                continue
            sr, p = best
            nb = [np.polyval(alpha[:, y + j, x + i][::-1], sr)
                  for j in (-1, 0, 1) for i in (-1, 0, 1) if (i, j) != (0, 0)]
            if (p > 0 and all(q < p for q in nb)) or (p < 0 and all(q > p for q in nb)):
                expect.add((x, y))
    got = {(int(c["ix"]), int(c["iy"])) for c in cands}
    assert len(expect) > 5
    assert got == expect


def _kp(octave, x, y, sigma, p, ix=0, iy=0):
    k = np.zeros(1, dtype=oracle.KP_DTYPE)
    k["octave"], k["x"], k["y"], k["sigma"], k["p"] = octave, x, y, sigma, p
    k["ix"], k["iy"] = ix, iy
    return k


def test_dedup_hand_built(O64):
    cases = [
        # (a, b, alive_a, alive_b)
        (_kp(0, 100.0, 100.0, 3.0, 20.0), _kp(1, 100.8, 100.5, 3.3, 25.0), 0, 1),   # close: weaker a loses
        (_kp(0, 100.0, 100.0, 3.0, 30.0), _kp(1, 100.8, 100.5, 3.3, 25.0), 1, 0),   # b weaker
        (_kp(0, 100.0, 100.0, 3.0, 20.0), _kp(1, 100.8, 100.5, 3.3, -25.0), 1, 1),  # opposite sign
        (_kp(0, 100.0, 100.0, 3.0, 20.0), _kp(1, 103.0, 100.0, 3.3, 25.0), 1, 1),   # 3 px > 2 px
        (_kp(0, 100.0, 100.0, 2.5, 20.0), _kp(1, 100.5, 100.0, 3.3, 25.0), 1, 1),   # ratio 1.32 > 2^0.25
        (_kp(0, 100.0, 100.0, 3.0, 25.0), _kp(1, 100.5, 100.0, 3.3, 25.0), 1, 0),   # tie: finer wins
        (_kp(0, 100.0, 100.0, 3.0, 20.0), _kp(2, 100.5, 100.0, 3.3, 25.0), 1, 1),   # not adjacent
        (_kp(2, 400.0, 400.0, 12.0, -9.0), _kp(3, 405.0, 403.0, 13.0, -8.0), 1, 0), # 5.8 px <= 8 px
    ]
    for a, b, ea, eb in cases:
        alive = O64.dedup(np.concatenate([a, b]))
        assert list(alive) == [ea, eb], (a, b, alive)


def test_dedup_order_independent(O64):
    rng = np.random.default_rng(9)
    n = 300
    c = np.zeros(n, dtype=oracle.KP_DTYPE)
    c["octave"] = rng.integers(0, 4, n)
    c["x"] = rng.uniform(0, 30, n)
    c["y"] = rng.uniform(0, 30, n)
    c["sigma"] = rng.uniform(1.6, 3.2, n) * 2.0 ** c["octave"]
    c["p"] = rng.uniform(-30, 30, n)
    alive = O64.dedup(c)
    perm = rng.permutation(n)
    alive2 = O64.dedup(c[perm])
    np.testing.assert_array_equal(alive[perm], alive2)
    assert 0 < alive.sum() < n


def test_select_matches_lexsort(O64):
    rng = np.random.default_rng(4)
    n = 500
    c = np.zeros(n, dtype=oracle.KP_DTYPE)
    c["octave"] = rng.integers(0, 5, n)
    c["ix"] = rng.integers(0, 100, n)
    c["iy"] = rng.integers(0, 100, n)
    c["p"] = np.round(rng.uniform(-5, 5, n), 1)          # many |p| ties
    alive = (rng.uniform(size=n) < 0.8).astype(np.int32)
    out = O64.select(c, alive, topk=120)
    keep = c[alive == 1]
    order = np.lexsort((keep["ix"], keep["iy"], keep["octave"], -np.abs(keep["p"])))
    ref = keep[order][:120]
    np.testing.assert_array_equal(out, ref)
