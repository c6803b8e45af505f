"""Pins for the oracle's orientation and descriptor stages (Algorithm 2)."""
import math

import numpy as np
import pytest

import oracle


def _ramp(N, phi, a=2.0, c=120.0):
    y, x = np.mgrid[0:N, 0:N].astype(np.float64)
    return c + a * (x * math.cos(phi) + y * math.sin(phi))


def _disk_mass(cx, cy, s, N, radius, wsig, g):
    """Sum over integer pixels strictly inside the disk (and 1..N-2) of
    g * exp(-d^2 / (2 (wsig s)^2)) -- brute force over the whole grid."""
    y, x = np.mgrid[0:N, 0:N].astype(np.float64)
    d2 = (x - cx) ** 2 + (y - cy) ** 2
    m = (d2 < (radius * s) ** 2) & (x >= 1) & (x <= N - 2) & (y >= 1) & (y <= N - 2)
    return float((g * np.exp(-d2 / (2 * (wsig * s) ** 2)))[m].sum())


@pytest.mark.parametrize("phi", [0.3, 1.0, 2.2, 3.9, 5.5])
def test_orientation_histogram_of_a_ramp(O64, phi):
    """A linear ramp has one gradient direction everywhere: the histogram holds
    the whole Gaussian-weighted magnitude in the two bins around phi, split
    linearly (bin b centred on b * 10 degrees)."""
    N, a = 64, 2.0
    G = _ramp(N, phi, a)
    cx, cy, s = 31.3, 30.6, 2.5
    h = O64.orient_hist(G, cx, cy, s)
    mass = _disk_mass(cx, cy, s, N, 3.96, 1.5, 2 * a)   # |grad| = 2a (central difference)
    fb = phi * 36 / (2 * math.pi)
    b0 = int(math.floor(fb)) % 36
    fr = fb - math.floor(fb)
    exp = np.zeros(36)
    exp[b0] = mass * (1 - fr)
    exp[(b0 + 1) % 36] = mass * fr
    np.testing.assert_allclose(h, exp, atol=1e-9 * mass)


@pytest.mark.parametrize("phi", [0.3, 1.0, 2.2, 3.9, 5.5])
def test_orientation_of_a_ramp(O64, phi):
    """Parabolic refinement of a two-bin split is biased by at most 0.17 bin
    (fr/(2-3fr) vs fr for fr in [0, 0.5]), i.e. < 2 degrees."""
    G = _ramp(64, phi)
    h = O64.orient_hist(G, 31.3, 30.6, 2.5)
    th, pk = O64.orient_peaks(h)
    assert len(th) == 1
    err = (th[0] - phi + math.pi) % (2 * math.pi) - math.pi
    assert abs(err) < math.radians(2.0)


def test_orientation_peaks_parabola_and_threshold(O64):
    # bins sampled from a parabola with vertex 7.3: refinement is exact
    b = np.arange(36, dtype=np.float64)
    h = np.maximum(0.0, 10.0 - (b - 7.3) ** 2)
    th, pk = O64.orient_peaks(h)
    assert len(th) == 1 and abs(th[0] - 7.3 * 2 * math.pi / 36) < 1e-12 and pk[0] == h[7]
    # second peak above / below 0.8 of the highest
    for second, n in ((8.1, 2), (7.9, 1), (8.0, 1)):
        h = np.zeros(36)
        h[5], h[20] = 10.0, second
        th, pk = O64.orient_peaks(h)
        assert len(th) == n
        assert pk[0] == 10.0
    # plateau: equal neighbouring bins are not strict maxima
    h = np.zeros(36)
    h[3] = h[4] = 5.0
    assert len(O64.orient_peaks(h)[0]) == 0
    # at most four, highest first; circular neighbourhood (bin 0 vs 35)
    h = np.zeros(36)
    for i, v in zip([0, 6, 12, 18, 24, 30], [9.0, 9.5, 8.5, 10.0, 8.8, 9.9]):
        h[i] = v
    th, pk = O64.orient_peaks(h)
    np.testing.assert_array_equal(pk, [10.0, 9.9, 9.5, 9.0])
    # flat histogram: no orientation
    assert len(O64.orient_peaks(np.zeros(36))[0]) == 0


@pytest.mark.parametrize("phi,theta", [(0.4, 0.0), (2.0, 1.1), (4.5, 5.9)])
def test_descriptor_orientation_split_of_a_ramp(O64, phi, theta):
    """One gradient direction: every cell's mass sits in the two orientation
    bins around (phi - theta), in the ratio (1 - a) : a before normalisation.
    Clamping is lifted so the ratio survives normalisation."""
    P = oracle.Oracle.default_params()
    P.desc_clamp = 1.0
    O = oracle.Oracle("f64", P)
    G = _ramp(96, phi)
    d = O.descriptor(G, 47.2, 48.7, 2.5, theta).reshape(16, 8)
    rel = (phi - theta) % (2 * math.pi)
    fo = rel * 8 / (2 * math.pi)
    o0 = int(math.floor(fo)) % 8
    ao = fo - math.floor(fo)
    other = [b for b in range(8) if b not in (o0, (o0 + 1) % 8)]
    assert np.all(d[:, other] == 0)
    cells = d.sum(axis=1) > 0
    assert cells.sum() == 16
    np.testing.assert_allclose(d[cells, o0] * ao, d[cells, (o0 + 1) % 8] * (1 - ao), atol=1e-12)
    assert abs(np.linalg.norm(d) - 1) < 1e-12


def test_descriptor_row_column_layout(O64):
    """Index = (row*4 + col)*8 + bin, row from the (rotated) y offset.  With
    theta = 0 and the support clipped on the left by the image edge, the
    column-0 cells are lighter than column-3 cells while rows stay symmetric."""
    P = oracle.Oracle.default_params()
    P.desc_clamp = 1.0
    O = oracle.Oracle("f64", P)
    N = 96
    G = _ramp(N, 0.7)
    cx, cy, s = 9.0, 48.0, 2.5      # support radius 15 px crosses x = 1
    d = O.descriptor(G, cx, cy, s, 0.0).reshape(4, 4, 8).sum(axis=2)
    assert d[:, 0].sum() < 0.5 * d[:, 3].sum()
    np.testing.assert_allclose(d[0, :], d[3, :], rtol=1e-12)
    np.testing.assert_allclose(d[1, :], d[2, :], rtol=1e-12)


def test_descriptor_unit_norm_and_clamp(O64, O32):
    rng = np.random.default_rng(2)
    G = rng.uniform(0, 255, size=(80, 80))
    for O, tol in ((O64, 1e-12), (O32, 1e-6)):
        for _ in range(10):
            cx, cy = rng.uniform(20, 60, size=2)
            s = rng.uniform(1.6, 3.2)
            d = O.descriptor(G.astype(O.dtype), cx, cy, s, rng.uniform(0, 2 * math.pi))
            assert abs(np.linalg.norm(d) - 1) < tol
            assert d.min() >= 0
    # flat patch: all-zero descriptor
    d = O64.descriptor(np.full((40, 40), 50.0), 20.0, 20.0, 2.0, 0.3)
    assert np.all(d == 0)


def test_scale_index(O64):
    # nearest scale image: k* = round(4 log2(s / 1.6))
    for s, k in [(1.6, 0), (1.7, 0), (1.8, 1), (2.0, 1), (2.1, 2), (2.5, 3), (2.9, 3), (3.0, 4), (3.19, 4)]:
        assert O64.scale_index(s) == k, s


def _cell_masses(N, cx, cy, s, theta, mag, radius=6.0, cell=3.0, wsig=6.0, strict=True):
    """Spatial mass of each of the 16 descriptor cells, straight from the
    definition (Sec. IV-B, Algorithm 2 stage B, weighting after Lowe 2004):
    every integer pixel (1..N-2 on both axes) strictly inside radius*sigma
    adds mag * exp(-d^2 / (2 (wsig sigma)^2)), split bilinearly between the two
    nearest cells per axis of its offset rotated by -theta and measured in
    cells of cell*sigma, cell centres at -1.5 .. 1.5."""
    m = np.zeros((4, 4))
    R = radius * s
    for v in range(1, N - 1):
        for u in range(1, N - 1):
            dx, dy = u - cx, v - cy
            d2 = dx * dx + dy * dy
            if not (d2 < R * R if strict else d2 <= R * R):
                continue
            wt = mag * math.exp(-d2 / (2 * (wsig * s) ** 2))
            rx = (math.cos(theta) * dx + math.sin(theta) * dy) / (cell * s)
            ry = (math.cos(theta) * dy - math.sin(theta) * dx) / (cell * s)
            for r in range(4):
                wy = max(0.0, 1 - abs(ry - (r - 1.5)))
                for c in range(4):
                    m[r, c] += wt * wy * max(0.0, 1 - abs(rx - (c - 1.5)))
    return m


@pytest.mark.parametrize("theta,phi,cx,cy,s", [(0.0, 0.3, 47.2, 48.7, 2.5), (math.pi / 3, 2.0, 46.6, 47.9, 2.2),
                                               (0.0, 1.1, 48.0, 48.0, 2.5)])
def test_descriptor_spatial_weighting(O64, theta, phi, cx, cy, s):
    """Pins the descriptor's spatial weighting: each cell's share of the
    descriptor (summed over its 8 bins) equals the brute-force cell mass of a
    constant-gradient ramp computed from the definition -- Gaussian of 6
    sigma, cells of 3 sigma, integer pixels strictly inside 6 sigma.  Clamping
    is lifted, so the normalised descriptor is proportional to the raw
    histogram.  A weighting sigma of 3 sigma, cells of 4 sigma, or a closed
    disk (<= 6 sigma, which adds the pixels exactly on the circle of the
    integer-centred cases) give cell masses that the oracle does not match."""
    P = oracle.Oracle.default_params()
    P.desc_clamp = 1.0
    O = oracle.Oracle("f64", P)
    N, a = 96, 2.0
    G = _ramp(N, phi, a)
    d = O.descriptor(G, cx, cy, s, theta).reshape(4, 4, 8).sum(axis=2)
    got = d / d.sum()

    def share(**kw):
        m = _cell_masses(N, cx, cy, s, theta, 2 * a, **kw)
        return m / m.sum()

    np.testing.assert_allclose(got, share(), rtol=0, atol=1e-9)
    for mutant in (dict(wsig=3.0), dict(cell=4.0)):
        assert np.abs(got - share(**mutant)).max() > 1e-3, mutant
    if cx == int(cx) and cy == int(cy) and 6 * s == int(6 * s):
        # pixels exactly 6 sigma away (e.g. (cx + 15, cy), (cx + 9, cy + 12))
        assert np.abs(got - share(strict=False)).max() > 1e-3
