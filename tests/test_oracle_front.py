"""Pins of the front-end downsampling oracle (oracle/front.py): the output
size rule, the area-average definition evaluated independently with exact
rationals over continuous pixel footprints, block means for integer
factors, mass conservation of the overlap weights, constants and ties."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import front as F


@pytest.mark.parametrize("wh,out", [
    ((1280, 960), (640, 480)), ((1920, 1080), (640, 360)), ((1000, 1000), (640, 640)),
    ((960, 1280), (480, 640)), ((641, 100), (640, 100)), ((640, 480), (640, 480)),
    ((480, 640), (480, 640)), ((17, 9), (17, 9)), ((8192, 16), (640, 1)), ((3000, 2000), (640, 427)),
])
def test_sizes(wh, out):
    assert F.front_size(*wh) == out


def _brute(img, m_w, m_h):
    """Area average from the continuous definition: input pixel (y, x) is the
    unit square [x, x+1) x [y, y+1); output pixel (l, j) covers
    [j W/m_w, (j+1) W/m_w) x [l H/m_h, (l+1) H/m_h); mean over the footprint
    with exact rationals, rounded half up."""
    H, W = img.shape
    sx, sy = Fraction(W, m_w), Fraction(H, m_h)
    out = np.zeros((m_h, m_w), dtype=np.uint8)

    def ov(a0, a1, b0, b1):
        return max(Fraction(0), min(a1, b1) - max(a0, b0))

    for l in range(m_h):
        for j in range(m_w):
            acc = Fraction(0)
            for y in range(H):
                oy = ov(Fraction(y), Fraction(y + 1), l * sy, (l + 1) * sy)
                if oy == 0:
                    continue
                for x in range(W):
                    ox = ov(Fraction(x), Fraction(x + 1), j * sx, (j + 1) * sx)
                    acc += ox * oy * int(img[y, x])
            mean = acc / (sx * sy)
            out[l, j] = int(mean + Fraction(1, 2))            # floor(mean + 1/2)
    return out


@pytest.mark.parametrize("shape,long_side", [((7, 5), 3), ((5, 9), 4), ((6, 6), 4), ((11, 4), 5), ((3, 13), 6)])
def test_matches_continuous_area_average(shape, long_side):
    rng = np.random.default_rng(sum(shape) * 7 + long_side)
    img = rng.integers(0, 256, size=shape).astype(np.uint8)
    wo, ho = F.front_size(shape[1], shape[0], long_side)
    assert max(wo, ho) == long_side
    np.testing.assert_array_equal(F.front(img, long_side), _brute(img, wo, ho))


def test_integer_factor_is_block_mean():
    rng = np.random.default_rng(5)
    img = rng.integers(0, 256, size=(960, 1280)).astype(np.int64)
    s = img.reshape(480, 2, 640, 2).sum(axis=(1, 3))
    np.testing.assert_array_equal(F.front(img.astype(np.uint8)), ((2 * s + 4) // 8).astype(np.uint8))


@pytest.mark.parametrize("n,m", [(1280, 640), (1000, 640), (641, 640), (8192, 640), (7, 3), (640, 640)])
def test_overlap_weights_conserve_mass(n, m):
    O = F.overlap_matrix(n, m)
    assert (O >= 0).all()
    np.testing.assert_array_equal(O.sum(axis=1), np.full(m, n))     # every output pixel is n long
    np.testing.assert_array_equal(O.sum(axis=0), np.full(n, m))     # every input pixel is fully shared out


def test_constant_and_ties():
    np.testing.assert_array_equal(F.front(np.full((750, 1000), 77, np.uint8)), np.full((480, 640), 77, np.uint8))
    # a mean exactly halfway between two values rounds up: (1 + 2) / 2 -> 2
    assert F.front(np.array([[1, 2]], np.uint8), long_side=1)[0, 0] == 2
    assert F.front(np.array([[2, 3, 3, 3]], np.uint8), long_side=2)[0, 0] == 3     # 2.5 -> 3
    assert F.front(np.array([[2, 2, 2, 3]], np.uint8), long_side=1)[0, 0] == 2     # 2.25 -> 2


def test_small_images_are_copied():
    rng = np.random.default_rng(1)
    img = rng.integers(0, 256, size=(480, 640)).astype(np.uint8)
    out = F.front(img)
    np.testing.assert_array_equal(out, img)
    assert out is not img
