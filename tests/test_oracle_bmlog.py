"""Pins of the BMLoG scale-space oracle (oracle/bmlog.py): the paper's block
count, unit DC gain, the exactness of block-circular filtering wherever the
kernel fits in the overlap (against a library spatial convolution with
clamped borders), and the octave-0 combined kernels away from the border
within their wrapped tail mass."""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import bmlog as B


def test_block_count_of_the_paper():
    # Sec. III-A: with N = 128 and R = 16 a 640x480 image gives 35 blocks
    nbx, nby = B.block_grid(640, 480)
    assert nbx * nby == 35
    assert B.block_grid(1280, 960) == (14, 10)


def test_taps_and_transfer():
    for k in range(5):
        t = B.taps(B.blur_sigma(k))
        assert len(t) == 2 * math.ceil(4 * B.blur_sigma(k)) + 1
        H = B.transfer(t)
        assert abs(H[0] - 1.0) < 1e-14                       # unit DC gain
        assert np.abs(H.imag).max() < 1e-14                   # symmetric taps: real response
        assert np.abs(H[1:] - H[1:][::-1]).max() < 1e-14      # even in frequency


def _spatial(X, t):
    """Separable correlation with clamp-to-edge borders (library)."""
    Y = ndi.correlate1d(X, t, axis=0, mode="nearest")
    return ndi.correlate1d(Y, t, axis=1, mode="nearest")


@pytest.mark.parametrize("shape", [(240, 320), (97, 130), (30, 40), (200, 96)])
def test_blocks_equal_spatial_when_the_kernel_fits(shape):
    """Radii 5..12 <= R: every kept pixel of every block equals the spatial
    filter, including at the image border (a clamped block is the clamped
    image)."""
    rng = np.random.default_rng(sum(shape))
    X = rng.uniform(0, 255, size=shape)
    ts = [B.taps(B.blur_sigma(k)) for k in range(1, 5)]
    outs = B.filter_blocks(X, [B.transfer(t) for t in ts])
    for out, t in zip(outs, ts):
        np.testing.assert_allclose(out, _spatial(X, t), rtol=0, atol=1e-9)


def test_octave0_combined_kernels_inside():
    """g0 then g_k (radius up to 19 > R): away from the image border by the
    combined radius, the block result equals the two spatial passes up to
    the mass of the combined kernel beyond R (which the circular block
    wraps), times the image's range."""
    rng = np.random.default_rng(7)
    img = rng.integers(0, 256, size=(240, 330)).astype(np.uint8)
    P = B.pyramid(img)[0]
    X = img.astype(np.float64)
    g0 = B.taps(B.blur_sigma(0))
    G00 = _spatial(X, g0)
    np.testing.assert_allclose(P[0][8:-8, 8:-8], G00[8:-8, 8:-8], rtol=0, atol=1e-9)   # radius 7 fits
    for k in range(1, 5):
        tk = B.taps(B.blur_sigma(k))
        ref = _spatial(G00, tk)
        comb = np.convolve(g0, tk)                              # combined 1-D kernel
        rc = (len(comb) - 1) // 2
        tail = comb[np.abs(np.arange(-rc, rc + 1)) > B.R].sum()
        bound = 2 * tail * 255 + 1e-9                           # wrapped mass, both axes
        m = rc + 1
        assert np.abs(P[k][m:-m, m:-m] - ref[m:-m, m:-m]).max() <= bound


def test_octaves_and_decimation():
    rng = np.random.default_rng(3)
    img = rng.integers(0, 256, size=(130, 200)).astype(np.uint8)
    P = B.pyramid(img)
    assert [p.shape[1:] for p in P] == [(130, 200), (65, 100), (33, 50), (17, 25)]
    for o in range(1, len(P)):
        np.testing.assert_array_equal(P[o][0], P[o - 1][4][::2, ::2])
