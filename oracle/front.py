"""Front-end downsampling oracle -- TEST INFRASTRUCTURE ONLY (numpy, exact
integer arithmetic).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may import this module; the GPU path shares nothing with it.

What it computes (the opening of Sec. III: the
encoder first brings every input image down to a low resolution whose
longer side is at most 640 pixels).  The paper names neither the output
size rule nor the filter; the readings taken here are:

  1. Size.  With L = max(W, H): an image with L <= 640 is left as it is;
     otherwise the longer side becomes 640 and the shorter one
     round(S * 640 / L), rounded half up, at least 1.
  2. Filter.  Area averaging: each output pixel is the mean of the input
     over the output pixel's footprint, every input pixel weighted by the
     area of its overlap with that footprint (separable: the product of
     the overlap lengths along x and along y).  In units where an input
     pixel along an axis of n inputs and m outputs is m long and an output
     pixel is n long, input i spans [i m, (i + 1) m), output j spans
     [j n, (j + 1) n), and their overlap is an integer, so the weighted sum
     N of an output pixel is an exact integer and the mean is N / (W H).
  3. Rounding.  The u8 output is the mean rounded half up,
     floor((2 N + W H) / (2 W H)), an exact integer decision.

The weighted sums are library matrix products (the overlap matrices applied
on both sides), evaluated in float64: every term and every partial sum is
an integer no larger than 255 W H < 2^53 (sides up to 8192), so float64
represents each exactly and the products are exact whatever their order of
summation -- the definition above evaluated exactly, at BLAS speed.
"""
from __future__ import annotations

import numpy as np

LONG_SIDE = 640


def front_size(width: int, height: int, long_side: int = LONG_SIDE):
    """Output (width, height) of the front end."""
    L = max(width, height)
    if L <= long_side:
        return width, height

    def scaled(s):
        return max(1, (2 * long_side * s + L) // (2 * L))     # round half up

    return scaled(width), scaled(height)


def overlap_matrix(n: int, m: int) -> np.ndarray:
    """O[j, i] = length of the overlap of input pixel i ([i m, (i+1) m)) and
    output pixel j ([j n, (j+1) n)), m outputs from n inputs (int64)."""
    j = np.arange(m, dtype=np.int64)[:, None]
    i = np.arange(n, dtype=np.int64)[None, :]
    lo = np.maximum(i * m, j * n)
    hi = np.minimum((i + 1) * m, (j + 1) * n)
    return np.maximum(hi - lo, 0)


def front(img: np.ndarray, long_side: int = LONG_SIDE) -> np.ndarray:
    """u8 H x W image -> u8 image of front_size (a copy when no resampling
    is needed)."""
    img = np.asarray(img)
    H, W = img.shape
    wo, ho = front_size(W, H, long_side)
    if (wo, ho) == (W, H):
        return img.astype(np.uint8).copy()
    oy = overlap_matrix(H, ho)               # ho x H
    ox = overlap_matrix(W, wo)               # wo x W
    assert 255 * W * H < 2 ** 53
    N = np.rint((oy.astype(np.float64) @ img.astype(np.float64)) @ ox.T.astype(np.float64)).astype(np.int64)
    d = np.int64(W) * np.int64(H)
    return ((2 * N + d) // (2 * d)).astype(np.uint8)
