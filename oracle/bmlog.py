"""BMLoG scale space oracle -- TEST INFRASTRUCTURE ONLY (numpy, float64).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may import this module; the GPU path shares nothing with it.

What it computes (Sec. III-A: the block-based mixture-domain LoG filtering
that the paper compares against before choosing spatial filters for the
GPU): the Gaussian scale images are filtered in the frequency domain,
block by block, and the Laplacian stays in the spatial domain (the detector
applies it as usual).  Each octave image is covered by N x N blocks that
overlap by R pixels on every side (the paper's N = 128, R = 16); a block is
transformed once (2-D DFT), multiplied by the transfer function of each
Gaussian, and transformed back once per scale image; only its central
(N - 2R) x (N - 2R) pixels are kept.

Readings (the paper gives the block scheme and its sizes, not the
details):
  * blocks are laid out from the octave image's origin with a stride of
    N - 2R = 96, block (bx, by) covering image columns [96 bx - 16,
    96 bx + 112) and rows likewise, pixels outside the image taken from the
    nearest edge pixel (the spatial definition's clamp-to-edge border); its
    central 96 x 96 pixels land on image columns [96 bx, 96 bx + 96);
  * the transfer function of a Gaussian is the DFT of its taps as the
    spatial definition samples, truncates and normalises them (radius
    ceil(4 s)), placed on the N-periodic grid -- real, as the taps are
    symmetric -- applied along both axes (the filters are separable);
  * octave 0 filters the u8 input itself: the base blur g0 (sigma0 = 1.6)
    gives G_{0,0}, and g0 followed by g_k gives G_{0,k} (the product of the
    two transfer functions), so one forward and five inverse transforms per
    block, as the paper counts them; octave o >= 1 filters its base
    G_{o,0} = G_{o-1,4} sampled at even pixels with g_1..g_4 (four
    inverse transforms);
  * octaves as the spatial scale space makes them (ceil-halving, the first
    octave with a short side below 32 is the last).

Where a kernel's radius is at most R, a block's central pixels see no wrap
of the circular convolution, so they equal the spatial filter; the
combined octave-0 kernels reach 7 + 12 = 19 pixels, and their taps beyond
16 wrap (a tail of relative mass below 1e-6).
"""
from __future__ import annotations

import math

import numpy as np

N = 128
R = 16
STEP = N - 2 * R
SIGMA0 = 1.6
INTERVALS = 4
MIN_SIDE = 32


def blur_sigma(k: int) -> float:
    """Direct blur of scale image k from the octave base (k >= 1), or the
    base blur (k = 0)."""
    return SIGMA0 if k == 0 else SIGMA0 * math.sqrt(2.0 ** (2.0 * k / INTERVALS) - 1.0)


def taps(s: float) -> np.ndarray:
    """Sampled Gaussian exp(-p^2 / (2 s^2)), |p| <= ceil(4 s), normalised."""
    r = math.ceil(4 * s)
    p = np.arange(-r, r + 1, dtype=np.float64)
    t = np.exp(-p * p / (2 * s * s))
    return t / t.sum()


def transfer(t: np.ndarray) -> np.ndarray:
    """DFT (length N) of taps placed on the N-periodic grid around 0."""
    r = (len(t) - 1) // 2
    h = np.zeros(N)
    for i, p in enumerate(range(-r, r + 1)):
        h[p % N] += t[i]
    return np.fft.fft(h)


def block_grid(w: int, h: int):
    """Blocks along x and y for a w x h image."""
    return -(-w // STEP), -(-h // STEP)


def filter_blocks(X: np.ndarray, transfers):
    """Frequency-domain filtering of image X (h x w) by block: one output
    image per 1-D transfer function H (applied along both axes)."""
    h, w = X.shape
    nbx, nby = block_grid(w, h)
    outs = [np.zeros((h, w)) for _ in transfers]
    for by in range(nby):
        rows = np.clip(np.arange(by * STEP - R, by * STEP - R + N), 0, h - 1)
        for bx in range(nbx):
            cols = np.clip(np.arange(bx * STEP - R, bx * STEP - R + N), 0, w - 1)
            F = np.fft.fft2(X[np.ix_(rows, cols)])
            y1, x1 = min(by * STEP + STEP, h), min(bx * STEP + STEP, w)
            for out, H in zip(outs, transfers):
                G = np.fft.ifft2(F * H[:, None] * H[None, :]).real
                out[by * STEP:y1, bx * STEP:x1] = G[R:R + y1 - by * STEP, R:R + x1 - bx * STEP]
    return outs


def octave_sizes(w: int, h: int):
    sizes = []
    while True:
        sizes.append((w, h))
        if min(w, h) < MIN_SIDE:
            return sizes
        w, h = (w + 1) // 2, (h + 1) // 2


def pyramid(img: np.ndarray):
    """u8 H x W image -> list over octaves of (5, h_o, w_o) float64 arrays
    G_{o,0..4}."""
    X = np.asarray(img, dtype=np.float64)
    H, W = X.shape
    g = [transfer(taps(blur_sigma(k))) for k in range(INTERVALS + 1)]
    out = []
    for o, (w, h) in enumerate(octave_sizes(W, H)):
        if o == 0:
            planes = filter_blocks(X, [g[0]] + [g[0] * g[k] for k in range(1, INTERVALS + 1)])
        else:
            base = out[-1][INTERVALS][::2, ::2]
            assert base.shape == (h, w)
            planes = [base] + filter_blocks(base, g[1:])
        out.append(np.stack(planes))
    return out
