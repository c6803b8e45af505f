"""Transform coding and ternary quantisation of local descriptors -- oracle,
TEST INFRASTRUCTURE ONLY (numpy).

Sec. III-C: each 8-bin cell histogram h = (h_0 .. h_7) of a descriptor goes
through an order-8 linear transform built from additions, subtractions and
power-of-two scalings; two transform sets are used, on neighbouring cells
alternately; each transformed element is quantised to -1, 0 or +1 with two
thresholds of its own, learned offline from that element's distribution.

Readings (the printed equations of both sets write every left-hand side as
v_0, and the paper does not say which cells take which set):
  * line k of a set defines v_k;
  * cell (row, col) of the 4 x 4 grid takes set A when row + col is even and
    set B when it is odd (a checkerboard: every pair of edge-neighbouring
    cells uses different sets);
  * element e = 8 * cell + k of the transformed descriptor is v_k of cell
    `cell`, the cells in the descriptor's own order (row * 4 + col);
  * q_e = +1 if v_e > hi_e, -1 if v_e < lo_e, else 0 (lo_e <= hi_e);
  * the code keeps the first n elements of a priority order (so the rate
    is 2n bits), element order[p] at position p, two bits per position
    (01 = +1, 10 = -1, 00 = 0), position p in word p // 16 at bits
    2 (p % 16) and up.
The transform is evaluated in float32, each expression left to right as
printed (parentheses first); the scalings by 1/2, 1/4, 1/8 are exact.  The
quantisation decisions are therefore taken in single precision, the
precision of the descriptors.
"""
from __future__ import annotations

import numpy as np

f32 = np.float32


def transform_a(h):
    """Set A on the last axis (8 bins) -> 8 values, float32."""
    h = np.asarray(h, dtype=f32)
    h0, h1, h2, h3, h4, h5, h6, h7 = (h[..., i] for i in range(8))
    v = [(h2 - h6) / f32(2), (h3 - h7) / f32(2), (h0 - h1) / f32(2), (h2 - h3) / f32(2),
         (h4 - h5) / f32(2), (h6 - h7) / f32(2), ((h0 + h4) - (h2 + h6)) / f32(4),
         ((h0 + h2 + h4 + h6) - (h1 + h3 + h5 + h7)) / f32(8)]
    return np.stack(v, axis=-1).astype(f32)


def transform_b(h):
    """Set B on the last axis (8 bins) -> 8 values, float32."""
    h = np.asarray(h, dtype=f32)
    h0, h1, h2, h3, h4, h5, h6, h7 = (h[..., i] for i in range(8))
    v = [(h0 - h4) / f32(2), (h1 - h5) / f32(2), (h7 - h0) / f32(2), (h1 - h2) / f32(2),
         (h3 - h4) / f32(2), (h5 - h6) / f32(2), ((h1 + h5) - (h3 + h7)) / f32(4),
         ((h0 + h1 + h2 + h3) - (h4 + h5 + h6 + h7)) / f32(8)]
    return np.stack(v, axis=-1).astype(f32)


def cell_uses_a(cell: int) -> bool:
    r, c = divmod(cell, 4)
    return (r + c) % 2 == 0


def transform(desc):
    """(..., 128) descriptors -> (..., 128) transformed elements, float32."""
    d = np.asarray(desc, dtype=f32).reshape(*np.shape(desc)[:-1], 16, 8)
    out = np.empty_like(d)
    for cell in range(16):
        out[..., cell, :] = (transform_a if cell_uses_a(cell) else transform_b)(d[..., cell, :])
    return out.reshape(*np.shape(desc)[:-1], 128)


def quantise(v, lo, hi):
    """Ternary symbols in {-1, 0, +1} (int8), thresholds per element."""
    v = np.asarray(v, dtype=f32)
    lo = np.asarray(lo, dtype=f32)
    hi = np.asarray(hi, dtype=f32)
    return np.where(v > hi, 1, np.where(v < lo, -1, 0)).astype(np.int8)


def pack(q, order, n):
    """Codes of the first n positions of the priority order -> 8 uint32 per
    descriptor (unused bits zero)."""
    q = np.asarray(q)
    words = np.zeros(q.shape[:-1] + (8,), dtype=np.uint32)
    for p in range(n):
        sym = q[..., order[p]]
        bits = np.where(sym > 0, 1, np.where(sym < 0, 2, 0)).astype(np.uint32)
        words[..., p // 16] |= bits << np.uint32(2 * (p % 16))
    return words


def unpack(words, order, n):
    """Inverse of pack: symbols by element (elements not coded are 0)."""
    words = np.asarray(words, dtype=np.uint32)
    q = np.zeros(words.shape[:-1] + (128,), dtype=np.int8)
    for p in range(n):
        bits = (words[..., p // 16] >> np.uint32(2 * (p % 16))) & np.uint32(3)
        q[..., order[p]] = np.where(bits == 1, 1, np.where(bits == 2, -1, 0))
    return q


def encode(desc, model, n=128):
    """Whole coding of descriptors (..., 128) with a model dict (lo, hi,
    order) -> (..., 8) uint32."""
    return pack(quantise(transform(desc), model["lo"], model["hi"]), model["order"], n)
