"""Keypoint / descriptor matching used by the GPU-vs-oracle parity tests.

A GPU record matches an oracle record of the same image and octave when
their base-image positions are within `tol_px` (default 0.5 px); pairs are
formed greedily by increasing distance, one to one.  Oriented records of one
keypoint share a position, so oriented matching adds the angular distance
(radians) as a tie-breaker and requires |d theta| <= tol_theta."""
from __future__ import annotations

import numpy as np


def _ang(a, b):
    d = np.abs(a - b) % (2 * np.pi)
    return np.minimum(d, 2 * np.pi - d)


def match(ref, got, tol_px=0.5, oriented=False, tol_theta=1e-2):
    """Returns list of (i_ref, j_got) pairs."""
    pairs = []
    if len(ref) == 0 or len(got) == 0:
        return pairs
    for o in np.union1d(np.unique(ref["octave"]), np.unique(got["octave"])):
        ia = np.nonzero(ref["octave"] == o)[0]
        jb = np.nonzero(got["octave"] == o)[0]
        if len(ia) == 0 or len(jb) == 0:
            continue
        ax, ay = ref["x"][ia].astype(np.float64), ref["y"][ia].astype(np.float64)
        bx, by = got["x"][jb].astype(np.float64), got["y"][jb].astype(np.float64)
        d = np.hypot(ax[:, None] - bx[None, :], ay[:, None] - by[None, :])
        ok = d <= tol_px
        cost = d.copy()
        if oriented:
            dt = _ang(ref["theta"][ia].astype(np.float64)[:, None], got["theta"][jb].astype(np.float64)[None, :])
            ok &= dt <= tol_theta
            cost = cost + dt
        ii, jj = np.nonzero(ok)
        order = np.argsort(cost[ii, jj], kind="stable")
        used_a, used_b = set(), set()
        for t in order:
            a, b = ii[t], jj[t]
            if a in used_a or b in used_b:
                continue
            used_a.add(a)
            used_b.add(b)
            pairs.append((int(ia[a]), int(jb[b])))
    return pairs


def rates(ref, got, **kw):
    pairs = match(ref, got, **kw)
    n = len(pairs)
    return (n / len(ref) if len(ref) else 1.0), (n / len(got) if len(got) else 1.0), pairs
