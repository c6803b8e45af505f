"""Keypoint relevance and selection -- oracle, TEST INFRASTRUCTURE ONLY (numpy).

Sec. III-B, Eqs. (4)-(5): the relevance of a keypoint is the product of
five conditional probabilities of correct matching, each a function of one
characteristic of the keypoint -- its scale sigma, its response p, its
distance d to the image centre, the Hessian ratio rho and the second
derivative p_ss of the response in scale -- read from tables over quantised
values of that characteristic:
    r = f1(sigma) f2(p) f3(d) f4(rho) f5(p_ss),
and the keypoints with the highest r are kept.  The standard's tables are
normative and not available here; the model is a stand-in of the same form
(per characteristic, 15 increasing bin edges and 16 table values).

Readings: sigma in base-image pixels; p taken as |p| (the response's sign
only tells a bright blob from a dark one); d = distance from the image
centre ((W-1)/2, (H-1)/2) over the centre's distance to a corner, in
[0, 1]; rho and p_ss as the detector writes them.  Bin b of a value v is
the number of edges e with e <= v.  Everything in single precision, the
products left to right, the distance without fused operations; ties in r
keep the input order.
"""
from __future__ import annotations

import numpy as np

f32 = np.float32
N_FEATURES = 5
N_BINS = 16


def features(kp, W, H):
    """(n, 5) float32 characteristics of keypoint records (fields x, y,
    sigma, p, rho and p_ss or pss)."""
    x, y = np.asarray(kp["x"], f32), np.asarray(kp["y"], f32)
    hx, hy = f32(0.5) * f32(W - 1), f32(0.5) * f32(H - 1)
    dx, dy = x - hx, y - hy
    d = np.sqrt(dx * dx + dy * dy) / np.sqrt(hx * hx + hy * hy)
    pss = kp["p_ss"] if "p_ss" in kp.dtype.names else kp["pss"]
    return np.stack([np.asarray(kp["sigma"], f32), np.abs(np.asarray(kp["p"], f32)), d.astype(f32),
                     np.asarray(kp["rho"], f32), np.asarray(pss, f32)], axis=1)


def bins(F, edges):
    """Bin index of every characteristic: the count of edges <= value."""
    F = np.asarray(F, f32)
    edges = np.asarray(edges, f32)
    return np.stack([(edges[k][None, :] <= F[:, k:k + 1]).sum(axis=1) for k in range(N_FEATURES)], axis=1)


def score(F, model):
    """r = f1 f2 f3 f4 f5, left to right in single precision."""
    b = bins(F, model["edges"])
    vals = np.asarray(model["values"], f32)
    r = vals[0][b[:, 0]]
    for k in range(1, N_FEATURES):
        r = (r * vals[k][b[:, k]]).astype(f32)
    return r.astype(f32)


def select(kp, W, H, model, n_keep):
    """Indices (into kp) of the n_keep keypoints of highest r, in that
    order; equal r keep the input order."""
    r = score(features(kp, W, H), model)
    order = np.lexsort((np.arange(len(r)), -r.astype(np.float64)))
    return order[:n_keep], r
