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


# -- whole-image checks against the oracle ----------------------------------
#
# End to end, a matched descriptor can differ from the oracle's by more than
# 1e-3 only because the two keypoints differ slightly (fp32 rounding of the
# extremal scale and the refined position moves the hard 6 sigma disk edge
# across a pixel centre).  describe_check proves that for every such pair:
# it recomputes the oracle's descriptor at the GPU record's own (x, y, sigma,
# theta) on the oracle's pyramid, where the bar is 1e-3.

def oracle_records(got):
    """GPU keypoint records (the binding's 48-byte dtype) as oracle records."""
    import oracle
    out = np.zeros(len(got), dtype=oracle.KP_DTYPE)
    for f in ("x", "y", "sigma", "p", "theta", "rho", "peak", "image", "octave", "ix", "iy"):
        out[f] = got[f]
    out["pss"] = got["p_ss"]
    return out


def oracle_stages(O, img, topk=None, mask=None, fmax=0.6):
    """Oracle detection (top-k, canonical), oriented records, descriptors
    and the oracle pyramid; with `mask` (uint8 per 4x4 cell) the gated
    detection."""
    H, W = img.shape
    _, flat = O.pyramid(img)
    cand = O.detect(flat, W, H) if mask is None else O.detect_masked(flat, W, H, mask, fmax)
    alive = O.dedup(cand)
    sel = O.select(cand, alive, topk)
    ori = O.orient(flat, W, H, sel)
    desc = O.describe(flat, W, H, ori)
    return sel, ori, desc, flat


def describe_check(O, flat, W, H, ori_ref, desc_ref, got, gdesc, tol=1e-3):
    """Oriented-keypoint match rates and descriptor agreement of one image."""
    q1, q2, pairs = rates(ori_ref, got, oriented=True)
    if not pairs:
        return dict(q1=q1, q2=q2, pairs=0, e2e_within=0, rechecked=0, shared_within=0, max_e2e=0.0,
                    mean_e2e=0.0, max_shared=0.0)
    ia = np.array([p[0] for p in pairs])
    jb = np.array([p[1] for p in pairs])
    err = np.abs(desc_ref[ia] - gdesc[jb]).max(axis=1)
    bad = err > tol
    max_shared, shared_within = 0.0, 0
    if bad.any():
        at_gpu = O.describe(flat, W, H, oracle_records(got[jb[bad]]))
        e2 = np.abs(at_gpu - gdesc[jb[bad]]).max(axis=1)
        max_shared, shared_within = float(e2.max()), int((e2 <= tol).sum())
    return dict(q1=q1, q2=q2, pairs=len(pairs), e2e_within=int((~bad).sum()), rechecked=int(bad.sum()),
                shared_within=shared_within, max_e2e=float(err.max()), mean_e2e=float(err.mean()),
                max_shared=max_shared)


def check_image(O, img, kp, ori, desc, topk=None, mask=None, fmax=0.6):
    """Keypoint rates (unoriented, top-k) and describe_check for one image."""
    H, W = img.shape
    sel, ori_ref, desc_ref, flat = oracle_stages(O, img, topk, mask, fmax)
    r1, r2, _ = rates(sel, kp)
    d = describe_check(O, flat, W, H, ori_ref, desc_ref, ori, desc)
    d.update(r1=r1, r2=r2, n_ref=len(sel), n_got=len(kp))
    return d


def check_images(O, imgs, kps, oris, descs, threads=16, masks=None, **kw):
    """check_image over many images on a thread pool (the oracle releases
    the interpreter lock while it runs); masks: per-image cell masks for
    gated detection, or None."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(lambda i: check_image(O, imgs[i], kps[i], oris[i], descs[i],
                                                 mask=None if masks is None else masks[i], **kw),
                           range(len(imgs))))


def summarize(results):
    """Aggregate rates over images: keypoint and oriented-keypoint match
    rates both ways (overall and worst image), the fraction of matched
    descriptors within 1e-3 end to end, and -- for the rest -- at shared
    keypoint geometry."""
    tot = lambda k: sum(r[k] for r in results)
    pairs = tot("pairs")
    return dict(
        images=len(results),
        kp_ref=sum(r["r1"] * r["n_ref"] for r in results) / max(1, tot("n_ref")),
        kp_got=sum(r["r2"] * r["n_got"] for r in results) / max(1, tot("n_got")),
        kp_min=min(min(r["r1"], r["r2"]) for r in results),
        ori_min=min(min(r["q1"], r["q2"]) for r in results),
        pairs=pairs,
        e2e_within=tot("e2e_within") / max(1, pairs),
        rechecked=tot("rechecked"),
        shared_miss=tot("rechecked") - tot("shared_within"),
        within_after_recheck=(tot("e2e_within") + tot("shared_within")) / max(1, pairs),
        max_e2e=max(r["max_e2e"] for r in results),
        max_shared=max(r["max_shared"] for r in results),
        mean_e2e=sum(r["mean_e2e"] * r["pairs"] for r in results) / max(1, pairs))


# Bars of the GPU parity tests (see tests/test_gpu_parity.py).
KP_RATE = 0.99
KP_RATE_IMAGE = 0.98   # worst single image of a batch (a near-tie at rank 1000 swaps one keypoint)
SHARED_MISS = 1e-4


def assert_parity(s, what):
    """The bars of this module on a summarize() result."""
    print(f"{what}: {s['images']} images; keypoints {s['kp_ref']:.4f}/{s['kp_got']:.4f} (worst image "
          f"{s['kp_min']:.4f}); oriented worst {s['ori_min']:.4f}; {s['pairs']} descriptor pairs, "
          f"{s['e2e_within']:.4f} within 1e-3 end to end, {s['rechecked']} rechecked at GPU geometry, "
          f"{s['shared_miss']} beyond 1e-3 there (max e2e {s['max_e2e']:.2e}, max at shared geometry "
          f"{s['max_shared']:.2e}, mean {s['mean_e2e']:.2e})", flush=True)
    assert s["kp_ref"] >= KP_RATE and s["kp_got"] >= KP_RATE
    assert s["kp_min"] >= KP_RATE_IMAGE and s["ori_min"] >= KP_RATE_IMAGE
    assert s["shared_miss"] <= SHARED_MISS * s["pairs"]
    assert s["within_after_recheck"] >= 1.0 - SHARED_MISS
