"""End-to-end pins for the oracle: closed forms and exact invariances."""
import math

import numpy as np
import pytest

import oracle
import synth


def _blob_image(N, cx, cy, s, A, bg=100.0):
    y, x = np.mgrid[0:N, 0:N].astype(np.float64)
    img = bg + A * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * s * s))
    return np.clip(np.floor(img + 0.5), 0, 255).astype(np.uint8)


@pytest.mark.parametrize("s", [2.0, 2.5, 4.0, 6.0, 8.0, 16.0, 24.0])
def test_blob_detected_at_its_scale(O64, s):
    """Continuous theory: the scale-normalised LoG at the centre of
    A exp(-r^2/2s^2) is -2 A s^2 sigma^2/(s^2+sigma^2)^2, extremal at sigma = s
    with value -A/2.  Exactly one strong keypoint, at the centre."""
    A, cx, cy = 60.0, 128.3, 127.6
    img = _blob_image(257, cx, cy, s, A)
    _, flat = O64.pyramid(img)
    cand = O64.detect(flat, 257, 257)
    alive = O64.dedup(cand)
    kp = O64.select(cand, alive, topk=0)
    strong = kp[np.abs(kp["p"]) > 0.5 * A / 2]
    assert len(strong) == 1
    k = strong[0]
    assert abs(k["sigma"] - s) < 0.05 * s
    assert abs(-k["p"] - A / 2) < 0.05 * A / 2
    assert math.hypot(k["x"] - cx, k["y"] - cy) < 0.1
    # its octave holds sigma* in [1.6, 3.2) octave pixels
    assert 1.6 <= k["sigma"] / 2 ** k["octave"] < 3.2


def _match(kp_a, kp_b, map_b_to_a):
    """Pair records by (octave, mapped integer position); the orientation
    records of one keypoint pair up in their stored (peak) order."""
    from collections import defaultdict
    ga, gb = defaultdict(list), defaultdict(list)
    for i, k in enumerate(kp_a):
        ga[(int(k["octave"]), int(k["ix"]), int(k["iy"]))].append(i)
    for j, k in enumerate(kp_b):
        ix, iy = map_b_to_a(int(k["ix"]), int(k["iy"]), int(k["octave"]))
        gb[(int(k["octave"]), ix, iy)].append(j)
    pairs = []
    for key, ii in ga.items():
        pairs.extend(zip(ii, gb.get(key, [])))
    return pairs


def test_rotation_by_90_degrees(O64):
    """On a (2^m+1)^2 image every stage commutes with a 90-degree rotation:
    clamp borders and even-sample decimation are symmetric, the 5-point
    Laplacian is isotropic, and 36 and 8 bins are multiples of 4.  Keypoints
    map, orientations shift by a quarter turn and descriptors are equal."""
    N = 257
    img = synth.image(11, 0, N, N, nblobs=60)
    rot = np.ascontiguousarray(np.rot90(img))      # rot[i, j] = img[j, N-1-i]
    ka, da, _ = O64.run(img)
    kb, db, _ = O64.run(rot)
    assert len(ka) > 100

    def b_to_a(ix, iy, o):
        n = (N - 1) // 2 ** o + 1               # octave size, exact for 2^m+1
        # point (x', y') in rot is (x, y) = (n-1-y', x') in img
        return n - 1 - iy, ix

    pairs = _match(ka, kb, b_to_a)
    assert len(pairs) >= 0.995 * len(ka)
    dth = []
    for i, j in pairs:
        d = (kb[j]["theta"] - ka[i]["theta"]) % (2 * math.pi)
        dth.append(d)
    # rot(x', y') = img(n-1-y', x'): the gradient (gx, gy) becomes (gy, -gx),
    # so every orientation turns by -pi/2 (records of one keypoint stay in
    # peak order, so they pair up one to one)
    dth = np.array(dth)
    quarter = np.abs(dth - 1.5 * math.pi) < 1e-6
    assert quarter.mean() > 0.99
    good = [(i, j) for (i, j), q in zip(pairs, quarter) if q]
    diff = max(np.abs(da[i] - db[j]).max() for i, j in good)
    assert diff < 1e-6


def test_brightness_offset_invariance(O64):
    """I + c (no clipping) leaves every Gaussian-image difference, hence every
    LoG, gradient, keypoint and descriptor unchanged (up to rounding)."""
    img = synth.image(12, 0, 200, 160, nblobs=40, amax=40.0)
    img = (img.astype(np.int32) // 2 + 30).astype(np.uint8)
    ka, da, sa = O64.run(img)
    kb, db, sb = O64.run((img + 50).astype(np.uint8))
    assert sa == sb
    np.testing.assert_allclose(ka["x"], kb["x"], atol=1e-9)
    np.testing.assert_allclose(ka["p"], kb["p"], atol=1e-9)
    np.testing.assert_allclose(da, db, atol=1e-9)


def test_contrast_scaling(O64):
    """2I with threshold 2T: every linear stage doubles exactly in binary
    floating point, the roots of p' and all ratios are unchanged, so the
    keypoints are identical with p doubled and descriptors equal."""
    img = synth.image(13, 0, 200, 160, nblobs=40)
    img = (img // 2).astype(np.uint8)
    P2 = oracle.Oracle.default_params()
    P2.contrast = 2 * P2.contrast
    O2 = oracle.Oracle("f64", P2)
    ka, da, sa = O64.run(img)
    kb, db, sb = O2.run((img * 2).astype(np.uint8))
    assert sa == sb
    np.testing.assert_array_equal(ka["x"], kb["x"])
    np.testing.assert_array_equal(ka["sigma"], kb["sigma"])
    np.testing.assert_array_equal(2 * ka["p"], kb["p"])
    np.testing.assert_allclose(da, db, atol=1e-12)


def test_f32_build_agrees_with_f64(O64, O32):
    img = synth.image(synth.SEED_SINGLE, 0, 640, 480)
    ka, da, sa = O64.run(img)
    kb, db, sb = O32.run(img)
    assert abs(sa["candidates"] - sb["candidates"]) <= 0.01 * sa["candidates"]
    # same keypoints (same octave, integer position) for >= 99% of records
    key = lambda k: (int(k["octave"]), int(k["ix"]), int(k["iy"]))
    sb_keys = {key(k) for k in kb}
    assert np.mean([key(k) in sb_keys for k in ka]) >= 0.99


def test_output_counts_and_ordering(O64):
    img = synth.image(synth.SEED_SINGLE, 0, 640, 480)
    kp, desc, st = O64.run(img)
    assert st["candidates"] >= st["deduped"] >= st["selected"]
    assert st["selected"] == 1000 and len(kp) == 1000
    # canonical order: |p| non-increasing
    assert np.all(np.diff(np.abs(kp["p"])) <= 0)
    assert np.all((kp["theta"] >= 0) & (kp["theta"] < 2 * math.pi))
    np.testing.assert_allclose(np.linalg.norm(desc, axis=1), 1.0, atol=1e-12)
    # every keypoint's sigma lies in its octave's range
    s_oct = kp["sigma"] / 2.0 ** kp["octave"]
    assert np.all((s_oct >= 1.6) & (s_oct < 3.2))
