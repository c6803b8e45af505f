"""Pins for the oracle's scale space (Eq. (1), Algorithm 1 stage A).

Each check compares the oracle with something other than itself: closed
forms, a library 2-D convolution, exact identities.
"""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi


@pytest.mark.parametrize("s", [0.8, 1.02977, 1.6, 2.16349, 2.77128, 5.0])
def test_gauss_taps_sum_symmetry_moment(O64, O32, s):
    r = O64.blur_radius(s)
    assert r == math.ceil(4 * s)
    for O, tol in ((O64, 1e-12), (O32, 1e-6)):
        t = O.gauss_taps(s, r).astype(np.float64)
        assert abs(t.sum() - 1.0) < tol
        np.testing.assert_array_equal(t, t[::-1])
        p = np.arange(-r, r + 1)
        # second moment of a sampled Gaussian truncated at 4s is s^2 to < 1e-3 s^2
        assert abs((t * p * p).sum() - s * s) < 1e-3 * s * s
        # unnormalised shape: ratio of neighbouring taps is exp(-(2p+1)/(2 s^2))
        ratio = t[r + 1] / t[r]
        assert abs(ratio - math.exp(-1.0 / (2 * s * s))) < 10 * tol


def test_scale_constants(O64):
    # sigma_k = 1.6 * 2^(k/4); direct blur sigma s_k adds sigma_k^2 - sigma0^2
    for k in range(5):
        assert abs(O64.scale_sigma(k) - 1.6 * 2 ** (k / 4)) < 1e-12
    assert abs(O64.blur_sigma(0) - 1.6) < 1e-15
    for k in range(1, 5):
        s = O64.blur_sigma(k)
        assert abs(1.6 ** 2 + s * s - O64.scale_sigma(k) ** 2) < 1e-12
    assert [O64.blur_radius(O64.blur_sigma(k)) for k in range(5)] == [7, 5, 7, 9, 12]


@pytest.mark.parametrize("shape", [(32, 32), (17, 29), (9, 40)])
@pytest.mark.parametrize("s", [1.02977, 2.77128])
def test_separable_blur_equals_2d_convolution(O64, O32, shape, s):
    rng = np.random.default_rng(11)
    img = rng.uniform(0, 255, size=shape)
    r = O64.blur_radius(s)
    k1 = O64.gauss_taps(s, r)
    ref = ndi.correlate(img, np.outer(k1, k1), mode="nearest")
    np.testing.assert_allclose(O64.blur(img, s, r), ref, atol=1e-10, rtol=0)
    np.testing.assert_allclose(O32.blur(img.astype(np.float32), s, r), ref, atol=1e-4 * 255, rtol=0)


def test_blur_preserves_constants_and_ramps(O64):
    # taps sum to 1 and are symmetric: constants and linear ramps pass unchanged
    # away from the clamped border
    s, r = 2.77128, 12
    y, x = np.mgrid[0:64, 0:64].astype(np.float64)
    ramp = 3.0 * x - 2.0 * y + 7.0
    out = O64.blur(ramp, s, r)
    np.testing.assert_allclose(out[r:-r, r:-r], ramp[r:-r, r:-r], atol=1e-10)
    np.testing.assert_allclose(O64.blur(np.full((20, 30), 42.0), s, r), 42.0, atol=1e-12)


@pytest.mark.parametrize("W,H,sizes", [
    (640, 480, [(640, 480), (320, 240), (160, 120), (80, 60), (40, 30)]),
    (1280, 960, [(1280, 960), (640, 480), (320, 240), (160, 120), (80, 60), (40, 30)]),
    (640, 427, [(640, 427), (320, 214), (160, 107), (80, 54), (40, 27)]),
    (640, 360, [(640, 360), (320, 180), (160, 90), (80, 45), (40, 23)]),
    (640, 640, [(640, 640), (320, 320), (160, 160), (80, 80), (40, 40), (20, 20)]),
    (480, 640, [(480, 640), (240, 320), (120, 160), (60, 80), (30, 40)]),
    (20, 16, [(20, 16)]),
])
def test_octave_sizes(O64, W, H, sizes):
    n = O64.num_octaves(W, H)
    assert [O64.octave_size(W, H, o) for o in range(n)] == sizes


def test_pyramid_structure(O64):
    rng = np.random.default_rng(3)
    img = rng.integers(0, 256, size=(70, 90), dtype=np.uint8)
    octs, _ = O64.pyramid(img)
    assert len(octs) == O64.num_octaves(90, 70)
    # G_{0,0}: the input pre-blurred by sigma0 (2-D library convolution)
    t0 = O64.gauss_taps(1.6, 7)
    np.testing.assert_allclose(octs[0][0], ndi.correlate(img.astype(np.float64), np.outer(t0, t0),
                                                         mode="nearest"), atol=1e-9)
    for o, planes in enumerate(octs):
        for k in range(1, 5):
            s = O64.blur_sigma(k)
            r = O64.blur_radius(s)
            t = O64.gauss_taps(s, r)
            np.testing.assert_allclose(planes[k], ndi.correlate(planes[0], np.outer(t, t), mode="nearest"),
                                       atol=1e-9)
        if o + 1 < len(octs):
            # decimation takes the even samples of G_{o,4}, exactly
            np.testing.assert_array_equal(octs[o + 1][0], planes[4][::2, ::2])


def test_laplacian_exact_on_quadratics_and_ramps(O64):
    y, x = np.mgrid[0:24, 0:31].astype(np.float64)
    sig = 1.9027
    q = x * x + y * y
    L = O64.laplacian(q, sig)
    np.testing.assert_allclose(L[1:-1, 1:-1], 4.0 * sig * sig, rtol=0, atol=1e-9)
    ramp = 2.5 * x - 1.25 * y + 9.0
    np.testing.assert_allclose(O64.laplacian(ramp, sig)[1:-1, 1:-1], 0.0, atol=1e-9)
    # a single impulse gives the 5-point stencil, scaled by sigma^2
    imp = np.zeros((5, 5))
    imp[2, 2] = 1.0
    L = O64.laplacian(imp, 2.0)
    exp = np.zeros((5, 5))
    exp[2, 2] = -4.0
    exp[1, 2] = exp[3, 2] = exp[2, 1] = exp[2, 3] = 1.0
    np.testing.assert_allclose(L, 4.0 * exp, atol=0)


def test_blob_scale_space_closed_form(O64):
    """A Gaussian blob A exp(-r^2/2s^2) blurred by sigma has scale-normalised
    LoG -2 A s^2 sigma^2 / (s^2+sigma^2)^2 at its centre (continuous theory);
    the pyramid planes plus the Laplacian reproduce it to a few percent."""
    s, A = 3.0, 60.0
    N = 129
    y, x = np.mgrid[0:N, 0:N].astype(np.float64)
    c = 64.0
    img = 100.0 + A * np.exp(-((x - c) ** 2 + (y - c) ** 2) / (2 * s * s))
    G0 = O64.blur(img, 1.6, 7)
    for k in range(5):
        sk = O64.scale_sigma(k)
        Gk = G0 if k == 0 else O64.blur(G0, O64.blur_sigma(k), O64.blur_radius(O64.blur_sigma(k)))
        L = O64.laplacian(Gk, sk)[64, 64]
        theory = -2 * A * s * s * sk * sk / (s * s + sk * sk) ** 2
        assert abs(L - theory) < 0.03 * abs(theory), (k, L, theory)
