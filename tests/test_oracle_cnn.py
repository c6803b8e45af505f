"""Pins for the surrogate-mask CNN oracle (oracle/cnn.py)."""
import math

import numpy as np
import pytest
import scipy.ndimage as ndi
import torch

from oracle import cnn


def test_param_count():
    assert cnn.N_PARAMS == 9382
    p = cnn.init_params(0)
    convs, Wh, bh = cnn.unpack(p)
    np.testing.assert_array_equal(cnn.pack(convs, Wh, bh).astype(np.float32), p)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 10, 5000), rng.uniform(-1, 1, 5000),
                        [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -0.0, 1e-30, 3.0e38]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cnn.bf16(x), ref)
    assert cnn.bf16(1.0 + 2 ** -8) == 1.0            # tie to even
    assert cnn.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6


def test_space_to_depth_layout_and_padding():
    rng = np.random.default_rng(1)
    img = rng.integers(0, 256, size=(10, 7), dtype=np.uint8)
    X = cnn.space_to_depth(img)
    assert X.shape == (3, 2, 16)
    for cy in range(3):
        for cx in range(2):
            for dy in range(4):
                for dx in range(4):
                    y, x = min(4 * cy + dy, 9), min(4 * cx + dx, 6)
                    assert X[cy, cx, 4 * dy + dx] == img[y, x] / 255.0


def test_conv3x3_matches_library_correlation():
    rng = np.random.default_rng(2)
    X = rng.normal(size=(6, 5, 3))
    W = rng.normal(size=(9, 3, 2))
    b = rng.normal(size=2)
    out = cnn.conv3x3(X, W, b)
    for co in range(2):
        ref = np.full((6, 5), b[co])
        for ci in range(3):
            k = W[:, ci, co].reshape(3, 3)          # k[dy+1, dx+1]
            ref += ndi.correlate(X[:, :, ci], k, mode="constant", cval=0.0)
        np.testing.assert_allclose(out[:, :, co], ref, atol=1e-12)


def test_conv_input_and_weight_grads_are_adjoints():
    """<dZ, conv(X, W)> is bilinear: its X- and W-derivatives equal the
    adjoint maps, checked through the inner-product identity."""
    rng = np.random.default_rng(3)
    X = rng.normal(size=(5, 4, 3))
    W = rng.normal(size=(9, 3, 2))
    dZ = rng.normal(size=(5, 4, 2))
    Xd = rng.normal(size=X.shape)
    Wd = rng.normal(size=W.shape)
    zero = np.zeros(2)
    lhs = np.sum(dZ * cnn.conv3x3(Xd, W, zero))
    assert abs(lhs - np.sum(Xd * cnn.conv3x3_input_grad(dZ, W))) < 1e-10
    lhs = np.sum(dZ * cnn.conv3x3(X, Wd, zero))
    assert abs(lhs - np.sum(Wd * cnn.conv3x3_weight_grad(X, dZ))) < 1e-10


def _problem(seed=4):
    rng = np.random.default_rng(seed)
    img = rng.integers(0, 256, size=(22, 19), dtype=np.uint8)
    params = cnn.init_params(seed).astype(np.float64)
    # biases away from zero so no ReLU sits on its kink
    convs, Wh, bh = cnn.unpack(params)
    convs = [(W, rng.uniform(0.05, 0.2, size=cnn.C)) for W, _ in convs]
    params = cnn.pack(convs, Wh, rng.normal(0, 0.5, size=cnn.NH))
    H4, W4 = cnn.grid_size(*img.shape)
    labels = rng.integers(0, 64, size=(H4, W4)).astype(np.uint8)
    pw = rng.uniform(1.0, 5.0, size=cnn.NH)
    return img, params, labels, pw


def test_gradient_matches_finite_differences():
    img, params, labels, pw = _problem()
    n_oct = 4
    loss, g = cnn.loss_and_grad(params, img, labels, pw, n_oct)
    rng = np.random.default_rng(5)
    idx = np.concatenate([rng.choice(cnn.N_PARAMS - 102, 60, replace=False),
                          np.arange(cnn.N_PARAMS - 102, cnn.N_PARAMS)[::5]])
    h = 1e-6
    for i in idx:
        pp, pm = params.copy(), params.copy()
        pp[i] += h
        pm[i] -= h
        fd = (cnn.loss_and_grad(pp, img, labels, pw, n_oct)[0] - cnn.loss_and_grad(pm, img, labels, pw, n_oct)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (i, fd, g[i])


def test_loss_closed_form_at_zero_logits():
    img, params, labels, pw = _problem()
    convs, Wh, bh = cnn.unpack(params)
    p0 = cnn.pack(convs, np.zeros_like(Wh), np.zeros(cnn.NH))
    n_oct = 5
    loss, g = cnn.loss_and_grad(p0, img, labels, pw, n_oct)
    y = ((labels[..., None] >> np.arange(cnn.NH)) & 1)[..., :n_oct]
    ref = np.mean(pw[:n_oct] * y * math.log(2) + (1 - y) * math.log(2))
    assert abs(loss - ref) < 1e-12
    # head bias gradient: mean of (1/2 (w y + 1 - y) - w y) per channel
    N = y.shape[0] * y.shape[1] * n_oct
    for o in range(n_oct):
        yo = y[..., o]
        ref_g = np.sum(0.5 * (pw[o] * yo + 1 - yo) - pw[o] * yo) / N
        assert abs(g[-cnn.NH + o] - ref_g) < 1e-12
    assert np.all(g[-cnn.NH + n_oct:] == 0)


def test_bf16_mode_close_to_fp64():
    img, params, labels, pw = _problem()
    l64, g64 = cnn.loss_and_grad(params, img, labels, pw, 4)
    l16, g16 = cnn.loss_and_grad(params, img, labels, pw, 4, bf16_mode=True)
    assert abs(l16 - l64) < 2e-2 * abs(l64)
    cos = g16 @ g64 / np.linalg.norm(g16) / np.linalg.norm(g64)
    assert cos > 0.99


def test_adam_first_step():
    rng = np.random.default_rng(6)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    p1, m, v = cnn.adam(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    # bias-corrected first step moves every parameter by lr * g / (|g| + eps)
    np.testing.assert_allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), atol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_labels_and_mask_bits():
    kp = np.zeros(3, dtype=[("octave", "i4"), ("ix", "i4"), ("iy", "i4")])
    kp[0] = (0, 9, 5)       # base (9, 5) -> cell (2, 1)
    kp[1] = (2, 3, 7)       # base (12, 28) -> cell (3, 7)
    kp[2] = (1, 4, 2)       # base (8, 4) -> cell (2, 1)
    lab = cnn.label_bits(kp, 40, 20)
    assert lab.shape == (10, 5)
    assert lab[1, 2] == 0b011 and lab[7, 3] == 0b100 and lab.sum() == 0b011 + 0b100
    z = np.full((2, 2, 6), -5.0)
    z[0, 1, 3] = 5.0
    z[1, 0, 5] = 5.0
    bits = cnn.mask_bits(z, 0.5, 5)
    assert bits[0, 1] == 8 and bits[1, 0] == 0 and bits.sum() == 8
