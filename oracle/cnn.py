"""Surrogate-mask CNN oracle -- TEST INFRASTRUCTURE ONLY (numpy).

Not from the paper: the learned candidate mask that gates ALP detection.
Plain numpy, float64 accumulation, written from the definition below so
that a reader can check each step by eye.  Optional `bf16=True` rounds, as
the GPU kernels do, the space-to-depth input, the conv weights and every
stored activation (and, in the backward pass, the MFMA operands dZ) to
bfloat16 with round-to-nearest-even.

Network (per image, at 1/4 resolution):
  X0 = space_to_depth(4)(u8 / 255): the image, edge-padded to a multiple
       of 4, as H4 x W4 cells of 16 channels (channel = 4*dy + dx);
  X_l = relu(conv3x3(X_{l-1}; W_l, b_l)), l = 1..4, 16 -> 16 channels,
       zero padding, tap t = 3*(dy+1) + (dx+1), W_l[t][ci][co];
  Z  = X_4 . Wh + bh  (1x1, 16 -> 6 logits, channel o = octave o);
  mask_o = sigmoid(Z_o) > tau.
Loss: mean over cells and the octave channels the image has of the
positive-weighted binary cross-entropy
  l = w_o y softplus(-z) + (1 - y) softplus(z).

Parameter vector (float32, 9382 entries): for l = 1..4, W_l (9*16*16,
[t][ci][co]) then b_l (16); then Wh (16*6, [c][o]) then bh (6).
"""
from __future__ import annotations

import numpy as np

C = 16
NL = 4
NH = 6
CONV_W = 9 * C * C
N_PARAMS = NL * (CONV_W + C) + C * NH + NH   # 9382


def bf16(a):
    """Round float values to the nearest bfloat16 (ties to even), as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(params):
    p = np.asarray(params, dtype=np.float64)
    assert p.size == N_PARAMS
    out, o = [], 0
    for _ in range(NL):
        W = p[o:o + CONV_W].reshape(9, C, C)
        o += CONV_W
        b = p[o:o + C]
        o += C
        out.append((W, b))
    Wh = p[o:o + C * NH].reshape(C, NH)
    o += C * NH
    bh = p[o:o + NH]
    return out, Wh, bh


def pack(convs, Wh, bh):
    parts = []
    for W, b in convs:
        parts += [np.asarray(W).reshape(-1), np.asarray(b).reshape(-1)]
    parts += [np.asarray(Wh).reshape(-1), np.asarray(bh).reshape(-1)]
    return np.concatenate(parts)


def init_params(seed=0):
    """He-normal conv weights, zero biases, small head."""
    rng = np.random.default_rng(seed)
    convs = [(rng.normal(0, np.sqrt(2.0 / (9 * C)), size=(9, C, C)), np.zeros(C)) for _ in range(NL)]
    Wh = rng.normal(0, np.sqrt(1.0 / C), size=(C, NH))
    bh = np.full(NH, -2.0)
    return pack(convs, Wh, bh).astype(np.float32)


def grid_size(H, W):
    return (H + 3) // 4, (W + 3) // 4


def space_to_depth(img):
    """(H, W) u8 -> (H4, W4, 16) float64 of value/255, edge padding."""
    img = np.asarray(img)
    H, W = img.shape
    H4, W4 = grid_size(H, W)
    pad = np.pad(img.astype(np.float64) / 255.0, ((0, 4 * H4 - H), (0, 4 * W4 - W)), mode="edge")
    X = pad.reshape(H4, 4, W4, 4).transpose(0, 2, 1, 3).reshape(H4, W4, 16)
    return X


def conv3x3(X, W, b):
    """out[y, x, co] = b[co] + sum_{dy, dx, ci} X[y+dy, x+dx, ci] W[3(dy+1)+(dx+1), ci, co],
    zero outside the grid."""
    H4, W4, _ = X.shape
    Xp = np.pad(X, ((1, 1), (1, 1), (0, 0)))
    out = np.broadcast_to(b, (H4, W4, W.shape[2])).copy()
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            t = 3 * (dy + 1) + (dx + 1)
            out += Xp[1 + dy:1 + dy + H4, 1 + dx:1 + dx + W4, :] @ W[t]
    return out


def conv3x3_input_grad(dZ, W):
    """d/dX of sum(dZ * conv3x3(X, W, .)): dX[y, x, ci] = sum_t dZ[y-dy, x-dx, :] W[t, ci, :]."""
    H4, W4, _ = dZ.shape
    dZp = np.pad(dZ, ((1, 1), (1, 1), (0, 0)))
    dX = np.zeros((H4, W4, W.shape[1]))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            t = 3 * (dy + 1) + (dx + 1)
            dX += dZp[1 - dy:1 - dy + H4, 1 - dx:1 - dx + W4, :] @ W[t].T
    return dX


def conv3x3_weight_grad(X, dZ):
    """dW[t, ci, co] = sum_{y, x} X[y+dy, x+dx, ci] dZ[y, x, co] (zero padding)."""
    H4, W4, Ci = X.shape
    Xp = np.pad(X, ((1, 1), (1, 1), (0, 0)))
    dW = np.zeros((9, Ci, dZ.shape[2]))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            t = 3 * (dy + 1) + (dx + 1)
            Xs = Xp[1 + dy:1 + dy + H4, 1 + dx:1 + dx + W4, :].reshape(-1, Ci)
            dW[t] = Xs.T @ dZ.reshape(-1, dZ.shape[2])
    return dW


def forward(params, img, bf16_mode=False):
    """Returns (logits (H4, W4, 6), activations [X0..X4])."""
    convs, Wh, bh = unpack(params)
    r = bf16 if bf16_mode else (lambda a: np.asarray(a, dtype=np.float64))
    X = r(space_to_depth(img))
    acts = [X]
    for W, b in convs:
        X = r(np.maximum(conv3x3(X, r(W), b), 0.0))
        acts.append(X)
    Z = X @ Wh + bh
    return Z, acts


def softplus(z):
    return np.logaddexp(0.0, z)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def loss_and_grad(params, img, labels, pos_weight, n_octaves, bf16_mode=False):
    """labels: (H4, W4) uint8, bit o = cell positive for octave o.
    pos_weight: 6 weights w_o.  Only channels o < n_octaves count.
    Returns (loss, gradient vector of N_PARAMS)."""
    convs, Wh, bh = unpack(params)
    r = bf16 if bf16_mode else (lambda a: np.asarray(a, dtype=np.float64))
    Z, acts = forward(params, img, bf16_mode)
    H4, W4, _ = Z.shape
    y = ((np.asarray(labels)[..., None] >> np.arange(NH)) & 1).astype(np.float64)
    valid = (np.arange(NH) < n_octaves).astype(np.float64)
    w = np.asarray(pos_weight, dtype=np.float64)
    N = H4 * W4 * n_octaves
    l = (w * y * softplus(-Z) + (1 - y) * softplus(Z)) * valid
    loss = l.sum() / N
    s = sigmoid(Z)
    dZ = (s * (w * y + 1 - y) - w * y) * valid / N
    X4 = acts[-1]
    gWh = X4.reshape(-1, C).T @ dZ.reshape(-1, NH)
    gbh = dZ.reshape(-1, NH).sum(0)
    dX = dZ @ Wh.T
    grads = []
    for l_i in range(NL - 1, -1, -1):
        W, b = convs[l_i]
        Xin, Xout = acts[l_i], acts[l_i + 1]
        dP = r(dX * (Xout > 0))                     # through the ReLU
        grads.append((conv3x3_weight_grad(Xin, dP), dP.reshape(-1, C).sum(0)))
        if l_i > 0:
            dX = conv3x3_input_grad(dP, r(W))
    grads.reverse()
    return loss, pack(grads, gWh, gbh)


def mask_bits(logits, tau, n_octaves):
    """(H4, W4) uint8: bit o set when sigmoid(z_o) > tau (o < n_octaves)."""
    on = sigmoid(logits) > tau
    on[..., n_octaves:] = False
    return (on.astype(np.uint8) << np.arange(NH, dtype=np.uint8)).sum(-1).astype(np.uint8)


def label_bits(keypoints, H, W):
    """(H4, W4) uint8: bit o set in the cell holding (ix 2^o, iy 2^o) / 4 of
    every keypoint of octave o."""
    H4, W4 = grid_size(H, W)
    lab = np.zeros((H4, W4), dtype=np.uint8)
    for k in keypoints:
        o = int(k["octave"])
        cx = (int(k["ix"]) << o) // 4
        cy = (int(k["iy"]) << o) // 4
        lab[min(cy, H4 - 1), min(cx, W4 - 1)] |= np.uint8(1 << o)
    return lab


def adam(params, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba 2015) with bias correction; returns new arrays."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
