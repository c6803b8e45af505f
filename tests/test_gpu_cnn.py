"""Surrogate CNN and gated detection on the GPU vs the CPU oracle.

Bars: forward activations and logits within relative L2 1e-2 of the oracle
run with the kernels' bf16 roundings; gradients cosine >= 0.999 and relative
L2 <= 2e-2; labels bit-exact; Adam within 1e-6; gating: an all-ones mask
reproduces the plain detector exactly, an all-zeros mask gives nothing, the
dense fallback reproduces the plain detector, and with a random mask every
keypoint lies in an active cell while >= 99% of the plain keypoints in
active cells are found.
"""
import numpy as np
import pytest

import json
import os

import oracle
import synth
from oracle import cnn
from parity import KP_RATE, assert_parity, check_images, oracle_stages, rates, summarize

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1705_09776_amd as cd  # noqa: E402


def _bf16_to_f32(t):
    u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32)


def _params(seed=0):
    p = cnn.init_params(seed).astype(np.float64)
    rng = np.random.default_rng(seed)
    convs, Wh, bh = cnn.unpack(p)
    convs = [(W, rng.uniform(-0.05, 0.1, size=cnn.C)) for W, _ in convs]
    return cnn.pack(convs, Wh, rng.normal(-1, 0.5, size=cnn.NH)).astype(np.float32)


def _images():
    return [synth.image(synth.SEED_SINGLE, 0, 640, 480), synth.image(7, 1, 97, 61, nblobs=10),
            synth.image(synth.SEED_RAGGED, 3, 480, 640, nblobs=150)]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.fixture(scope="module")
def fwd():
    imgs = _images()
    pipe = cd.Pipeline([(im.shape[1], im.shape[0]) for im in imgs])
    pipe.upload(imgs)
    P = _params(1)
    dP = torch.from_numpy(P).cuda()
    pipe.cnn_forward(dP, tau=0.3)
    torch.cuda.synchronize()
    return imgs, pipe, P, dP


def test_forward_matches_oracle(fwd):
    imgs, pipe, P, _ = fwd
    acts = _bf16_to_f32(pipe.d_acts).reshape(cnn.NL, pipe.ncells, cnn.C)
    logits = pipe.d_logits.cpu().numpy()
    mask = pipe.d_mask.cpu().numpy()
    for i, im in enumerate(imgs):
        c0, w4, h4 = pipe.cell_layout(i)
        Z, A = cnn.forward(P, im, bf16_mode=True)
        for l in range(cnn.NL):
            g = acts[l, c0:c0 + w4 * h4].reshape(h4, w4, cnn.C)
            r = _rel(g, A[l + 1])
            assert r <= 1e-2, (i, l, r)
        gz = logits[c0:c0 + w4 * h4].reshape(h4, w4, cnn.NH)
        assert _rel(gz, Z) <= 1e-2
        n_oct = pipe.num_octaves(i)
        ref = cnn.mask_bits(Z, 0.3, min(n_oct, cnn.NH))
        got = mask[c0:c0 + w4 * h4].reshape(h4, w4)
        # bits can only differ where the logit sits at the threshold
        zthr = np.log(0.3 / 0.7)
        near = (np.abs(Z - zthr) < 1e-2).any(-1)
        assert np.all((got == ref) | near)
        assert (got == ref).mean() > 0.999


def test_backward_matches_oracle(fwd):
    imgs, pipe, P, dP = fwd
    rng = np.random.default_rng(3)
    labels = rng.integers(0, 64, size=pipe.ncells).astype(np.uint32)
    pw = rng.uniform(1, 8, size=cnn.NH).astype(np.float32)
    d_lab = torch.from_numpy(labels.view(np.int32)).cuda()
    d_pw = torch.from_numpy(pw).cuda()
    work = torch.empty(2 * pipe.ncells * cnn.C, dtype=torch.int16, device="cuda")
    grad = torch.empty(cnn.N_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    cd.cdvs_cnn_backward(pipe.ctx, pipe.d_images, dP, pipe.d_acts, pipe.d_logits, d_lab, d_pw, work, grad, loss)
    torch.cuda.synchronize()
    g_ref = np.zeros(cnn.N_PARAMS)
    l_ref = 0.0
    for i, im in enumerate(imgs):
        c0, w4, h4 = pipe.cell_layout(i)
        lab = labels[c0:c0 + w4 * h4].reshape(h4, w4).astype(np.uint8)
        l, g = cnn.loss_and_grad(P, im, lab, pw, min(pipe.num_octaves(i), cnn.NH), bf16_mode=True)
        l_ref += l / len(imgs)
        g_ref += g / len(imgs)
    g = grad.cpu().numpy().astype(np.float64)
    cos = g @ g_ref / np.linalg.norm(g) / np.linalg.norm(g_ref)
    print(f"loss gpu {loss.item():.6f} oracle {l_ref:.6f}; grad cos {cos:.6f} rel {_rel(g, g_ref):.2e}")
    assert abs(loss.item() - l_ref) <= 1e-3 * abs(l_ref)
    assert cos >= 0.999 and _rel(g, g_ref) <= 2e-2
    # every block of the parameter vector agrees, not only the head
    off = 0
    for l in range(cnn.NL):
        blk = slice(off, off + cnn.CONV_W)
        assert _rel(g[blk], g_ref[blk]) <= 3e-2, l
        off += cnn.CONV_W + cnn.C


def test_adam_matches_oracle():
    rng = np.random.default_rng(4)
    p = rng.normal(size=cnn.N_PARAMS)
    m = np.zeros(cnn.N_PARAMS)
    v = np.zeros(cnn.N_PARAMS)
    pipe = cd.Pipeline([(64, 48)])
    t = [torch.from_numpy(a.astype(np.float32)).cuda() for a in (p, m, v)]
    for step in (1, 2, 3):
        g = rng.normal(size=cnn.N_PARAMS)
        dg = torch.from_numpy(g.astype(np.float32)).cuda()
        cd.cdvs_cnn_adam(pipe.ctx, t[0], dg, t[1], t[2], step, lr=1e-3)
        p, m, v = cnn.adam(p, g.astype(np.float32).astype(np.float64), m, v, step, lr=1e-3)
    torch.cuda.synchronize()
    np.testing.assert_allclose(t[0].cpu().numpy(), p, atol=1e-6)


def test_labels_from_oracle_keypoints(O32):
    img = synth.image(synth.SEED_SINGLE, 0, 640, 480)
    pipe = cd.Pipeline([(640, 480)])
    pipe.upload([img])
    pipe.cnn_buffers()
    kp, _, _ = O32.run(img, with_desc=False)
    rec = np.zeros((1, pipe.kp_capacity), dtype=cd.KP_DTYPE)
    for f in ("octave", "ix", "iy"):
        rec[f][0, :len(kp)] = kp[f]
    pipe.d_kp.copy_(torch.from_numpy(rec.view(np.int32).reshape(1, pipe.kp_capacity, 12)))
    pipe.d_count.fill_(len(kp))
    lab = torch.empty(pipe.ncells, dtype=torch.int32, device="cuda")
    cd.cdvs_cnn_labels(pipe.ctx, pipe.d_kp, pipe.d_count, lab)
    torch.cuda.synchronize()
    c0, w4, h4 = pipe.cell_layout(0)
    ref = cnn.label_bits(kp, 480, 640)
    np.testing.assert_array_equal(lab.cpu().numpy().reshape(h4, w4).astype(np.uint8), ref)


def _gated(imgs, mask_fn, fmax=0.6, topk=4096):
    p = cd.default_params()
    p.topk = topk
    p.mask_fmax = fmax
    pipe = cd.Pipeline([(im.shape[1], im.shape[0]) for im in imgs], params=p, kp_capacity=topk)
    pipe.upload(imgs)
    pipe.cnn_buffers()
    pipe.pyramid()
    pipe.detect()
    torch.cuda.synchronize()
    plain = [k.copy() for k in pipe.keypoints()]
    m = mask_fn(pipe)
    pipe.d_mask.copy_(torch.from_numpy(m))
    pipe.detect(mask=pipe.d_mask)
    torch.cuda.synchronize()
    assert pipe.sync_status() == cd.CDVS_OK
    return pipe, plain, pipe.keypoints(), m


_KEYS = ["x", "y", "sigma", "p", "octave", "ix", "iy"]


def test_gate_all_ones_and_all_zeros():
    imgs = list(synth.fixed_batch(synth.SEED_BATCH, 2))
    pipe, plain, gated, _ = _gated(imgs, lambda pp: np.full(pp.ncells, 0x3F, dtype=np.uint8), fmax=1.0)
    for a, b in zip(plain, gated):
        np.testing.assert_array_equal(a[_KEYS], b[_KEYS])
    pipe, plain, gated, _ = _gated(imgs, lambda pp: np.zeros(pp.ncells, dtype=np.uint8), fmax=0.6)
    assert all(len(g) == 0 for g in gated)


def test_gate_dense_fallback():
    imgs = list(synth.fixed_batch(synth.SEED_BATCH, 2))
    rng = np.random.default_rng(5)
    _, plain, gated, _ = _gated(imgs, lambda pp: rng.integers(0, 64, pp.ncells).astype(np.uint8), fmax=0.0)
    for a, b in zip(plain, gated):
        np.testing.assert_array_equal(a[_KEYS], b[_KEYS])


def test_gate_random_mask():
    imgs = list(synth.fixed_batch(synth.SEED_BATCH, 2))
    rng = np.random.default_rng(6)
    pipe, plain, gated, m = _gated(imgs, lambda pp: (rng.random((pp.ncells, 6)) < 0.3).astype(np.uint8)
                                   .dot(1 << np.arange(6)).astype(np.uint8), fmax=1.0)

    def active(i, k):
        c0, w4, h4 = pipe.cell_layout(i)
        o = int(k["octave"])
        cx = min((int(k["ix"]) << o) >> 2, w4 - 1)
        cy = min((int(k["iy"]) << o) >> 2, h4 - 1)
        return (m[c0 + cy * w4 + cx] >> o) & 1

    for i in range(len(imgs)):
        assert all(active(i, k) for k in gated[i])
        want = {(int(k["octave"]), int(k["ix"]), int(k["iy"])) for k in plain[i] if active(i, k)}
        got = {(int(k["octave"]), int(k["ix"]), int(k["iy"])) for k in gated[i]}
        assert len(want & got) >= 0.99 * len(want)
        assert 0.2 * len(plain[i]) < len(gated[i]) < 0.5 * len(plain[i])


def test_fused_inference_equals_training_forward(fwd):
    """The fused inference kernel (no activations stored) gives the training
    forward's logits and mask bit for bit, on ragged sizes with partial
    tiles."""
    imgs, pipe, P, dP = fwd
    logits = pipe.d_logits.cpu().numpy().copy()
    mask = pipe.d_mask.cpu().numpy().copy()
    pipe.d_logits.fill_(float("nan"))
    pipe.d_mask.fill_(0xAA)
    cd.cdvs_cnn_forward(pipe.ctx, pipe.d_images, dP, None, pipe.d_logits, pipe.d_mask, 0.3)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(pipe.d_logits.cpu().numpy().view(np.uint32), logits.view(np.uint32))
    np.testing.assert_array_equal(pipe.d_mask.cpu().numpy(), mask)


_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _image_masks(pipe, mask):
    out = []
    for i in range(pipe.n):
        c0, w4, h4 = pipe.cell_layout(i)
        out.append(mask[c0:c0 + w4 * h4].reshape(h4, w4).copy())
    return out


@pytest.mark.parametrize("which", ["trained", "random"])
def test_gated_detection_matches_oracle(O32, which):
    """The gated pass against the oracle's own gated detection (a centre is
    examined iff its cell bit is set, neighbours read in full, dense above
    mask_fmax, stage C and the top-k afterwards) under the same mask: the
    trained 640x480 network's mask at its stored threshold, and a random mask
    with 30% of the (cell, octave) bits set; keypoints, orientations and
    descriptors to the plain path's bars."""
    imgs = list(synth.fixed_batch(synth.SEED_EVAL, 16, first=3000))
    pipe = cd.Pipeline([(640, 480)] * len(imgs))
    pipe.upload(imgs)
    pipe.cnn_buffers()
    if which == "trained":
        from paper_1705_09776_amd import surrogate
        w = os.path.join(_ROOT, "paper_1705_09776_amd", "weights", "surrogate_640x480.npz")
        tau = float(json.load(open(os.path.splitext(w)[0] + ".json"))["tau"])
        params = torch.from_numpy(surrogate.load_checkpoint(w)["params"]).cuda()
        pipe.run_gated(params, tau)
    else:
        rng = np.random.default_rng(11)
        m = (rng.random((pipe.ncells, 6)) < 0.3).astype(np.uint8).dot(1 << np.arange(6)).astype(np.uint8)
        pipe.d_mask.copy_(torch.from_numpy(m))
        pipe.pyramid()
        pipe.detect(mask=pipe.d_mask)
        pipe.orient()
        pipe.describe()
    torch.cuda.synchronize()
    assert pipe.sync_status() == cd.CDVS_OK
    masks = _image_masks(pipe, pipe.d_mask.cpu().numpy())
    res = check_images(O32, imgs, pipe.keypoints(), pipe.oriented(), pipe.descriptors(), masks=masks,
                       fmax=pipe.params.mask_fmax)
    assert_parity(summarize(res), f"gated ({which} mask)")


def test_gated_bench_configuration_every_image(O32):
    """The benchmark's gated launch configuration: the trained 640x480
    network's mask at its stored threshold over the 256-image batch, then
    the gated pass; every image against the oracle's gated detection under
    the GPU's mask, to the plain path's bars."""
    from paper_1705_09776_amd import surrogate
    imgs = list(synth.fixed_batch(synth.SEED_BATCH, 256))
    pipe = cd.Pipeline([(640, 480)] * len(imgs))
    pipe.upload(imgs)
    pipe.cnn_buffers()
    w = os.path.join(_ROOT, "paper_1705_09776_amd", "weights", "surrogate_640x480.npz")
    tau = float(json.load(open(os.path.splitext(w)[0] + ".json"))["tau"])
    params = torch.from_numpy(surrogate.load_checkpoint(w)["params"]).cuda()
    pipe.run_gated(params, tau)
    torch.cuda.synchronize()
    assert pipe.sync_status() == cd.CDVS_OK
    masks = _image_masks(pipe, pipe.d_mask.cpu().numpy())
    res = check_images(O32, imgs, pipe.keypoints(), pipe.oriented(), pipe.descriptors(), masks=masks,
                       fmax=pipe.params.mask_fmax)
    assert_parity(summarize(res), "gated (trained mask, 256-image batch)")


def test_gated_graph_replay_equals_eager():
    """The captured gated pass (fused CNN mask, pyramid, gated detection,
    orientation, descriptors) replayed several times, with the outputs and
    the mask cleared and an eager gated pass on the same buffers in between,
    reproduces the eager gated run: the mask bit for bit, keypoints and
    descriptors to the plain pass's replay bars."""
    from paper_1705_09776_amd import surrogate
    imgs = list(synth.fixed_batch(synth.SEED_BATCH, 4))
    pipe = cd.Pipeline([(640, 480)] * len(imgs))
    pipe.upload(imgs)
    pipe.cnn_buffers()
    w = os.path.join(_ROOT, "paper_1705_09776_amd", "weights", "surrogate_640x480.npz")
    tau = float(json.load(open(os.path.splitext(w)[0] + ".json"))["tau"])
    params = torch.from_numpy(surrogate.load_checkpoint(w)["params"]).cuda()
    pipe.run_gated(params, tau)
    torch.cuda.synchronize()
    assert pipe.sync_status() == cd.CDVS_OK
    m0 = pipe.d_mask.cpu().numpy().copy()
    k0 = [k.copy() for k in pipe.oriented()]
    d0 = [d.copy() for d in pipe.descriptors()]
    pipe.capture_gated(params, tau)
    for r in range(3):
        for t in (pipe.d_mask, pipe.d_kp, pipe.d_count, pipe.d_kp_ori, pipe.d_count_ori, pipe.d_desc, pipe.d_pyr):
            t.zero_()
        torch.cuda.synchronize()
        pipe.replay()
        torch.cuda.synchronize()
        assert pipe.sync_status() == cd.CDVS_OK
        np.testing.assert_array_equal(pipe.d_mask.cpu().numpy(), m0)
        k1, d1 = pipe.oriented(), pipe.descriptors()
        for i in range(len(imgs)):
            np.testing.assert_array_equal(k1[i][["x", "y", "sigma", "p", "octave", "ix", "iy"]],
                                          k0[i][["x", "y", "sigma", "p", "octave", "ix", "iy"]])
            np.testing.assert_allclose(k1[i]["theta"], k0[i]["theta"], atol=1e-5)
            np.testing.assert_allclose(d1[i], d0[i], atol=1e-5)
        pipe.run_gated(params, tau)   # eager pass between replays
        torch.cuda.synchronize()


def test_gated_capture_arguments_rejected():
    """Capturing the gated pass refuses a threshold outside (0, 1), a null
    buffer and enabled event timing before the capture begins, keeping the
    graph captured earlier; a misaligned pyramid is refused by the recorded
    pyramid call, which ends the capture and leaves no graph."""
    imgs = list(synth.fixed_batch(synth.SEED_BATCH, 1))
    pipe = cd.Pipeline([(640, 480)])
    pipe.upload(imgs)
    pipe.cnn_buffers()
    params = torch.zeros(cd.CNN_PARAMS, dtype=torch.float32, device="cuda")
    pipe.run()
    pipe.capture()
    args = [pipe.d_images, params, 0.5, pipe.d_mask, pipe.d_pyr, pipe.d_kp, pipe.d_count, pipe.d_kp_ori,
            pipe.d_count_ori, pipe.d_desc]
    cases = [(2, 0.0), (2, 1.0), (2, float("nan")), (3, None), (1, None)]
    for idx, val in cases:
        a = list(args)
        a[idx] = val
        with pytest.raises(cd.CdvsError) as e:
            cd.cdvs_graph_capture_gated(pipe.ctx, *a)
        assert e.value.status == cd.CDVS_ERR_ARG, (idx, val)
    cd.cdvs_profile_enable(pipe.ctx, True)
    with pytest.raises(cd.CdvsError) as e:
        cd.cdvs_graph_capture_gated(pipe.ctx, *args)
    assert e.value.status == cd.CDVS_ERR_STATE
    cd.cdvs_profile_enable(pipe.ctx, False)
    # the plain graph captured above is still there and still runs
    k0 = [k.copy() for k in pipe.keypoints()]
    pipe.d_count.zero_()
    pipe.replay()
    torch.cuda.synchronize()
    assert pipe.sync_status() == cd.CDVS_OK
    for a, b in zip(pipe.keypoints(), k0):
        np.testing.assert_array_equal(a, b)
    a = list(args)
    a[4] = pipe.d_pyr[1:]
    with pytest.raises(cd.CdvsError) as e:
        cd.cdvs_graph_capture_gated(pipe.ctx, *a)
    assert e.value.status == cd.CDVS_ERR_ARG
    with pytest.raises(cd.CdvsError) as e:
        pipe.replay()
    assert e.value.status == cd.CDVS_ERR_STATE


def test_gate_leaves_octaves_beyond_its_bits_dense(O32):
    """A 2048x1536 image has octaves 0..6; the mask has bits for octaves 0..5
    only, so octave 6 is always examined densely: an all-ones mask gives
    exactly the plain keypoints, and an all-zeros mask gives the oracle's
    gated detection under the same mask (every keypoint in octave 6)."""
    img = synth.image(synth.SEED_HIRES, 11, 2048, 1536, nblobs=900, smax=40.0)
    pipe, plain, gated, _ = _gated([img], lambda pp: np.full(pp.ncells, 0x3F, dtype=np.uint8), fmax=1.0)
    assert pipe.num_octaves(0) == 7
    np.testing.assert_array_equal(plain[0][_KEYS], gated[0][_KEYS])
    pipe, plain, gated, m = _gated([img], lambda pp: np.zeros(pp.ncells, dtype=np.uint8), fmax=1.0)
    g = gated[0]
    assert len(g) > 0 and np.all(g["octave"] == 6)
    ref, _, _, _ = oracle_stages(O32, img, topk=4096, mask=_image_masks(pipe, m)[0], fmax=1.0)
    r_ref, r_got, _ = rates(ref, g)
    assert r_ref >= KP_RATE and r_got >= KP_RATE
