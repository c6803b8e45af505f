"""Front-end downsampling on the GPU (cdvs_front_end) against the oracle
(oracle/front.py).  The output is an integer decision made in exact integer
arithmetic on both sides, so the bar is bit-exact on every pixel.  Covered:
non-integer and integer factors, either side longer, extreme aspect ratios,
images already within 640 (copied), the largest side, a source that does
not fit its context image (latched, the others still written), and the
whole detector run on the GPU's output against the detector run on the
oracle's output (identical inputs give identical keypoints)."""
import numpy as np
import pytest

import synth
from oracle import front as F

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1705_09776_amd as cd  # noqa: E402


def _sources(sizes, seed):
    rng = np.random.default_rng(seed)
    imgs = []
    for (w, h) in sizes:
        if w * h <= 1 << 21:
            imgs.append(rng.integers(0, 256, size=(h, w)).astype(np.uint8))
        else:   # large: a smooth field plus noise, cheaper to draw
            y, x = np.mgrid[0:h, 0:w]
            f = 128 + 60 * np.sin(x / 37.0) * np.cos(y / 23.0) + rng.integers(-20, 21, size=(h, w))
            imgs.append(np.clip(f, 0, 255).astype(np.uint8))
    return imgs


def _run(imgs, out_sizes=None):
    buf, sdesc = cd.pack_images(imgs)
    sizes = out_sizes or [cd.cdvs_front_size(im.shape[1], im.shape[0]) for im in imgs]
    pipe = cd.Pipeline(sizes)
    d_src = torch.from_numpy(buf).cuda()
    d_sd = cd.descs_to_device(sdesc)
    pipe.d_images.fill_(7)
    pipe.front_end(d_src, d_sd)
    st = pipe.sync_status()
    host = pipe.d_images.cpu().numpy()
    outs = [host[d.offset:d.offset + d.pitch * d.height].reshape(d.height, d.pitch)[:, :d.width] for d in pipe.descs]
    return pipe, outs, st


SIZES = [(1280, 960), (1000, 750), (1023, 767), (641, 480), (2000, 3000), (8192, 256), (256, 8192), (640, 480),
         (333, 222), (4096, 4096), (700, 700), (1920, 1080), (8192, 8192)]


def test_bit_exact_against_oracle():
    imgs = _sources(SIZES, 3)
    _, outs, st = _run(imgs)
    assert st == cd.CDVS_OK
    for im, out in zip(imgs, outs):
        ref = F.front(im)
        assert out.shape == ref.shape
        np.testing.assert_array_equal(out, ref, err_msg=f"source {im.shape}")


def test_mismatched_source_latched():
    imgs = _sources([(1280, 960), (1000, 750), (800, 600)], 4)
    sizes = [cd.cdvs_front_size(im.shape[1], im.shape[0]) for im in imgs]
    sizes[1] = (640, 481)                      # not what 1000 x 750 maps to
    _, outs, st = _run(imgs, sizes)
    assert st == cd.CDVS_ERR_SHAPE
    np.testing.assert_array_equal(outs[0], F.front(imgs[0]))
    np.testing.assert_array_equal(outs[2], F.front(imgs[2]))
    assert (outs[1] == 7).all()                # skipped, left untouched


def test_detector_on_front_end_output():
    """High-resolution synthetic scenes (the stream's recipe, 1280x960 and a
    non-integer 1000x750) through the front end, then the whole plain
    pass: the same keypoints and descriptors as the pass over the oracle's
    downsampled images uploaded directly."""
    imgs = [synth.image(synth.SEED_HIRES, i, 1280, 960, nblobs=600, smax=40.0) for i in range(2)]
    imgs.append(synth.image(synth.SEED_HIRES, 2, 1000, 750, nblobs=400, smax=40.0))
    pipe, outs, st = _run(imgs)
    assert st == cd.CDVS_OK
    pipe.run()
    torch.cuda.synchronize()
    kp_a, desc_a = pipe.keypoints(), pipe.descriptors()
    ref = cd.Pipeline(pipe.sizes)
    ref.upload([F.front(im) for im in imgs])
    ref.run()
    torch.cuda.synchronize()
    for a, b in zip(kp_a, ref.keypoints()):
        np.testing.assert_array_equal(a, b)
    for a, b in zip(desc_a, ref.descriptors()):
        np.testing.assert_array_equal(a, b)


def test_bench_configuration_every_image():
    """The benchmark's launch configuration: 256 high-resolution scenes of
    1280x960 rendered on the device, brought to 640x480 in one launch; every
    output image bit-exact against the oracle on its source."""
    W, H, n = 1280, 960, 256
    src = synth.device_batch(synth.SEED_HIRES, n, W, H, 400, 1200, smax=40.0)
    d_sd = cd.descs_to_device([cd.ImageDesc(i * W * H, W, H, W, 0) for i in range(n)])
    wo, ho = cd.cdvs_front_size(W, H)
    pipe = cd.Pipeline([(wo, ho)] * n)
    pipe.front_end(src, d_sd)
    torch.cuda.synchronize()
    assert pipe.sync_status() == cd.CDVS_OK
    host = pipe.d_images.cpu().numpy()
    srch = src.cpu().numpy()
    for i, d in enumerate(pipe.descs):
        out = host[d.offset:d.offset + d.pitch * d.height].reshape(d.height, d.pitch)[:, :d.width]
        ref = F.front(srch[i * W * H:(i + 1) * W * H].reshape(H, W))
        np.testing.assert_array_equal(out, ref, err_msg=f"image {i}")
