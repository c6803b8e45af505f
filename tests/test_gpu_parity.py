"""GPU (HIP path through the C ABI) vs the CPU oracle on the same seeded inputs.

Bars:
  * keypoints: >= 99% of oracle keypoints have a GPU keypoint in the same image
    and octave within 0.5 base-image px, and the reverse;
  * descriptors: over matched oriented keypoints (|d theta| <= 1e-2 rad),
    every descriptor is within max |d| <= 1e-3 of the oracle's after
    normalisation -- end to end, or, where the two keypoints' fp32 geometry
    differs enough to move a pixel across the disk edge, at the GPU's own
    (x, y, sigma, theta) (tests/parity.py describe_check); at most 1e-4 of
    the pairs may miss both (an fp32 tie in the nearest-scale-image choice);
  * pyramid planes: max |d| <= 1e-3 on the 0..255 scale against the fp64
    oracle (fp32 sums of <= 25 taps per pass, two passes, values <= 255:
    the accumulated rounding stays near 1e-4).
Decisions are compared against the fp32 oracle build, which takes them in
the kernels' precision.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from parity import KP_RATE, assert_parity, check_images, describe_check, match, rates, summarize

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1705_09776_amd as cd  # noqa: E402

DESC_TOL = 1e-3
DESC_RATE = 0.99
PLANE_TOL = 1e-3


def _run(images, params=None, kp_capacity=None):
    sizes = [(im.shape[1], im.shape[0]) for im in images]
    pipe = cd.Pipeline(sizes, params=params, kp_capacity=kp_capacity)
    pipe.upload(images)
    pipe.run()
    torch.cuda.synchronize()
    assert pipe.sync_status() == cd.CDVS_OK
    return pipe


def _oracle_stages(O, img, topk=None):
    """Oracle detection (top-k, canonical) and oriented records + descriptors."""
    H, W = img.shape
    _, flat = O.pyramid(img)
    cand = O.detect(flat, W, H)
    alive = O.dedup(cand)
    sel = O.select(cand, alive, topk)
    ori = O.orient(flat, W, H, sel)
    desc = O.describe(flat, W, H, ori)
    return sel, ori, desc, flat


@pytest.fixture(scope="module")
def single():
    img = synth.image(synth.SEED_SINGLE, 0, 640, 480)
    pipe = _run([img])
    return img, pipe


@pytest.fixture(scope="module")
def single_oracle(single, O32):
    img, _ = single
    return _oracle_stages(O32, img)


def test_pyramid_planes_match_oracle(single, O64):
    img, pipe = single
    octs, _ = O64.pyramid(img)
    assert pipe.num_octaves(0) == len(octs) == 5
    worst = 0.0
    for o, planes in enumerate(octs):
        for k in range(5):
            g = pipe.plane(0, o, k)
            assert g.shape == planes[k].shape
            worst = max(worst, float(np.abs(g - planes[k]).max()))
    print("max |G_gpu - G_oracle64| =", worst)
    assert worst <= PLANE_TOL


def test_keypoints_match_oracle(single, single_oracle):
    _, pipe = single
    sel, _, _, _ = single_oracle
    got = pipe.keypoints()[0]
    assert len(got) == len(sel) == 1000
    r_ref, r_got, pairs = rates(sel, got)
    print(f"keypoint match: oracle->gpu {r_ref:.4f}, gpu->oracle {r_got:.4f}")
    assert r_ref >= KP_RATE and r_got >= KP_RATE
    # matched responses and scales agree closely
    dp = np.array([abs(sel["p"][i] - got["p"][j]) / abs(sel["p"][i]) for i, j in pairs])
    ds = np.array([abs(sel["sigma"][i] - got["sigma"][j]) / sel["sigma"][i] for i, j in pairs])
    print(f"rel |dp| p99 {np.quantile(dp, 0.99):.2e}, rel |dsigma| p99 {np.quantile(ds, 0.99):.2e}")
    # sigma* is the root of p'(sigma): its rounding error is dp'/p'', large
    # where the extremum is flat, so it gets a looser bar than p
    assert np.quantile(dp, 0.99) < 1e-3 and np.quantile(ds, 0.99) < 5e-3
    # canonical order
    assert np.all(np.diff(np.abs(got["p"])) <= 0)


def test_descriptors_match_oracle(single, single_oracle, O32):
    """End to end on the single image: every matched descriptor within 1e-3
    of the oracle's, or, where it is not, within 1e-3 of the oracle's
    descriptor at the GPU keypoint's own geometry."""
    img, pipe = single
    _, ori, desc, flat = single_oracle
    got = pipe.oriented()[0]
    gdesc = pipe.descriptors()[0]
    d = describe_check(O32, flat, 640, 480, ori, desc, got, gdesc)
    d.update(r1=1.0, r2=1.0, n_ref=1, n_got=1)
    assert_parity(summarize([d]), "single image")
    assert d["q1"] >= KP_RATE and d["q2"] >= KP_RATE
    np.testing.assert_allclose(np.linalg.norm(gdesc, axis=1), 1.0, atol=1e-5)
    assert gdesc.min() >= 0


def test_orient_and_describe_on_oracle_keypoints(single, single_oracle, O32):
    """Stage isolation: the GPU orients and describes the oracle's own
    keypoints, so records pair one to one."""
    img, _ = single
    pipe = _run([img])
    sel, ori, desc, _ = single_oracle
    rec = np.zeros((1, pipe.kp_capacity), dtype=cd.KP_DTYPE)
    for f in ("x", "y", "sigma", "p", "rho"):
        rec[f][0, :len(sel)] = sel[f]
    rec["p_ss"][0, :len(sel)] = sel["pss"]
    for f in ("image", "octave", "ix", "iy"):
        rec[f][0, :len(sel)] = sel[f]
    pipe.d_kp.copy_(torch.from_numpy(rec.view(np.int32).reshape(1, pipe.kp_capacity, 12)))
    pipe.d_count.fill_(len(sel))
    pipe.orient()
    pipe.describe()
    torch.cuda.synchronize()
    got = pipe.oriented()[0]
    gdesc = pipe.descriptors()[0]
    # same expansion when the orientation peaks agree
    same = 0
    for i in range(min(len(ori), len(got))):
        if (ori["ix"][i], ori["iy"][i], ori["octave"][i]) == (got["ix"][i], got["iy"][i], got["octave"][i]):
            same += 1
    assert same >= 0.99 * len(ori)
    r_ref, r_got, pairs = rates(ori, got, oriented=True, tol_theta=1e-3)
    assert r_ref >= KP_RATE and r_got >= KP_RATE
    err = np.array([np.abs(desc[i] - gdesc[j]).max() for i, j in pairs])
    print(f"isolated descriptor max|d|: max {err.max():.2e} mean {err.mean():.2e}")
    assert np.mean(err <= DESC_TOL) >= DESC_RATE


def test_full_batch_every_image(O32):
    """256 x 640x480 in one context (the benchmark's launch configuration),
    every image against the oracle."""
    n = 256
    imgs = synth.fixed_batch(synth.SEED_BATCH, n)
    pipe = _run(list(imgs))
    kps, oris, descs = pipe.keypoints(), pipe.oriented(), pipe.descriptors()
    for i in range(n):
        assert len(kps[i]) == 1000 and len(oris[i]) == 1000
        assert np.all(kps[i]["image"] == i)
        assert np.all(np.diff(np.abs(kps[i]["p"])) <= 0)
        np.testing.assert_allclose(np.linalg.norm(descs[i], axis=1), 1.0, atol=1e-5)
    assert_parity(summarize(check_images(O32, list(imgs), kps, oris, descs)), "256-image batch")


def test_ragged_batch_equals_single_runs(O32):
    imgs = synth.ragged_batch(synth.SEED_RAGGED, 6)
    batch = _run(imgs)
    bk, bo, bd = batch.keypoints(), batch.oriented(), batch.descriptors()
    for i, im in enumerate(imgs):
        one = _run([im])
        k1, o1, d1 = one.keypoints()[0], one.oriented()[0], one.descriptors()[0]
        for f in ("x", "y", "sigma", "p", "octave", "ix", "iy"):
            np.testing.assert_array_equal(bk[i][f], k1[f])
        np.testing.assert_array_equal(bo[i]["octave"], o1["octave"])
        np.testing.assert_allclose(bo[i]["theta"], o1["theta"], atol=1e-5)
        np.testing.assert_allclose(bd[i], d1, atol=1e-5)
    # and the ragged images agree with the oracle
    for i in (0, 3):
        sel, ori, desc, _ = _oracle_stages(O32, imgs[i])
        r1, r2, _ = rates(sel, bk[i])
        assert min(r1, r2) >= KP_RATE


def test_edge_cases(O32):
    rng = np.random.default_rng(1)
    tiny = rng.integers(0, 256, size=(16, 16), dtype=np.uint8)
    odd = synth.image(21, 0, 97, 61, nblobs=10)
    flat = np.full((64, 80), 117, dtype=np.uint8)
    pipe = _run([tiny, odd, flat])
    kps, oris = pipe.keypoints(), pipe.oriented()
    assert len(kps[2]) == 0 and len(oris[2]) == 0
    for i, im in enumerate([tiny, odd]):
        sel, ori, _, _ = _oracle_stages(O32, im)
        r1, r2, _ = rates(sel, kps[i])
        assert abs(len(sel) - len(kps[i])) <= max(1, 0.01 * len(sel))
        if len(sel):
            assert min(r1, r2) >= 0.95
    assert pipe.num_octaves(0) == 1 and pipe.num_octaves(1) == 2


def test_small_topk(O32):
    p = cd.default_params()
    p.topk = 10
    img = synth.image(synth.SEED_SINGLE, 0, 640, 480)
    pipe = _run([img], params=p, kp_capacity=16)
    got = pipe.keypoints()[0]
    assert len(got) == 10 and len(pipe.oriented()[0]) == 10
    sel, _, _, _ = _oracle_stages(O32, img, topk=10)
    assert [tuple(r) for r in sel[["octave", "ix", "iy"]]] == [tuple(r) for r in got[["octave", "ix", "iy"]]]


@pytest.mark.parametrize("cap", [1, 7])
def test_small_capacities_per_image(O32, cap):
    """Keypoint capacities of 1 (the slot divider's identity case) and 7 (a
    general divisor) over a batch of three images: each image's top-k
    matches the oracle's, and its oriented records and descriptors are
    those of the same image run alone, so no slot lands in another image."""
    p = cd.default_params()
    p.topk = cap
    imgs = list(synth.fixed_batch(synth.SEED_BATCH, 3))
    pipe = _run(imgs, params=p, kp_capacity=cap)
    for i, img in enumerate(imgs):
        got = pipe.keypoints()[i]
        sel, _, _, _ = _oracle_stages(O32, img, topk=cap)
        assert [tuple(r) for r in sel[["octave", "ix", "iy"]]] == [tuple(r) for r in got[["octave", "ix", "iy"]]]
        alone = _run([img], params=p, kp_capacity=cap)
        fields = [f for f in cd.KP_DTYPE.names if f != "image"]   # the batch index differs
        np.testing.assert_array_equal(pipe.oriented()[i][fields], alone.oriented()[0][fields])
        assert np.all(pipe.oriented()[i]["image"] == i)
        np.testing.assert_array_equal(pipe.descriptors()[i], alone.descriptors()[0])


def test_repeatable(single):
    img, _ = single
    pipe = _run([img])
    k1 = pipe.keypoints()[0].copy()
    d1 = pipe.descriptors()[0].copy()
    pipe.run()
    torch.cuda.synchronize()
    k2 = pipe.keypoints()[0]
    np.testing.assert_array_equal(k1[["x", "y", "sigma", "p", "octave", "ix", "iy"]],
                                  k2[["x", "y", "sigma", "p", "octave", "ix", "iy"]])
    np.testing.assert_allclose(pipe.descriptors()[0], d1, atol=1e-6)


def test_graph_replay_equals_eager():
    """The captured pass (kernel nodes only) replayed several times, with
    eager work on the same buffers in between, reproduces the eager run."""
    imgs = list(synth.fixed_batch(synth.SEED_BATCH, 4))
    pipe = _run(imgs)
    k0 = [k.copy() for k in pipe.oriented()]
    d0 = [d.copy() for d in pipe.descriptors()]
    pipe.capture()
    for r in range(3):
        for t in (pipe.d_kp, pipe.d_count, pipe.d_kp_ori, pipe.d_count_ori, pipe.d_desc, pipe.d_pyr):
            t.zero_()
        torch.cuda.synchronize()
        pipe.replay()
        torch.cuda.synchronize()
        assert pipe.sync_status() == cd.CDVS_OK
        k1, d1 = pipe.oriented(), pipe.descriptors()
        for i in range(len(imgs)):
            np.testing.assert_array_equal(k1[i][["x", "y", "sigma", "p", "octave", "ix", "iy"]],
                                          k0[i][["x", "y", "sigma", "p", "octave", "ix", "iy"]])
            np.testing.assert_allclose(k1[i]["theta"], k0[i]["theta"], atol=1e-5)
            np.testing.assert_allclose(d1[i], d0[i], atol=1e-5)
        pipe.run()          # eager pass between replays
        torch.cuda.synchronize()


def test_scale_tile_variants_identical(tmp_path):
    """Every tile shape of the scale-plane kernel writes the same planes bit
    for bit (ragged sizes, so each shape has partial tiles), and the
    autotuner picks one of them, caches it and reads the cache back."""
    imgs = [synth.image(synth.SEED_RAGGED, i, w, h, nblobs=40)
            for i, (w, h) in enumerate([(640, 480), (333, 217), (97, 61), (480, 640)])]
    pipe = cd.Pipeline([(im.shape[1], im.shape[0]) for im in imgs])
    pipe.upload(imgs)
    ref = None
    for v in range(cd.TUNE_VARIANTS):
        cd.cdvs_tune_set(pipe.ctx, cd.KERNEL_SCALES, v)
        pipe.d_pyr.fill_(float("nan"))
        pipe.pyramid()
        torch.cuda.synchronize()
        got = pipe.d_pyr.cpu().numpy().view(np.uint32)
        if ref is None:
            ref = got.copy()
        else:
            np.testing.assert_array_equal(got, ref, err_msg=f"variant {v}")
    cache = str(tmp_path / "tune.json")
    cd.cdvs_autotune(pipe.ctx, pipe.d_images, pipe.d_pyr, cache)
    v = cd.cdvs_tune_get(pipe.ctx, cd.KERNEL_SCALES)
    dv = cd.cdvs_tune_get(pipe.ctx, cd.KERNEL_DETECT)
    assert 0 <= v < cd.TUNE_VARIANTS and 0 <= dv < cd.DETECT_VARIANTS
    import json
    entries = json.load(open(cache))
    e = list(entries.values())[0]
    assert len(entries) == 1 and e["variant"] == v and e["detect"] == dv and len(e["detect_us"]) == cd.DETECT_VARIANTS
    cd.cdvs_tune_set(pipe.ctx, cd.KERNEL_SCALES, (v + 1) % cd.TUNE_VARIANTS)
    cd.cdvs_tune_set(pipe.ctx, cd.KERNEL_DETECT, (dv + 1) % cd.DETECT_VARIANTS)
    cd.cdvs_autotune(pipe.ctx, pipe.d_images, pipe.d_pyr, cache)   # cache hit
    assert cd.cdvs_tune_get(pipe.ctx, cd.KERNEL_SCALES) == v
    assert cd.cdvs_tune_get(pipe.ctx, cd.KERNEL_DETECT) == dv
    # a corrupt cache is replaced by a valid one
    bad = str(tmp_path / "bad.json")
    open(bad, "w").write("not json {\n\"x\": }\n")
    cd.cdvs_autotune(pipe.ctx, pipe.d_images, pipe.d_pyr, bad)
    assert len(json.load(open(bad))) == 1


def test_ragged_1024_every_image(O32):
    """The uneven-size workload at its full size (1024 images, one packed
    context, captured graph, autotuned tile shape), every image against the
    oracle."""
    imgs = synth.ragged_batch(synth.SEED_RAGGED, 1024)
    pipe = cd.Pipeline([(im.shape[1], im.shape[0]) for im in imgs])
    pipe.upload(imgs)
    cd.cdvs_autotune(pipe.ctx, pipe.d_images, pipe.d_pyr, None)
    pipe.capture()
    pipe.replay()
    torch.cuda.synchronize()
    assert pipe.sync_status() == cd.CDVS_OK
    kps, oris, descs = pipe.keypoints(), pipe.oriented(), pipe.descriptors()
    for i in range(len(imgs)):
        assert 0 < len(kps[i]) <= 1000 and len(oris[i]) <= 1000
        assert np.all(kps[i]["image"] == i)
        assert np.all(np.diff(np.abs(kps[i]["p"])) <= 0)
        np.testing.assert_allclose(np.linalg.norm(descs[i], axis=1), 1.0, atol=1e-5)
    assert_parity(summarize(check_images(O32, imgs, kps, oris, descs)), "1024-image ragged batch")


def test_misaligned_pyramid_rejected():
    """Host-side argument checks: a pyramid pointer off the 256-byte
    alignment is refused by every call that reads it, before any launch."""
    pipe = cd.Pipeline([(64, 48)])
    bad = pipe.d_pyr[1:]
    for call in (lambda: cd.cdvs_pyramid(pipe.ctx, pipe.d_images, bad),
                 lambda: cd.cdvs_alp_detect(pipe.ctx, bad, None, pipe.d_kp, pipe.d_count),
                 lambda: cd.cdvs_orient(pipe.ctx, bad, pipe.d_kp, pipe.d_count, pipe.d_kp_ori, pipe.d_count_ori),
                 lambda: cd.cdvs_describe(pipe.ctx, bad, pipe.d_kp_ori, pipe.d_count_ori, pipe.d_desc)):
        with pytest.raises(cd.CdvsError) as e:
            call()
        assert e.value.status == cd.CDVS_ERR_ARG


def _lattice(W, H, period):
    """128 + 100 sin(2 pi x / period) sin(2 pi y / period): four blob-like
    extrema per period squared, far denser than natural images."""
    y, x = np.mgrid[0:H, 0:W]
    v = 128 + 100 * np.sin(2 * np.pi * x / period) * np.sin(2 * np.pi * y / period)
    return np.clip(np.rint(v), 0, 255).astype(np.uint8)


@pytest.fixture(scope="module")
def large(O32):
    """A 4096x4096 image: ~58k candidates, more than the 8192 that stage C
    and the top-k hold per image, so the GPU first keeps the 8192 strongest."""
    img = synth.image(synth.SEED_SINGLE, 1, 4096, 4096, nblobs=2000)
    _, flat = O32.pyramid(img)
    cand = O32.detect(flat, 4096, 4096, cap=1 << 18)
    assert 8192 < len(cand) < (1 << 18)
    alive = O32.dedup(cand)
    return img, cand, alive


def test_large_image_strongest_selection_exact(large, O32):
    img, cand, alive = large
    sel = O32.select(cand, alive)
    pipe = _run([img])   # asserts CDVS_OK: the top-1000 was provably exact
    assert pipe.candidate_capacity() >= len(cand)
    got = pipe.keypoints()[0]
    assert len(got) == len(sel) == 1000
    r_ref, r_got, _ = rates(sel, got)
    print(f"4096x4096: {len(cand)} candidates, match {r_ref:.4f} / {r_got:.4f}")
    assert r_ref >= KP_RATE and r_got >= KP_RATE
    assert np.all(np.diff(np.abs(got["p"])) <= 0)


def test_large_image_inexact_topk_latched(large, O32):
    """topk = 8192 on that image reaches the weakest of the 8192 strongest
    candidates: the result is flagged, and what is written is still the
    exact ranking down to the selection threshold."""
    img, cand, alive = large
    p = cd.default_params()
    p.topk = 8192
    pipe = cd.Pipeline([(4096, 4096)], params=p, kp_capacity=8192)
    pipe.upload([img])
    pipe.run()
    assert pipe.sync_status() == cd.CDVS_ERR_CAPACITY
    assert pipe.sync_status() == cd.CDVS_OK   # the latch was cleared
    got = pipe.keypoints()[0]
    thr = np.sort(np.abs(cand["p"]))[::-1][8191]
    ref = O32.select(cand, alive, 8192)
    ref = ref[np.abs(ref["p"]) > thr * (1 + 1e-3)]
    got = got[np.abs(got["p"]) > thr * (1 + 1e-3)]
    r_ref, r_got, _ = rates(ref, got)
    print(f"above threshold: {len(ref)} oracle, {len(got)} gpu, match {r_ref:.4f} / {r_got:.4f}")
    assert len(ref) > 4000
    assert r_ref >= KP_RATE and r_got >= KP_RATE


def test_candidate_overflow_latched(O32):
    """A period-11 sine lattice gives ~9800 candidates in 640x480, more than
    its 8192-candidate capacity: the overflow is reported, and every keypoint
    written is one of the oracle's candidates."""
    img = _lattice(640, 480, 11)
    _, flat = O32.pyramid(img)
    cand = O32.detect(flat, 640, 480, cap=1 << 18)
    assert len(cand) > 8192
    pipe = cd.Pipeline([(640, 480)])
    assert pipe.candidate_capacity() == 8192
    pipe.upload([img])
    pipe.run()
    assert pipe.sync_status() == cd.CDVS_ERR_CAPACITY
    got = pipe.keypoints()[0]
    assert len(got) == 1000
    _, r_got, _ = rates(cand, got)
    assert r_got >= KP_RATE


def test_max_side_images(O32):
    """The longest sides the library accepts (8192) in a ragged pair."""
    a = synth.image(synth.SEED_SINGLE, 2, 8192, 64, nblobs=100)
    b = synth.image(synth.SEED_SINGLE, 3, 64, 8192, nblobs=100)
    pipe = _run([a, b])
    kps = pipe.keypoints()
    for i, im in enumerate([a, b]):
        sel, _, _, _ = _oracle_stages(O32, im)
        assert len(sel) > 100
        r1, r2, _ = rates(sel, kps[i])
        assert min(r1, r2) >= KP_RATE
        assert pipe.num_octaves(i) == O32.num_octaves(im.shape[1], im.shape[0])


@pytest.mark.parametrize("gated", [False, True])
def test_detect_launch_forms_identical(gated):
    """Both launch forms of the detection (one wave per strip; persistent
    with per-XCD work counters) give the same keypoints, plain and gated, on
    a ragged batch (partial strips, several octaves)."""
    imgs = [synth.image(synth.SEED_RAGGED, i, w, h, nblobs=60)
            for i, (w, h) in enumerate([(640, 480), (333, 217), (97, 61), (480, 640), (1280, 96)])]
    pipe = cd.Pipeline([(im.shape[1], im.shape[0]) for im in imgs])
    pipe.upload(imgs)
    pipe.pyramid()
    mask = None
    if gated:
        rng = np.random.default_rng(5)
        ncell = cd.cdvs_cnn_cells(pipe.ctx)
        mask = torch.from_numpy(rng.integers(0, 256, size=ncell, dtype=np.uint8)).cuda()
    got = []
    for v in range(cd.DETECT_VARIANTS):
        cd.cdvs_tune_set(pipe.ctx, cd.KERNEL_DETECT, v)
        pipe.d_kp.zero_()
        pipe.detect(mask=mask)
        torch.cuda.synchronize()
        assert pipe.sync_status() == cd.CDVS_OK
        got.append(pipe.keypoints())
    for a, b in zip(got[0], got[1]):
        assert len(a) == len(b) > 0
        for f in ("x", "y", "sigma", "p", "octave", "ix", "iy"):
            np.testing.assert_array_equal(a[f], b[f])


def test_persistent_detection_matches_oracle(O32):
    """The persistent launch form on its own against the oracle (same bars as
    the one-wave-per-strip form), on ragged sizes."""
    imgs = [synth.image(synth.SEED_RAGGED, 20 + i, w, h, nblobs=120)
            for i, (w, h) in enumerate([(640, 480), (333, 217), (480, 640)])]
    pipe = cd.Pipeline([(im.shape[1], im.shape[0]) for im in imgs])
    pipe.upload(imgs)
    cd.cdvs_tune_set(pipe.ctx, cd.KERNEL_DETECT, 1)
    pipe.run()
    torch.cuda.synchronize()
    assert pipe.sync_status() == cd.CDVS_OK
    for im, got in zip(imgs, pipe.keypoints()):
        sel, _, _, _ = _oracle_stages(O32, im)
        r_ref, r_got, _ = rates(sel, got)
        assert r_ref >= KP_RATE and r_got >= KP_RATE, (im.shape, r_ref, r_got)


def test_keypoints_outside_the_histogram_bounds(single, single_oracle):
    """Caller-supplied records the histogram kernels cannot take (scale in
    octave units above 2 sigma0 -- the bound the fixed-point histograms are
    sized for --, zero scale, a non-finite position, an octave out of range)
    get no orientation and an all-zero descriptor; a valid record among them
    is unaffected."""
    img, _ = single
    pipe = _run([img])
    sel = single_oracle[0]
    good = sel[0]
    rec = np.zeros((1, pipe.kp_capacity), dtype=cd.KP_DTYPE)

    def put(j, **kw):
        for f in ("x", "y", "sigma", "p", "rho", "octave", "ix", "iy"):
            rec[f][0, j] = good[f]
        for f, v in kw.items():
            rec[f][0, j] = v

    o = int(good["octave"])
    put(0)
    put(1, sigma=3.3 * 2 ** o)
    put(2, sigma=0.0)
    put(3, x=np.float32("nan"))
    put(4, octave=20)
    put(5)
    pipe.d_kp.copy_(torch.from_numpy(rec.view(np.int32).reshape(1, pipe.kp_capacity, 12)))
    pipe.d_count.fill_(6)
    pipe.d_kp_ori.zero_()
    pipe.orient()
    torch.cuda.synchronize()
    ori = pipe.oriented()[0]
    n1 = len(ori) // 2
    assert len(ori) == 2 * n1 and n1 >= 1
    np.testing.assert_array_equal(ori["x"][:n1], ori["x"][n1:])
    # the same records as oriented input to the descriptor kernel
    for j in range(6):
        rec["theta"][0, j] = 0.5
    pipe.d_kp_ori.copy_(torch.from_numpy(rec.view(np.int32).reshape(1, pipe.kp_capacity, 12)))
    pipe.d_count_ori.fill_(6)
    pipe.d_desc.fill_(7.0)
    pipe.describe()
    torch.cuda.synchronize()
    d = pipe.descriptors()[0]
    assert abs(np.linalg.norm(d[0]) - 1) < 1e-5
    np.testing.assert_array_equal(d[0], d[5])
    assert np.all(d[1:5] == 0)
