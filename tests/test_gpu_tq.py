"""Transform coding and ternary quantisation on the GPU (cdvs_encode) against
the oracle (oracle/tq.py) with the stand-in thresholds.

The code is an integer result decided by single-precision comparisons, and
both sides evaluate the same single-precision expressions, so on the same
descriptors the codes must be bit-identical.  End to end (GPU descriptors
against oracle descriptors of matched keypoints, which agree to 1e-3), a
symbol may differ only where the oracle's transformed value lies within
1e-3 of a threshold (every transformed element moves by at most the
largest change of the bins it combines)."""
import os

import numpy as np
import pytest

import synth
from oracle import tq
from parity import oracle_stages, rates

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1705_09776_amd as cd  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MODEL = os.path.join(ROOT, "paper_1705_09776_amd", "weights", "tq_standin.npz")


@pytest.fixture(scope="module")
def model():
    return dict(np.load(MODEL))


def _encode(model, descs, counts, kp_cap, n_el):
    n = len(descs)
    params = cd.default_params()
    params.topk = min(params.topk, kp_cap)      # the context requires topk <= capacity
    pipe = cd.Pipeline([(64, 64)] * n, params=params, kp_capacity=kp_cap)
    host = np.zeros((n, kp_cap, 128), dtype=np.float32)
    for i, d in enumerate(descs):
        host[i, :len(d)] = d
    pipe.d_desc.copy_(torch.from_numpy(host))
    pipe.d_count_ori.copy_(torch.from_numpy(np.asarray(counts, dtype=np.int32)))
    codes = torch.full((n, kp_cap, 8), -1, dtype=torch.int32, device="cuda")
    cd.cdvs_encode(pipe.ctx, cd.Tq(model), n_el, pipe.d_desc, pipe.d_count_ori, codes)
    torch.cuda.synchronize()
    return codes.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("n_el", [128, 100, 16, 1])
def test_codes_bit_exact_on_oracle_descriptors(model, O32, n_el):
    imgs = synth.fixed_batch(synth.SEED_BATCH, 2)
    d0 = O32.run(imgs[0])[1].astype(np.float32)
    d1 = O32.run(imgs[1])[1].astype(np.float32)[:37]
    got = _encode(model, [d0, d1, np.zeros((0, 128), np.float32)], [len(d0), 37, 0], 1000, n_el)
    np.testing.assert_array_equal(got[0, :len(d0)], tq.encode(d0, model, n_el))
    np.testing.assert_array_equal(got[1, :37], tq.encode(d1, model, n_el))
    assert np.all(got[1, 37:] == 0xFFFFFFFF) and np.all(got[2] == 0xFFFFFFFF)   # untouched


def test_ties_at_the_thresholds(model):
    """Thresholds placed exactly on transformed values: a value equal to a
    threshold codes as 0 on both sides."""
    rng = np.random.default_rng(4)
    d = rng.gamma(0.5, 1.0, (64, 128))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    v = tq.transform(d)
    m = dict(model)
    m["lo"] = v[3].copy()
    m["hi"] = v[5].copy()
    m["lo"], m["hi"] = np.minimum(m["lo"], m["hi"]), np.maximum(m["lo"], m["hi"])
    got = _encode(m, [d], [64], 64, 128)
    np.testing.assert_array_equal(got[0], tq.encode(d, m, 128))
    q = tq.unpack(got[0], m["order"], 128)
    assert np.all(q[3][v[3] == m["lo"]] == 0) and np.all(q[5][v[5] == m["hi"]] == 0)


def test_end_to_end_symbols(model, O32):
    img = synth.image(synth.SEED_SINGLE, 0, 640, 480)
    pipe = cd.Pipeline([(640, 480)])
    pipe.upload([img])
    pipe.run()
    codes = torch.zeros((1, pipe.kp_capacity, 8), dtype=torch.int32, device="cuda")
    cd.cdvs_encode(pipe.ctx, cd.Tq(model), 128, pipe.d_desc, pipe.d_count_ori, codes)
    torch.cuda.synchronize()
    got = pipe.oriented()[0]
    gq = tq.unpack(codes.cpu().numpy().view(np.uint32)[0, :len(got)], model["order"], 128)
    _, ori, desc, _ = oracle_stages(O32, img)
    _, _, pairs = rates(ori, got, oriented=True)
    ia = np.array([p[0] for p in pairs])
    jb = np.array([p[1] for p in pairs])
    close = np.abs(desc[ia] - pipe.descriptors()[0][jb]).max(axis=1) <= 1e-3
    v = tq.transform(desc[ia][close].astype(np.float32)).astype(np.float64)
    rq = tq.quantise(v, model["lo"], model["hi"])
    margin = np.minimum(np.abs(v - model["lo"]), np.abs(v - model["hi"]))
    sure = margin > 1e-3
    print(f"{close.sum()} descriptor pairs within 1e-3; {sure.mean():.4f} of their symbols away from a threshold")
    assert close.sum() >= 0.85 * len(pairs)
    np.testing.assert_array_equal(gq[jb[close]][sure], rq[sure])


def test_bench_configuration_every_image(model):
    """The benchmark's launch configuration: all 128 elements of the 1000
    descriptors of each of the 256 images of the plain pass coded in one
    launch; on the GPU's own descriptors the oracle's codes must come out
    identical for every descriptor."""
    imgs = synth.fixed_batch(synth.SEED_BATCH, 256)
    pipe = cd.Pipeline([(640, 480)] * len(imgs))
    pipe.upload(list(imgs))
    pipe.run()
    codes = torch.full((len(imgs), pipe.kp_capacity, cd.TQ_WORDS), -1, dtype=torch.int32, device="cuda")
    cd.cdvs_encode(pipe.ctx, cd.Tq(model), 128, pipe.d_desc, pipe.d_count_ori, codes)
    torch.cuda.synchronize()
    assert pipe.sync_status() == cd.CDVS_OK
    got = codes.cpu().numpy().view(np.uint32)
    desc = pipe.d_desc.cpu().numpy()
    cnt = pipe.d_count_ori.cpu().numpy()
    assert cnt.min() > 0
    for i in range(len(imgs)):
        np.testing.assert_array_equal(got[i, :cnt[i]], tq.encode(desc[i, :cnt[i]], model, 128), err_msg=f"image {i}")
