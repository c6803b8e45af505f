"""cdvs_scfv_noalloc (SCFV with no device allocation, scratch in the
library's static device array) against cdvs_scfv, its context-based form,
and against the float64 oracle, called through the C ABI.

Two calls in a row on the split path (a batch small enough to be split into
parts: the second call has fewer images and fewer descriptors, so stale
partial sums of the first would show), then a batch large enough for the
one-workgroup-per-image path.  The two entry points sum in different orders,
so they agree to single-precision rounding: the bar is the SCFV parity bar,
1e-3 of the image's largest |entry| for the gradients and delta; the order
must sort the call's own delta and rank the other's delta within that
tolerance; sign bits agree wherever the entry is farther than the tolerance
from zero.  The call must not allocate through torch either."""
import os

import numpy as np
import pytest

import synth
from oracle import scfv

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1705_09776_amd as cd  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MODEL = os.path.join(ROOT, "paper_1705_09776_amd", "weights", "scfv_standin.npz")
TOL = 1e-3
CAP = 1000


@pytest.fixture(scope="module")
def model():
    return dict(np.load(MODEL))


def _agree(a, b):
    """a, b: (gm, gv, delta, order, bits) of one image from two sources."""
    gm, gv, dl, order, bits = a
    rgm, rgv, rdl, rorder, _ = b
    gmax, vmax, dmax = np.abs(rgm).max(), np.abs(rgv).max(), rdl.max()
    if gmax == 0:
        assert not gm.any() and not gv.any() and not dl.any()
        np.testing.assert_array_equal(order, np.arange(512))
        return
    assert np.abs(gm - rgm).max() <= TOL * gmax
    assert np.abs(gv - rgv).max() <= TOL * vmax
    assert np.abs(dl - rdl).max() <= TOL * dmax
    np.testing.assert_array_equal(order, scfv.rank(dl))
    assert np.abs(rdl[order] - rdl[rorder]).max() <= TOL * dmax
    for bb, g, gx in ((bits[:, 0], rgm, gmax), (bits[:, 1], rgv, vmax)):
        sure = np.abs(g) > TOL * gx
        got = ((bb[:, None] >> np.arange(32, dtype=np.uint32)[None, :]) & 1).astype(bool)
        np.testing.assert_array_equal(got[sure], (g > 0)[sure])


def _inputs(descs):
    n = len(descs)
    host = np.zeros((n, CAP, 128), dtype=np.float32)
    for i, d in enumerate(descs):
        host[i, :len(d)] = d
    return torch.from_numpy(host).cuda(), torch.tensor([len(d) for d in descs], dtype=torch.int32).cuda()


def _context_form(model, d_desc, d_count, n):
    """The same batch through cdvs_scfv (a context of n small images whose
    capacity is CAP)."""
    pipe = cd.Pipeline([(64, 64)] * n, kp_capacity=CAP)
    S = cd.Scfv(model, n)
    cd.cdvs_scfv(pipe.ctx, S, d_desc, d_count)
    torch.cuda.synchronize()
    return S.outputs()


def _noalloc(S, d_desc, d_count, n):
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated(), torch.cuda.memory_reserved()
    cd.cdvs_scfv_noalloc(S, d_desc, d_count, n, CAP)
    torch.cuda.synchronize()
    assert (torch.cuda.memory_allocated(), torch.cuda.memory_reserved()) == before
    return S.outputs()


def _check_all(got, ref_ctx, descs, model):
    m64 = {k: v.astype(np.float64) for k, v in model.items()}
    for i, d in enumerate(descs):
        _agree(tuple(x[i] for x in got), tuple(x[i] for x in ref_ctx))
        o = scfv.scfv(d.astype(np.float64), m64)
        _agree(tuple(x[i] for x in got), (o["gm"], o["gv"], o["delta"], o["order"], None))


def test_two_calls_split_path(model, O32):
    imgs = synth.fixed_batch(synth.SEED_BATCH, 3)
    full = [O32.run(im)[1].astype(np.float32) for im in imgs]
    # first call: 3 images (1000, 33 and no descriptors) -> split into parts
    descs1 = [full[0], full[1][:33], np.zeros((0, 128), np.float32)]
    assert cd.lib().cdvs_scfv_noalloc is not None
    S = cd.Scfv(model, 3)
    d_desc, d_count = _inputs(descs1)
    got1 = _noalloc(S, d_desc, d_count, 3)
    _check_all(got1, _context_form(model, d_desc, d_count, 3), descs1, model)
    # second call, smaller: 1 image with 200 descriptors (more parts, fewer
    # of them filled), into fresh output buffers
    descs2 = [full[2][:200]]
    S2 = cd.Scfv(model, 1)
    d_desc2, d_count2 = _inputs(descs2)
    got2 = _noalloc(S2, d_desc2, d_count2, 1)
    _check_all(got2, _context_form(model, d_desc2, d_count2, 1), descs2, model)


def test_one_workgroup_per_image_path(model):
    """40 images (above the split limit): one workgroup per image, seeded
    random clamped unit descriptors with ragged counts."""
    rng = np.random.default_rng(11)
    descs = []
    for i in range(40):
        k = int(rng.integers(0, CAP + 1)) if i % 5 else CAP
        d = rng.gamma(0.5, 1.0, (k, 128))
        d /= np.maximum(np.linalg.norm(d, axis=1, keepdims=True), 1e-12)
        d = np.minimum(d, 0.2)
        d /= np.maximum(np.linalg.norm(d, axis=1, keepdims=True), 1e-12)
        descs.append(d.astype(np.float32))
    S = cd.Scfv(model, 40)
    d_desc, d_count = _inputs(descs)
    got = _noalloc(S, d_desc, d_count, 40)
    ref = _context_form(model, d_desc, d_count, 40)
    for i in range(40):
        _agree(tuple(x[i] for x in got), tuple(x[i] for x in ref))


def test_arguments_rejected_before_launch(model):
    S = cd.Scfv(model, 1)
    d_desc, d_count = _inputs([np.zeros((1, 128), np.float32)])
    L = cd.lib()
    st = L.cdvs_scfv_noalloc(cd.ctypes.byref(S.model), cd._ptr(d_desc), cd._ptr(d_count), 1,
                             cd.MAX_KP_CAPACITY + 1, cd._ptr(S.gm), cd._ptr(S.gv), cd._ptr(S.delta),
                             cd._ptr(S.order), cd._ptr(S.bits), None)
    assert st == cd.CDVS_ERR_ARG
    assert b"maximum" in L.cdvs_last_error(None)
