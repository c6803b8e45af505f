"""The device generator renders the host generator's images byte for byte
(same recipe, same seeds; fixed blob count, drawn blob count, padded pitch)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def _dev(seed, n, w, h, nmin, nmax, smax, first=0, pitch=None):
    pitch = pitch or w
    t = synth.device_batch(seed, n, w, h, nmin, nmax, smax=smax, first=first, pitch=pitch)
    torch.cuda.synchronize()
    return t.cpu().numpy().reshape(n, h, pitch)


def test_fixed_batch_matches_host():
    host = synth.fixed_batch(synth.SEED_BATCH, 3, first=10)
    dev = _dev(synth.SEED_BATCH, 3, 640, 480, 200, 200, 20.0, first=10)
    print("differing bytes:", int((host != dev).sum()))
    np.testing.assert_array_equal(dev, host)


def test_hires_batch_matches_host():
    host = synth.hires_batch(synth.SEED_HIRES, 2, first=7)
    dev = _dev(synth.SEED_HIRES, 2, 1280, 960, 400, 1200, 40.0, first=7)
    print("differing bytes:", int((host != dev).sum()))
    np.testing.assert_array_equal(dev, host)


def test_padded_pitch():
    w, h, pitch = 333, 217, 384
    dev = _dev(9, 2, w, h, 30, 60, 20.0, pitch=pitch)
    lib = synth._load()
    for i in range(2):
        ref = np.empty((h, w), dtype=np.uint8)
        nb = lib.synth_blob_count(9, i, 30, 60)
        assert lib.synth_image(9, i, w, h, w, nb, 2.0, 20.0, 80.0, ref.ctypes.data) == 0
        np.testing.assert_array_equal(dev[i, :, :w], ref)
        assert dev[i, :, w:].max() == 0
