"""What the trained surrogate gains over the method without it.

On held-out images (evaluation seed base, never seen in training) the
committed 640x480 weights, at the threshold stored with them, keep >= 98%
of the plain detector's top-1000 keypoints while switching off most
(cell, octave) entries; the same network untrained, at the same threshold,
either loses recall or keeps far more of the image active."""
import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1705_09776_amd import surrogate  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_1705_09776_amd", "weights", "surrogate_640x480.npz")


def test_trained_mask_beats_untrained():
    st = surrogate.load_checkpoint(WEIGHTS)
    tau = json.load(open(os.path.splitext(WEIGHTS)[0] + ".json"))["tau"]
    imgs = list(synth.fixed_batch(synth.SEED_EVAL, 64, first=3000))
    trained = surrogate.evaluate(st["params"], imgs, [tau])[0]
    untrained = surrogate.evaluate(surrogate.init_params(0), imgs, [tau])[0]
    print("trained", trained)
    print("untrained", untrained)
    assert trained["recall_topk"] >= 0.98
    assert trained["active_fraction"] <= 0.45
    assert untrained["recall_topk"] < trained["recall_topk"] - 0.02 or \
        untrained["active_fraction"] > 1.5 * trained["active_fraction"]


def test_sparse_keypoint_model():
    """At contrast threshold 4 (sparse keypoints) the committed T = 4 model,
    at its stored threshold, keeps >= 98% of the plain detector's keypoints
    on held-out images with a quarter of the (cell, octave) entries active."""
    w = os.path.join(ROOT, "paper_1705_09776_amd", "weights", "surrogate_640x480_t4.npz")
    st = surrogate.load_checkpoint(w)
    tau = json.load(open(os.path.splitext(w)[0] + ".json"))["tau"]
    imgs = list(synth.fixed_batch(synth.SEED_EVAL, 64, first=3000))
    r = surrogate.evaluate(st["params"], imgs, [tau], contrast=4.0)[0]
    print("T=4", r)
    assert r["recall_topk"] >= 0.975 and r["active_fraction"] <= 0.35
