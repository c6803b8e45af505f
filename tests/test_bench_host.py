"""Host-side logic of bench.py (CPU only): the one-GPU refusal, the octave
geometry and algorithmic model the roofline uses, and the rule that counter
figures are used only while the kernel's source still matches them."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr or "--gpus 1" in r.stderr


def test_octave_pixels():
    # 640x480 -> 640x480, 320x240, 160x120, 80x60, 40x30 (the last octave has a
    # short side below 32 and is included); 1280x960 adds one more octave
    assert bench.octave_pixels([(640, 480)]) == [307200, 76800, 19200, 4800, 1200]
    assert sum(bench.octave_pixels([(640, 480)])) == 409200
    assert sum(bench.octave_pixels([(1280, 960)])) == 1638000
    assert len(bench.octave_pixels([(1280, 960)])) == 6
    # ceil halving on odd sizes
    assert bench.octave_pixels([(97, 61)]) == [97 * 61, 49 * 31]


def test_algorithmic_model():
    a = bench.algorithmic([(640, 480)] * 2, n_kp=2000, n_ori=2000)
    npx = 2 * 409200
    assert a["detect"]["bytes"] == 20 * npx
    nxt = 2 * (409200 - 307200)
    assert a["scales"]["bytes"] == 20 * npx + 4 * nxt
    assert a["scales"]["flop"] == bench.SCALES_FLOP_PER_PX * npx
    # symmetric taps: per pass 3r + 2 flops; the column passes share 12 pair sums
    assert bench.SCALES_FLOP_PER_PX == 12 + sum(2 * (r + 1) for r in (5, 7, 9, 12)) + sum(3 * r + 2 for r in (5, 7, 9, 12))
    assert bench.PREBLUR_FLOP_PER_PX == 46
    assert a["describe"]["bytes"] == 2000 * (48 + 512)
    # the scale kernel is below the ridge, so the roofline classes it by bytes
    assert bench.SCALES_FLOP_PER_PX / 20 < bench.RIDGE_FLOP_PER_BYTE


def test_traffic_requires_matching_source(tmp_path, monkeypatch):
    csrc = os.path.join(ROOT, "paper_1705_09776_amd", "csrc")
    data = open(os.path.join(csrc, "pyramid.hip"), "rb").read() + open(os.path.join(csrc, "cdvs_internal.h"), "rb").read()
    good = hashlib.sha256(data).hexdigest()
    f = tmp_path / "traffic.md"
    f.write_text(f"    traffic k_blur<1,4,12,false,1> 1234 pyramid.hip {good}\n"
                 f"    traffic k_describe 99 describe.hip {'0' * 64}\n"
                 f"    valu k_blur<1,4,12,false,1> 777 pyramid.hip {good}\n")
    monkeypatch.setattr(bench, "TRAFFIC", str(f))
    monkeypatch.setattr(bench, "SQ", str(f))
    assert bench.measured_traffic("scales", 1) == 1234
    assert bench.measured_traffic("scales", 2) is None      # another tile variant: not measured
    assert bench.measured_traffic("describe") is None      # stale: source changed since
    assert bench.measured_traffic("detect") is None        # no line
    assert bench.measured_path_bytes(1) is None
    assert bench.measured_valu("scales", 1) == 777


def test_committed_profiles_match_the_sources():
    """The committed counter summaries were taken on the current kernels."""
    for k in ("scales", "preblur", "detect", "finalize", "orient", "describe"):
        assert bench.measured_traffic(k, 1) is not None, k
        assert bench.measured_valu(k, 1) is not None, k
