"""Pins for the oracle's gated detection (the learned gate; not part of the
paper): a centre of octave o is examined iff bit o of its 4x4 cell is set,
neighbours are still read in full, an octave whose mask is denser than fmax
(or o >= 6, bits the gate never sets) is examined densely, and stage C runs
afterwards on whatever was found.  Since neighbours are read in full, the
gated candidates must be exactly the plain candidates whose cell bit is set
-- checked here by brute force against the ungated detector."""
import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def scene(O32):
    img = synth.image(synth.SEED_SINGLE, 4, 200, 152, nblobs=40)
    H, W = img.shape
    _, flat = O32.pyramid(img)
    plain = O32.detect(flat, W, H)
    assert len(plain) > 50 and len(np.unique(plain["octave"])) >= 3
    return img, flat, plain


def _key(k):
    return (int(k["octave"]), int(k["ix"]), int(k["iy"]))


def _cell_bit(mask, k):
    o = int(k["octave"])
    return (mask[(int(k["iy"]) << o) >> 2, (int(k["ix"]) << o) >> 2] >> o) & 1


def test_all_ones_mask_is_plain(O32, scene):
    img, flat, plain = scene
    H, W = img.shape
    mask = np.full(((H + 3) // 4, (W + 3) // 4), 0x3F, dtype=np.uint8)
    got = O32.detect_masked(flat, W, H, mask, fmax=2.0)   # never dense by fraction
    np.testing.assert_array_equal(got, plain)


def test_all_zeros_mask_finds_nothing(O32, scene):
    img, flat, _ = scene
    H, W = img.shape
    mask = np.zeros(((H + 3) // 4, (W + 3) // 4), dtype=np.uint8)
    assert len(O32.detect_masked(flat, W, H, mask, fmax=0.6)) == 0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_mask_selects_plain_candidates(O32, scene, seed):
    """Sparse random masks (well under fmax): gated = {plain candidates whose
    cell bit is set}, with identical records (neighbours are read in full)."""
    img, flat, plain = scene
    H, W = img.shape
    rng = np.random.default_rng(seed)
    mask = (rng.random(((H + 3) // 4, (W + 3) // 4, 6)) < 0.3).astype(np.uint8)
    mask = (mask << np.arange(6, dtype=np.uint8)).sum(axis=2).astype(np.uint8)
    got = O32.detect_masked(flat, W, H, mask, fmax=0.6)
    want = plain[np.array([_cell_bit(mask, k) == 1 for k in plain])]
    assert 0 < len(want) < len(plain)
    got_s = got[np.lexsort((got["ix"], got["iy"], got["octave"]))]
    want_s = want[np.lexsort((want["ix"], want["iy"], want["octave"]))]
    np.testing.assert_array_equal(got_s, want_s)


def test_dense_fallback_and_high_octaves(O32, scene):
    """An octave whose active cells exceed fmax of the image's cells is
    examined in full; a mask of exactly fmax is not (strict comparison)."""
    img, flat, plain = scene
    H, W = img.shape
    H4, W4 = (H + 3) // 4, (W + 3) // 4
    ncell = H4 * W4
    mask = np.zeros((H4, W4), dtype=np.uint8)
    flat_mask = mask.reshape(-1)
    n_on = int(0.5 * ncell) + 1                       # just above fmax = 0.5 for octave 0
    flat_mask[:n_on] |= 1
    got = O32.detect_masked(flat, W, H, mask, fmax=0.5)
    assert {_key(k) for k in got} == {_key(k) for k in plain if k["octave"] == 0}
    # exactly at the fraction: gated (only the first n cells)
    mask[:] = 0
    n_eq = ncell // 2 if ncell % 2 == 0 else None
    if n_eq is not None:
        flat_mask[:n_eq] |= 1
        got = O32.detect_masked(flat, W, H, mask, fmax=0.5)
        want = {_key(k) for k in plain if k["octave"] == 0 and _cell_bit(mask, k)}
        assert {_key(k) for k in got} == want


def test_octaves_beyond_the_gate_are_dense(O32):
    """Octaves 6 and up have no gate bit: an all-zero mask still finds every
    plain candidate there (a 2048x2048 image has 8 octaves)."""
    img = synth.image(synth.SEED_SINGLE, 5, 2048, 2048, nblobs=300, smax=60.0)
    _, flat = O32.pyramid(img)
    assert O32.num_octaves(2048, 2048) == 8
    plain = O32.detect(flat, 2048, 2048, cap=1 << 17)
    mask = np.zeros((512, 512), dtype=np.uint8)
    got = O32.detect_masked(flat, 2048, 2048, mask, fmax=0.6, cap=1 << 17)
    assert len(got) == int((plain["octave"] >= 6).sum()) > 0
    assert np.all(got["octave"] >= 6)
