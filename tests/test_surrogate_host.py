"""Host-side parts of the surrogate trainer: parameter layout, checkpoints."""
import numpy as np
import pytest

from oracle import cnn
from paper_1705_09776_amd import surrogate


def test_init_params_layout():
    p = surrogate.init_params(3)
    assert p.shape == (cnn.N_PARAMS,) and p.dtype == np.float32
    convs, Wh, bh = cnn.unpack(p)
    for W, b in convs:
        assert np.all(b == 0) and 0.05 < W.std() < 0.2
    assert np.all(bh == -2.0)


def _state(seed=0):
    rng = np.random.default_rng(seed)
    return {"params": rng.normal(size=cnn.N_PARAMS).astype(np.float32),
            "m": rng.normal(size=cnn.N_PARAMS).astype(np.float32),
            "v": rng.random(cnn.N_PARAMS).astype(np.float32),
            "pos_weight": np.array([20, 10, 5, 3, 2, 1], dtype=np.float32),
            "step": np.array([17], dtype=np.int64), "cursor": np.array([544], dtype=np.int64),
            "data_seed": np.array([4], dtype=np.int64)}


def test_checkpoint_round_trip(tmp_path):
    st = _state()
    path = str(tmp_path / "c.npz")
    surrogate.save_checkpoint(path, st)
    back = surrogate.load_checkpoint(path)
    for k in st:
        np.testing.assert_array_equal(back[k], st[k])


def test_checkpoint_corruption_detected(tmp_path):
    st = _state()
    path = str(tmp_path / "c.npz")
    surrogate.save_checkpoint(path, st)
    # rewrite one parameter but keep the old checksum
    with np.load(path) as z:
        d = {k: z[k] for k in z.files}
    d["params"] = d["params"].copy()
    d["params"][100] += 1.0
    np.savez(path, **d)
    with pytest.raises(ValueError):
        surrogate.load_checkpoint(path)
