"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/cdvs.h declares, and rejects bad arguments on the host."""
import ctypes
import os
import re

import pytest

import paper_1705_09776_amd as cd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "cdvs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cdvs_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert _declared_functions() == sorted(cd.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = cd.lib()
    for name in _declared_functions():
        assert hasattr(L, name), name
    out = os.popen(f"nm -D --defined-only {cd.LIB_PATH}").read()
    for name in _declared_functions():
        assert re.search(rf"\bT {name}\b", out), name


def test_struct_sizes():
    assert ctypes.sizeof(cd.Params) == 76
    assert ctypes.sizeof(cd.ImageDesc) == 24
    assert cd.KP_DTYPE.itemsize == 48


def test_default_params():
    p = cd.default_params()
    assert p.version == cd.CDVS_PARAMS_VERSION
    assert abs(p.sigma0 - 1.6) < 1e-7 and p.intervals == 4 and p.min_side == 32
    assert abs(p.contrast - 1.5) < 1e-7 and p.border == 4 and p.topk == 1000
    assert abs(p.ori_radius - 3.96) < 1e-6 and abs(p.ori_peak - 0.8) < 1e-7 and p.max_ori == 4
    assert p.desc_cell == 3 and p.desc_radius == 6 and abs(p.desc_clamp - 0.2) < 1e-7
    assert abs(p.mask_fmax - 0.6) < 1e-7


def test_defaults_agree_with_oracle_constants():
    import oracle
    o = oracle.Oracle.default_params()
    p = cd.default_params()
    for f in ["sigma0", "intervals", "min_side", "contrast", "edge_r", "border", "max_offset", "dedup_dlog2",
              "ori_radius", "ori_wsigma", "ori_peak", "max_ori", "topk", "desc_cell", "desc_radius",
              "desc_wsigma", "desc_clamp"]:
        assert abs(getattr(o, f) - getattr(p, f)) < 1e-6, f


def _desc(w=640, h=480, pitch=None, off=0):
    return cd.ImageDesc(off, w, h, pitch or w, 0)


@pytest.mark.parametrize("mutate,code", [
    (lambda p, d: setattr(p, "version", 7), cd.CDVS_ERR_VERSION),
    (lambda p, d: setattr(p, "sigma0", 1.5), cd.CDVS_ERR_ARG),
    (lambda p, d: setattr(p, "intervals", 3), cd.CDVS_ERR_ARG),
    (lambda p, d: setattr(p, "border", 0), cd.CDVS_ERR_ARG),
    (lambda p, d: setattr(p, "max_ori", 5), cd.CDVS_ERR_ARG),
    (lambda p, d: setattr(p, "topk", 5000), cd.CDVS_ERR_ARG),
    (lambda p, d: setattr(p, "ori_peak", 0.0), cd.CDVS_ERR_ARG),
    (lambda p, d: setattr(p, "mask_fmax", 1.5), cd.CDVS_ERR_ARG),
    (lambda p, d: d.__setitem__(0, _desc(15, 480)), cd.CDVS_ERR_SHAPE),
    (lambda p, d: d.__setitem__(0, _desc(640, 8193)), cd.CDVS_ERR_SHAPE),
    (lambda p, d: d.__setitem__(0, _desc(640, 480, pitch=600)), cd.CDVS_ERR_SHAPE),
    (lambda p, d: d.__setitem__(0, _desc(640, 480, off=-1)), cd.CDVS_ERR_SHAPE),
])
def test_validation_errors(mutate, code):
    p = cd.default_params()
    d = [_desc()]
    mutate(p, d)
    st, msg = cd.cdvs_validate(p, d, 1000)
    assert st == code and msg
    # cdvs_ctx_create validates before it touches any device
    with pytest.raises(cd.CdvsError) as e:
        cd.cdvs_ctx_create(p, d, 1000)
    assert e.value.status == code


def test_validation_counts():
    p = cd.default_params()
    assert cd.cdvs_validate(p, [_desc()], 1000)[0] == cd.CDVS_OK
    assert cd.cdvs_validate(p, [_desc()], 0)[0] == cd.CDVS_ERR_SHAPE
    assert cd.cdvs_validate(p, [_desc()], 9000)[0] == cd.CDVS_ERR_SHAPE
    assert cd.cdvs_validate(p, [], 1000)[0] == cd.CDVS_ERR_SHAPE
    L = cd.lib()
    assert L.cdvs_validate(None, None, 1, 1000, None, 0) == cd.CDVS_ERR_ARG
    assert L.cdvs_validate(ctypes.byref(p), None, 1, 1000, None, 0) == cd.CDVS_ERR_ARG
    # null context
    assert L.cdvs_pyramid(None, None, None, None) == cd.CDVS_ERR_STATE
    assert L.cdvs_sync_status(None, None) == cd.CDVS_ERR_STATE
    assert L.cdvs_pyramid_bytes(None) == -1


def test_pack_images():
    import numpy as np
    a = np.arange(20 * 17, dtype=np.uint8).reshape(17, 20)
    b = np.ones((30, 70), dtype=np.uint8)
    buf, descs = cd.pack_images([a, b])
    assert descs[0].pitch == 64 and descs[1].pitch == 128 and descs[1].offset == 64 * 17
    np.testing.assert_array_equal(buf[:64 * 17].reshape(17, 64)[:, :20], a)


def test_tune_api_host_checks():
    L = cd.lib()
    assert L.cdvs_tune_get(None, cd.KERNEL_SCALES) == -1
    assert L.cdvs_tune_get(None, cd.KERNEL_DETECT) == -1
    assert L.cdvs_tune_set(None, cd.KERNEL_DETECT, 1) == cd.CDVS_ERR_STATE
    assert L.cdvs_tune_set(None, cd.KERNEL_SCALES, 0) == cd.CDVS_ERR_STATE
    assert L.cdvs_autotune(None, None, None, None, None) == cd.CDVS_ERR_STATE


def test_standin_consumer_on_host():
    """The stand-in consumer is host code: check its coding and bounds."""
    import numpy as np
    L = cd.lib()
    n, cap = 3, 5
    rng = np.random.default_rng(2)
    desc = rng.uniform(0, 0.6, size=(n, cap, 128)).astype(np.float32)
    desc[0, 0, :4] = [0.0, 255.5 / 512, 254.5 / 512, 1.0]
    counts = np.array([5, 2, 0], dtype=np.int32)
    out = np.zeros((2 * n, cap, 128), dtype=np.uint8)
    kept = np.full(2 * n, -1, dtype=np.int32)
    sink = cd.StandinSink(out.ctypes.data, kept.ctypes.data, 2 * n, 4, 2)
    rc = L.cdvs_standin_consume(ctypes.addressof(sink), 1, n, cap, counts.ctypes.data, None, desc.ctypes.data)
    assert rc == 0
    assert list(kept) == [-1, -1, -1, 4, 2, 0]
    q = np.clip(np.floor(desc * np.float32(512) + np.float32(0.5)), 0, 255).astype(np.uint8)
    np.testing.assert_array_equal(out[3, :4], q[0, :4])
    np.testing.assert_array_equal(out[4, :2], q[1, :2])
    assert out[3, 4].max() == 0 and out[5].max() == 0 and out[:3].max() == 0
    assert list(out[3, 0, :4]) == [0, 255, 255, 255]
    # a chunk past the sink's size is refused
    assert L.cdvs_standin_consume(ctypes.addressof(sink), 2, n, cap, counts.ctypes.data, None, desc.ctypes.data) != 0
    assert L.cdvs_stream(None, None, 0, 0, None, None, None, None) == cd.CDVS_ERR_STATE


def test_scfv_noalloc_rejects_arguments_without_a_gpu():
    """The allocation-free SCFV entry point checks its arguments on the host
    before any device call: null pointers, a capacity beyond the maximum,
    an image count out of range and misalignment, each with a message."""
    import ctypes
    import paper_1705_09776_amd as cd
    L = cd.lib()
    m = cd.ScfvModel(16, 16, 16, 16, 16)       # fake, never dereferenced
    fake = ctypes.c_void_p(4096)

    def call(model, desc, n, cap):
        return L.cdvs_scfv_noalloc(model, desc, fake, n, cap, fake, fake, fake, fake, fake, None)

    assert call(None, fake, 1, 100) == cd.CDVS_ERR_ARG
    assert b"null" in L.cdvs_last_error(None)
    assert call(ctypes.byref(m), fake, 1, cd.MAX_KP_CAPACITY + 1) == cd.CDVS_ERR_ARG
    assert b"maximum" in L.cdvs_last_error(None)
    assert call(ctypes.byref(m), fake, -1, 100) == cd.CDVS_ERR_ARG
    assert call(ctypes.byref(m), ctypes.c_void_p(4100), 1, 100) == cd.CDVS_ERR_ARG
    assert b"aligned" in L.cdvs_last_error(None)
    assert call(ctypes.byref(m), fake, 0, 100) == cd.CDVS_OK       # nothing to do, nothing enqueued


def test_front_size_matches_oracle_rule():
    """cdvs_front_size (host logic, no GPU) against the oracle's size rule on
    seeded random sizes and the edges; sizes outside 1..8192 are refused."""
    import numpy as np
    import paper_1705_09776_amd as cd
    from oracle import front as F
    rng = np.random.default_rng(9)
    cases = [(1, 1), (640, 640), (641, 641), (8192, 1), (1, 8192), (8192, 8192), (1281, 961)]
    cases += [tuple(int(v) for v in rng.integers(1, 8193, 2)) for _ in range(2000)]
    for w, h in cases:
        assert cd.cdvs_front_size(w, h) == F.front_size(w, h), (w, h)
    for w, h in ((0, 10), (10, 0), (8193, 10)):
        try:
            cd.cdvs_front_size(w, h)
        except cd.CdvsError as e:
            assert e.status == cd.CDVS_ERR_SHAPE
        else:
            raise AssertionError("accepted an invalid size")
