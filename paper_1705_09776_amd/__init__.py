"""Python binding of the gfx950 CDVS front-half library (libcdvs.so).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch provides device memory and streams.  The functions keep the
names of the C ABI (include/cdvs.h); ``Pipeline`` owns the buffers of one
batch layout and runs the four stages.

Importing this package never compiles anything; ``build()`` does.  If the
library has not been built, ``lib()`` raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcdvs.so")
_lib = None

CDVS_OK = 0
CDVS_ERR_ARG = -1
CDVS_ERR_SHAPE = -2
CDVS_ERR_CAPACITY = -3
CDVS_ERR_HIP = -4
CDVS_ERR_STATE = -5
CDVS_ERR_VERSION = -6
CDVS_PARAMS_VERSION = 2
CNN_PARAMS = 9382
CNN_CHANNELS = 16
CNN_HEADS = 6
CNN_LAYERS = 4
DESC_DIM = 128
MAX_KP_CAPACITY = 8192      # CDVS_MAX_KP_CAPACITY

_STATUS = {0: "CDVS_OK", -1: "CDVS_ERR_ARG", -2: "CDVS_ERR_SHAPE", -3: "CDVS_ERR_CAPACITY",
           -4: "CDVS_ERR_HIP", -5: "CDVS_ERR_STATE", -6: "CDVS_ERR_VERSION"}


class CdvsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("version", ctypes.c_int32), ("sigma0", ctypes.c_float), ("intervals", ctypes.c_int32),
                ("min_side", ctypes.c_int32), ("contrast", ctypes.c_float), ("edge_r", ctypes.c_float),
                ("border", ctypes.c_int32), ("max_offset", ctypes.c_float), ("dedup_dlog2", ctypes.c_float),
                ("ori_radius", ctypes.c_float), ("ori_wsigma", ctypes.c_float), ("ori_peak", ctypes.c_float),
                ("max_ori", ctypes.c_int32), ("desc_cell", ctypes.c_float), ("desc_radius", ctypes.c_float),
                ("desc_wsigma", ctypes.c_float), ("desc_clamp", ctypes.c_float), ("topk", ctypes.c_int32),
                ("mask_fmax", ctypes.c_float)]


class ImageDesc(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("pitch", ctypes.c_int32), ("reserved", ctypes.c_int32)]


# 48-byte cdvs_keypoint
KP_DTYPE = np.dtype([("x", "f4"), ("y", "f4"), ("sigma", "f4"), ("p", "f4"), ("theta", "f4"),
                     ("rho", "f4"), ("p_ss", "f4"), ("peak", "f4"), ("image", "i4"), ("octave", "i4"),
                     ("ix", "i4"), ("iy", "i4")])
assert KP_DTYPE.itemsize == 48

# Every symbol include/cdvs.h declares.
EXPORTS = ["cdvs_default_params", "cdvs_validate", "cdvs_ctx_create", "cdvs_ctx_destroy", "cdvs_last_error",
           "cdvs_pyramid_bytes", "cdvs_num_octaves", "cdvs_plane_layout", "cdvs_pyramid", "cdvs_alp_detect",
           "cdvs_orient", "cdvs_describe", "cdvs_sync_status", "cdvs_candidate_capacity",
           "cdvs_graph_capture", "cdvs_graph_capture_gated", "cdvs_graph_launch", "cdvs_profile_enable",
           "cdvs_profile_read",
           "cdvs_cnn_cells", "cdvs_cnn_cell_layout", "cdvs_cnn_forward", "cdvs_cnn_labels", "cdvs_cnn_backward",
           "cdvs_cnn_adam", "cdvs_autotune", "cdvs_tune_get", "cdvs_tune_set",
           "cdvs_stream", "cdvs_standin_consume", "cdvs_scfv", "cdvs_scfv_noalloc", "cdvs_encode", "cdvs_front_size", "cdvs_front_end", "cdvs_pyramid_bmlog",
           "cdvs_relevance_select"]
TUNE_VARIANTS = 4
DETECT_VARIANTS = 2

KERNEL_SCALES = 1
KERNEL_DETECT = 3
KERNEL_NAMES = ["preblur", "scales", "clear", "detect", "finalize", "orient", "orient_compact", "describe",
                "cnn_forward", "mask_count", "scfv", "encode", "relevance", "front", "bmlog"]
TQ_WORDS = 8
SCFV_COMPONENTS = 512
SCFV_DIM = 32


class RelevanceModel(ctypes.Structure):
    _fields_ = [("d_edges", ctypes.c_void_p), ("d_values", ctypes.c_void_p)]


class TqModel(ctypes.Structure):
    _fields_ = [("d_lo", ctypes.c_void_p), ("d_hi", ctypes.c_void_p), ("d_order", ctypes.c_void_p)]


class ScfvModel(ctypes.Structure):
    _fields_ = [("d_pca_mean", ctypes.c_void_p), ("d_pca_matrix", ctypes.c_void_p), ("d_weights", ctypes.c_void_p),
                ("d_means", ctypes.c_void_p), ("d_variances", ctypes.c_void_p)]


def build() -> str:
    from . import hipbuild
    return hipbuild.build()


def lib():
    """The loaded libcdvs.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1705_09776_amd.hipbuild`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    P = ctypes.POINTER(Params)
    sig = {
        "cdvs_default_params": (Params, []),
        "cdvs_validate": (i32, [P, ctypes.POINTER(ImageDesc), i32, i32, ctypes.c_char_p, i32]),
        "cdvs_ctx_create": (i32, [P, ctypes.POINTER(ImageDesc), i32, i32, ctypes.POINTER(vp)]),
        "cdvs_ctx_destroy": (None, [vp]),
        "cdvs_last_error": (ctypes.c_char_p, [vp]),
        "cdvs_pyramid_bytes": (i64, [vp]),
        "cdvs_num_octaves": (i32, [vp, i32]),
        "cdvs_plane_layout": (i32, [vp, i32, i32, i32, ctypes.POINTER(i64), ctypes.POINTER(i32),
                                    ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "cdvs_pyramid": (i32, [vp, vp, vp, vp]),
        "cdvs_alp_detect": (i32, [vp, vp, vp, vp, vp, vp]),
        "cdvs_orient": (i32, [vp, vp, vp, vp, vp, vp, vp]),
        "cdvs_describe": (i32, [vp, vp, vp, vp, vp, vp]),
        "cdvs_sync_status": (i32, [vp, vp]),
        "cdvs_candidate_capacity": (i32, [vp]),
        "cdvs_autotune": (i32, [vp, vp, vp, ctypes.c_char_p, vp]),
        "cdvs_tune_get": (i32, [vp, i32]),
        "cdvs_tune_set": (i32, [vp, i32, i32]),
        "cdvs_stream": (i32, [vp, vp, i64, i32, ctypes.POINTER(StreamBuffers), vp, vp, vp]),
        "cdvs_standin_consume": (i32, [vp, i32, i32, i32, vp, vp, vp]),
        "cdvs_cnn_cells": (i64, [vp]),
        "cdvs_cnn_cell_layout": (i32, [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "cdvs_cnn_forward": (i32, [vp, vp, vp, vp, vp, vp, ctypes.c_float, vp]),
        "cdvs_cnn_labels": (i32, [vp, vp, vp, vp, vp]),
        "cdvs_cnn_backward": (i32, [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
        "cdvs_cnn_adam": (i32, [vp, vp, vp, vp, vp, i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                ctypes.c_float, vp]),
        "cdvs_graph_capture": (i32, [vp, vp, vp, vp, vp, vp, vp, vp]),
        "cdvs_graph_capture_gated": (i32, [vp, vp, vp, ctypes.c_float, vp, vp, vp, vp, vp, vp, vp]),
        "cdvs_graph_launch": (i32, [vp, vp]),
        "cdvs_profile_enable": (i32, [vp, i32]),
        "cdvs_profile_read": (i32, [vp, vp, vp]),
        "cdvs_scfv": (i32, [vp, ctypes.POINTER(ScfvModel), vp, vp, vp, vp, vp, vp, vp, vp]),
        "cdvs_pyramid_bmlog": (i32, [vp, vp, vp, vp]),
        "cdvs_front_size": (i32, [i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "cdvs_front_end": (i32, [vp, vp, vp, vp, vp]),
        "cdvs_scfv_noalloc": (i32, [ctypes.POINTER(ScfvModel), vp, vp, i32, i32, vp, vp, vp, vp, vp, vp]),
        "cdvs_encode": (i32, [vp, ctypes.POINTER(TqModel), i32, vp, vp, vp, vp]),
        "cdvs_relevance_select": (i32, [vp, ctypes.POINTER(RelevanceModel), vp, vp, i32, vp, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def default_params() -> Params:
    return lib().cdvs_default_params()


def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    return int(getattr(stream, "cuda_stream", stream))


def _check(ctx, st: int):
    if st != CDVS_OK:
        raise CdvsError(st, lib().cdvs_last_error(ctx).decode(errors="replace"))


def cdvs_validate(params: Params, descs, kp_capacity: int):
    arr = (ImageDesc * len(descs))(*descs)
    buf = ctypes.create_string_buffer(256)
    st = lib().cdvs_validate(ctypes.byref(params), arr, len(descs), kp_capacity, buf, 256)
    return st, buf.value.decode()


def cdvs_ctx_create(params: Params, descs, kp_capacity: int):
    arr = (ImageDesc * len(descs))(*descs)
    out = ctypes.c_void_p()
    st = lib().cdvs_ctx_create(ctypes.byref(params), arr, len(descs), kp_capacity, ctypes.byref(out))
    _check(None, st)
    return out


def cdvs_ctx_destroy(ctx):
    lib().cdvs_ctx_destroy(ctx)


def cdvs_pyramid(ctx, d_images, d_pyr, stream=None):
    _check(ctx, lib().cdvs_pyramid(ctx, _ptr(d_images), _ptr(d_pyr), _stream(stream)))


def cdvs_alp_detect(ctx, d_pyr, d_mask, d_kp, d_count, stream=None):
    _check(ctx, lib().cdvs_alp_detect(ctx, _ptr(d_pyr), _ptr(d_mask), _ptr(d_kp), _ptr(d_count), _stream(stream)))


def cdvs_orient(ctx, d_pyr, d_kp_in, d_count_in, d_kp_out, d_count_out, stream=None):
    _check(ctx, lib().cdvs_orient(ctx, _ptr(d_pyr), _ptr(d_kp_in), _ptr(d_count_in), _ptr(d_kp_out),
                                  _ptr(d_count_out), _stream(stream)))


def cdvs_describe(ctx, d_pyr, d_kp, d_count, d_desc, stream=None):
    _check(ctx, lib().cdvs_describe(ctx, _ptr(d_pyr), _ptr(d_kp), _ptr(d_count), _ptr(d_desc), _stream(stream)))


def cdvs_sync_status(ctx, stream=None) -> int:
    """The latched device-side status (CDVS_OK, CDVS_ERR_CAPACITY or
    CDVS_ERR_SHAPE); raises on any other error."""
    st = lib().cdvs_sync_status(ctx, _stream(stream))
    if st not in (CDVS_OK, CDVS_ERR_CAPACITY, CDVS_ERR_SHAPE):
        _check(ctx, st)
    return st


def cdvs_autotune(ctx, d_images, d_pyr, cache_path=None, stream=None):
    _check(ctx, lib().cdvs_autotune(ctx, _ptr(d_images), _ptr(d_pyr),
                                    cache_path.encode() if cache_path else None, _stream(stream)))


def cdvs_tune_get(ctx, kernel: int) -> int:
    return int(lib().cdvs_tune_get(ctx, kernel))


def cdvs_tune_set(ctx, kernel: int, variant: int):
    _check(ctx, lib().cdvs_tune_set(ctx, kernel, variant))


def cdvs_candidate_capacity(ctx) -> int:
    return int(lib().cdvs_candidate_capacity(ctx))


def cdvs_cnn_cells(ctx) -> int:
    return int(lib().cdvs_cnn_cells(ctx))


def cdvs_cnn_cell_layout(ctx, image: int):
    c0, w4, h4 = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
    _check(ctx, lib().cdvs_cnn_cell_layout(ctx, image, ctypes.byref(c0), ctypes.byref(w4), ctypes.byref(h4)))
    return c0.value, w4.value, h4.value


def cdvs_cnn_forward(ctx, d_images, d_params, d_acts, d_logits=None, d_mask=None, tau=0.5, stream=None):
    _check(ctx, lib().cdvs_cnn_forward(ctx, _ptr(d_images), _ptr(d_params), _ptr(d_acts), _ptr(d_logits),
                                       _ptr(d_mask), float(tau), _stream(stream)))


def cdvs_cnn_labels(ctx, d_kp, d_count, d_labels, stream=None):
    _check(ctx, lib().cdvs_cnn_labels(ctx, _ptr(d_kp), _ptr(d_count), _ptr(d_labels), _stream(stream)))


def cdvs_cnn_backward(ctx, d_images, d_params, d_acts, d_logits, d_labels, d_pos_weight, d_work, d_grad, d_loss,
                      stream=None):
    _check(ctx, lib().cdvs_cnn_backward(ctx, _ptr(d_images), _ptr(d_params), _ptr(d_acts), _ptr(d_logits),
                                        _ptr(d_labels), _ptr(d_pos_weight), _ptr(d_work), _ptr(d_grad), _ptr(d_loss),
                                        _stream(stream)))


def cdvs_cnn_adam(ctx, d_params, d_grad, d_m, d_v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(ctx, lib().cdvs_cnn_adam(ctx, _ptr(d_params), _ptr(d_grad), _ptr(d_m), _ptr(d_v), int(step), float(lr),
                                    float(beta1), float(beta2), float(eps), _stream(stream)))


def cdvs_graph_capture(ctx, d_images, d_pyr, d_kp, d_count, d_kp_ori, d_count_ori, d_desc):
    _check(ctx, lib().cdvs_graph_capture(ctx, _ptr(d_images), _ptr(d_pyr), _ptr(d_kp), _ptr(d_count),
                                         _ptr(d_kp_ori), _ptr(d_count_ori), _ptr(d_desc)))


def cdvs_graph_capture_gated(ctx, d_images, d_params, tau, d_mask, d_pyr, d_kp, d_count, d_kp_ori, d_count_ori,
                             d_desc):
    _check(ctx, lib().cdvs_graph_capture_gated(ctx, _ptr(d_images), _ptr(d_params), float(tau), _ptr(d_mask),
                                               _ptr(d_pyr), _ptr(d_kp), _ptr(d_count), _ptr(d_kp_ori),
                                               _ptr(d_count_ori), _ptr(d_desc)))


def cdvs_graph_launch(ctx, stream=None):
    _check(ctx, lib().cdvs_graph_launch(ctx, _stream(stream)))


def cdvs_profile_enable(ctx, enable: bool):
    _check(ctx, lib().cdvs_profile_enable(ctx, 1 if enable else 0))


def cdvs_profile_read(ctx):
    """{kernel name: (total ms, launches)} since the last read."""
    ms = np.zeros(len(KERNEL_NAMES), dtype=np.float64)
    n = np.zeros(len(KERNEL_NAMES), dtype=np.int32)
    _check(ctx, lib().cdvs_profile_read(ctx, ms.ctypes.data, n.ctypes.data))
    return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_NAMES)}


class Scfv:
    """Device copy of an SCFV model (PCA mean and matrix, GMM weights, means
    and variances; see include/cdvs.h) and the output buffers of cdvs_scfv
    for n images."""

    def __init__(self, model: dict, n_images: int, device="cuda"):
        import torch
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
        self.tensors = {k: t(model[k]) for k in ("pca_mean", "pca_matrix", "weights", "means", "variances")}
        assert self.tensors["pca_mean"].shape == (DESC_DIM,)
        assert self.tensors["pca_matrix"].shape == (SCFV_DIM, DESC_DIM)
        assert self.tensors["weights"].shape == (SCFV_COMPONENTS,)
        assert self.tensors["means"].shape == self.tensors["variances"].shape == (SCFV_COMPONENTS, SCFV_DIM)
        tt = self.tensors
        self.model = ScfvModel(_ptr(tt["pca_mean"]), _ptr(tt["pca_matrix"]), _ptr(tt["weights"]),
                               _ptr(tt["means"]), _ptr(tt["variances"]))
        n, C, Dm = n_images, SCFV_COMPONENTS, SCFV_DIM
        self.gm = torch.zeros((n, C, Dm), dtype=torch.float32, device=device)
        self.gv = torch.zeros((n, C, Dm), dtype=torch.float32, device=device)
        self.delta = torch.zeros((n, C), dtype=torch.float32, device=device)
        self.order = torch.zeros((n, C), dtype=torch.int32, device=device)
        self.bits = torch.zeros((n, C, 2), dtype=torch.int32, device=device)

    def outputs(self):
        """(gm, gv, delta, order, bits) as numpy arrays (bits as uint32)."""
        return (self.gm.cpu().numpy(), self.gv.cpu().numpy(), self.delta.cpu().numpy(), self.order.cpu().numpy(),
                self.bits.cpu().numpy().view(np.uint32))


class Relevance:
    """Device copy of relevance tables (edges 5 x 15, values 5 x 16)."""

    def __init__(self, model: dict, device="cuda"):
        import torch
        self.edges = torch.from_numpy(np.ascontiguousarray(model["edges"], dtype=np.float32)).to(device)
        self.values = torch.from_numpy(np.ascontiguousarray(model["values"], dtype=np.float32)).to(device)
        assert self.edges.shape == (5, 15) and self.values.shape == (5, 16)
        self.model = RelevanceModel(_ptr(self.edges), _ptr(self.values))


def cdvs_relevance_select(ctx, rel: Relevance, d_kp_in, d_count_in, n_keep, d_kp_out, d_count_out, d_score=None,
                          stream=None):
    _check(ctx, lib().cdvs_relevance_select(ctx, ctypes.byref(rel.model), _ptr(d_kp_in), _ptr(d_count_in),
                                            int(n_keep), _ptr(d_kp_out), _ptr(d_count_out), _ptr(d_score),
                                            _stream(stream)))


class Tq:
    """Device copy of a ternary-quantiser model (thresholds lo, hi and the
    element priority order; see include/cdvs.h)."""

    def __init__(self, model: dict, device="cuda"):
        import torch
        self.lo = torch.from_numpy(np.ascontiguousarray(model["lo"], dtype=np.float32)).to(device)
        self.hi = torch.from_numpy(np.ascontiguousarray(model["hi"], dtype=np.float32)).to(device)
        self.order = torch.from_numpy(np.ascontiguousarray(model["order"], dtype=np.int32)).to(device)
        assert self.lo.shape == self.hi.shape == self.order.shape == (DESC_DIM,)
        self.model = TqModel(_ptr(self.lo), _ptr(self.hi), _ptr(self.order))


def cdvs_encode(ctx, tq: Tq, n_elements, d_desc, d_count, d_codes, stream=None):
    _check(ctx, lib().cdvs_encode(ctx, ctypes.byref(tq.model), int(n_elements), _ptr(d_desc), _ptr(d_count),
                                  _ptr(d_codes), _stream(stream)))


def cdvs_scfv(ctx, scfv: Scfv, d_desc, d_count, stream=None):
    _check(ctx, lib().cdvs_scfv(ctx, ctypes.byref(scfv.model), _ptr(d_desc), _ptr(d_count), _ptr(scfv.gm),
                                _ptr(scfv.gv), _ptr(scfv.delta), _ptr(scfv.order), _ptr(scfv.bits),
                                _stream(stream)))


def cdvs_pyramid_bmlog(ctx, d_images, d_pyr, stream=None):
    """The block frequency-domain (BMLoG) scale space into d_pyr (same
    layout as cdvs_pyramid)."""
    _check(ctx, lib().cdvs_pyramid_bmlog(ctx, _ptr(d_images), _ptr(d_pyr), _stream(stream)))


def cdvs_front_size(width: int, height: int):
    """(width, height) of the front end's output for a width x height image."""
    w, h = ctypes.c_int32(), ctypes.c_int32()
    _check(None, lib().cdvs_front_size(int(width), int(height), ctypes.byref(w), ctypes.byref(h)))
    return w.value, h.value


def cdvs_front_end(ctx, d_src, d_src_desc, d_images, stream=None):
    """Front end into the context's image layout (d_src_desc: device tensor
    of n x 24-byte cdvs_image_desc records)."""
    _check(ctx, lib().cdvs_front_end(ctx, _ptr(d_src), _ptr(d_src_desc), _ptr(d_images), _stream(stream)))


def cdvs_scfv_noalloc(scfv: Scfv, d_desc, d_count, n_images: int, kp_capacity: int, stream=None):
    """cdvs_scfv without a context, on the library's static scratch (no
    device allocation); outputs to scfv's buffers."""
    _check(None, lib().cdvs_scfv_noalloc(ctypes.byref(scfv.model), _ptr(d_desc), _ptr(d_count), int(n_images),
                                         int(kp_capacity), _ptr(scfv.gm), _ptr(scfv.gv), _ptr(scfv.delta),
                                         _ptr(scfv.order), _ptr(scfv.bits), _stream(stream)))


def cdvs_plane_layout(ctx, image: int, octave: int, k: int):
    off, w, h, p = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(ctx, lib().cdvs_plane_layout(ctx, image, octave, k, ctypes.byref(off), ctypes.byref(w),
                                        ctypes.byref(h), ctypes.byref(p)))
    return off.value, w.value, h.value, p.value


def pack_images(images):
    """Pack a list of 2-D uint8 arrays (or an (n, H, W) array) into one byte
    buffer with 64-byte-aligned rows; returns (buffer, descriptors)."""
    descs, off, chunks = [], 0, []
    for im in images:
        im = np.ascontiguousarray(im, dtype=np.uint8)
        h, w = im.shape
        pitch = (w + 63) // 64 * 64
        buf = np.zeros((h, pitch), dtype=np.uint8)
        buf[:, :w] = im
        descs.append(ImageDesc(off, w, h, pitch, 0))
        chunks.append(buf.reshape(-1))
        off += buf.size
    return np.concatenate(chunks), descs


def descs_to_device(descs, device="cuda"):
    """A list of ImageDesc as a device tensor of 24-byte records (the
    cdvs_image_desc array cdvs_front_end takes)."""
    import torch
    arr = (ImageDesc * len(descs))(*descs)
    host = np.frombuffer(bytes(arr), dtype=np.uint8).copy()
    return torch.from_numpy(host).to(device)


class StreamBuffers(ctypes.Structure):
    _fields_ = [("d_pyr", ctypes.c_void_p), ("d_kp", ctypes.c_void_p), ("d_count", ctypes.c_void_p),
                ("d_kp_ori", ctypes.c_void_p), ("d_count_ori", ctypes.c_void_p), ("d_desc", ctypes.c_void_p),
                ("d_cnn_params", ctypes.c_void_p), ("d_acts", ctypes.c_void_p), ("d_mask", ctypes.c_void_p),
                ("tau", ctypes.c_float), ("h_count", ctypes.c_void_p * 2), ("h_kp", ctypes.c_void_p * 2),
                ("h_desc", ctypes.c_void_p * 2)]


class StandinSink(ctypes.Structure):
    _fields_ = [("out", ctypes.c_void_p), ("kept", ctypes.c_void_p), ("total_images", ctypes.c_int64),
                ("keep", ctypes.c_int32), ("threads", ctypes.c_int32)]


# consumer(user, chunk, n_images, kp_capacity, h_count, h_kp, h_desc) -> int32 (0 = continue)
CHUNK_CONSUMER = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


def cdvs_stream(ctx, d_images, chunk_stride: int, n_chunks: int, bufs: StreamBuffers, consumer, user, stream=None):
    """consumer: a CHUNK_CONSUMER instance or a raw function address (int)."""
    fn = consumer if isinstance(consumer, int) else ctypes.cast(consumer, ctypes.c_void_p).value
    _check(ctx, lib().cdvs_stream(ctx, _ptr(d_images), chunk_stride, n_chunks, ctypes.byref(bufs), fn, user,
                                  _stream(stream)))


def standin_consumer_address() -> int:
    return ctypes.cast(lib().cdvs_standin_consume, ctypes.c_void_p).value


class Pipeline:
    """Device buffers and context for one batch layout.

    ``run()`` enqueues cdvs_pyramid -> cdvs_alp_detect -> cdvs_orient ->
    cdvs_describe on the current torch stream."""

    def __init__(self, sizes, params: Params | None = None, kp_capacity: int | None = None, device="cuda"):
        import torch
        self.torch = torch
        self.params = params if params is not None else default_params()
        self.kp_capacity = kp_capacity or max(1, self.params.topk)
        self.sizes = [tuple(s) for s in sizes]          # (width, height)
        self.descs, off = [], 0
        for (w, h) in self.sizes:
            pitch = (w + 63) // 64 * 64
            self.descs.append(ImageDesc(off, w, h, pitch, 0))
            off += pitch * h
        self.image_bytes = off
        self.n = len(self.sizes)
        self.ctx = cdvs_ctx_create(self.params, self.descs, self.kp_capacity)
        L = lib()
        self.pyr_bytes = int(L.cdvs_pyramid_bytes(self.ctx))
        dev = torch.device(device)
        self.d_images = torch.zeros(self.image_bytes, dtype=torch.uint8, device=dev)
        self.d_pyr = torch.empty(self.pyr_bytes // 4, dtype=torch.float32, device=dev)
        self.d_kp = torch.zeros((self.n, self.kp_capacity, 12), dtype=torch.int32, device=dev)
        self.d_count = torch.zeros(self.n, dtype=torch.int32, device=dev)
        self.d_kp_ori = torch.zeros((self.n, self.kp_capacity, 12), dtype=torch.int32, device=dev)
        self.d_count_ori = torch.zeros(self.n, dtype=torch.int32, device=dev)
        self.d_desc = torch.zeros((self.n, self.kp_capacity, DESC_DIM), dtype=torch.float32, device=dev)

    def close(self):
        if getattr(self, "ctx", None):
            cdvs_ctx_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pack(self, images) -> np.ndarray:
        """The batch laid out as the context's image table says (host bytes)."""
        assert len(images) == self.n
        host = np.zeros(self.image_bytes, dtype=np.uint8)
        for im, d in zip(images, self.descs):
            im = np.asarray(im, dtype=np.uint8)
            assert im.shape == (d.height, d.width)
            host[d.offset:d.offset + d.pitch * d.height].reshape(d.height, d.pitch)[:, :d.width] = im
        return host

    def upload(self, images):
        self.d_images.copy_(self.torch.from_numpy(self.pack(images)))

    def front_end(self, d_src, d_src_desc, stream=None):
        """cdvs_front_end: sources (packed u8 on the device, descriptors from
        descs_to_device) brought down into this batch's images; the context
        must have been made with cdvs_front_size of each source."""
        cdvs_front_end(self.ctx, d_src, d_src_desc, self.d_images, stream)

    # -- streaming ----------------------------------------------------------
    def stream(self, d_all, n_chunks, params=None, tau=0.1, consumer=None, user=None, keep=None, threads=8,
               stream=None, sink=None):
        """cdvs_stream over n_chunks batches packed back to back in d_all
        (chunk stride = image_bytes).  With consumer None the library's
        stand-in consumer runs and (codes, kept) are returned: codes
        (n_chunks * n, kp_capacity, 128) uint8, kept (n_chunks * n) int32
        (pass them as `sink` to reuse arrays)."""
        t = self.torch
        assert d_all.numel() >= n_chunks * self.image_bytes
        if getattr(self, "_slots", None) is None:
            n, cap = self.n, self.kp_capacity
            self._slots = [(t.empty(n, dtype=t.int32, pin_memory=True),
                            t.empty(n * cap * 12, dtype=t.int32, pin_memory=True),
                            t.empty(n * cap * DESC_DIM, dtype=t.float32, pin_memory=True)) for _ in range(2)]
        b = StreamBuffers()
        b.d_pyr, b.d_kp, b.d_count = _ptr(self.d_pyr), _ptr(self.d_kp), _ptr(self.d_count)
        b.d_kp_ori, b.d_count_ori, b.d_desc = _ptr(self.d_kp_ori), _ptr(self.d_count_ori), _ptr(self.d_desc)
        if params is not None:
            self.cnn_buffers()
            b.d_cnn_params, b.d_acts, b.d_mask, b.tau = _ptr(params), None, _ptr(self.d_mask), tau
        for i in range(2):
            b.h_count[i], b.h_kp[i], b.h_desc[i] = (_ptr(x) for x in self._slots[i])
        result = None
        if consumer is None:
            if sink is None:
                sink = (np.zeros((n_chunks * self.n, self.kp_capacity, DESC_DIM), dtype=np.uint8),
                        np.zeros(n_chunks * self.n, dtype=np.int32))
            codes, kept = sink
            assert codes.shape[0] >= n_chunks * self.n and codes.dtype == np.uint8 and codes.flags.c_contiguous
            assert codes.shape[1:] == (self.kp_capacity, DESC_DIM)
            assert kept.dtype == np.int32 and kept.size >= n_chunks * self.n
            c_sink = StandinSink(codes.ctypes.data, kept.ctypes.data, n_chunks * self.n,
                                 self.kp_capacity if keep is None else keep, threads)
            consumer, user, result = standin_consumer_address(), ctypes.addressof(c_sink), (codes, kept)
        cdvs_stream(self.ctx, d_all, self.image_bytes, n_chunks, b, consumer, user, stream)
        return result

    def pyramid(self, stream=None):
        cdvs_pyramid(self.ctx, self.d_images, self.d_pyr, stream)

    def detect(self, stream=None, mask=None):
        cdvs_alp_detect(self.ctx, self.d_pyr, mask, self.d_kp, self.d_count, stream)

    # -- surrogate CNN ----------------------------------------------------
    def cnn_buffers(self):
        """Allocate (once) the CNN activation, logit and mask buffers."""
        if getattr(self, "d_acts", None) is None:
            t = self.torch
            self.ncells = cdvs_cnn_cells(self.ctx)
            dev = self.d_pyr.device
            self.d_acts = t.empty(CNN_LAYERS * self.ncells * CNN_CHANNELS, dtype=t.int16, device=dev)
            self.d_logits = t.empty((self.ncells, CNN_HEADS), dtype=t.float32, device=dev)
            self.d_mask = t.empty(self.ncells, dtype=t.uint8, device=dev)
        return self.d_acts

    def cnn_forward(self, params, tau=None, logits=True, stream=None, keep_acts=True):
        """keep_acts: store every layer's activations (training); otherwise
        the fused inference kernel runs."""
        self.cnn_buffers()
        cdvs_cnn_forward(self.ctx, self.d_images, params, self.d_acts if keep_acts else None,
                         self.d_logits if logits else None, self.d_mask if tau is not None else None,
                         0.5 if tau is None else tau, stream)

    def run_gated(self, params, tau, stream=None):
        """CNN mask (fused inference) -> pyramid -> gated detection ->
        orientation -> descriptors."""
        self.cnn_forward(params, tau=tau, logits=False, stream=stream, keep_acts=False)
        self.pyramid(stream)
        self.detect(stream, mask=self.d_mask)
        self.orient(stream)
        self.describe(stream)

    def cell_layout(self, image):
        return cdvs_cnn_cell_layout(self.ctx, image)

    def orient(self, stream=None):
        cdvs_orient(self.ctx, self.d_pyr, self.d_kp, self.d_count, self.d_kp_ori, self.d_count_ori, stream)

    def describe(self, stream=None):
        cdvs_describe(self.ctx, self.d_pyr, self.d_kp_ori, self.d_count_ori, self.d_desc, stream)

    def run(self, stream=None):
        self.pyramid(stream)
        self.detect(stream)
        self.orient(stream)
        self.describe(stream)

    def capture(self):
        """Capture the whole pass on this pipeline's buffers into a HIP graph."""
        cdvs_graph_capture(self.ctx, self.d_images, self.d_pyr, self.d_kp, self.d_count, self.d_kp_ori,
                           self.d_count_ori, self.d_desc)

    def capture_gated(self, params, tau):
        """Capture the whole gated pass (fused CNN mask, pyramid, gated
        detection, orientation, descriptors) into the context's graph."""
        self.cnn_buffers()
        cdvs_graph_capture_gated(self.ctx, self.d_images, params, tau, self.d_mask, self.d_pyr, self.d_kp,
                                 self.d_count, self.d_kp_ori, self.d_count_ori, self.d_desc)

    def replay(self, stream=None):
        cdvs_graph_launch(self.ctx, stream)

    def sync_status(self, stream=None) -> int:
        return cdvs_sync_status(self.ctx, stream)

    # -- host read-back helpers (tests) ---------------------------------
    def plane(self, image, octave, k):
        off, w, h, pitch = cdvs_plane_layout(self.ctx, image, octave, k)
        flat = self.d_pyr[off:off + pitch * h].view(h, pitch)[:, :w]
        return flat.cpu().numpy()

    def num_octaves(self, image):
        return int(lib().cdvs_num_octaves(self.ctx, image))

    def max_octaves(self):
        """The largest octave count of the batch (cdvs_pyramid's scale-kernel launches)."""
        return max(self.num_octaves(i) for i in range(self.n))

    def candidate_capacity(self):
        return cdvs_candidate_capacity(self.ctx)

    @staticmethod
    def _records(t, counts):
        arr = t.cpu().numpy().view(KP_DTYPE).reshape(t.shape[0], t.shape[1])
        return [arr[i, :counts[i]].copy() for i in range(arr.shape[0])]

    def keypoints(self):
        counts = self.d_count.cpu().numpy()
        return self._records(self.d_kp, counts)

    def oriented(self):
        counts = self.d_count_ori.cpu().numpy()
        return self._records(self.d_kp_ori, counts)

    def descriptors(self):
        counts = self.d_count_ori.cpu().numpy()
        d = self.d_desc.cpu().numpy()
        return [d[i, :counts[i]].copy() for i in range(self.n)]
