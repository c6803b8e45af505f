"""CPU oracle for the CDVS front half -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The product path (the HIP
library and its Python binding) never imports it, and shares no code with it.

The C source (``cdvs_oracle.c``) is built twice:

* ``f64`` -- REAL = double; the reference for the mathematical pins;
* ``f32`` -- REAL = float; decisions (thresholds, strict NMS, disk membership,
  peak tests) taken in the precision of the GPU kernels, used for parity.

Both are compiled with ``-O2 -ffp-contract=off`` and no fast-math.  A third
build, ``f32n`` (REAL = float, ``-O3 -march=native -fno-fast-math
-ffp-contract=off``), is compiled on demand on the machine that runs it and
serves only to time the oracle as a CPU baseline.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cdvs_oracle.c")
_LIBS = {"f64": os.path.join(_HERE, "liboracle_f64.so"),
         "f32": os.path.join(_HERE, "liboracle_f32.so")}
_REAL = {"f64": "double", "f32": "float"}
_cache: dict = {}

KP_DTYPE = np.dtype([("x", "f8"), ("y", "f8"), ("sigma", "f8"), ("p", "f8"),
                     ("theta", "f8"), ("rho", "f8"), ("pss", "f8"), ("peak", "f8"),
                     ("image", "i4"), ("octave", "i4"), ("ix", "i4"), ("iy", "i4")])


class Params(ctypes.Structure):
    _fields_ = [("sigma0", ctypes.c_double), ("intervals", ctypes.c_int32),
                ("min_side", ctypes.c_int32), ("contrast", ctypes.c_double),
                ("edge_r", ctypes.c_double), ("border", ctypes.c_int32),
                ("ori_bins", ctypes.c_int32), ("max_offset", ctypes.c_double),
                ("dedup_dlog2", ctypes.c_double), ("ori_radius", ctypes.c_double),
                ("ori_wsigma", ctypes.c_double), ("ori_peak", ctypes.c_double),
                ("max_ori", ctypes.c_int32), ("topk", ctypes.c_int32),
                ("desc_cell", ctypes.c_double), ("desc_radius", ctypes.c_double),
                ("desc_wsigma", ctypes.c_double), ("desc_clamp", ctypes.c_double)]


def build() -> None:
    """Compile both portable oracle variants with gcc (always recompiles)."""
    for prec in ("f64", "f32"):
        lib = _LIBS[prec]
        tmp = lib + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-Wall",
                               "-ffp-contract=off", "-fno-fast-math",
                               f"-DREAL={_REAL[prec]}", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, lib)


def build_native(out_dir: str) -> str:
    """Compile the fp32 oracle for this host's CPU (``-O3 -march=native``,
    still ``-fno-fast-math -ffp-contract=off``) into out_dir; returns the
    library path.  Used for the CPU-baseline timing only."""
    path = os.path.join(out_dir, "liboracle_f32_native.so")
    subprocess.check_call(["gcc", "-O3", "-march=native", "-fPIC", "-shared", "-std=c99", "-Wall",
                           "-ffp-contract=off", "-fno-fast-math", "-DREAL=float", "-o", path, _SRC, "-lm"])
    return path


def use_native(path: str) -> None:
    """Register a library written by build_native as the ``f32n`` build."""
    _LIBS["f32n"] = path
    _REAL["f32n"] = "float"
    _cache.pop("f32n", None)


def _load(prec: str):
    if prec in _cache:
        return _cache[prec]
    path = _LIBS[prec]
    if prec != "f32n" and (not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC)):
        build()
    lib = ctypes.CDLL(path)
    vp, i32, f64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    P = ctypes.POINTER(Params)
    sig = {
        "or_default_params": (None, [P]),
        "or_real_size": (i32, []),
        "or_num_octaves": (i32, [i32, i32, i32]),
        "or_octave_size": (None, [i32, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "or_pyramid_len": (ctypes.c_int64, [i32, i32, P]),
        "or_plane_offset": (ctypes.c_int64, [i32, i32, P, i32, i32]),
        "or_scale_sigma": (f64, [P, i32]),
        "or_blur_sigma": (f64, [P, i32]),
        "or_blur_radius": (i32, [f64]),
        "or_gauss_taps": (None, [f64, i32, vp]),
        "or_blur": (i32, [vp, i32, i32, f64, i32, vp]),
        "or_pyramid": (i32, [vp, i32, i32, i32, P, vp]),
        "or_laplacian": (None, [vp, i32, i32, f64, vp]),
        "or_alp_beta": (i32, [P, vp]),
        "or_alp_fit": (None, [vp, i32, vp, vp]),
        "or_alp_extremum": (i32, [vp, f64, f64, vp, vp, vp]),
        "or_refine3x3": (i32, [vp, f64, f64, vp, vp, vp, vp]),
        "or_detect": (i32, [vp, i32, i32, P, i32, vp, i32]),
        "or_detect_masked": (i32, [vp, i32, i32, P, i32, vp, f64, vp, i32]),
        "or_dedup": (None, [vp, i32, P, vp]),
        "or_select": (i32, [vp, i32, vp, i32, vp]),
        "or_scale_index": (i32, [P, f64]),
        "or_orient_hist": (None, [vp, i32, i32, f64, f64, f64, P, vp]),
        "or_orient_peaks": (i32, [vp, P, vp, vp]),
        "or_orient": (i32, [vp, i32, i32, P, vp, i32, vp, i32]),
        "or_descriptor": (None, [vp, i32, i32, f64, f64, f64, f64, P, vp]),
        "or_describe": (None, [vp, i32, i32, P, vp, i32, vp]),
        "or_run": (i32, [vp, i32, i32, i32, P, i32, vp, vp, i32, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    # or_alp_extremum / or_refine3x3 take REAL scalars (not double) by value
    # through pointers only, so the f64 argtypes above are for lo/hi/edge_r/
    # max_off, which are REAL in C; fix them per build.
    rt = ctypes.c_double if prec == "f64" else ctypes.c_float
    lib.or_alp_extremum.argtypes = [vp, rt, rt, vp, vp, vp]
    lib.or_refine3x3.argtypes = [vp, rt, rt, vp, vp, vp, vp]
    _cache[prec] = lib
    return lib


class Oracle:
    """Thin ctypes wrapper around one precision build of the oracle."""

    def __init__(self, prec: str = "f64", params: Params | None = None):
        self.prec = prec
        self.lib = _load(prec)
        self.dtype = np.float64 if _REAL[prec] == "double" else np.float32
        assert self.lib.or_real_size() == np.dtype(self.dtype).itemsize
        if params is None:
            params = Params()
            self.lib.or_default_params(ctypes.byref(params))
        self.P = params

    # -- parameters ------------------------------------------------------
    @staticmethod
    def default_params() -> Params:
        p = Params()
        _load("f64").or_default_params(ctypes.byref(p))
        return p

    def params_dict(self) -> dict:
        return {f: getattr(self.P, f) for f, _ in Params._fields_}

    # -- geometry --------------------------------------------------------
    def num_octaves(self, W, H):
        return self.lib.or_num_octaves(W, H, self.P.min_side)

    def octave_size(self, W, H, o):
        w, h = ctypes.c_int(), ctypes.c_int()
        self.lib.or_octave_size(W, H, o, ctypes.byref(w), ctypes.byref(h))
        return w.value, h.value

    def scale_sigma(self, k):
        return self.lib.or_scale_sigma(ctypes.byref(self.P), k)

    def blur_sigma(self, k):
        return self.lib.or_blur_sigma(ctypes.byref(self.P), k)

    def blur_radius(self, s):
        return self.lib.or_blur_radius(s)

    # -- filters ---------------------------------------------------------
    def gauss_taps(self, s, r):
        t = np.empty(2 * r + 1, dtype=self.dtype)
        self.lib.or_gauss_taps(s, r, t.ctypes.data)
        return t

    def blur(self, img, s, r):
        a = np.ascontiguousarray(img, dtype=self.dtype)
        out = np.empty_like(a)
        rc = self.lib.or_blur(a.ctypes.data, a.shape[1], a.shape[0], s, r, out.ctypes.data)
        assert rc == 0
        return out

    def laplacian(self, G, sigma_k):
        a = np.ascontiguousarray(G, dtype=self.dtype)
        out = np.empty_like(a)
        self.lib.or_laplacian(a.ctypes.data, a.shape[1], a.shape[0], sigma_k, out.ctypes.data)
        return out

    def pyramid(self, img):
        """Returns a list over octaves of arrays (S+1, h_o, w_o)."""
        img = np.ascontiguousarray(img, dtype=np.uint8)
        H, W = img.shape
        n = self.lib.or_pyramid_len(W, H, ctypes.byref(self.P))
        flat = np.empty(n, dtype=self.dtype)
        rc = self.lib.or_pyramid(img.ctypes.data, W, H, W, ctypes.byref(self.P), flat.ctypes.data)
        assert rc == 0
        return self._split(flat, W, H), flat

    def _split(self, flat, W, H):
        out = []
        K = self.P.intervals + 1
        for o in range(self.num_octaves(W, H)):
            w, h = self.octave_size(W, H, o)
            off = self.lib.or_plane_offset(W, H, ctypes.byref(self.P), o, 0)
            out.append(flat[off:off + K * w * h].reshape(K, h, w))
        return out

    # -- ALP -------------------------------------------------------------
    def alp_beta(self):
        K = self.P.intervals + 1
        b = np.empty(K * 4, dtype=np.float64)
        assert self.lib.or_alp_beta(ctypes.byref(self.P), b.ctypes.data) == 0
        return b.reshape(K, 4)

    def alp_fit(self, L):
        K = self.P.intervals + 1
        beta = self.alp_beta().astype(self.dtype).ravel()
        lk = np.ascontiguousarray(L, dtype=self.dtype)
        a = np.empty(4, dtype=self.dtype)
        self.lib.or_alp_fit(beta.ctypes.data, K, lk.ctypes.data, a.ctypes.data)
        return a

    def alp_extremum(self, alpha, lo=None, hi=None):
        lo = self.scale_sigma(0) if lo is None else lo
        hi = self.scale_sigma(self.P.intervals) if hi is None else hi
        a = np.ascontiguousarray(alpha, dtype=self.dtype)
        s, p, pss = (np.zeros(1, dtype=self.dtype) for _ in range(3))
        ok = self.lib.or_alp_extremum(a.ctypes.data, lo, hi, s.ctypes.data, p.ctypes.data,
                                      pss.ctypes.data)
        return (bool(ok), float(s[0]), float(p[0]), float(pss[0]))

    def refine3x3(self, v):
        a = np.ascontiguousarray(np.asarray(v).reshape(9), dtype=self.dtype)
        ox, oy, pr, rho = (np.zeros(1, dtype=self.dtype) for _ in range(4))
        ok = self.lib.or_refine3x3(a.ctypes.data, self.P.edge_r, self.P.max_offset,
                                   ox.ctypes.data, oy.ctypes.data, pr.ctypes.data, rho.ctypes.data)
        return (bool(ok), float(ox[0]), float(oy[0]), float(pr[0]), float(rho[0]))

    # -- stages ------------------------------------------------------------
    def detect(self, flat, W, H, image=0, cap=1 << 16):
        out = np.zeros(cap, dtype=KP_DTYPE)
        n = self.lib.or_detect(flat.ctypes.data, W, H, ctypes.byref(self.P), image,
                               out.ctypes.data, cap)
        assert n >= 0
        return out[:min(n, cap)].copy()

    def detect_masked(self, flat, W, H, mask, fmax=0.6, image=0, cap=1 << 16):
        """Stages A-B examining only the centres the cell mask switches on
        (mask: uint8 per 4x4 cell, shape (ceil(H/4), ceil(W/4)))."""
        m = np.ascontiguousarray(mask, dtype=np.uint8)
        assert m.shape == ((H + 3) // 4, (W + 3) // 4)
        out = np.zeros(cap, dtype=KP_DTYPE)
        n = self.lib.or_detect_masked(flat.ctypes.data, W, H, ctypes.byref(self.P), image, m.ctypes.data,
                                      float(fmax), out.ctypes.data, cap)
        assert n >= 0
        return out[:min(n, cap)].copy()

    def dedup(self, cand):
        cand = np.ascontiguousarray(cand, dtype=KP_DTYPE)
        alive = np.zeros(len(cand), dtype=np.int32)
        self.lib.or_dedup(cand.ctypes.data, len(cand), ctypes.byref(self.P), alive.ctypes.data)
        return alive

    def select(self, cand, alive, topk=None):
        topk = self.P.topk if topk is None else topk
        cand = np.ascontiguousarray(cand, dtype=KP_DTYPE)
        alive = np.ascontiguousarray(alive, dtype=np.int32)
        out = np.zeros(max(1, len(cand)), dtype=KP_DTYPE)
        m = self.lib.or_select(cand.ctypes.data, len(cand), alive.ctypes.data, topk,
                               out.ctypes.data)
        return out[:m].copy()

    def scale_index(self, s_oct):
        return self.lib.or_scale_index(ctypes.byref(self.P), s_oct)

    def orient_hist(self, G, cx, cy, s):
        a = np.ascontiguousarray(G, dtype=self.dtype)
        hist = np.zeros(self.P.ori_bins, dtype=self.dtype)
        self.lib.or_orient_hist(a.ctypes.data, a.shape[1], a.shape[0], cx, cy, s,
                                ctypes.byref(self.P), hist.ctypes.data)
        return hist

    def orient_peaks(self, hist):
        h = np.ascontiguousarray(hist, dtype=self.dtype)
        th = np.zeros(64, dtype=self.dtype)
        pk = np.zeros(64, dtype=self.dtype)
        c = self.lib.or_orient_peaks(h.ctypes.data, ctypes.byref(self.P), th.ctypes.data,
                                     pk.ctypes.data)
        return th[:c].astype(np.float64), pk[:c].astype(np.float64)

    def orient(self, flat, W, H, kps, cap=None):
        kps = np.ascontiguousarray(kps, dtype=KP_DTYPE)
        cap = cap or max(1, 4 * len(kps))
        out = np.zeros(cap, dtype=KP_DTYPE)
        m = self.lib.or_orient(flat.ctypes.data, W, H, ctypes.byref(self.P), kps.ctypes.data,
                               len(kps), out.ctypes.data, cap)
        return out[:m].copy()

    def descriptor(self, G, cx, cy, s, theta):
        a = np.ascontiguousarray(G, dtype=self.dtype)
        d = np.zeros(128, dtype=self.dtype)
        self.lib.or_descriptor(a.ctypes.data, a.shape[1], a.shape[0], cx, cy, s, theta,
                               ctypes.byref(self.P), d.ctypes.data)
        return d.astype(np.float64)

    def describe(self, flat, W, H, kps):
        kps = np.ascontiguousarray(kps, dtype=KP_DTYPE)
        d = np.zeros((max(1, len(kps)), 128), dtype=np.float64)
        self.lib.or_describe(flat.ctypes.data, W, H, ctypes.byref(self.P), kps.ctypes.data,
                             len(kps), d.ctypes.data)
        return d[:len(kps)]

    def run(self, img, image=0, cap=None, with_desc=True):
        """Whole front half for one image -> (keypoints, descriptors, stats)."""
        img = np.ascontiguousarray(img, dtype=np.uint8)
        H, W = img.shape
        cap = cap or max(1, 4 * (self.P.topk if self.P.topk > 0 else 65536))
        kp = np.zeros(cap, dtype=KP_DTYPE)
        desc = np.zeros((cap, 128), dtype=np.float64) if with_desc else None
        stats = np.zeros(4, dtype=np.int32)
        n = self.lib.or_run(img.ctypes.data, W, H, W, ctypes.byref(self.P), image, kp.ctypes.data,
                            desc.ctypes.data if with_desc else None, cap, stats.ctypes.data)
        assert n >= 0
        return kp[:n].copy(), (desc[:n].copy() if with_desc else None), dict(
            candidates=int(stats[0]), deduped=int(stats[1]), selected=int(stats[2]),
            oriented=int(stats[3]))
