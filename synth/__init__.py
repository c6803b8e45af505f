"""Seeded synthetic grayscale images (the only module shared by the oracle's
tests and the GPU path's tests and benchmark).

It holds none of the method's arithmetic: a horizontal ramp, Gaussian blobs,
uniform noise and 8-bit quantisation, drawn from a counter-based SplitMix64
hash (the recipe is stated at the top of ``synth.c``).

Workload recipes (640x480-class images, blob scale and amplitude ranges):

* ``fixed_batch``  -- n images of one size, ``nblobs`` blobs each
  (single-image and fixed-shape batch workloads).
* ``ragged_batch`` -- n images with long side 640 and aspect ratio drawn from
  {4:3, 3:2, 16:9, 1:1, 3:4}, 100..400 blobs each.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None

# Seed bases, one per workload.
SEED_SINGLE = 1
SEED_BATCH = 2
SEED_RAGGED = 3
SEED_TRAIN = 4
SEED_EVAL = 5
SEED_HIRES = 6
SEED_HIRES_TRAIN = 7


def build() -> str:
    """Compile libsynth.so with gcc (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-Wall",
                           "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


_DEV_SRC = os.path.join(_HERE, "synth_dev.hip")
_DEV_LIB = os.path.join(_HERE, "libsynth_dev.so")
_dev = None


def build_device() -> str:
    """Compile the device twin libsynth_dev.so for gfx950 (always recompiles)."""
    tmp = _DEV_LIB + ".tmp"
    subprocess.check_call(["hipcc", "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
                           "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-o", tmp, _DEV_SRC])
    os.replace(tmp, _DEV_LIB)
    return _DEV_LIB


def _load_device():
    global _dev
    if _dev is None:
        if not os.path.exists(_DEV_LIB):
            raise RuntimeError(f"{_DEV_LIB} is missing: run synth.build_device()")
        lib = ctypes.CDLL(_DEV_LIB)
        lib.synth_dev_batch.restype = ctypes.c_int
        lib.synth_dev_batch.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
        _dev = lib
    return _dev


def device_batch(seed: int, n: int, width: int, height: int, nmin: int, nmax: int | None = None,
                 smin: float = 2.0, smax: float = 20.0, amax: float = 80.0, first: int = 0,
                 out=None, pitch: int | None = None, image_stride: int | None = None):
    """Images first..first+n-1 rendered on the current GPU into `out` (a
    uint8 torch tensor, allocated when None) on torch's current stream;
    image i at byte i * image_stride, rows of `pitch` bytes.  Byte for byte
    the host generator's output (fixed_batch: nmin = nmax = nblobs;
    hires_batch: nmin..nmax)."""
    import torch
    pitch = pitch or width
    image_stride = image_stride or pitch * height
    if out is None:
        out = torch.empty(n * image_stride, dtype=torch.uint8, device="cuda")
    assert out.dtype == torch.uint8 and out.is_cuda and out.numel() >= n * image_stride
    rc = _load_device().synth_dev_batch(seed, first, n, width, height, pitch, nmin,
                                        nmin if nmax is None else nmax, smin, smax, amax, out.data_ptr(),
                                        image_stride, torch.cuda.current_stream().cuda_stream)
    if rc != 0:
        raise ValueError(f"synth_dev_batch failed ({rc})")
    return out


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    u64 = ctypes.c_uint64
    lib.synth_sm64.restype = u64
    lib.synth_sm64.argtypes = [u64]
    lib.synth_hash.restype = u64
    lib.synth_hash.argtypes = [u64, u64, u64, u64]
    lib.synth_uniform.restype = ctypes.c_double
    lib.synth_uniform.argtypes = [u64, u64, u64, u64]
    lib.synth_blob_count.restype = ctypes.c_int
    lib.synth_blob_count.argtypes = [u64, u64, ctypes.c_int, ctypes.c_int]
    lib.synth_aspect_size.restype = None
    lib.synth_aspect_size.argtypes = [u64, u64, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.synth_image.restype = ctypes.c_int
    lib.synth_image.argtypes = [u64, u64, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_void_p]
    _lib = lib
    return lib


def sm64(x: int) -> int:
    return int(_load().synth_sm64(x))


def hash64(seed: int, image: int, field: int, idx: int) -> int:
    return int(_load().synth_hash(seed, image, field, idx))


def uniform(seed: int, image: int, field: int, idx: int) -> float:
    return float(_load().synth_uniform(seed, image, field, idx))


def image(seed: int, index: int, width: int, height: int, nblobs: int = 200,
          smin: float = 2.0, smax: float = 20.0, amax: float = 80.0) -> np.ndarray:
    """One uint8 image of shape (height, width)."""
    out = np.empty((height, width), dtype=np.uint8)
    rc = _load().synth_image(seed, index, width, height, width, nblobs, smin, smax, amax,
                             out.ctypes.data)
    if rc != 0:
        raise ValueError("synth_image: bad arguments")
    return out


def _pool_size(n: int) -> int:
    return max(1, min(n, 16, os.cpu_count() or 1))


def fixed_batch(seed: int, n: int, width: int = 640, height: int = 480, nblobs: int = 200,
                smin: float = 2.0, smax: float = 20.0, amax: float = 80.0,
                first: int = 0) -> np.ndarray:
    """n images (indices first..first+n-1), shape (n, height, width), uint8."""
    out = np.empty((n, height, width), dtype=np.uint8)
    lib = _load()

    def one(i):
        rc = lib.synth_image(seed, first + i, width, height, width, nblobs, smin, smax, amax,
                             out[i].ctypes.data)
        if rc != 0:
            raise ValueError("synth_image: bad arguments")

    with ThreadPoolExecutor(_pool_size(n)) as ex:
        list(ex.map(one, range(n)))
    return out


def hires_batch(seed: int, n: int, width: int = 1280, height: int = 960, nmin: int = 400, nmax: int = 1200,
                smin: float = 2.0, smax: float = 40.0, amax: float = 80.0, first: int = 0) -> np.ndarray:
    """n images of one size with a per-image blob count drawn from U{nmin..nmax}
    (the high-resolution stream recipe), shape (n, height, width), uint8."""
    out = np.empty((n, height, width), dtype=np.uint8)
    lib = _load()

    def one(i):
        nb = lib.synth_blob_count(seed, first + i, nmin, nmax)
        rc = lib.synth_image(seed, first + i, width, height, width, nb, smin, smax, amax, out[i].ctypes.data)
        if rc != 0:
            raise ValueError("synth_image: bad arguments")

    with ThreadPoolExecutor(_pool_size(n)) as ex:
        list(ex.map(one, range(n)))
    return out


def ragged_sizes(seed: int, n: int, long_side: int = 640, first: int = 0):
    lib = _load()
    sizes = []
    for i in range(n):
        w, h = ctypes.c_int(), ctypes.c_int()
        lib.synth_aspect_size(seed, first + i, long_side, ctypes.byref(w), ctypes.byref(h))
        sizes.append((w.value, h.value))
    return sizes


def ragged_batch(seed: int, n: int, long_side: int = 640, nmin: int = 100, nmax: int = 400,
                 smin: float = 2.0, smax: float = 20.0, amax: float = 80.0, first: int = 0):
    """List of n uint8 images of uneven size (aspect ratio drawn per image)."""
    lib = _load()
    sizes = ragged_sizes(seed, n, long_side, first)
    imgs = [np.empty((h, w), dtype=np.uint8) for (w, h) in sizes]

    def one(i):
        w, h = sizes[i]
        nb = lib.synth_blob_count(seed, first + i, nmin, nmax)
        rc = lib.synth_image(seed, first + i, w, h, w, nb, smin, smax, amax, imgs[i].ctypes.data)
        if rc != 0:
            raise ValueError("synth_image: bad arguments")

    with ThreadPoolExecutor(_pool_size(n)) as ex:
        list(ex.map(one, range(n)))
    return imgs
