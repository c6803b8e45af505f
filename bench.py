#!/usr/bin/env python3
"""Throughput of the CDVS front half on one MI355X.

One step = the whole hot path over one batch already resident in HBM:
cdvs_pyramid -> cdvs_alp_detect -> cdvs_orient -> cdvs_describe on a batch of
256 seeded synthetic 640x480 u8 images (top 1000 keypoints described per
image).  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--batch B] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0        # MI355X HBM3E
PEAK_FP32_TFLOPS = 157.3     # MI355X FP32 vector, published (256 CU x 2.4 GHz x 256 FLOP/clk, packed FP32)
# The library is built with packed FP32 switched off, so its kernels issue at
# most one FP32 fused multiply-add per lane per cycle: 256 CU x 4 SIMD x 16
# lanes x 2 FLOP x 2.4 GHz = 78.6 TFLOP/s.  The ridge that decides whether a
# kernel is bandwidth- or arithmetic-bound uses this usable rate.
USABLE_FP32_TFLOPS = 78.6

# Minimum arithmetic per pixel of the separable Gaussians with symmetric
# taps: one pass of radius r is r pair additions and r+1 multiply-adds
# (3r + 2 flops); the four scale images (r = 5, 7, 9, 12) take two passes
# each, and their column passes share the pair sums of one input column
# (12 additions, then r+1 multiply-adds per image).
SCALES_FLOP_PER_PX = (12 + sum(2 * (r + 1) for r in (5, 7, 9, 12))) + sum(3 * r + 2 for r in (5, 7, 9, 12))  # 193
PREBLUR_FLOP_PER_PX = 2 * (3 * 7 + 2)                                # 46
RIDGE_FLOP_PER_BYTE = USABLE_FP32_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)  # 9.8


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def octave_pixels(sizes, min_side=32):
    """Per octave: total pixels over the batch."""
    tot = {}
    for (w, h) in sizes:
        o = 0
        while True:
            tot[o] = tot.get(o, 0) + w * h
            if min(w, h) < min_side:
                break
            w, h = (w + 1) // 2, (h + 1) // 2
            o += 1
    return [tot[o] for o in sorted(tot)]


def algorithmic(sizes, n_kp, n_ori):
    """Algorithmic bytes and flops of one step, per kernel."""
    npx = octave_pixels(sizes)
    n0 = npx[0]
    nxt = sum(npx[1:])
    allpx = sum(npx)
    return {
        "preblur": {"bytes": n0 * (1 + 4), "flop": n0 * PREBLUR_FLOP_PER_PX},
        # read G_{o,0}, write G_{o,1..4}, write G_{o+1,0}
        "scales": {"bytes": allpx * (4 + 16) + nxt * 4, "flop": allpx * SCALES_FLOP_PER_PX},
        # read five planes
        "detect": {"bytes": allpx * 20, "flop": allpx * 70},
        "finalize": {"bytes": None, "flop": None},
        "orient": {"bytes": n_kp * 48 + n_ori * 48, "flop": None},
        "orient_compact": {"bytes": None, "flop": None},
        "describe": {"bytes": n_ori * (48 + 512), "flop": None},
        "clear": {"bytes": None, "flop": None},
    }


WEIGHTS = os.path.join(ROOT, "paper_1705_09776_amd", "weights", "surrogate_640x480.npz")
WEIGHTS_HIRES = os.path.join(ROOT, "paper_1705_09776_amd", "weights", "surrogate_1280x960.npz")
WEIGHTS_T4 = os.path.join(ROOT, "paper_1705_09776_amd", "weights", "surrogate_640x480_t4.npz")
TRAFFIC = os.path.join(ROOT, "profiles", "traffic_plain_batch256_640x480.md")
SQ = os.path.join(ROOT, "profiles", "sq_counters_plain_batch256_640x480.md")
SIMDS, CLOCK_HZ = 1024, 2.4e9      # 256 CUs x 4 SIMDs; a wave64 VALU instruction takes 4 cycles of a SIMD
# kernel names in the profile summaries (the scale kernel's carries its tile variant)
_PROFILE_NAME = {"detect": "k_detect_strip<false,false>", "describe": "k_describe", "scales": "k_blur<1,4,12,false,{v}>",
                 "orient": "k_orient", "finalize": "k_finalize", "preblur": "k_blur<0,1,7,true,4>",
                 "orient_compact": "k_orient_compact"}


def measured_path_bytes(variant):
    """HBM bytes per step of the whole plain path from the committed counter
    summary (every kernel's source unchanged), else None."""
    total = 0
    for k in ("detect", "scales", "describe", "orient", "finalize", "preblur"):
        b = measured_traffic(k, variant)
        if b is None:
            return None
        total += b
    return total


def achievable_hbm_gbs(nbytes=2 << 30, reps=5):
    """Read + write streaming rate (bytes read and written per second) of
    plain device-to-device kernels over 2 GiB: the better of torch's copy_
    and an elementwise add into another buffer (the add streams faster on
    this GPU)."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    best = 0.0
    for op in (lambda: b.copy_(a), lambda: torch.add(a, 1.0, out=b)):
        op()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            op()
        e1.record()
        torch.cuda.synchronize()
        dt = e0.elapsed_time(e1) * 1e-3 / reps
        best = max(best, 2 * nbytes / dt / 1e9)
    del a, b
    torch.cuda.empty_cache()
    return best


def single_leg(reps=200):
    """One 640x480 image (the single-image workload): latency of one captured
    pass, launch-bound rather than bandwidth-bound."""
    import torch
    import synth
    import paper_1705_09776_amd as cd
    img = synth.image(synth.SEED_SINGLE, 0, 640, 480)
    pipe = cd.Pipeline([(640, 480)])
    pipe.upload([img])
    pipe.run()
    pipe.capture()
    for _ in range(10):
        pipe.replay()
    torch.cuda.synchronize()
    lat = []
    for _ in range(reps):
        t0 = time.perf_counter()
        pipe.replay()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    lat.sort()
    return {"latency_ms_median": round(lat[len(lat) // 2] * 1e3, 4), "latency_ms_p90": round(lat[int(0.9 * len(lat))] * 1e3, 4),
            "keypoints": int(pipe.d_count_ori.item()),
            "timing": f"{reps} replays of the captured pass, each followed by a device synchronisation"}


def _profile_figure(path, tag, kernel, variant):
    """A per-step figure of `kernel` from a committed counter summary (256
    images 640x480), or None when there is none or the kernel's source has
    changed since the counters were taken."""
    import hashlib
    name = _PROFILE_NAME.get(kernel)
    if name is None or not os.path.exists(path):
        return None
    name = name.format(v=variant)
    csrc = os.path.join(ROOT, "paper_1705_09776_amd", "csrc")
    for line in open(path):
        f = line.split()
        if len(f) == 5 and f[0] == tag and f[1] == name:
            data = open(os.path.join(csrc, f[3]), "rb").read() + open(os.path.join(csrc, "cdvs_internal.h"), "rb").read()
            return int(f[2]) if hashlib.sha256(data).hexdigest() == f[4] else None
    return None


def measured_traffic(kernel, variant=1):
    """HBM bytes per step of `kernel` (rocprofv3 FETCH_SIZE and WRITE_SIZE)."""
    return _profile_figure(TRAFFIC, "traffic", kernel, variant)


def measured_valu(kernel, variant=1):
    """Wave-level VALU instructions per step of `kernel` (rocprofv3 SQ_INSTS_VALU)."""
    return _profile_figure(SQ, "valu", kernel, variant)


def gated_leg(pipe, steps, B, plain_kp):
    """The surrogate-gated pass on the same batch: CNN mask -> pyramid ->
    gated detection -> orientation -> descriptors: K eager steps with
    per-kernel events, then K replays of the pass captured as one hipGraph;
    recall of the plain top-1000 keypoints."""
    import numpy as np
    import torch
    import paper_1705_09776_amd as cd
    from paper_1705_09776_amd import surrogate
    st = surrogate.load_checkpoint(WEIGHTS)
    with open(os.path.splitext(WEIGHTS)[0] + ".json") as f:
        tau = float(json.load(f)["tau"])
    params = torch.from_numpy(st["params"]).cuda()
    pipe.cnn_buffers()
    for _ in range(2):
        pipe.run_gated(params, tau)
    torch.cuda.synchronize()
    cd.cdvs_profile_enable(pipe.ctx, True)
    t0 = time.perf_counter()
    for _ in range(steps):
        pipe.run_gated(params, tau)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = cd.cdvs_profile_read(pipe.ctx)
    cd.cdvs_profile_enable(pipe.ctx, False)
    if pipe.sync_status() != cd.CDVS_OK:
        raise RuntimeError("capacity overflow in the gated leg")
    gk = pipe.keypoints()
    key = lambda k: (int(k["octave"]), int(k["ix"]), int(k["iy"]))
    hit = sum(len({key(k) for k in a} & {key(k) for k in b}) for a, b in zip(plain_kp, gk))
    mask = pipe.d_mask.cpu().numpy()
    act = sum(int(((mask >> o) & 1).sum()) for o in range(5))
    eager_ms = (t1 - t0) * 1e3 / steps
    # the same gated pass captured as one hipGraph, timed by back-to-back replays
    pipe.capture_gated(params, tau)
    for _ in range(2):
        pipe.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pipe.replay()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    if pipe.sync_status() != cd.CDVS_OK:
        raise RuntimeError("capacity overflow in the gated leg's replays")
    return {"value": round(B / (ms * 1e-3), 1), "unit": "images/s", "ms_per_step": round(ms, 4),
            "eager_images_per_s": round(B / (eager_ms * 1e-3), 1), "eager_ms_per_step": round(eager_ms, 4),
            "tau": tau, "recall_top1000": round(hit / max(1, sum(len(a) for a in plain_kp)), 5),
            "active_cell_fraction": round(act / (5 * mask.size), 4),
            "timing": "value: K hipGraph replays of the gated pass (CNN mask, pyramid, gated detection, "
                      "orientation, descriptors); kernels: K eager steps with per-kernel events",
            "kernels_ms_per_step": {k: round(v[0] / steps, 4) for k, v in prof.items() if v[1]}}


def sparse_leg(imgs, steps, contrast=4.0):
    """Sensitivity point with sparse keypoints: the same batch with contrast
    threshold T = 4 (instead of 1.5), plain pass against the pass gated by a
    network trained on T = 4 labels, both as graph replays and eager steps."""
    import torch
    import paper_1705_09776_amd as cd
    from paper_1705_09776_amd import surrogate
    B = len(imgs)
    p = cd.default_params()
    p.contrast = contrast
    pipe = cd.Pipeline([(640, 480)] * B, params=p)
    pipe.upload(list(imgs))
    # each form gets the same warm-up (three untimed passes) before its timing
    for _ in range(3):
        pipe.run()
    pipe.capture()
    for _ in range(3):
        pipe.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pipe.replay()
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / steps
    for _ in range(3):
        pipe.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pipe.run()
    torch.cuda.synchronize()
    t_plain_eager = (time.perf_counter() - t0) / steps
    plain_kp = [k.copy() for k in pipe.keypoints()]
    st = surrogate.load_checkpoint(WEIGHTS_T4)
    with open(os.path.splitext(WEIGHTS_T4)[0] + ".json") as f:
        tau = float(json.load(f)["tau"])
    params = torch.from_numpy(st["params"]).cuda()
    for _ in range(3):
        pipe.run_gated(params, tau)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pipe.run_gated(params, tau)
    torch.cuda.synchronize()
    t_gated_eager = (time.perf_counter() - t0) / steps
    pipe.capture_gated(params, tau)
    for _ in range(3):
        pipe.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pipe.replay()
    torch.cuda.synchronize()
    t_gated = (time.perf_counter() - t0) / steps
    if pipe.sync_status() != cd.CDVS_OK:
        raise RuntimeError("capacity overflow in the sparse leg")
    gk = pipe.keypoints()
    key = lambda k: (int(k["octave"]), int(k["ix"]), int(k["iy"]))
    hit = sum(len({key(k) for k in a} & {key(k) for k in b}) for a, b in zip(plain_kp, gk))
    mask = pipe.d_mask.cpu().numpy()
    act = sum(int(((mask >> o) & 1).sum()) for o in range(5))
    return {"contrast": contrast, "tau": tau, "keypoints_per_image": round(sum(len(k) for k in plain_kp) / B, 1),
            "plain_images_per_s": round(B / t_plain, 1), "plain_eager_images_per_s": round(B / t_plain_eager, 1),
            "gated_images_per_s": round(B / t_gated, 1), "gated_eager_images_per_s": round(B / t_gated_eager, 1),
            "gated_vs_plain_graph": round(t_plain / t_gated, 4),
            "gated_vs_plain_eager": round(t_plain_eager / t_gated_eager, 4),
            "net": ("loss: the gate's CNN costs more than the detection it skips" if t_gated > t_plain
                    else "gain"),
            "recall_top1000": round(hit / max(1, sum(len(a) for a in plain_kp)), 5),
            "active_cell_fraction": round(act / (5 * mask.size), 4),
            "timing": "plain and gated: K graph replays each (and K eager steps each)"}


def ragged_leg(steps, n=1024):
    """Uneven sizes: n images, long side 640, aspect drawn from {4:3, 3:2,
    16:9, 1:1, 3:4}, 100-400 blobs each, in one packed ragged context; the
    scale-plane tile shape and the detection's launch form (one wave per
    strip or persistent) are picked by the autotuner, then K replays of the
    captured pass are timed."""
    import tempfile
    import torch
    import synth
    import paper_1705_09776_amd as cd
    imgs = synth.ragged_batch(synth.SEED_RAGGED, n)
    sizes = [(im.shape[1], im.shape[0]) for im in imgs]
    pipe = cd.Pipeline(sizes)
    pipe.upload(imgs)
    pipe.run()
    torch.cuda.synchronize()
    with tempfile.TemporaryDirectory() as td:
        cache = os.path.join(td, "tune.json")
        t0 = time.perf_counter()
        cd.cdvs_autotune(pipe.ctx, pipe.d_images, pipe.d_pyr, cache)
        t_tune = time.perf_counter() - t0
        tune = list(json.load(open(cache)).values())[0]
    pipe.capture()
    pipe.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pipe.replay()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if pipe.sync_status() != cd.CDVS_OK:
        raise RuntimeError("capacity overflow in the ragged leg")
    ms = (t1 - t0) * 1e3 / steps
    npx = sum(octave_pixels(sizes))
    return {"value": round(n / (ms * 1e-3), 1), "unit": "images/s", "ms_per_step": round(ms, 4), "images": n,
            "octave_px_per_image": round(npx / n, 1),
            "tile_variant": tune["variant"], "tile_variant_us": tune["us"],
            "detect_variant": tune["detect"], "detect_variant_us": tune["detect_us"], "autotune_s": round(t_tune, 3),
            "launches_per_stage": {"pyramid": 1 + pipe.max_octaves(), "detect": 1, "finalize": 1, "orient": 2,
                                   "describe": 1},
            "persistent_detect": ("built and tested (same keypoints, and oracle parity), kept only when the "
                                  "autotuner measures it faster: it is slower here (detect_variant_us[1])"),
            "timing": "K hipGraph replays of the whole plain pass over the packed ragged batch"}


HIRES = (1280, 960)


def stream_leg(n_images=4096, chunk=256, threads=16):
    """High-resolution stream: n_images 1280x960 (400-1200 blobs, sigma up to
    40 px) resident in HBM, surrogate-gated, in chunks of `chunk` images;
    descriptors of the top 1000 keypoints per image go to pinned host
    buffers and a host stand-in consumer (u8 coding of the descriptors, in
    place of the CPU-side compression) overlapped with the next chunk."""
    import numpy as np
    import torch
    import synth
    import paper_1705_09776_amd as cd
    from paper_1705_09776_amd import surrogate
    W, H = HIRES
    pipe = cd.Pipeline([(W, H)] * chunk)
    n_chunks = n_images // chunk
    d_all = synth.device_batch(synth.SEED_HIRES, n_chunks * chunk, W, H, 400, 1200, smax=40.0)
    torch.cuda.synchronize()
    wpath = WEIGHTS_HIRES if os.path.exists(WEIGHTS_HIRES) else WEIGHTS
    st = surrogate.load_checkpoint(wpath)
    with open(os.path.splitext(wpath)[0] + ".json") as f:
        tau = float(json.load(f)["tau"])
    params = torch.from_numpy(st["params"]).cuda()
    sink = (np.zeros((n_chunks * chunk, pipe.kp_capacity, cd.DESC_DIM), dtype=np.uint8),
            np.zeros(n_chunks * chunk, dtype=np.int32))
    sink[0][:] = 1                                    # touch the pages before timing
    # recall of the gated detector on the first chunk
    ib = pipe.image_bytes
    pipe.d_images = d_all[:ib]
    pipe.run()
    torch.cuda.synchronize()
    plain = [k.copy() for k in pipe.keypoints()]
    pipe.run_gated(params, tau)
    torch.cuda.synchronize()
    gk = pipe.keypoints()
    key = lambda k: (int(k["octave"]), int(k["ix"]), int(k["iy"]))
    hit = sum(len({key(k) for k in a} & {key(k) for k in b}) for a, b in zip(plain, gk))
    recall = hit / max(1, sum(len(a) for a in plain))
    mask = pipe.d_mask.cpu().numpy()
    active = sum(int(((mask >> o) & 1).sum()) for o in range(6)) / (6 * mask.size)
    # GPU only: the same chunks, gated, without the hand-off
    pipe.stream(d_all, 1, params=params, tau=tau, threads=threads, sink=sink)      # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in range(n_chunks):
        pipe.d_images = d_all[c * ib:(c + 1) * ib]
        pipe.run_gated(params, tau)
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    # end to end: compute, D2H into pinned slots, host consumer, overlapped
    t0 = time.perf_counter()
    pipe.stream(d_all, n_chunks, params=params, tau=tau, threads=threads, sink=sink)
    t_e2e = time.perf_counter() - t0
    n = n_chunks * chunk
    d2h = n * pipe.kp_capacity * (cd.DESC_DIM * 4 + 48)
    return {"value": round(n / t_e2e, 1), "unit": "images/s", "images": n, "chunk": chunk, "width": W, "height": H,
            "gpu_only_images_per_s": round(n / t_gpu, 1), "overlap_efficiency": round(t_gpu / t_e2e, 4),
            "d2h_gb": round(d2h / 1e9, 3), "weights": os.path.basename(wpath), "tau": tau,
            "recall_first_chunk": round(recall, 5),
            "active_cell_fraction_first_chunk": round(active, 4), "consumer_threads": threads,
            "descriptors_kept": int(sink[1][:n].sum()),
            "timing": "end to end over the stream (inputs resident in HBM; ends when the host consumer has "
                      "finished the last chunk); gpu_only: the same chunks gated, eager, no hand-off"}


SCFV_MODEL = os.path.join(ROOT, "paper_1705_09776_amd", "weights", "scfv_standin.npz")
TQ_MODEL = os.path.join(ROOT, "paper_1705_09776_amd", "weights", "tq_standin.npz")
REL_MODEL = os.path.join(ROOT, "paper_1705_09776_amd", "weights", "relevance_standin.npz")
PEAK_FP32_MFMA_TFLOPS = 157.3    # MI355X dense FP32 matrix rate
# SCFV arithmetic per descriptor: PCA 32 x 128, then logits and gradient
# sums against 512 components over the 64 columns [x | x.*x] (multiply-adds
# as two flops)
SCFV_FLOP_PER_DESC = 2 * 32 * 128 + 2 * 512 * 64 + 2 * 512 * 64


def _timed(fn, steps):
    """Mean ms of fn() over `steps` runs on torch's current stream (events)."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def aggregate_leg(pipe, steps, B):
    """The steps the paper places beside description (Sec. III-B to III-D)
    on the plain pass's outputs, each kernel timed with events on its own
    stream: relevance selection of 300 of each image's 1000 detected
    keypoints, transform coding of the 1000 descriptors per image (all 128
    elements), SCFV aggregation of the same descriptors (stand-in models);
    and the allocation-free SCFV on one image (split over workgroups)
    against the context form on one image."""
    import numpy as np
    import torch
    import paper_1705_09776_amd as cd
    rel = cd.Relevance(dict(np.load(REL_MODEL)))
    tq = cd.Tq(dict(np.load(TQ_MODEL)))
    S = cd.Scfv(dict(np.load(SCFV_MODEL)), B)
    kp_out, cnt_out = torch.zeros_like(pipe.d_kp), torch.zeros_like(pipe.d_count)
    codes = torch.zeros((B, pipe.kp_capacity, cd.TQ_WORDS), dtype=torch.int32, device="cuda")
    n_keep = 300

    def one():
        cd.cdvs_relevance_select(pipe.ctx, rel, pipe.d_kp, pipe.d_count, n_keep, kp_out, cnt_out)
        cd.cdvs_encode(pipe.ctx, tq, 128, pipe.d_desc, pipe.d_count_ori, codes)
        cd.cdvs_scfv(pipe.ctx, S, pipe.d_desc, pipe.d_count_ori)

    one()
    torch.cuda.synchronize()
    cd.cdvs_profile_enable(pipe.ctx, True)
    for _ in range(steps):
        one()
    torch.cuda.synchronize()
    prof = cd.cdvs_profile_read(pipe.ctx)
    cd.cdvs_profile_enable(pipe.ctx, False)
    n_kp = int(pipe.d_count.sum().item())
    n_desc = int(pipe.d_count_ori.sum().item())
    ms = {k: prof[k][0] / steps for k in ("relevance", "encode", "scfv")}
    rel_bytes = n_kp * 48 + int(cnt_out.sum().item()) * (48 + 4)
    enc_bytes = n_desc * (512 + 4 * cd.TQ_WORDS)
    scfv_flop = n_desc * SCFV_FLOP_PER_DESC
    out = {
        "relevance": {"ms": round(ms["relevance"], 4), "images_per_s": round(B / (ms["relevance"] * 1e-3), 1),
                      "keep": n_keep,
                      "roofline": {"bound": "hbm", "achieved": round(rel_bytes / (ms["relevance"] * 1e-3) / 1e9, 1),
                                   "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                   "frac": round(rel_bytes / (ms["relevance"] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}},
        "encode": {"ms": round(ms["encode"], 4), "descriptors_per_s": round(n_desc / (ms["encode"] * 1e-3), 1),
                   "roofline": {"bound": "hbm", "achieved": round(enc_bytes / (ms["encode"] * 1e-3) / 1e9, 1),
                                "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                "frac": round(enc_bytes / (ms["encode"] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}},
        "scfv": {"ms": round(ms["scfv"], 4), "images_per_s": round(B / (ms["scfv"] * 1e-3), 1),
                 "roofline": {"bound": "mfma", "achieved": round(scfv_flop / (ms["scfv"] * 1e-3) / 1e12, 2),
                              "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                              "frac": round(scfv_flop / (ms["scfv"] * 1e-3) / 1e12 / PEAK_FP32_MFMA_TFLOPS, 4)}},
        "descriptors_per_image": round(n_desc / B, 1),
    }
    # one image: the context form (one workgroup) and the allocation-free
    # form (the image split into parts over workgroups)
    S1 = cd.Scfv(dict(np.load(SCFV_MODEL)), 1)
    d1, c1 = pipe.d_desc[:1].contiguous(), pipe.d_count_ori[:1].contiguous()
    one_ctx = cd.Pipeline([(640, 480)])
    out["scfv_one_image_ms"] = {
        "context_form": round(_timed(lambda: cd.cdvs_scfv(one_ctx.ctx, S1, d1, c1), 50), 4),
        "noalloc_split": round(_timed(lambda: cd.cdvs_scfv_noalloc(S1, d1, c1, 1, pipe.kp_capacity), 50), 4)}
    out["timing"] = (f"{steps} rounds of the three calls, per-kernel events; one-image SCFV: mean of 50 calls "
                     "between events (model constants included)")
    return out


def bmlog_leg(pipe, steps, B):
    """The BMLoG scale space (block frequency-domain Gaussians, Sec. III-A)
    on the same batch against the spatial one, per-kernel events; and the
    detector's keypoints on it against those on the spatial planes."""
    import torch
    import paper_1705_09776_amd as cd
    cd.cdvs_pyramid_bmlog(pipe.ctx, pipe.d_images, pipe.d_pyr)
    torch.cuda.synchronize()
    cd.cdvs_profile_enable(pipe.ctx, True)
    for _ in range(steps):
        cd.cdvs_pyramid_bmlog(pipe.ctx, pipe.d_images, pipe.d_pyr)
    for _ in range(steps):
        pipe.pyramid()
    torch.cuda.synchronize()
    prof = cd.cdvs_profile_read(pipe.ctx)
    cd.cdvs_profile_enable(pipe.ctx, False)
    bm = prof["bmlog"][0] / steps
    sp = (prof["preblur"][0] + prof["scales"][0]) / steps
    # keypoints from the BMLoG planes against the spatial ones (the pipeline
    # buffers hold the spatial pass again afterwards)
    cd.cdvs_pyramid_bmlog(pipe.ctx, pipe.d_images, pipe.d_pyr)
    pipe.detect()
    kb = pipe.keypoints()
    pipe.run()
    torch.cuda.synchronize()
    ks = pipe.keypoints()
    key = lambda k: (int(k["octave"]), int(k["ix"]), int(k["iy"]))
    same = sum(len({key(k) for k in a} & {key(k) for k in b}) for a, b in zip(kb, ks))
    return {"bmlog_ms": round(bm, 4), "spatial_ms": round(sp, 4), "bmlog_over_spatial": round(bm / sp, 3),
            "bmlog_images_per_s": round(B / (bm * 1e-3), 1),
            "keypoints_shared_with_spatial": round(same / max(1, sum(len(a) for a in ks)), 4),
            "timing": f"{steps} calls of each scale space on the batch, per-kernel events"}


def front_leg(steps, n=256):
    """The front end on n images 1280x960 (the high-resolution recipe,
    rendered on the device) brought down to 640x480, then the plain pass:
    the front-end kernel's rate and the whole pass's images/s from the
    high-resolution inputs."""
    import torch
    import paper_1705_09776_amd as cd
    import synth
    W, H = 1280, 960
    src = synth.device_batch(synth.SEED_HIRES, n, W, H, 400, 1200, smax=40.0)
    sdesc = [cd.ImageDesc(i * W * H, W, H, W, 0) for i in range(n)]
    d_sd = cd.descs_to_device(sdesc)
    wo, ho = cd.cdvs_front_size(W, H)
    pipe = cd.Pipeline([(wo, ho)] * n)
    pipe.front_end(src, d_sd)
    if pipe.sync_status() != cd.CDVS_OK:
        raise RuntimeError("front end rejected the batch")
    front_ms = _timed(lambda: pipe.front_end(src, d_sd), steps)

    def whole():
        pipe.front_end(src, d_sd)
        pipe.run()

    whole_ms = _timed(whole, steps)
    fb = n * (W * H + wo * ho)
    return {"images": n, "source": f"{W}x{H}", "output": f"{wo}x{ho}", "front_ms": round(front_ms, 4),
            "front_images_per_s": round(n / (front_ms * 1e-3), 1),
            "roofline": {"bound": "hbm", "achieved": round(fb / (front_ms * 1e-3) / 1e9, 1), "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": round(fb / (front_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)},
            "front_plus_plain_images_per_s": round(n / (whole_ms * 1e-3), 1),
            "timing": f"mean of {steps} eager runs between events (inputs resident in HBM)"}


def host_cpu():
    """CPU model name (from /proc/cpuinfo) and logical CPU counts."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"cpu": model or platform.processor() or platform.machine(), "nproc": os.cpu_count(),
            "usable_cpus": usable}


def cpu_baseline(imgs, seconds: float, ragged_seconds: float):
    """The oracle as it stands, built for this host (fp32, -O3 -march=native,
    -fno-fast-math -ffp-contract=off), over bounded samples of the same
    workloads: one image per thread, as many threads as the process may use
    up to 16 (the host CPUs one GPU of this machine is given).  The batch
    sample cycles through the 256 images; the ragged sample takes the first
    images of the 1024-image uneven-size batch in order."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    import synth
    with tempfile.TemporaryDirectory() as td:
        oracle.use_native(oracle.build_native(td))
        O = oracle.Oracle("f32n")
        cores = max(1, min(16, host_cpu()["usable_cpus"]))
        single = []
        for _ in range(5):                     # one image, one thread: median of 5
            t0 = time.perf_counter()
            O.run(imgs[0], image=0)
            single.append(time.perf_counter() - t0)
        per = sorted(single)[2]
        # about `seconds` of wall time on all threads
        n = max(cores, int(seconds * cores / max(per, 1e-3)))
        t0 = time.perf_counter()
        with ThreadPoolExecutor(cores) as ex:
            list(ex.map(lambda i: O.run(imgs[i % len(imgs)], image=i), range(n)))
        dt = time.perf_counter() - t0
        nr = max(cores, int(ragged_seconds * cores / max(per, 1e-3)))
        rag = synth.ragged_batch(synth.SEED_RAGGED, min(nr, 1024))
        t0 = time.perf_counter()
        with ThreadPoolExecutor(cores) as ex:
            list(ex.map(lambda i: O.run(rag[i], image=i), range(len(rag))))
        dtr = time.perf_counter() - t0
    return {"value": round(n / dt, 3), "unit": "images/s", "cores": cores, "kind": "oracle",
            "build": "fp32, gcc -O3 -march=native -fno-fast-math -ffp-contract=off",
            "single_thread_ms_per_image": round(per * 1e3, 1),
            "ragged_images_per_s": round(len(rag) / dtr, 3),
            "sample": f"{n} images drawn in order from the {len(imgs)}-image 640x480 batch (cycling), whole path "
                      f"per image, one image per thread, {cores} threads, {dt:.1f} s; ragged: the first "
                      f"{len(rag)} of the 1024 uneven-size images, same pool, {dtr:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-ragged-seconds", type=float, default=6.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gated", action="store_true")
    ap.add_argument("--no-ragged", action="store_true")
    ap.add_argument("--no-stream", action="store_true")
    ap.add_argument("--no-single", action="store_true")
    ap.add_argument("--no-sparse", action="store_true")
    ap.add_argument("--stream-images", type=int, default=4096)
    ap.add_argument("--no-aggregate", action="store_true")
    ap.add_argument("--no-front", action="store_true")
    ap.add_argument("--no-bmlog", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(images would shard across GPUs with no exchange); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    import paper_1705_09776_amd as cd

    B = args.batch
    log(f"[bench] generating {B} images 640x480")
    imgs = synth.fixed_batch(synth.SEED_BATCH, B)
    sizes = [(640, 480)] * B
    pipe = cd.Pipeline(sizes)
    pipe.upload(list(imgs))
    torch.cuda.synchronize()
    # the library's autotuner picks the scale tile shape and the detection's
    # launch form for this batch (outside the timed region)
    cd.cdvs_autotune(pipe.ctx, pipe.d_images, pipe.d_pyr, None)
    tuned = {"scale_tile_variant": cd.cdvs_tune_get(pipe.ctx, cd.KERNEL_SCALES),
             "detect_variant": cd.cdvs_tune_get(pipe.ctx, cd.KERNEL_DETECT)}

    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        pipe.run()
    torch.cuda.synchronize()
    if pipe.sync_status() != cd.CDVS_OK:
        raise RuntimeError("capacity overflow during warmup")

    # timed region: K replays of the captured pass (one hipGraph per step)
    pipe.capture()
    pipe.replay()
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} graph replays")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        pipe.replay()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if pipe.sync_status() != cd.CDVS_OK:
        raise RuntimeError("capacity overflow in the timed region")
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = B / (ms_per_step * 1e-3)

    # per-kernel durations: the same K steps launched eagerly, every kernel
    # bracketed by HIP events on the stream it runs on
    cd.cdvs_profile_enable(pipe.ctx, True)
    torch.cuda.synchronize()
    e0 = time.perf_counter()
    for _ in range(args.steps):
        pipe.run()
    torch.cuda.synchronize()
    e1 = time.perf_counter()
    prof = cd.cdvs_profile_read(pipe.ctx)
    cd.cdvs_profile_enable(pipe.ctx, False)
    eager_ms = (e1 - e0) * 1e3 / args.steps

    n_kp = int(pipe.d_count.sum().item())
    n_ori = int(pipe.d_count_ori.sum().item())
    alg = algorithmic(sizes, n_kp, n_ori)
    kernels = {}
    for name, (ms, launches) in prof.items():
        if launches == 0:
            continue
        per_step = launches / args.steps
        kernels[name] = {"ms_per_step": round(ms / args.steps, 4), "launches_per_step": per_step,
                         "avg_launch_us": round(ms * 1e3 / launches, 2)}
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    d = kernels[dom]
    t_step_s = d["ms_per_step"] * 1e-3
    a = alg[dom]
    # roofline of the dominant kernel: its algorithmic bytes (or flops) over its
    # own event-timed duration, per launch averaged over the timed region
    if a["bytes"] is not None and a["flop"] is not None and a["flop"] / a["bytes"] > RIDGE_FLOP_PER_BYTE:
        roof = {"bound": "alu", "achieved": round(a["flop"] / t_step_s / 1e12, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s"}
    elif a["bytes"] is not None:
        roof = {"bound": "hbm", "achieved": round(a["bytes"] / t_step_s / 1e9, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s"}
    else:
        roof = {"bound": "alu", "achieved": None, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s"}
    roof["frac"] = round(roof["achieved"] / roof["peak"], 4) if roof["achieved"] is not None else None
    tv = tuned["scale_tile_variant"]
    step_bytes = measured_traffic(dom, tv) if B == 256 else None   # HBM bytes per step (rocprofv3 counters)
    roof["traffic"] = round(step_bytes / d["launches_per_step"]) if step_bytes is not None else None  # per launch
    roof["kernel"] = dom
    roof["launch_us"] = d["avg_launch_us"]
    hbm_bytes = sum(v["bytes"] for v in alg.values() if v["bytes"] is not None)

    ach = achievable_hbm_gbs()
    path_bytes = measured_path_bytes(tv) if B == 256 else None
    # each kernel's VALU issue fraction: its counted wave instructions x 4
    # cycles over the SIMD-cycles of its event-timed duration
    for name, kd in kernels.items():
        vi = measured_valu(name, tv) if B == 256 else None
        if vi is not None and kd["ms_per_step"] > 0:
            kd["valu_issue"] = round(vi * 4 / (SIMDS * CLOCK_HZ * kd["ms_per_step"] * 1e-3), 3)
    roof["valu_issue"] = kernels[dom].get("valu_issue")
    hbm = {"model_gbs": round(hbm_bytes * args.steps / (t1 - t0) / 1e9, 1), "achievable_stream_gbs": round(ach, 1),
           "model_frac_of_peak": round(hbm_bytes * args.steps / (t1 - t0) / 1e9 / PEAK_HBM_GBS, 4),
           "model_frac_of_achievable": round(hbm_bytes * args.steps / (t1 - t0) / 1e9 / ach, 4)}
    if path_bytes is not None:
        g = path_bytes / (ms_per_step * 1e-3) / 1e9
        hbm.update({"counter_gbs": round(g, 1), "counter_frac_of_peak": round(g / PEAK_HBM_GBS, 4),
                    "counter_frac_of_achievable": round(g / ach, 4)})
    # the target for the plain batched path: 70% of the achievable rate by
    # model bytes; the scale-space and keypoint kernels are bound by vector
    # issue, and the detection, which streams at nearly the achievable rate,
    # moves 1.28x its model bytes (strip halos), so the path falls short of it
    hbm["target_frac_of_achievable"] = 0.70
    hbm["target_met"] = hbm["model_frac_of_achievable"] >= 0.70
    out = {
        "metric": "images/s at 640x480 (plain vs surrogate-gated @>=98% kp recall); HBM GB/s",
        "value": round(value, 1),
        "unit": "images/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded blobs on a ramp with noise, 640x480 u8)",
        "config": {"workload": f"plain path, batch of {B} images 640x480, top-1000 keypoints described per image",
                   "batch": B, "width": 640, "height": 480, "topk": 1000, "path": "plain", **tuned},
        "model_hbm_gbs": round(hbm_bytes * args.steps / (t1 - t0) / 1e9, 1),
        "hbm": hbm,
        "timing": "value: K back-to-back hipGraph replays of the whole pass; kernels: K eager steps with "
                  "per-kernel HIP events",
        "eager_ms_per_step": round(eager_ms, 4),
        "keypoints_per_image": round(n_kp / B, 1),
        "oriented_per_image": round(n_ori / B, 1),
        "kernels": kernels,
        "roofline": roof,
    }
    if os.path.exists(WEIGHTS) and not args.no_gated:
        log("[bench] surrogate-gated leg")
        plain_kp = [k.copy() for k in pipe.keypoints()]
        out["plain_eager_images_per_s"] = round(B / (eager_ms * 1e-3), 1)
        out["gated"] = gated_leg(pipe, args.steps, B, plain_kp)
        g = out["gated"]
        g["vs_plain_eager"] = round(g["eager_images_per_s"] / out["plain_eager_images_per_s"], 4)
        g["vs_plain_graph"] = round(g["value"] / out["value"], 4)
        g["net"] = ("loss: the gate's CNN costs more than the detection it skips"
                    if g["value"] < out["value"] else "gain")
    if not args.no_aggregate and os.path.exists(SCFV_MODEL):
        log("[bench] relevance, transform coding and SCFV on the plain pass's outputs")
        out["aggregate"] = aggregate_leg(pipe, args.steps, B)
    if not args.no_bmlog:
        log("[bench] BMLoG scale space against the spatial one")
        out["bmlog"] = bmlog_leg(pipe, args.steps, B)
    if not args.no_front:
        log("[bench] front end (1280x960 -> 640x480) and plain pass")
        out["front"] = front_leg(args.steps)
    if not args.no_single:
        log("[bench] single image latency")
        out["single"] = single_leg()
    if os.path.exists(WEIGHTS_T4) and not args.no_gated and not args.no_sparse:
        log("[bench] sparse-keypoint sensitivity leg (contrast 4)")
        out["sparse_t4"] = sparse_leg(imgs, args.steps)
    if not args.no_ragged:
        log("[bench] ragged leg (1024 images of uneven size)")
        out["ragged"] = ragged_leg(args.steps)
    if os.path.exists(WEIGHTS) and not args.no_stream:
        log(f"[bench] high-resolution stream ({args.stream_images} images 1280x960)")
        del pipe
        torch.cuda.empty_cache()
        out["stream"] = stream_leg(args.stream_images)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(imgs, args.cpu_seconds, args.cpu_ragged_seconds)
    out["host"] = host_cpu()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
