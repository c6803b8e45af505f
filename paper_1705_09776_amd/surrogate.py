"""Training and evaluation of the surrogate candidate mask (driving the
library's own forward, backward and Adam kernels; Python only marshals).

Labels come from the plain detector: every keypoint it keeps (top-k set
high, so all of them) marks the cell of its integer position, per octave.
The loss is the positive-weighted cross-entropy of the library (weights
n_neg / n_pos per octave, clamped to 50, estimated on the first batch).
Checkpoints hold the fp32 parameters, both Adam moments, the step and the
data cursor, with a SHA-256 over all of them.
"""
from __future__ import annotations

import hashlib
import io
import time

import numpy as np

from . import (CNN_CHANNELS, CNN_HEADS, CNN_LAYERS, CNN_PARAMS, Pipeline, cdvs_cnn_adam, cdvs_cnn_backward,
               cdvs_cnn_labels, default_params)

LABEL_TOPK = 4096


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal 3x3 weights, zero conv biases, small head with bias -2."""
    rng = np.random.default_rng(seed)
    parts = []
    for _ in range(CNN_LAYERS):
        parts.append(rng.normal(0.0, np.sqrt(2.0 / (9 * CNN_CHANNELS)), size=9 * CNN_CHANNELS * CNN_CHANNELS))
        parts.append(np.zeros(CNN_CHANNELS))
    parts.append(rng.normal(0.0, np.sqrt(1.0 / CNN_CHANNELS), size=CNN_CHANNELS * CNN_HEADS))
    parts.append(np.full(CNN_HEADS, -2.0))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == CNN_PARAMS
    return p


def label_pipeline(batch: int, width=640, height=480, contrast=None) -> Pipeline:
    p = default_params()
    p.topk = LABEL_TOPK
    if contrast is not None:
        p.contrast = contrast
    return Pipeline([(width, height)] * batch, params=p, kp_capacity=LABEL_TOPK)


# Training recipes: image size and generator arguments.
RECIPES = {
    "vga": dict(width=640, height=480, nmin=200, nmax=200, smax=20.0),
    "hires": dict(width=1280, height=960, nmin=400, nmax=1200, smax=40.0),
}


class Trainer:
    """recipe "vga": 640x480, 200 blobs, sigma U[2, 20] (host generator);
    recipe "hires": 1280x960, 400-1200 blobs, sigma U[2, 40], rendered on the
    device straight into the batch buffer."""

    def __init__(self, batch=32, width=None, height=None, lr=1e-3, seed=0, data_seed=4, dataset=20000,
                 recipe="vga", contrast=None):
        import torch
        self.torch = torch
        self.recipe = RECIPES[recipe]
        width = width or self.recipe["width"]
        height = height or self.recipe["height"]
        self.batch, self.lr, self.data_seed = batch, lr, data_seed
        self.dataset = dataset   # training images are indices 0..dataset-1, visited in order, epoch after epoch
        self.width, self.height = width, height
        self.on_device = recipe == "hires"
        self.contrast = contrast    # detector contrast threshold of the labels (None: the default)
        self.pipe = label_pipeline(batch, width, height, contrast)
        self.pipe.cnn_buffers()
        dev = self.pipe.d_pyr.device
        self.params = torch.from_numpy(init_params(seed)).to(dev)
        self.m = torch.zeros(CNN_PARAMS, dtype=torch.float32, device=dev)
        self.v = torch.zeros_like(self.m)
        self.grad = torch.zeros_like(self.m)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.labels = torch.zeros(self.pipe.ncells, dtype=torch.int32, device=dev)
        self.work = torch.empty(2 * self.pipe.ncells * CNN_CHANNELS, dtype=torch.int16, device=dev)
        self.pos_weight = None
        self.step = 0
        self.cursor = 0          # index of the next training image

    # -- data -----------------------------------------------------------
    def render_next(self):
        """Render the next batch on the device into the pipeline's image buffer."""
        import synth
        r, first = self.recipe, self.cursor % self.dataset
        n = min(self.batch, self.dataset - first)
        stride = self.pipe.image_bytes // self.batch
        assert stride == self.width * self.height
        kw = dict(smax=r["smax"])
        synth.device_batch(self.data_seed, n, self.width, self.height, r["nmin"], r["nmax"], first=first,
                           out=self.pipe.d_images, **kw)
        if n < self.batch:
            synth.device_batch(self.data_seed, self.batch - n, self.width, self.height, r["nmin"], r["nmax"], first=0,
                               out=self.pipe.d_images[n * stride:], **kw)
        self.cursor += self.batch

    def next_images(self):
        import synth
        first = self.cursor % self.dataset
        n = min(self.batch, self.dataset - first)
        imgs = list(synth.fixed_batch(self.data_seed, n, self.width, self.height, first=first))
        if n < self.batch:
            imgs += list(synth.fixed_batch(self.data_seed, self.batch - n, self.width, self.height, first=0))
        self.cursor += self.batch
        return list(imgs)

    def make_labels(self):
        self.pipe.pyramid()
        self.pipe.detect()
        cdvs_cnn_labels(self.pipe.ctx, self.pipe.d_kp, self.pipe.d_count, self.labels)

    def estimate_pos_weight(self):
        lab = self.labels.cpu().numpy().view(np.uint32)
        w = []
        for o in range(CNN_HEADS):
            pos = int(((lab >> o) & 1).sum())
            neg = lab.size - pos
            w.append(min(50.0, neg / pos) if pos else 1.0)
        self.pos_weight = self.torch.tensor(w, dtype=self.torch.float32, device=self.params.device)

    # -- one step ---------------------------------------------------------
    def train_step(self, images=None) -> float:
        if images is None and self.on_device:
            self.render_next()
        else:
            self.pipe.upload(images if images is not None else self.next_images())
        self.make_labels()
        if self.pos_weight is None:
            self.estimate_pos_weight()
        self.pipe.cnn_forward(self.params, tau=None, logits=True)
        cdvs_cnn_backward(self.pipe.ctx, self.pipe.d_images, self.params, self.pipe.d_acts, self.pipe.d_logits,
                          self.labels, self.pos_weight, self.work, self.grad, self.loss)
        self.step += 1
        cdvs_cnn_adam(self.pipe.ctx, self.params, self.grad, self.m, self.v, self.step, lr=self.lr)
        return float(self.loss.item())

    def train(self, n_images: int, log_every=50, log=print):
        t0 = time.perf_counter()
        losses = []
        while self.cursor < n_images:
            losses.append(self.train_step())
            if log and self.step % log_every == 0:
                log(f"step {self.step} images {self.cursor} loss {np.mean(losses[-log_every:]):.5f} "
                    f"{time.perf_counter() - t0:.1f}s")
        return losses

    # -- checkpoints --------------------------------------------------------
    def state(self) -> dict:
        return {"params": self.params.cpu().numpy(), "m": self.m.cpu().numpy(), "v": self.v.cpu().numpy(),
                "pos_weight": (self.pos_weight.cpu().numpy() if self.pos_weight is not None
                               else np.zeros(0, dtype=np.float32)),
                "step": np.array([self.step], dtype=np.int64), "cursor": np.array([self.cursor], dtype=np.int64),
                "data_seed": np.array([self.data_seed], dtype=np.int64)}

    def save(self, path: str):
        save_checkpoint(path, self.state())

    def load(self, path: str):
        st = load_checkpoint(path)
        t = self.torch
        dev = self.params.device
        self.params.copy_(t.from_numpy(st["params"]).to(dev))
        self.m.copy_(t.from_numpy(st["m"]).to(dev))
        self.v.copy_(t.from_numpy(st["v"]).to(dev))
        self.pos_weight = (t.from_numpy(st["pos_weight"]).to(dev) if st["pos_weight"].size else None)
        self.step = int(st["step"][0])
        self.cursor = int(st["cursor"][0])
        self.data_seed = int(st["data_seed"][0])


_CKPT_KEYS = ["params", "m", "v", "pos_weight", "step", "cursor", "data_seed"]


def _digest(state: dict) -> str:
    h = hashlib.sha256()
    for k in _CKPT_KEYS:
        a = np.ascontiguousarray(state[k])
        h.update(k.encode())
        h.update(str(a.dtype).encode())
        h.update(a.tobytes())
    return h.hexdigest()


def save_checkpoint(path: str, state: dict):
    buf = io.BytesIO()
    np.savez(buf, sha256=np.frombuffer(_digest(state).encode(), dtype=np.uint8), **{k: state[k] for k in _CKPT_KEYS})
    with open(path, "wb") as f:
        f.write(buf.getvalue())


def load_checkpoint(path: str) -> dict:
    """Loads a checkpoint written by save_checkpoint; raises ValueError when
    its checksum does not match its contents."""
    with np.load(path, allow_pickle=False) as z:
        state = {k: z[k] for k in _CKPT_KEYS}
        stored = bytes(z["sha256"]).decode()
    if _digest(state) != stored:
        raise ValueError(f"checkpoint {path}: checksum mismatch")
    return state


def evaluate(params, images, taus, topk=1000, fmax=None, contrast=None):
    """Recall of the gated detector against the plain one on `images`.

    Returns one dict per tau: recall over all final keypoints (top-k set to
    the label capacity) and over the top-`topk`, and the fraction of active
    (cell, octave) entries of the mask."""
    import torch
    from . import cdvs_alp_detect
    sizes = [(im.shape[1], im.shape[0]) for im in images]
    out = []
    p = default_params()
    p.topk = topk
    if fmax is not None:
        p.mask_fmax = fmax
    if contrast is not None:
        p.contrast = contrast
    pipe_k = Pipeline(sizes, params=p, kp_capacity=max(topk, 1))
    pipe_all = label_pipeline(len(images), *sizes[0], contrast=contrast) if len(set(sizes)) == 1 else None
    pipe_k.upload(images)
    pipe_k.cnn_buffers()
    pipe_k.pyramid()
    pipe_k.detect()
    plain_k = pipe_k.keypoints()
    plain_all = None
    if pipe_all is not None:
        pipe_all.upload(images)
        pipe_all.pyramid()
        pipe_all.detect()
        plain_all = pipe_all.keypoints()
        pipe_all.cnn_buffers()
    dparams = params if hasattr(params, "data_ptr") else torch.from_numpy(np.asarray(params, np.float32)).cuda()
    key = lambda k: (int(k["octave"]), int(k["ix"]), int(k["iy"]))
    for tau in taus:
        pipe_k.cnn_forward(dparams, tau=tau, logits=False, keep_acts=False)
        cdvs_alp_detect(pipe_k.ctx, pipe_k.d_pyr, pipe_k.d_mask, pipe_k.d_kp, pipe_k.d_count)
        gk = pipe_k.keypoints()
        hit = sum(len({key(k) for k in a} & {key(k) for k in b}) for a, b in zip(plain_k, gk))
        rec = {"tau": tau, "recall_topk": hit / max(1, sum(len(a) for a in plain_k))}
        mask = pipe_k.d_mask.cpu().numpy()
        n_oct = [pipe_k.num_octaves(i) for i in range(len(images))]
        rec["active_fraction_per_octave"] = []
        for o in range(CNN_HEADS):
            a = t = 0
            for i in range(len(images)):
                if o < n_oct[i]:
                    c0, w4, h4 = pipe_k.cell_layout(i)
                    a += int(((mask[c0:c0 + w4 * h4] >> o) & 1).sum())
                    t += w4 * h4
            if t:
                rec["active_fraction_per_octave"].append(round(a / t, 4))
        act, tot = 0, 0
        for i in range(len(images)):
            c0, w4, h4 = pipe_k.cell_layout(i)
            m = mask[c0:c0 + w4 * h4]
            for o in range(min(n_oct[i], CNN_HEADS)):
                act += int(((m >> o) & 1).sum())
                tot += m.size
        rec["active_fraction"] = act / max(1, tot)
        if pipe_all is not None:
            pipe_all.d_mask.copy_(pipe_k.d_mask)
            cdvs_alp_detect(pipe_all.ctx, pipe_all.d_pyr, pipe_all.d_mask, pipe_all.d_kp, pipe_all.d_count)
            ga = pipe_all.keypoints()
            hit = sum(len({key(k) for k in a} & {key(k) for k in b}) for a, b in zip(plain_all, ga))
            rec["recall_all"] = hit / max(1, sum(len(a) for a in plain_all))
        out.append(rec)
    torch.cuda.synchronize()
    return out
