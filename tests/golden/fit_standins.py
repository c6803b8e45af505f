"""Writes the stand-in parameters of the descriptor coding and aggregation
steps, fitted on oracle descriptors of seeded synthetic images:

* SCFV (Sec. III-D): a PCA (128 -> 32) and a 512-component diagonal GMM,
  fitted the usual way (PCA by the eigenvectors of the descriptor
  covariance; GMM by expectation-maximisation in float64);
* keypoint relevance (Sec. III-B, Eqs. (4)-(5)): per characteristic
  (sigma, |p|, distance to the centre, rho, p_ss), 15 bin edges at its
  quantiles over all detected keypoints, and per bin the rate at which a
  keypoint is found again (same octave, within 1 base pixel) when the same
  image gets fresh pixel noise (uniform +-6 levels, added here, rounded
  and clipped) -- the stand-in for "correctly matched" (Laplace-smoothed);
* transform coding (Sec. III-C): per transformed element, the two ternary
  thresholds at its 1/3 and 2/3 quantiles (so that each symbol is about
  equally likely), and a priority order of the elements by the entropy of
  their symbols, highest first (ties: lower element first).

They stand in for the MPEG-CDVS normative parameters, which are not
available here: same shapes, but fitted on synthetic blob images, so they
carry no claim about real images.  Only the oracle computes the
descriptors they are fitted on.

Run from the repository root (about a minute):
    python tests/golden/fit_standins.py
Writes paper_1705_09776_amd/weights/scfv_standin.npz, tq_standin.npz and
relevance_standin.npz (float32 / int32) with a .json note beside each.
"""
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
import synth  # noqa: E402
from oracle import relevance, tq  # noqa: E402

SEED_FIT = 8          # seed base of the fitting images (no other workload uses it)
N_IMAGES = 48
COMPONENTS = 512
PDIM = 32
EM_ITERATIONS = 30
OUT = os.path.join(ROOT, "paper_1705_09776_amd", "weights", "scfv_standin.npz")
OUT_TQ = os.path.join(ROOT, "paper_1705_09776_amd", "weights", "tq_standin.npz")
OUT_REL = os.path.join(ROOT, "paper_1705_09776_amd", "weights", "relevance_standin.npz")
REL_IMAGES = 32
NOISE = 6


def descriptors():
    O = oracle.Oracle("f64")
    imgs = synth.fixed_batch(SEED_FIT, N_IMAGES)
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        out = list(ex.map(lambda i: O.run(imgs[i], image=i)[1], range(N_IMAGES)))
    return np.concatenate(out)


def fit_pca(D):
    m = D.mean(axis=0)
    C = np.cov((D - m).T)
    ev, V = np.linalg.eigh(C)
    A = V[:, np.argsort(ev)[::-1][:PDIM]].T
    # fix each direction's sign: its largest-magnitude entry is positive
    A *= np.sign(A[np.arange(PDIM), np.abs(A).argmax(axis=1)])[:, None]
    return m, A


def fit_gmm(X, rng):
    n = len(X)
    mu = X[rng.choice(n, COMPONENTS, replace=False)].copy()
    floor = 1e-3 * X.var(axis=0).mean()
    var = np.tile(X.var(axis=0), (COMPONENTS, 1))
    w = np.full(COMPONENTS, 1.0 / COMPONENTS)
    for _ in range(EM_ITERATIONS):
        # E step: log w_i + log N(x; mu_i, var_i), normalised per descriptor
        L = (np.log(w)[None, :] - 0.5 * np.sum(np.log(2 * np.pi * var), axis=1)[None, :]
             - 0.5 * ((X * X) @ (1 / var).T - 2 * X @ (mu / var).T + np.sum(mu * mu / var, axis=1)[None, :]))
        L -= L.max(axis=1, keepdims=True)
        G = np.exp(L)
        G /= G.sum(axis=1, keepdims=True)
        # M step; a component that lost all its mass is re-seeded on a random point
        nk = G.sum(axis=0)
        dead = nk < 1e-8
        nk = np.maximum(nk, 1e-12)
        mu = (G.T @ X) / nk[:, None]
        var = np.maximum((G.T @ (X * X)) / nk[:, None] - mu * mu, floor)
        if dead.any():
            mu[dead] = X[rng.choice(n, int(dead.sum()), replace=False)]
            var[dead] = X.var(axis=0)
        w = nk / nk.sum()
    return w, mu, var


def fit_tq(D):
    V = tq.transform(D.astype(np.float32)).astype(np.float64)
    lo = np.quantile(V, 1.0 / 3.0, axis=0)
    hi = np.quantile(V, 2.0 / 3.0, axis=0)
    q = tq.quantise(V, lo.astype(np.float32), hi.astype(np.float32))
    ent = np.zeros(128)
    for s in (-1, 0, 1):
        p = (q == s).mean(axis=0)
        ent -= np.where(p > 0, p * np.log2(np.where(p > 0, p, 1.0)), 0.0)
    order = np.lexsort((np.arange(128), -np.round(ent, 12)))
    return lo, hi, order, ent


def _all_keypoints(O, img):
    H, W = img.shape
    _, flat = O.pyramid(img)
    cand = O.detect(flat, W, H)
    return O.select(cand, O.dedup(cand), 0)


def fit_relevance():
    O = oracle.Oracle("f64")
    imgs = synth.fixed_batch(SEED_FIT, REL_IMAGES)
    rng = np.random.default_rng(SEED_FIT + 1)
    views = [np.clip(np.rint(im.astype(np.float64) + rng.uniform(-NOISE, NOISE, im.shape)), 0, 255).astype(np.uint8)
             for im in imgs]
    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        a = list(ex.map(lambda im: _all_keypoints(O, im), imgs))
        b = list(ex.map(lambda im: _all_keypoints(O, im), views))
    F, hit = [], []
    for ka, kb in zip(a, b):
        H, W = imgs[0].shape
        F.append(relevance.features(ka, W, H))
        m = np.zeros(len(ka), bool)
        for o in np.unique(ka["octave"]):
            ia, jb = np.nonzero(ka["octave"] == o)[0], np.nonzero(kb["octave"] == o)[0]
            if len(jb):
                d = np.hypot(ka["x"][ia, None] - kb["x"][None, jb], ka["y"][ia, None] - kb["y"][None, jb])
                m[ia] = d.min(axis=1) <= 1.0
        hit.append(m)
    F, hit = np.concatenate(F), np.concatenate(hit)
    edges = np.stack([np.quantile(F[:, k].astype(np.float64), np.arange(1, 16) / 16.0) for k in range(5)])
    edges = edges.astype(np.float32)
    b = relevance.bins(F, edges)
    values = np.zeros((5, 16))
    for k in range(5):
        for j in range(16):
            sel = b[:, k] == j
            values[k, j] = (hit[sel].sum() + 1.0) / (sel.sum() + 2.0)
    return edges, values.astype(np.float32), len(F), float(hit.mean())


def main():
    t0 = time.time()
    D = descriptors()
    m, A = fit_pca(D)
    X = (D - m) @ A.T
    w, mu, var = fit_gmm(X, np.random.default_rng(SEED_FIT))
    np.savez(OUT, pca_mean=m.astype(np.float32), pca_matrix=A.astype(np.float32), weights=w.astype(np.float32),
             means=mu.astype(np.float32), variances=var.astype(np.float32))
    note = {"what": "stand-in SCFV parameters (PCA 128->32, 512-component diagonal GMM), fitted on oracle "
                    "descriptors of seeded synthetic images; not the MPEG-CDVS normative parameters",
            "images": N_IMAGES, "seed_base": SEED_FIT, "descriptors": int(len(D)), "em_iterations": EM_ITERATIONS,
            "min_weight": float(w.min()), "max_weight": float(w.max()),
            "pca_variance_kept": float(np.var(X, axis=0).sum() / np.var(D, axis=0).sum()),
            "fit_s": round(time.time() - t0, 1)}
    with open(os.path.splitext(OUT)[0] + ".json", "w") as f:
        json.dump(note, f, indent=1)
    print(json.dumps(note))
    lo, hi, order, ent = fit_tq(D)
    np.savez(OUT_TQ, lo=lo.astype(np.float32), hi=hi.astype(np.float32), order=order.astype(np.int32))
    note = {"what": "stand-in ternary-quantisation thresholds (1/3 and 2/3 quantiles of each transformed element) "
                    "and element priority (symbol entropy, highest first) fitted on oracle descriptors of seeded "
                    "synthetic images; not the MPEG-CDVS normative thresholds",
            "images": N_IMAGES, "seed_base": SEED_FIT, "descriptors": int(len(D)),
            "entropy_bits_first_16": [round(float(e), 4) for e in ent[order[:16]]],
            "entropy_bits_total": round(float(ent.sum()), 2)}
    with open(os.path.splitext(OUT_TQ)[0] + ".json", "w") as f:
        json.dump(note, f, indent=1)
    print(json.dumps(note))
    edges, values, nkp, rate = fit_relevance()
    np.savez(OUT_REL, edges=edges, values=values)
    note = {"what": "stand-in relevance tables (per characteristic sigma, |p|, centre distance, rho, p_ss: 15 "
                    "quantile bin edges and 16 repeat rates) fitted on oracle keypoints of seeded synthetic images "
                    "against a re-noised copy; not the MPEG-CDVS normative tables",
            "images": REL_IMAGES, "seed_base": SEED_FIT, "keypoints": nkp, "noise_levels": NOISE,
            "repeat_rate": round(rate, 4),
            "value_range": [[round(float(v.min()), 4), round(float(v.max()), 4)] for v in values]}
    with open(os.path.splitext(OUT_REL)[0] + ".json", "w") as f:
        json.dump(note, f, indent=1)
    print(json.dumps(note))


if __name__ == "__main__":
    main()
