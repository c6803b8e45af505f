"""Writes synth_sha256.txt: SHA-256 of a few generated images, frozen when
first generated so that any later change to the input recipe is noticed.
Run from the repository root: python tests/golden/make_synth_golden.py"""
import hashlib
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
import synth  # noqa: E402

CASES = [  # (seed, index, width, height, nblobs, smax)
    (synth.SEED_SINGLE, 0, 640, 480, 200, 20.0),
    (synth.SEED_BATCH, 0, 640, 480, 200, 20.0),
    (synth.SEED_BATCH, 255, 640, 480, 200, 20.0),
    (synth.SEED_HIRES, 3, 1280, 960, 800, 40.0),
]


def main():
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "synth_sha256.txt")
    with open(out, "w") as f:
        f.write("# seed index width height nblobs smax sha256\n")
        for seed, idx, w, h, nb, smax in CASES:
            img = synth.image(seed, idx, w, h, nblobs=nb, smax=smax)
            f.write(f"{seed} {idx} {w} {h} {nb} {smax} {hashlib.sha256(img.tobytes()).hexdigest()}\n")
    print("wrote", out)


if __name__ == "__main__":
    main()
