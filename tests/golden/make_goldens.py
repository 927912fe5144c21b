"""Write the FP64 oracle embeddings the full-size GPU parity tests compare
against, one .npy per case plus the index goldens.json (model, precision,
seeds, image sizes).  Calls only oracle/ and synth/:

    python tests/golden/make_goldens.py [case ...]      (about 5 minutes)

Cases: every image of the ViT-B/16 224 px batch (64, FP32 and BF16 weights),
of the ViT-L/14 336 px batch (32, BF16), of the mixed-resolution ViT-B/16
batch (96 images from {224, 336, 448}, BF16), two ViT-L/14 images at each
serving resolution {224, 336, 384, 448} with e4m3 per-row weights, and two
ViT-L/14 336 px images with FP32 weights.  Seeds follow the workloads'
convention (weights 1000+k, images 2000+k, resolutions 4000+k).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import vit64 as O  # noqa: E402


def cases():
    mixed = synth.draw_resolutions(96, (224, 336, 448), 4003)
    out = {
        "b16_224_fp32": ("b16", "fp32", 1001, 2001, [(224, 224)] * 64),
        "b16_224_bf16": ("b16", "bf16", 1001, 2001, [(224, 224)] * 64),
        "l14_336_bf16": ("l14", "bf16", 1002, 2002, [(336, 336)] * 32),
        "b16_mixed_bf16": ("b16", "bf16", 1003, 2003, [(r, r) for r in mixed]),
        "l14_336_fp32": ("l14", "fp32", 1002, 2002, [(336, 336)] * 2),
    }
    for r in (224, 336, 384, 448):
        out[f"l14_fp8w_{r}"] = ("l14", "fp8w", 1004, 2004 + r, [(r, r)] * 2)
    return out


def main(argv):
    want = set(argv) or None
    idx_path = os.path.join(HERE, "goldens.json")
    index = json.load(open(idx_path)) if os.path.exists(idx_path) else {}
    for name, (model, prec, w_seed, i_seed, sizes) in cases().items():
        if want and name not in want:
            continue
        t0 = time.time()
        c = synth.MODELS[model]
        p = O.weights_for(synth.make_params(c, w_seed), prec)
        imgs = synth.make_images(sizes, i_seed)
        emb = O.encode(imgs, p, c)
        np.save(os.path.join(HERE, f"{name}.npy"), emb)
        index[name] = {"model": model, "precision": prec, "weights_seed": w_seed,
                       "images_seed": i_seed, "sizes": [list(s) for s in sizes],
                       "file": f"{name}.npy"}
        print(f"{name}: {len(imgs)} images in {time.time() - t0:.1f} s", flush=True)
    with open(idx_path, "w") as f:
        json.dump(index, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
