"""Shared helpers of the parity tests: input packing and error metrics."""
from __future__ import annotations

import functools
from typing import List, Sequence, Tuple

import numpy as np

import synth


@functools.lru_cache(maxsize=4)
def blob(model: str, seed: int) -> np.ndarray:
    return synth.make_blob(synth.MODELS[model], seed)


def params(model: str, seed: int):
    return synth.blob_to_params(synth.MODELS[model], blob(model, seed))


def pack(images: Sequence[np.ndarray]) -> np.ndarray:
    return np.ascontiguousarray(np.concatenate([im.reshape(-1) for im in images]))


def sizes_of(images: Sequence[np.ndarray]) -> List[Tuple[int, int]]:
    return [(int(im.shape[1]), int(im.shape[2])) for im in images]


def rel_err(got: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Per-row ||got - ref|| / ||ref||."""
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    return np.linalg.norm(got - ref, axis=-1) / np.linalg.norm(ref, axis=-1)


def cosine(got: np.ndarray, ref: np.ndarray) -> np.ndarray:
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    return (got * ref).sum(-1) / np.linalg.norm(got, axis=-1) / np.linalg.norm(ref, axis=-1)


def certified_top1(logits_ref: np.ndarray, emb_err: np.ndarray, scale: float):
    """Rows whose reference top-1 / top-2 logit gap exceeds 2*scale*||de||:
    for those, no perturbation of that size can change the argmax."""
    s = np.sort(logits_ref, axis=1)
    gap = s[:, -1] - s[:, -2]
    return gap > 2.0 * scale * emb_err


def rescale_excursion(s_log2: np.ndarray, tile: int = 64) -> float:
    """Largest amount, over the rows of a score matrix in log2 units, by which
    a key tile's maximum exceeds the maximum of all earlier tiles (-inf
    entries are masked keys).  Above 8, the BF16 attention kernel's lazy
    rescale runs for that row."""
    n = s_log2.shape[1]
    run = np.max(s_log2[:, :tile], axis=1)
    best = -np.inf
    for t in range(1, (n + tile - 1) // tile):
        tm = np.max(s_log2[:, tile * t:tile * (t + 1)], axis=1)
        ok = np.isfinite(tm) & np.isfinite(run)
        if ok.any():
            best = max(best, float(np.max(tm[ok] - run[ok])))
        run = np.maximum(run, tm)
    return best
