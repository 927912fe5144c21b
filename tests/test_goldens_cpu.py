"""The stored full-size oracle embeddings are the oracle's: re-derive the
first image of every case from oracle/ and synth/ and compare (CPU)."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import vit64 as O

GOLDEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
GOLDENS = json.load(open(os.path.join(GOLDEN_DIR, "goldens.json")))


def test_every_case_has_its_file():
    for name, g in GOLDENS.items():
        ref = np.load(os.path.join(GOLDEN_DIR, g["file"]))
        assert ref.shape == (len(g["sizes"]), synth.MODELS[g["model"]].proj_dim), name
        assert ref.dtype == np.float64
        assert np.allclose(np.linalg.norm(ref, axis=1), 1.0, atol=1e-12)


@pytest.mark.parametrize("name", sorted(GOLDENS))
def test_first_image_rederived(name):
    g = GOLDENS[name]
    c = synth.MODELS[g["model"]]
    h, w = g["sizes"][0]
    img = synth.make_images([(h, w)], g["images_seed"])[0]
    p = O.weights_for(synth.make_params(c, g["weights_seed"]), g["precision"])
    ref = np.load(os.path.join(GOLDEN_DIR, g["file"]))
    assert np.max(np.abs(O.encode([img], p, c)[0] - ref[0])) <= 1e-12
