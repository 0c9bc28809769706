"""Regression pin: the oracle still reproduces the values its own committed
script (tests/golden/make_golden.py) stored."""
import json
import os

import numpy as np

from paper_2006_10004_amd import synth

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_small64_seed0.json")


def test_oracle_matches_stored_values(orc):
    g = json.load(open(GOLD))
    c = g["case"]
    f = synth.shapes_image(synth.SMALL_64, c["seed"])
    r = orc.decompose(f, c["dt"], c["K"], c["iters"], c["edges"], tau=c["tau"])
    assert np.allclose(r["S"][0], g["S"], rtol=1e-12, atol=1e-12)
    assert np.allclose(np.abs(r["bands"][:, 0]).sum(axis=(1, 2)), g["band_l1"], rtol=1e-12)
    for j, row in enumerate(g["band_pixels"]):
        for (i, k), v in zip(g["pixels"], row):
            assert abs(r["bands"][j, 0, i, k] - v) < 1e-14
    for (i, k), v in zip(g["pixels"], g["residual_pixels"]):
        assert abs(r["residual"][0, i, k] - v) < 1e-14
