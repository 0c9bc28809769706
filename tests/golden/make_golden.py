"""Write tests/golden/oracle_small64_seed0.json from the FP64 oracle.

Calls only the oracle (and the input generator).  The stored values pin the
oracle against unintended changes of its arithmetic: the 64x64 shape image
of seed 0 decomposed with dt = 0.005, K = 60 samples, 200 Chambolle
iterations per ROF solve, tau = 0.248, cold start (every solve from p = 0,
the oracle's default), dyadic edges
{0, 1, 2, 4, 60}.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2006_10004_amd import synth  # noqa: E402

CASE = dict(seed=0, dt=0.005, K=60, iters=200, tau=0.248, edges=[0, 1, 2, 4, 60])
PIXELS = [(0, 0), (5, 17), (31, 32), (40, 7), (63, 63)]


def compute():
    f = synth.shapes_image(synth.SMALL_64, CASE["seed"])
    r = oracle.decompose(f, CASE["dt"], CASE["K"], CASE["iters"], CASE["edges"], tau=CASE["tau"])
    return {
        "case": CASE,
        "S": r["S"][0].tolist(),
        "band_l1": np.abs(r["bands"][:, 0]).sum(axis=(1, 2)).tolist(),
        "pixels": PIXELS,
        "band_pixels": [[float(r["bands"][j, 0, i, k]) for (i, k) in PIXELS] for j in range(4)],
        "residual_pixels": [float(r["residual"][0, i, k]) for (i, k) in PIXELS],
    }


if __name__ == "__main__":
    with open(os.path.join(HERE, "oracle_small64_seed0.json"), "w") as fh:
        json.dump(compute(), fh, indent=1)
