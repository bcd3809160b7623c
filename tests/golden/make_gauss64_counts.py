"""Write gauss64_counts.json: the extremum and cell counts of the 64^3
Gaussian-sum parity field (8 bumps, seed 0), computed by the CPU oracle
alone.

These are regression values of the oracle, not an independent pin: the
oracle itself is pinned by the exhaustive, closed-form, library and
worked-example tests.  The file guards the parity field against drift of
the input generator or the oracle, and gives the GPU test an expected count.

    python tests/golden/make_gauss64_counts.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2409_03771_amd import synth  # noqa: E402


def main():
    f = synth.config_field("gauss64")
    asc, desc, ms = O.segment(f)
    out = {
        "field": "gauss64: 64^3 float32, sum of 8 Gaussians + U[-1e-4,1e-4] "
                 "noise, seed 0",
        "source": "oracle/ (serial C oracle), written by "
                  "tests/golden/make_gauss64_counts.py",
        "n_maxima": int(np.unique(asc).size),
        "n_minima": int(np.unique(desc).size),
        "n_cells": int(np.unique(ms).size),
    }
    path = os.path.join(HERE, "gauss64_counts.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(path, out)


if __name__ == "__main__":
    main()
