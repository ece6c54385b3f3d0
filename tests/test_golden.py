"""Values fixed by the paper's printed formulas (no GPU)."""
import json
import os

import numpy as np

from paper_1911_10487_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_paper_model_solution_values():
    with open(os.path.join(GOLD, "paper_model_solution.json")) as fh:
        g = json.load(fh)
    for pt in g["points"]:
        x, y, z = pt["xyz"]
        assert abs(synth.paper_contrast(x, y, z, g["a0"]) - pt["xi"]) < 1e-14, pt["why"]
