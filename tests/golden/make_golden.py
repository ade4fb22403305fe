"""Writes tests/golden/oracle_c1_sample.json from the CPU oracle only.

The paper prints no worked numeric example for the renderer, so the stored
values here are the oracle's own outputs on a seeded input (a regression
fixture: any later change to the oracle's arithmetic must name the passage
that justifies it).  Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_2604_10982_amd import scenes  # noqa: E402

PIXELS = [(17, 23), (64, 64), (90, 31), (101, 77), (5, 120), (127, 0)]


def compute():
    sc, cam, K, _ = scenes.config("c1_box2k")
    pix = [y * cam.width + x for x, y in PIXELS]
    r = O.render(sc, cam, K, O.TOPK, pix=pix)
    rf = O.render(sc, cam, K, O.FULL, pix=pix)
    out = {"config": "c1_box2k", "K": K, "pixels": PIXELS,
           "pairs": {m: O.keystage(sc, cam, m, pairs=False)["P"] for m in ("sphere", "aabb", "ellipse")},
           "rgb": r["rgb"].tolist(), "depth": r["depth"].tolist(), "alpha": r["alpha"].tolist(),
           "feat_topk_0_4": r["feat"][:, :4].tolist(), "feat_full_0_4": rf["feat"][:, :4].tolist(),
           "sel_id": r["sel_id"].tolist()}
    return out


if __name__ == "__main__":
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_c1_sample.json")
    with open(path, "w") as f:
        json.dump(compute(), f, indent=1)
    print("wrote", path)
