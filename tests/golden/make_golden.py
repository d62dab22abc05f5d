"""Writes tests/golden/config0_oracle.json from the FP64 oracle alone.

The paper prints no worked example (its figures are images of LOFAR fields and
its tables are timings), so the stored values here are the oracle's own
output on the seeded tiny configuration: a regression fixture that makes any
later change to the oracle's arithmetic visible.  Run:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2411_07321_amd import synth  # noqa: E402


def summary():
    ds = synth.config0()
    inp = oracle.Inputs.make(ds.uvw, ds.freq_hz, ds.vis, ds.weights, ds.flags)
    prm = oracle.Params(ds.grid_n, ds.n_wplanes, ds.support, ds.cell_rad, ds.kernel_sigma)
    out = oracle.image(inp, prm)
    img = out["image"][0]
    src = []
    for l, m in zip(ds.sky.l, ds.sky.m):
        p = int(round(l / ds.cell_rad)) + ds.grid_n // 2
        q = int(round(m / ds.cell_rad)) + ds.grid_n // 2
        src.append([q, p, float(img[q, p])])
    st = out["stats"][0]
    return {
        "config": "config0 (seed 1000): 256^2, 8 w-planes, support 7, sigma 0.9, FP64",
        "stats": {k: (float(v) if isinstance(v, float) else int(v)) for k, v in st.items()},
        "image_sum": float(img.sum()),
        "image_l2": float(np.linalg.norm(img)),
        "image_max": float(img.max()),
        "source_pixels": src,
    }


if __name__ == "__main__":
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config0_oracle.json")
    with open(path, "w") as f:
        json.dump(summary(), f, indent=1)
    print("wrote", path)
