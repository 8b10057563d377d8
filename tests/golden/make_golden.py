"""Writes oracle_values.json: oracle outputs on small seeded inputs, kept as
a regression record of the oracle itself.  Every value comes from oracle/
(nothing from the GPU path); the paper prints no pixel values to store.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import oracle as o  # noqa: E402


def cases():
    tiny = synth.tiny_shot()
    pix_t = synth.pixel_sample(tiny, 64, 1)
    micro_s = synth.micro_shot()
    micro_g = synth.micro_shot(shape=synth.SHAPE_GAUSS)
    pm = micro_s.pixel_list()
    g = np.array([1.0, -0.5, 0.25, 2.0])
    wide = micro_s.replace(n_fast=3, n_slow=2, pixel=6.0e-3, beam_f=-1.4e-2, beam_s=-6.0e-3, roi=None)
    return {
        "tiny_sincg_64px": (pix_t, o.simulate(tiny, pix_t)),
        "micro_sincg": (pm, o.simulate(micro_s, pm)),
        "micro_gauss": (pm, o.simulate(micro_g, pm)),
        "micro_gauss_gradient": (pm, o.gradient(micro_g, pm, g)),
        "tiny_water_background_64px": (pix_t, o.background(tiny, synth.water_background(), pix_t)),
        "wide_air_background": (wide.pixel_list(), o.background(wide, synth.air_background(), wide.pixel_list())),
    }


def main():
    out = {"about": "oracle outputs on seeded synthetic inputs (synth/), written by tests/golden/make_golden.py "
                    "from oracle/ only; pixels are (i_fast, i_slow)",
           "cases": {k: {"pixels": p.tolist(), "values": [float(x) for x in np.ravel(v)]}
                     for k, (p, v) in cases().items()}}
    with open(os.path.join(HERE, "oracle_values.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
