"""Write tests/golden/fp32_sensitivity.json: how much the FP64 oracle's own
result moves under the disturbances FP32 brings, over the 100 steps of the
full-size FP32 comparisons, on the same recipes at sizes the oracle runs in
minutes (the 256^3 turbulent box recipe at 64^3, the eight-group 128^3 box
recipe at 32^3).  The disturbances are those of fp32_response in
tests/gpu_common.py: E and F held in FP32 (rounded at the start and after
every step) and the reconstructed face values perturbed at the FP32
rounding level ("fp32") or 2^6 times above it ("flip", certain to flip
face-fix decisions).  Per field: rel-L1 = sum|d| / sum|ref|,
rel-Linf = max|d| / max|ref|, and the fraction of cells with
|d| > 1e-5 max|ref| (the cells a flip has reached).

It calls only the oracle, the shared input generator and the test
helpers' disturbance runs.

    python tests/golden/make_fp32_sensitivity.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from paper_2606_26268_amd import inputs as I  # noqa: E402
from tests import gpu_common as G  # noqa: E402

FIELDS = ("E", "Fx", "Fy", "Fz", "mx", "my", "mz", "Eg")
STEPS = 100


def cases():
    box = I.make_turbulent_box(64, 1, 5.2083e-5 * 128 / 64, STEPS, "box64")
    mg = I.make_multigroup(8, (32, 32, 32), steps=STEPS)
    return {"turbulent_box_64": box, "multigroup8_box_32": mg}


def stats(a, ref):
    out = {}
    for k, v in G._field_stats(a, ref, FIELDS).items():
        out[k] = {"rel_l1": float(v["l1"]), "rel_linf": float(v["linf"]),
                  "frac_above": v["flips"] / a[k].size}
    return out


def main():
    res = {"steps": STEPS, "threshold": G.FLIP_THRESHOLD, "face_noise": G.FACE_NOISE,
           "flip_noise": G.FLIP_NOISE, "cases": {}}
    for name, p in cases().items():
        t0 = time.perf_counter()
        mg = p.groups is not None
        o = orc.Oracle(p)
        ref = (o.run_mg if mg else o.run)(p.fields, p.dt, STEPS)[0]
        resp = G.fp32_response(orc, p, STEPS)
        res["cases"][name] = {"cells": int(np.prod(p.n)), "dt": p.dt,
                              "fp32": stats(resp["fp32"], ref), "flip": stats(resp["flip"], ref)}
        print(f"{name}: {time.perf_counter() - t0:.0f} s", flush=True)
        for kind in ("fp32", "flip"):
            r = res["cases"][name][kind]
            print("  " + kind + " " + " ".join(f"{k}:{v['rel_l1']:.1e}/{v['rel_linf']:.1e}/{v['frac_above']:.1e}"
                                              for k, v in r.items()), flush=True)
    with open(os.path.join(HERE, "fp32_sensitivity.json"), "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
