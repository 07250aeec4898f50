"""Filter-step tile plans for MI355X, found by the library's autotuner (chfsi_autotune_filter).

``python -m paper_1206_3768_amd.autotune`` (on the GPU) times every candidate plan for the listed
shapes and writes ``tuned_plans.json`` next to this file; :func:`load` puts a table into a handle.
Shapes not in the table use the nearest tuned n (within a factor 1.5) or the built-in heuristic.
"""
from __future__ import annotations

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuned_plans.json")

# (n, widths) of the workloads: the n=2048 sequence (m = 192), the n=4096 sequence (m = 320), the
# n=8192 mixed-precision sequence (m = 480) and the batched k-point sizes
SHAPES = [(2048, [192, 144, 96, 48, 32]), (4096, [320, 240, 160, 80, 32]), (8192, [480, 360, 240, 120, 32]),
          (1024, [64, 32]), (512, [48, 32]), (3000, [216, 160, 96, 48]), (6000, [432, 320, 200, 96])]


def load(handle, path: str = TABLE) -> int:
    """Sets every plan of the table in the handle; returns the number of entries (0 if no table)."""
    if not os.path.exists(path):
        return 0
    with open(path) as fh:
        entries = json.load(fh)["plans"]
    for e in entries:
        handle.set_filter_plan(e["n"], e["m"], e["prec"], e["plan"])
    return len(entries)


def main() -> int:
    from . import chfsi
    h = chfsi.Handle(0)
    out = []
    for n, widths in SHAPES:
        for w in widths:
            for prec in (chfsi.FP64, chfsi.FP32, chfsi.BF16X3, chfsi.BF16X6):
                plan, ms = h.autotune_filter(n, w, prec)
                tf = 8.0 * n * n * w / (ms * 1e-3) / 1e12
                out.append({"n": n, "m": w, "prec": prec, "plan": plan, "ms": round(ms, 5), "tflops": round(tf, 2)})
                print(json.dumps(out[-1]), flush=True)
    with open(TABLE, "w") as fh:
        json.dump({"device": "MI355X (gfx950)", "plans": out}, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
