"""Writes tests/golden/batch16_oracle.json: the CPU oracle's results for the
first nine problems of the sixteen-problem batch (one per (refinement, nz)
pair: refinements 4, 5, 6 x nz 32, 64, 128, quadratic grading, seeded
uniform right-hand sides), for the batched-solve parity test at the batch's
own shape.

Calls only oracle/ and synth/ (the seeded inputs). Stored per problem: the
FP64 and mixed (FP32 V-cycle) FCG iteration counts at rtol 1e-8, values of
the FP64 solution at 64 seeded sample cells, and the relative distance
between the oracle's own mixed and FP64 solutions at those samples.

usage: python tests/golden/make_batch16.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import tpmg  # noqa: E402


def main():
    t0 = time.time()
    out = {"source": "oracle/ (CPU FP64 TPMG-FCG), tests/golden/make_batch16.py", "problems": []}
    for i, w in enumerate(synth.batch_list()[:9]):
        h = tpmg.build(w.refinement, w.r_faces(), w.omega2)
        fine = h.meshes[-1]
        f = synth.make_rhs(w, fine.centre, fine.area, h.vert.vk)
        rng = np.random.default_rng(5000 + i)
        cells = np.sort(rng.choice(fine.n, 64, replace=False))
        levels = rng.integers(0, w.nz, 64)
        s64 = tpmg.solve(h, f, rtol=1e-8)
        s32 = tpmg.solve(h, f, rtol=1e-8, precision="fp32")
        x64 = s64.x[cells, levels]
        x32 = s32.x[cells, levels]
        out["problems"].append({
            "index": i, "name": w.name, "refinement": w.refinement, "nz": w.nz,
            "sample_cells": cells.tolist(), "sample_levels": levels.tolist(),
            "fp64_iters": s64.iters, "mixed_iters": s32.iters,
            "fp64_x_samples": x64.tolist(),
            "mixed_vs_fp64": float(np.max(np.abs(x32 - x64)) / np.max(np.abs(x64))),
        })
        print(f"{w.name} ref {w.refinement} nz {w.nz}: fp64 {s64.iters}, mixed {s32.iters} iterations, "
              f"{time.time() - t0:.1f} s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch16_oracle.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
