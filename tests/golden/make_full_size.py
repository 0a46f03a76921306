"""Writes tests/golden/<workload>_oracle.json: the CPU oracle's results on a
full-size workload, for the GPU parity tests at that size.

Calls only oracle/ and synth/ (the seeded inputs). Stored: FP64 and mixed
FCG iteration counts and residual histories (rtol 1e-8), and values at 256
seeded sample cells of the FP64 solution, of one FP64 V-cycle applied to the
right-hand side, and of A x for a seeded random x. With --rates also the
V-cycle convergence factors (Section 5.2: the V-cycle in the Richardson
iteration, f = 0, 12 cycles from seeded U[-1, 1] values, seed 7) of the FP64
and of the FP32 V-cycle.

usage: python tests/golden/make_full_size.py [workload] [--rates]
       (default ico6_nz128)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import operator as opm, tpmg  # noqa: E402


def main(name="ico6_nz128", *flags):
    w = synth.workload(name)
    t0 = time.time()
    h = tpmg.build(w.refinement, w.r_faces(), w.omega2)
    fine = h.meshes[-1]
    f = synth.make_rhs(w, fine.centre, fine.area, h.vert.vk)
    rng = np.random.default_rng(1234)
    cells = np.sort(rng.choice(fine.n, 256, replace=False))
    levels = rng.integers(0, w.nz, 256)
    x = np.random.default_rng(99).standard_normal(f.shape)
    ax = opm.apply(h.finest, x)
    del x
    z = tpmg.vcycle(h, f)
    print(f"setup + spmv + vcycle {time.time() - t0:.1f} s", flush=True)
    s64 = tpmg.solve(h, f, rtol=1e-8)
    print(f"fp64 solve: {s64.iters} iterations, {time.time() - t0:.1f} s", flush=True)
    out = {
        "workload": name,
        "source": "oracle/ (CPU FP64 TPMG-FCG), tests/golden/make_full_size.py",
        "sample_cells": cells.tolist(),
        "sample_levels": levels.tolist(),
        "spmv_x_seed": 99,
        "spmv_samples": ax[cells, levels].tolist(),
        "vcycle_samples": z[cells, levels].tolist(),
        "vcycle_norm": float(np.linalg.norm(z)),
        "fp64": {"iters": s64.iters, "history": s64.history, "x_samples": s64.x[cells, levels].tolist(),
                 "x_norm": float(np.linalg.norm(s64.x))},
    }
    del s64, z, ax
    s32 = tpmg.solve(h, f, rtol=1e-8, precision="fp32")
    print(f"mixed solve: {s32.iters} iterations, {time.time() - t0:.1f} s", flush=True)
    out["mixed"] = {"iters": s32.iters, "history": s32.history, "x_norm": float(np.linalg.norm(s32.x))}
    del s32
    if "--rates" in flags:
        out["rate_seed"] = 7
        out["rate_cycles"] = [12, 4]
        out["fp64"]["vcycle_rate"] = tpmg.richardson_rate(h, seed=7, cycles=12, skip=4)
        print(f"fp64 rate {out['fp64']['vcycle_rate']:.6f}, {time.time() - t0:.1f} s", flush=True)
        out["mixed"]["vcycle_rate"] = tpmg.richardson_rate(h, seed=7, cycles=12, skip=4, precision="fp32")
        print(f"fp32 rate {out['mixed']['vcycle_rate']:.6f}, {time.time() - t0:.1f} s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_oracle.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main(*sys.argv[1:])
