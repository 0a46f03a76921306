"""Shared helpers of the GPU parity tests: build the same problem on the
oracle (CPU, FP64) and on the HIP library, from the same seeded inputs."""
import numpy as np

import synth
from oracle import tpmg as otpmg

CASES = {
    # name: (refinement, nz, grading, seed, random profiles)
    "ico2_nz8_rand": (2, 8, "uniform", 1, True),          # coarse grids padded (80 -> 128, 20 -> 64 columns)
    "ico3_nz13_quad": (3, 13, "quadratic", 2, True),      # ragged level chunks
    "ico3_nz16": (3, 16, "uniform", 0, False),            # the 20,480-unknown manufactured-solution solve
    "ico4_nz32_quad": (4, 32, "quadratic", 3, True),
}


def make(case, **setup):
    import paper_1408_2981_amd as T

    ref, nz, grading, seed, rand = CASES[case]
    r = synth.vertical_faces(nz, synth.H10KM, grading)
    om2 = synth.omega_for(ref) ** 2
    prof = synth.profiles_random(nz, synth.n_cells(ref), seed=seed + 100) if rand else None
    h = otpmg.build(ref, r, om2, profiles=prof)
    P = T.Problem(ref, r, om2, profiles=prof).setup(**setup)
    fine = h.meshes[-1]
    if case == "ico3_nz16":
        f = synth.make_rhs(synth.workload("ico3_nz16"), fine.centre, fine.area, h.vert.vk)
    else:
        f = synth.cell_integral(synth.uniform_noise(fine.n, nz, seed), fine.area, h.vert.vk)
    return h, P, f


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
