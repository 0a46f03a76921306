"""Parity at the benchmark's full size (10,485,760 unknowns: icosahedral
refinement 6 x 128 quadratically graded levels), in the configuration
bench.py times (kernels launched one by one, autotuned, FP64 and mixed;
graph replay is covered at smaller sizes). The oracle's results for this
workload are stored in tests/golden/ico6_nz128_oracle.json by
tests/golden/make_full_size.py (it calls only oracle/ and synth/): sampled
values of A x, of one V-cycle and of the FP64 solution, the iteration counts
and residual histories."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1408_2981_amd as T  # noqa: E402
import synth  # noqa: E402
from oracle import mesh  # noqa: E402

GOLD = os.path.join(os.path.dirname(__file__), "golden", "ico6_nz128_oracle.json")


@pytest.fixture(scope="module")
def setup():
    g = json.load(open(GOLD))
    w = synth.workload(g["workload"])
    fine = mesh.hierarchy(w.refinement)[-1]
    P64 = T.Problem(w.refinement, w.r_faces(), w.omega2).setup(precond_fp32=False, use_graph=False, autotune=1)
    f = synth.make_rhs(w, fine.centre, fine.area, P64.vk())
    return g, w, f, P64


def _samples(P, tiled, g):
    u = P.unpack(tiled)
    return u[np.array(g["sample_cells"]), np.array(g["sample_levels"])], u


def test_full_size_spmv(setup):
    g, w, f, P = setup
    x = np.random.default_rng(g["spmv_x_seed"]).standard_normal((w.n, w.nz))
    y = P.device_vector()
    P.spmv(P.pack(x), y)
    P.synchronize()
    got, _ = _samples(P, y, g)
    ref = np.array(g["spmv_samples"])
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_full_size_vcycle_fp64(setup):
    g, w, f, P = setup
    z = P.device_vector()
    P.vcycle(P.pack(f), z)
    P.synchronize()
    got, full = _samples(P, z, g)
    ref = np.array(g["vcycle_samples"])
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    nrm = abs(np.linalg.norm(full) / g["vcycle_norm"] - 1)
    print(f"full-size V-cycle: sampled max rel diff {err:.2e}, norm rel diff {nrm:.2e}")
    assert err <= 1e-10 and nrm <= 1e-10


def test_full_size_solve_fp64(setup):
    g, w, f, P = setup
    u = P.device_vector()
    st, iters, relres, hist, ms = P.solve(P.pack(f), u, rtol=1e-8, maxit=100)
    got, full = _samples(P, u, g)
    ref = np.array(g["fp64"]["x_samples"])
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    nrm = abs(np.linalg.norm(full) / g["fp64"]["x_norm"] - 1)
    print(f"full-size FP64 solve: {iters} iterations (oracle {g['fp64']['iters']}), {ms:.2f} ms, "
          f"sampled max rel diff {err:.2e}, norm rel diff {nrm:.2e}")
    assert st == T.TPMG_OK and iters == g["fp64"]["iters"]
    assert np.allclose(hist, g["fp64"]["history"], rtol=1e-6, atol=0)
    assert err <= 1e-10 and nrm <= 1e-10


def test_full_size_solve_mixed(setup):
    g, w, f, P64 = setup
    P = T.Problem(w.refinement, w.r_faces(), w.omega2).setup(precond_fp32=True, use_graph=False, autotune=1)
    u = P.device_vector()
    st, iters, relres, hist, ms = P.solve(P.pack(f), u, rtol=1e-8, maxit=100)
    got, full = _samples(P, u, g)
    ref = np.array(g["fp64"]["x_samples"])
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    nrm = abs(np.linalg.norm(full) / g["fp64"]["x_norm"] - 1)
    print(f"full-size mixed solve: {iters} iterations (oracle mixed {g['mixed']['iters']}), {ms:.2f} ms, "
          f"relres {relres:.2e}; vs oracle FP64 solution: sampled max rel diff {err:.2e}, norm rel diff {nrm:.2e}")
    assert st == T.TPMG_OK and relres <= 1e-8
    assert abs(iters - g["mixed"]["iters"]) <= 1
    assert err <= 1e-6 and nrm <= 1e-6
    P.close()
