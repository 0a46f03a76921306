"""The largest workload: icosahedral refinement 7 x 128 quadratically graded
levels (41,943,040 unknowns), at both ends of the anisotropy sweep
(H = 1e-1 and 1e-3 x the horizontal spacing), in the configuration bench.py times
(graph replay, autotuned kernels). The oracle cannot run the full solve
here in seconds, so the checks are what holds at any size, with the
oracle's own FP64 operator as the reference: the operator against the oracle's
on a random field, and both solves' true residual f - A u, evaluated by the
oracle, below the stopping tolerance."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1408_2981_amd as T  # noqa: E402
import synth  # noqa: E402
from oracle import operator as opm, tpmg as otpmg  # noqa: E402


@pytest.fixture(scope="module", params=["0.1", "0.001"])
def config3(request):
    w = synth.workload(f"ico7_nz128_ar{request.param}")
    h = otpmg.build(w.refinement, w.r_faces(), w.omega2)
    fine = h.meshes[-1]
    f = synth.make_rhs(w, fine.centre, fine.area, h.vert.vk)
    return w, h, f


def _residual_and_floor(h, f, u):
    """||f - A u|| / ||f|| with the oracle's operator, and the rounding floor
    of that evaluation relative to ||f||: || |A| |u| || eps / ||f||, where
    |A| = 2 D - A (D the diagonal; A is an M-matrix, so |A||u| sums the
    magnitudes of every stencil term)."""
    op = h.finest
    l, m, e = opm.column_bands(op)
    a = np.abs(u)
    abs_au = 2.0 * (e + l + m) * a - opm.apply(op, a)
    fn = np.linalg.norm(f)
    r = f - opm.apply(op, u)
    return float(np.linalg.norm(r) / fn), float(np.linalg.norm(abs_au) * np.finfo(np.float64).eps / fn)


def test_config3_operator(config3):
    w, h, f = config3
    P = T.Problem(w.refinement, w.r_faces(), w.omega2).setup(precond_fp32=False, use_graph=True, autotune=1)
    x = np.random.default_rng(3).standard_normal((w.n, w.nz))
    y = P.device_vector()
    P.spmv(P.pack(x), y)
    P.synchronize()
    got = P.unpack(y)
    ref = opm.apply(h.finest, x)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"config 3 {w.name} operator: max rel diff {err:.2e}")
    assert err <= 1e-12
    P.close()


@pytest.mark.parametrize("fp32", [False, True])
def test_config3_solve_true_residual(config3, fp32):
    w, h, f = config3
    P = T.Problem(w.refinement, w.r_faces(), w.omega2).setup(precond_fp32=fp32, use_graph=True, autotune=1)
    u = P.device_vector()
    st, iters, relres, hist, ms = P.solve(P.pack(f), u, rtol=1e-8, maxit=100)
    true, floor = _residual_and_floor(h, f, P.unpack(u))
    print(f"config 3 {w.name} {'mixed' if fp32 else 'FP64'}: {iters} iterations, {ms:.1f} ms, relres {relres:.2e}, "
          f"true residual (oracle operator) {true:.2e}, rounding floor of its evaluation {floor:.2e}")
    assert st == T.TPMG_OK and relres <= 1e-8
    # The recurrence residual and the true one part by rounding only: the
    # evaluation of f - A u itself (at most 8 stencil terms per row) and the
    # drift of the recurrence over the iterations, each a multiple of
    # eps || |A| |u| ||; at this anisotropy that floor is far above 1e-8.
    assert true <= 1e-8 + (8 + iters) * floor
    assert iters <= (25 if fp32 else 15)
    P.close()
