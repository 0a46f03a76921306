"""The multicolour block-SOR smoother (the paper's block-SOR, Section 5,
taken colour by colour; tpmg_mg_params.smoother_order = 1) against the
oracle's (oracle/tpmg.py with_sor: the same greedy colouring, colours
ascending before the coarse-grid correction and descending after): FP64
V-cycle and solution within 1e-10, identical iteration counts and residual
histories, Richardson factor within 1e-7 relative, for relaxation factors
1 (the paper's) and 1.2, factorised and full profiles; the mixed path to
the FP32 bars."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1408_2981_amd as T  # noqa: E402
import synth  # noqa: E402
from gpu_common import CASES, rel  # noqa: E402
from oracle import operator as opm, tpmg as otpmg  # noqa: E402


def _make(case, omega, **setup):
    ref, nz, grading, seed, rand = CASES[case]
    r = synth.vertical_faces(nz, synth.H10KM, grading)
    om2 = synth.omega_for(ref) ** 2
    prof = synth.profiles_random(nz, synth.n_cells(ref), seed=seed + 100) if rand else None
    h = otpmg.build(ref, r, om2, profiles=prof).with_sor(omega)
    P = T.Problem(ref, r, om2, profiles=prof).setup(smoother_order=T.SMOOTHER_ORDER_SOR, omega_relax=omega, **setup)
    fine = h.meshes[-1]
    f = synth.cell_integral(synth.uniform_noise(fine.n, nz, seed), fine.area, h.vert.vk)
    return h, P, f


@pytest.mark.parametrize("omega", [1.0, 1.2])
@pytest.mark.parametrize("case", ["ico2_nz8_rand", "ico3_nz13_quad", "ico4_nz32_quad"])
def test_sor_fp64_against_oracle(case, omega):
    h, P, f = _make(case, omega)
    z = P.device_vector()
    P.vcycle(P.pack(f), z)
    P.synchronize()
    zerr = rel(P.unpack(z), otpmg.vcycle(h, f))
    ref = otpmg.solve(h, f, rtol=1e-8, maxit=200)
    u = P.device_vector()
    st, iters, relres, hist, _ = P.solve(P.pack(f), u, rtol=1e-8, maxit=200)
    err = rel(P.unpack(u), ref.x)
    u0 = synth.uniform_noise(f.shape[0], f.shape[1], 7)
    rate, _ = T.tpmg_richardson_rate(P.mg, P.pack(u0), 12, 4)
    rate_o = otpmg.richardson_rate(h, seed=7)
    print(f"{case} SOR omega {omega}: V-cycle {zerr:.2e}; {iters} iterations (oracle {ref.iters}), solution {err:.2e}; "
          f"factor GPU {rate:.6f} oracle {rate_o:.6f}")
    assert zerr <= 1e-10
    assert st == T.TPMG_OK and iters == ref.iters and err <= 1e-10
    assert np.allclose(hist, ref.history, rtol=1e-6, atol=1e-12)
    # (after 12 cycles the residual is ~rho^12 of the start while the
    # stencil terms it is formed from stay near |A||u|: on these strongly
    # anisotropic columns the FP64 evaluation of ||r_12|| carries ~1e-8
    # relative rounding, of which the rate keeps an eighth; the two sides
    # also round the column solves in different orders: bar 1e-7)
    assert abs(rate - rate_o) <= 1e-7 * rate_o
    P.close()


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("case", ["ico3_nz16", "ico4_nz32_quad"])
def test_sor_mixed(case, graph):
    h, P, f = _make(case, 1.0, precond_fp32=True, use_graph=graph)
    o32 = otpmg.solve(h, f, rtol=1e-8, maxit=200, precision="fp32")
    u = P.device_vector()
    st, iters, *_ = P.solve(P.pack(f), u, rtol=1e-8, maxit=200)
    assert st == T.TPMG_OK and abs(iters - o32.iters) <= 1
    tight = otpmg.solve(h, f, rtol=1e-13, maxit=400)
    u = P.device_vector()
    st, it11, relres, *_ = P.solve(P.pack(f), u, rtol=1e-11, maxit=400)
    err = rel(P.unpack(u), tight.x)
    print(f"{case} SOR mixed graph={graph}: {iters} iterations (oracle FP32 {o32.iters}); rtol 1e-11 error {err:.2e}")
    assert st == T.TPMG_OK and err <= 1e-6
    P.close()


def test_sor_with_full_profiles():
    """Multicolour block-SOR on the V-cycle of profiles that do not factorise
    (TPMG^(full)), FP64, against the oracle."""
    ref, nz = 3, 13
    r = synth.vertical_faces(nz, synth.H10KM, "quadratic")
    om2 = synth.omega_for(ref) ** 2
    n = synth.n_cells(ref)
    rng = np.random.default_rng(61)
    full = opm.FullProfiles(rng.uniform(0.5, 2.0, (n, nz + 1)), rng.uniform(0.5, 2.0, (n, nz)),
                            rng.uniform(0.5, 2.0, (n, nz)))
    prof = synth.profiles_random(nz, n, seed=62)
    h = otpmg.build(ref, r, om2, profiles=prof, full=full).with_sor(1.0)
    P = T.Problem(ref, r, om2, profiles=prof, full=full).setup(smoother_order=T.SMOOTHER_ORDER_SOR, omega_relax=1.0,
                                                               precond_profiles=T.PRECOND_FULL)
    f = synth.cell_integral(synth.uniform_noise(n, nz, 63), h.meshes[-1].area, h.vert.vk)
    ref_s = otpmg.solve(h, f, rtol=1e-8, maxit=200)
    u = P.device_vector()
    st, iters, *_ = P.solve(P.pack(f), u, rtol=1e-8, maxit=200)
    err = rel(P.unpack(u), ref_s.x)
    print(f"full profiles + SOR: {iters} iterations (oracle {ref_s.iters}), solution {err:.2e}")
    assert st == T.TPMG_OK and iters == ref_s.iters and err <= 1e-10
    # batches take SOR problems, with profiles that factorise or not
    # (test_gpu_batch runs them)
    stream = P.stream
    Q = T.Problem(ref, r, om2).setup(precond_fp32=True, use_graph=True, stream=stream,
                                     smoother_order=T.SMOOTHER_ORDER_SOR, omega_relax=1.0)
    assert T.tpmg_batch_workspace_size([Q.mg]) > 0
    assert T.tpmg_batch_workspace_size([P.mg]) > 0
    P.close()
    Q.close()
