"""The operator with vertical advection (Section 2.1, eq. HelmholtzVector;
Appendix A "Vertical advection"; balanced flow of Section 5.2, whose xi_r =
Lambda rho d_r theta) and the paper's outer solvers, preconditioned
Richardson and BiCGStab (Section 5.2), against the oracle: FP64 operator
within 1e-12, V-cycle within 1e-10, identical iteration counts and residual
histories (1e-6), solutions within 1e-10; mixed precision within one
iteration of the oracle's FP32 V-cycle; the FCG solve refuses the
non-symmetric operator."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1408_2981_amd as T  # noqa: E402
import synth  # noqa: E402
from oracle import mesh, operator as opm, tpmg as otpmg  # noqa: E402

MODES = {"full": (T.PRECOND_FULL, otpmg.FULL_TERMS_ADV), "factorised": (T.PRECOND_FACTORISED, ()),
         "partial": (T.PRECOND_PARTIAL, ("alpha_r",))}


def _case(eps, ref=3, nz=16):
    r = synth.vertical_faces(nz, synth.H10KM, "quadratic")
    om = synth.omega_for(ref)
    m = mesh.hierarchy(ref)[-1]
    bf = synth.balanced_flow(eps, m.centre, r, om)
    f = synth.cell_integral(synth.uniform_noise(m.n, nz, 81), m.area, opm.vertical(r).vk)
    return ref, r, om * om, bf, f


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("eps", [0.5, 1.23])
@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("method", ["bicgstab", "richardson"])
def test_advection_fp64_against_oracle(eps, mode, method):
    ref, r, om2, bf, f = _case(eps)
    code, terms = MODES[mode]
    A = otpmg.build(ref, r, om2, profiles=bf.factorised, full=bf, full_terms=otpmg.FULL_TERMS_ADV).finest
    h = otpmg.build(ref, r, om2, profiles=bf.factorised, full=bf if terms else None, full_terms=terms)
    P = T.Problem(ref, r, om2, profiles=bf.factorised, full=bf, advection=True).setup(precond_profiles=code)
    x = np.random.default_rng(5).standard_normal(f.shape)
    y = P.device_vector()
    P.spmv(P.pack(x), y)
    P.synchronize()
    ax = opm.apply(A, x)
    assert np.max(np.abs(P.unpack(y) - ax)) <= 1e-12 * np.max(np.abs(ax))
    z = P.device_vector()
    P.vcycle(P.pack(f), z)
    P.synchronize()
    zerr = _rel(P.unpack(z), otpmg.vcycle(h, f))
    ref_s = otpmg.solve(h, f, rtol=1e-8, maxit=200, outer=A, method=method)
    u = P.device_vector()
    d = (T.tpmg_solve_bicgstab if method == "bicgstab" else T.tpmg_solve_richardson)(P.mg, P.pack(f), u, 1e-8, 200)
    err = _rel(P.unpack(u), ref_s.x)
    print(f"eps {eps} {method} TPMG {mode}: V-cycle {zerr:.2e}; {d['iters']} iterations (oracle {ref_s.iters}), "
          f"solution {err:.2e}")
    assert zerr <= 1e-10
    assert d["status"] == T.TPMG_OK and d["iters"] == ref_s.iters and err <= 1e-10
    assert np.allclose(d["history"], ref_s.history, rtol=1e-6, atol=1e-12)
    P.close()


@pytest.mark.parametrize("method", ["bicgstab", "richardson"])
def test_advection_mixed(method):
    ref, r, om2, bf, f = _case(1.23)
    A = otpmg.build(ref, r, om2, profiles=bf.factorised, full=bf, full_terms=otpmg.FULL_TERMS_ADV)
    P = T.Problem(ref, r, om2, profiles=bf.factorised, full=bf, advection=True).setup(
        precond_fp32=True, precond_profiles=T.PRECOND_FULL)
    o32 = otpmg.solve(A, f, rtol=1e-8, maxit=200, precision="fp32", method=method)
    u = P.device_vector()
    fn = T.tpmg_solve_bicgstab if method == "bicgstab" else T.tpmg_solve_richardson
    d = fn(P.mg, P.pack(f), u, 1e-8, 200)
    xd = otpmg.direct_solve(A.finest, f)
    err = _rel(P.unpack(u), xd)
    print(f"{method} mixed: {d['iters']} iterations (oracle FP32 {o32.iters}); error vs direct {err:.2e}")
    assert d["status"] == T.TPMG_OK and abs(d["iters"] - o32.iters) <= 1
    assert err <= 1e-6
    P.close()


def test_fcg_refuses_advection_and_outer_solvers_on_spd():
    ref, r, om2, bf, f = _case(0.5)
    P = T.Problem(ref, r, om2, profiles=bf.factorised, full=bf, advection=True).setup()
    u = P.device_vector()
    with pytest.raises(T.TpmgError) as e:
        P.solve(P.pack(f), u)
    assert e.value.status == T.TPMG_ERR_ARG
    P.close()
    # without advection the outer solvers run on the symmetric operator too
    h = otpmg.build(ref, r, om2, profiles=bf.factorised, full=bf)
    Q = T.Problem(ref, r, om2, profiles=bf.factorised, full=bf).setup()
    for method, fn in (("bicgstab", T.tpmg_solve_bicgstab), ("richardson", T.tpmg_solve_richardson)):
        o = otpmg.solve(h, f, rtol=1e-8, maxit=200, method=method)
        u = Q.device_vector()
        d = fn(Q.mg, Q.pack(f), u, 1e-8, 200)
        assert d["iters"] == o.iters and _rel(Q.unpack(u), o.x) <= 1e-10
    Q.close()
