"""Profiles that do not factorise (Section 4.2; Section 5.2 balanced flow,
Section 5.3): the operator of the equation with coefficients per (T, k),
preconditioned by the V-cycle of the full operator (TPMG^(full)), of the
approximate factorisation (TPMG^(x)) or of the full alpha_r with the rest
factorised (TPMG^(partial)), against the oracle's hierarchies of the same
three kinds (FP64: operator within 1e-12, V-cycle and solution within
1e-10, identical iteration counts and residual histories, V-cycle
convergence factor within 1e-8 relative; mixed: the FP32 V-cycle bars of
the factorised case)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1408_2981_amd as T  # noqa: E402
import synth  # noqa: E402
from oracle import mesh, operator as opm, tpmg as otpmg  # noqa: E402

MODES = {"full": (T.PRECOND_FULL, otpmg.FULL_TERMS), "factorised": (T.PRECOND_FACTORISED, ()),
         "partial": (T.PRECOND_PARTIAL, ("alpha_r",))}


def _case(name):
    if name.startswith("balanced"):
        eps = float(name.split("_")[1])
        ref, nz = 3, 16
        r = synth.vertical_faces(nz, synth.H10KM, "quadratic")
        om = synth.omega_for(ref)
        m = mesh.hierarchy(ref)[-1]
        bf = synth.balanced_flow(eps, m.centre, r, om)
        return ref, r, om * om, bf.factorised, bf, synth.cell_integral(synth.uniform_noise(m.n, nz, 41), m.area,
                                                                        opm.vertical(r).vk)
    ref, nz = 3, 13
    r = synth.vertical_faces(nz, synth.H10KM, "quadratic")
    om2 = synth.omega_for(ref) ** 2
    n = synth.n_cells(ref)
    rng = np.random.default_rng(42)
    full = opm.FullProfiles(rng.uniform(0.5, 2.0, (n, nz + 1)), rng.uniform(0.5, 2.0, (n, nz)),
                            rng.uniform(0.5, 2.0, (n, nz)))
    prof = synth.profiles_random(nz, n, seed=43)
    m = mesh.hierarchy(ref)[-1]
    return ref, r, om2, prof, full, synth.cell_integral(synth.uniform_noise(n, nz, 44), m.area, opm.vertical(r).vk)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


CASES = ["balanced_0.5", "balanced_1.23", "random"]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("mode", list(MODES))
def test_profiles_fp64_against_oracle(case, mode):
    ref, r, om2, prof, full, f = _case(case)
    code, terms = MODES[mode]
    A = otpmg.build(ref, r, om2, profiles=prof, full=full).finest
    h = otpmg.build(ref, r, om2, profiles=prof, full=full if terms else None, full_terms=terms)
    P = T.Problem(ref, r, om2, profiles=prof, full=full).setup(precond_profiles=code)
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
    ref_s = otpmg.solve(h, f, rtol=1e-8, maxit=200, outer=A)
    u = P.device_vector()
    st, iters, relres, hist, _ = P.solve(P.pack(f), u, rtol=1e-8, maxit=200)
    err = _rel(P.unpack(u), ref_s.x)
    u0 = synth.uniform_noise(f.shape[0], f.shape[1], 7)
    rate, _ = T.tpmg_richardson_rate(P.mg, P.pack(u0), 12, 4)
    rate_o = otpmg.richardson_rate(h, seed=7, outer=A)
    print(f"{case} TPMG {mode}: V-cycle {zerr:.2e}; {iters} iterations (oracle {ref_s.iters}), solution {err:.2e}; "
          f"Richardson factor GPU {rate:.6f}, oracle {rate_o:.6f}")
    assert zerr <= 1e-10
    assert st == T.TPMG_OK and iters == ref_s.iters and err <= 1e-10
    assert np.allclose(hist, ref_s.history, rtol=1e-6, atol=1e-12)
    assert abs(rate - rate_o) <= 1e-8 * rate_o
    P.close()


@pytest.mark.parametrize("case", ["balanced_1.23", "random"])
@pytest.mark.parametrize("mode", list(MODES))
def test_profiles_mixed(case, mode):
    """FP32 V-cycle of each kind inside the FP64 Krylov method: converges,
    iteration count within one of the oracle's FP32 V-cycle solve, and the
    solution within 1e-6 of the oracle's tight FP64 solve when solved to
    rtol 1e-11."""
    ref, r, om2, prof, full, f = _case(case)
    code, terms = MODES[mode]
    A = otpmg.build(ref, r, om2, profiles=prof, full=full).finest
    h = otpmg.build(ref, r, om2, profiles=prof, full=full if terms else None, full_terms=terms)
    P = T.Problem(ref, r, om2, profiles=prof, full=full).setup(precond_fp32=True, precond_profiles=code)
    o32 = otpmg.solve(h, f, rtol=1e-8, maxit=200, outer=A, precision="fp32")
    u = P.device_vector()
    st, iters, relres, hist, _ = P.solve(P.pack(f), u, rtol=1e-8, maxit=200)
    assert st == T.TPMG_OK and abs(iters - o32.iters) <= 1
    tight = otpmg.solve(h, f, rtol=1e-13, maxit=400, outer=A)
    u = P.device_vector()
    st, iters11, relres, hist, _ = P.solve(P.pack(f), u, rtol=1e-11, maxit=400)
    err = _rel(P.unpack(u), tight.x)
    print(f"{case} TPMG {mode} mixed: {iters} iterations (oracle FP32 {o32.iters}); at rtol 1e-11 error {err:.2e}")
    assert st == T.TPMG_OK and err <= 1e-6
    P.close()


def test_profile_mode_restrictions():
    ref, r, om2, prof, full, f = _case("random")
    P = T.Problem(ref, r, om2, profiles=prof, full=full)
    with pytest.raises(T.TpmgError) as e:
        P.setup(precond_profiles=T.PRECOND_FULL, smoother=T.SMOOTHER_LDS)
    assert e.value.status == T.TPMG_ERR_ARG
    with pytest.raises(T.TpmgError):
        P.setup(precond_profiles=T.PRECOND_PARTIAL, scan_levels=4)
    P.setup(precond_fp32=True, use_graph=True, precond_profiles=T.PRECOND_FULL)
    tun = P.tuning()
    assert all(t["smoother"] == T.SMOOTHER_SCAN and t["scan_levels"] in (8, 16) for t in tun)
    # a batch takes problems of either kind together (test_gpu_batch solves one)
    stream = P.stream
    Q = T.Problem(ref, r, om2, profiles=prof).setup(precond_fp32=True, use_graph=True, stream=stream)
    assert T.tpmg_batch_workspace_size([P.mg, Q.mg]) > 0
    # graph replay and the autotuner with full profiles: the same result as
    # launches one by one with the built-in choices
    u1 = P.device_vector()
    st1, it1, *_ = P.solve(P.pack(f), u1)
    R = T.Problem(ref, r, om2, profiles=prof, full=full).setup(precond_fp32=True, use_graph=False, autotune=1,
                                                              precond_profiles=T.PRECOND_FULL)
    u2 = R.device_vector()
    st2, it2, *_ = R.solve(R.pack(f), u2)
    assert st1 == st2 == T.TPMG_OK and abs(it1 - it2) <= 1
    P.close()
    Q.close()
    R.close()


@pytest.mark.parametrize("mode", list(MODES))
def test_relax_on_the_vcycle_operator(mode):
    """tpmg_relax with profiles that do not factorise runs on the finest
    operator of the V-cycle (full, factorised or partial): against the
    oracle's sweep with damping 1 on that operator, entrywise within the
    rounding bar of test_gpu_mlp.test_relax_matches_oracle."""
    ref, r, om2, prof, full, f = _case("random")
    code, terms = MODES[mode]
    h = otpmg.build(ref, r, om2, profiles=prof, full=full if terms else None, full_terms=terms)
    P = T.Problem(ref, r, om2, profiles=prof, full=full).setup(precond_profiles=code, precond_fp32=True)
    op = h.finest
    l, m, e = opm.column_bands(op)
    u_in = synth.uniform_noise(f.shape[0], f.shape[1], 9) * 1e-3
    out = P.device_vector()
    P.relax(P.pack(f), P.pack(u_in), out)
    P.synchronize()
    got = P.unpack(out)
    ref_u = otpmg.smooth(op, f, u_in, 1.0)
    a = np.abs(u_in)
    bound = 2 * (8 + f.shape[1]) * np.finfo(np.float64).eps * otpmg.thomas_margin(
        l, m, e, np.abs(f) + 2.0 * (e + l + m) * a - opm.apply(op, a))
    ratio = float(np.max(np.abs(got - ref_u) / bound))
    print(f"{mode}: relax vs oracle {ratio:.2e} of the rounding bar")
    assert ratio <= 1.0
    P.close()
