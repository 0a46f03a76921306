"""GPU parity of the HIP path against the CPU oracle (through the C ABI):
layout conversion, the matrix-free SpMV (eq. ColumnEquation), one V-cycle
(Algorithm 1) in FP64 and FP32, and the full flexible-CG solve. FP64 bar:
relative error <= 1e-10 and identical iteration counts; mixed bar: <= 1e-6
against the oracle's FP64 solution."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import synth  # noqa: E402
from oracle import operator as opm, tpmg as otpmg  # noqa: E402
from gpu_common import CASES, make, rel  # noqa: E402


@pytest.mark.parametrize("case", list(CASES))
def test_pack_unpack_roundtrip(case):
    h, P, f = make(case)
    t = P.pack(f)
    back = P.unpack(t)
    assert np.array_equal(back, f)
    tiled = t.cpu().numpy()
    assert np.count_nonzero(tiled) <= f.size
    assert tiled.size == P.len and P.len % 64 == 0


@pytest.mark.parametrize("case", list(CASES))
def test_spmv(case):
    h, P, f = make(case)
    x = np.random.default_rng(7).standard_normal(f.shape)
    xd = P.pack(x)
    yd = P.device_vector()
    P.spmv(xd, yd)
    P.synchronize()
    y = P.unpack(yd)
    ref = opm.apply(h.finest, x)
    assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref))
    # padding entries stay zero
    assert np.count_nonzero(yd.cpu().numpy()) <= y.size


@pytest.mark.parametrize("case", list(CASES))
def test_vcycle_fp64(case):
    h, P, f = make(case)
    zd = P.device_vector()
    P.vcycle(P.pack(f), zd)
    P.synchronize()
    z = P.unpack(zd)
    ref = otpmg.vcycle(h, f)
    print(f"{case}: FP64 V-cycle rel diff {rel(z, ref):.2e}")
    assert rel(z, ref) <= 1e-10, rel(z, ref)


def _anorm(op, v):
    return float(np.sqrt(np.sum(v * opm.apply(op, v))))


@pytest.mark.parametrize("case", list(CASES))
def test_vcycle_fp32(case):
    """The FP32 V-cycle is a different rounding of the same operator, and the
    problem's conditioning amplifies FP32 rounding differently in different
    norms. Bar: the GPU FP32 V-cycle is as close to the exact FP64 V-cycle as
    the oracle's own FP32 V-cycle is (within 10x, plus 1e-7), in the l2 norm
    and in the energy norm of A."""
    h, P, f = make(case, precond_fp32=True)
    zd = P.device_vector()
    P.vcycle(P.pack(f), zd)
    P.synchronize()
    z = P.unpack(zd)
    z64 = otpmg.vcycle(h, f)
    z32 = otpmg.make_preconditioner(h, "fp32")(f)
    op = h.finest
    for name, norm in (("l2", np.linalg.norm), ("A", lambda v: _anorm(op, v))):
        e_gpu = norm(z - z64) / norm(z64)
        e_orc = norm(z32 - z64) / norm(z64)
        print(f"{case}: FP32 V-cycle {name}-error vs FP64 V-cycle: GPU {e_gpu:.2e}, oracle FP32 {e_orc:.2e}")
        assert e_gpu <= 10 * e_orc + 1e-7


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("graph", [False, True])
def test_solve_fp64(case, graph):
    h, P, f = make(case, use_graph=graph)
    ref = otpmg.solve(h, f, rtol=1e-8)
    ud = P.device_vector()
    st, iters, relres, hist, _ = P.solve(P.pack(f), ud, rtol=1e-8, maxit=100)
    u = P.unpack(ud)
    print(f"{case} graph={graph}: iters {iters} (oracle {ref.iters}), rel err {rel(u, ref.x):.2e}")
    assert st == 0 and ref.status == "converged"
    assert iters == ref.iters
    assert rel(u, ref.x) <= 1e-10
    assert np.allclose(hist, ref.history, rtol=1e-6, atol=0)


@pytest.mark.parametrize("case", list(CASES))
def test_solve_mixed(case):
    """Mixed path (FP32 V-cycle in FP64 FCG). At rtol 1e-8 the error against
    the exact solution is limited by the conditioning, for the FP64 path too
    (the 20,480-unknown case: 7e-6), so the 1e-6 bar is applied at rtol 1e-11;
    at 1e-8 the GPU's error must be within 10x of the oracle's mixed solve."""
    h, P, f = make(case, precond_fp32=True, use_graph=True)
    tight = otpmg.solve(h, f, rtol=1e-13, maxit=400)
    ref32 = otpmg.solve(h, f, rtol=1e-8, precision="fp32")
    fd = P.pack(f)
    ud = P.device_vector()
    st, iters, relres, hist, _ = P.solve(fd, ud, rtol=1e-8, maxit=100)
    u = P.unpack(ud)
    e_gpu, e_orc = rel(u, tight.x), rel(ref32.x, tight.x)
    print(f"{case}: mixed rtol 1e-8: iters {iters} (oracle mixed {ref32.iters}); error vs exact: GPU {e_gpu:.2e}, "
          f"oracle mixed {e_orc:.2e}")
    assert st == 0 and relres <= 1e-8
    assert abs(iters - ref32.iters) <= 1
    assert e_gpu <= max(1e-6, 10 * e_orc)
    ud2 = P.device_vector()
    st, iters2, relres2, _, _ = P.solve(fd, ud2, rtol=1e-11, maxit=200)
    e_tight = rel(P.unpack(ud2), tight.x)
    print(f"{case}: mixed rtol 1e-11: iters {iters2}, error vs exact {e_tight:.2e}")
    assert st == 0 and e_tight <= 1e-6


def test_graph_replays_match_eager():
    h, P, f = make("ico3_nz13_quad", use_graph=True)
    _, Pe, _ = make("ico3_nz13_quad", use_graph=False)
    fd, fe = P.pack(f), Pe.pack(f)
    outs = []
    for _ in range(3):
        ud = P.device_vector()
        P.solve(fd, ud, rtol=1e-8, maxit=100)
        outs.append(P.unpack(ud))
        torch.cuda.synchronize()
        _ = (fd * 2).sum().item()          # unrelated eager work between replays
    ue = Pe.device_vector()
    Pe.solve(fe, ue, rtol=1e-8, maxit=100)
    eager = Pe.unpack(ue)
    for o in outs:
        assert np.array_equal(o, eager)


def test_deterministic_fp64():
    h, P, f = make("ico4_nz32_quad")
    fd = P.pack(f)
    a, b = P.device_vector(), P.device_vector()
    P.solve(fd, a, rtol=1e-8, maxit=100)
    P.solve(fd, b, rtol=1e-8, maxit=100)
    assert torch.equal(a, b)


@pytest.mark.parametrize("graph", [False, True])
def test_iteration_queued_after_convergence_changes_nothing(graph):
    """The solve queues iteration k+1 before it has read iteration k's
    residual norm. The same solve stopped by maxit at the converged iteration
    count (nothing queued beyond it) returns the same bits, and so does a run
    whose maxit leaves it one iteration short (status: not converged)."""
    import paper_1408_2981_amd as T

    h, P, f = make("ico4_nz32_quad", use_graph=graph)
    fd = P.pack(f)
    a = P.device_vector()
    st, iters, _, hist_a, _ = P.solve(fd, a, rtol=1e-8, maxit=100)
    assert st == T.TPMG_OK
    b = P.device_vector()
    st_b, iters_b, _, hist_b, _ = P.solve(fd, b, rtol=1e-8, maxit=iters)
    assert st_b == T.TPMG_OK and iters_b == iters
    assert torch.equal(a, b) and np.array_equal(hist_a, hist_b)
    c = P.device_vector()
    st_c, iters_c, _, _, _ = P.solve(fd, c, rtol=1e-8, maxit=iters - 1)
    assert st_c == T.TPMG_NOT_CONVERGED and iters_c == iters - 1
    assert not torch.equal(a, c)


@pytest.mark.parametrize("case", ["ico2_nz8_rand", "ico3_nz16", "ico4_nz32_quad"])
def test_vcycle_rate(case):
    """V-cycle convergence factor in the Richardson iteration (f = 0, seeded
    start, 12 cycles, rate over the last 8) against the oracle's."""
    import paper_1408_2981_amd as T

    h, P, f = make(case)
    u0 = synth.uniform_noise(f.shape[0], f.shape[1], 7)
    rate, norms = T.tpmg_richardson_rate(P.mg, P.pack(u0), 12, 4)
    ref = otpmg.richardson_rate(h, seed=7)
    print(f"{case}: V-cycle rate GPU {rate:.6f}, oracle {ref:.6f}")
    assert abs(rate - ref) <= 1e-8 * ref
    h32, P32, _ = make(case, precond_fp32=True)
    rate32, _ = T.tpmg_richardson_rate(P32.mg, P32.pack(u0), 12, 4)
    ref32 = otpmg.richardson_rate(h, seed=7, precision="fp32")
    print(f"{case}: mixed V-cycle rate GPU {rate32:.6f}, oracle FP32 {ref32:.6f}, FP64 {ref:.6f}")
    # Against the oracle's own FP32 V-cycle (the same algorithm, rounded in
    # another order). The residual left after a few cycles lies in the
    # components the V-cycle reduces slowest, and on those an FP32 V-cycle is
    # a poor copy of the FP64 one: measured with the oracle on these cases,
    # |A (M32 r - M64 r)| / |r| reaches 0.09 (ico4_nz32_quad) to 0.56
    # (ico3_nz16) from the sixth cycle on. A per-cycle residual perturbation
    # of eta moves the per-cycle factor by at most eta; two FP32 V-cycles
    # each within eta of the FP64 one differ by at most 2 eta. The bar, 0.1,
    # is the smallest of those perturbations (and above twice the oracle's
    # own FP32-to-FP64 difference on these cases, 0.036 at most).
    assert rate32 < 1.0
    assert abs(rate32 - ref32) <= 0.1


def test_extreme_anisotropy_fp32():
    """H/h = 1e-3 (ratio of the vertical extent to the horizontal spacing, the
    far end of the anisotropy sweep of the robustness tables) on a small
    sphere: the FP32 V-cycle stays a contraction with the FP64 V-cycle's
    factor (within the bar above) and stays close to the FP64 V-cycle (the
    oracle's FP32 V-cycle is 2.6e-7 away; bar 1e-4)."""
    import paper_1408_2981_amd as T

    ref_level, nz = 4, 32
    r = synth.vertical_faces(nz, 1e-3 * synth.nominal_spacing(ref_level), "quadratic")
    om2 = synth.omega_for(ref_level) ** 2
    h = otpmg.build(ref_level, r, om2)
    fine = h.meshes[-1]
    f = synth.cell_integral(synth.uniform_noise(fine.n, nz, 3), fine.area, h.vert.vk)
    z64 = otpmg.vcycle(h, f)
    P = T.Problem(ref_level, r, om2).setup(precond_fp32=True)
    zd = P.device_vector()
    P.vcycle(P.pack(f), zd)
    P.synchronize()
    err = rel(P.unpack(zd), z64)
    u0 = synth.uniform_noise(fine.n, nz, 7)
    # this problem reaches its asymptotic factor late: rate over cycles 10-20
    rate32, _ = T.tpmg_richardson_rate(P.mg, P.pack(u0), 20, 10)
    ref = otpmg.richardson_rate(h, seed=7, cycles=20, skip=10)
    print(f"H/h 1e-3: FP32 V-cycle vs FP64 V-cycle {err:.2e}; mixed rate {rate32:.4f}, FP64 oracle rate {ref:.4f}")
    assert err <= 1e-4
    assert rate32 < 1.0 and abs(rate32 - ref) <= 0.1


@pytest.mark.parametrize("fp32", [False, True])
def test_caller_samples_on_coarse_grids(fp32):
    """Horizontal factors sampled by the caller on coarse grids
    (tpmg_op_create_levels) on top of random finest-grid profiles: FP64
    V-cycle and solve against the oracle built from the same samples (1e-10,
    identical iteration counts and histories); mixed: iterations within one
    of the oracle's mixed solve and the error against the exact solution
    within the bar of test_solve_mixed."""
    ref, nz = 3, 13
    r = synth.vertical_faces(nz, synth.H10KM, "quadratic")
    om2 = synth.omega_for(ref) ** 2
    prof = synth.profiles_random(nz, synth.n_cells(ref), seed=31)
    rng = np.random.default_rng(32)
    lv = {2: (rng.uniform(0.5, 2.0, 320), None, rng.uniform(0.5, 2.0, 320)),
          1: (None, rng.uniform(0.5, 2.0, 80), None)}
    h = otpmg.build(ref, r, om2, profiles=prof, level_factors=lv)
    import paper_1408_2981_amd as T

    P = T.Problem(ref, r, om2, profiles=prof, level_factors=lv).setup(precond_fp32=fp32)
    fine = h.meshes[-1]
    f = synth.cell_integral(synth.uniform_noise(fine.n, nz, 33), fine.area, h.vert.vk)
    ud = P.device_vector()
    st, iters, relres, hist, _ = P.solve(P.pack(f), ud, rtol=1e-8, maxit=100)
    u = P.unpack(ud)
    ref64 = otpmg.solve(h, f, rtol=1e-8)
    assert st == 0
    if not fp32:
        zd = P.device_vector()
        P.vcycle(P.pack(f), zd)
        P.synchronize()
        assert rel(P.unpack(zd), otpmg.vcycle(h, f)) <= 1e-10
        assert iters == ref64.iters
        assert rel(u, ref64.x) <= 1e-10
        assert np.allclose(hist, ref64.history, rtol=1e-6, atol=0)
    else:
        ref32 = otpmg.solve(h, f, rtol=1e-8, precision="fp32")
        tight = otpmg.solve(h, f, rtol=1e-13, maxit=400)
        assert abs(iters - ref32.iters) <= 1
        assert rel(u, tight.x) <= max(1e-6, 10 * rel(ref32.x, tight.x))
    print(f"caller samples, {'mixed' if fp32 else 'FP64'}: {iters} iterations (oracle FP64 {ref64.iters}), "
          f"solution vs oracle FP64 {rel(u, ref64.x):.2e}")
    P.close()
