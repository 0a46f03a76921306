"""C-ABI failure paths on the GPU, forced from the host: breakdown on a
non-finite right-hand side, maxit reached, zero right-hand side, workspace
too small, aliasing arguments."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1408_2981_amd as T  # noqa: E402
from gpu_common import make  # noqa: E402


def test_nan_rhs_is_breakdown():
    h, P, f = make("ico2_nz8_rand")
    f = f.copy()
    f[3, 2] = np.nan
    ud = P.device_vector()
    st, iters, *_ = P.solve(P.pack(f), ud, rtol=1e-8, maxit=20)
    assert st == T.TPMG_ERR_BREAKDOWN


def test_maxit_not_converged_keeps_iterate():
    h, P, f = make("ico3_nz13_quad")
    ud = P.device_vector()
    st, iters, relres, hist, _ = P.solve(P.pack(f), ud, rtol=1e-14, maxit=1)
    assert st == T.TPMG_NOT_CONVERGED and iters == 1
    u = P.unpack(ud)
    assert np.all(np.isfinite(u)) and relres < 1.0


def test_zero_rhs():
    h, P, f = make("ico2_nz8_rand")
    ud = P.device_vector()
    st, iters, *_ = P.solve(P.pack(np.zeros_like(f)), ud, rtol=1e-8, maxit=10)
    assert st == T.TPMG_OK and iters == 0
    assert not torch.any(ud)


def test_converged_guess_and_maxit_zero_leave_u_unchanged():
    """The first iteration is queued before the host reads the initial
    residual: when the guess already meets the tolerance, or maxit is 0, the
    solve reports 0 iterations and returns the guess bit for bit."""
    h, P, f = make("ico3_nz13_quad")
    fd = P.pack(f)
    ud = P.device_vector()
    st, iters, *_ = P.solve(fd, ud, rtol=1e-8, maxit=100)
    assert st == T.TPMG_OK and iters > 0
    u0 = ud.clone()
    st, iters, relres, *_ = P.solve(fd, ud, rtol=1e-6, maxit=100)
    assert st == T.TPMG_OK and iters == 0 and relres <= 1e-6
    assert torch.equal(ud, u0)
    st, iters, *_ = P.solve(fd, ud, rtol=1e-14, maxit=0)
    assert st == T.TPMG_NOT_CONVERGED and iters == 0
    assert torch.equal(ud, u0)
    # and a following solve from that guess still converges
    st, iters, relres, *_ = P.solve(fd, ud, rtol=1e-10, maxit=100)
    assert st == T.TPMG_OK and iters > 0 and relres <= 1e-10


def test_workspace_too_small_and_alias():
    h, P, f = make("ico2_nz8_rand")
    p = T.tpmg_mg_params_default()
    need = T.tpmg_mg_workspace_size(P.op, p)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    with pytest.raises(T.TpmgError) as e:
        T.tpmg_mg_setup(P.op, p, ws.data_ptr(), need // 2, torch.cuda.current_stream().cuda_stream)
    assert e.value.status == T.TPMG_ERR_NOMEM
    v = P.device_vector()
    with pytest.raises(T.TpmgError) as e:
        T.tpmg_spmv(P.mg, v, v)
    assert e.value.status == T.TPMG_ERR_ARG


def test_divergence_stop_forced_from_host():
    """The divergence stop (||r_k|| > div_tol ||r_0|| -> TPMG_ERR_BREAKDOWN),
    forced by a bound below what the first iteration reaches: the solve stops
    after that iteration with a finite iterate, its residual recorded, and a
    message naming the divergence; a bound of 1e3 leaves the same solve
    alone."""
    h, P, f = make("ico3_nz13_quad")
    fd = P.pack(f)
    ud = P.device_vector()
    d = T.tpmg_solve_details(P.mg, fd, ud, 1e-8, 50, div_tol=1e-6)
    assert d["status"] == T.TPMG_ERR_BREAKDOWN and d["iters"] == 1
    assert "divergence" in d["message"]
    assert 1e-6 < d["history"][1] / d["history"][0] < 1.0
    assert torch.all(torch.isfinite(ud)) and torch.any(ud)
    ud.zero_()
    torch.cuda.synchronize()
    d = T.tpmg_solve_details(P.mg, fd, ud, 1e-8, 50, div_tol=1e3)
    assert d["status"] == T.TPMG_OK
    with pytest.raises(T.TpmgError) as e:
        T.tpmg_solve_details(P.mg, fd, ud, 1e-8, 50, div_tol=-1.0)
    assert e.value.status == T.TPMG_ERR_ARG


@pytest.mark.parametrize("fp32", [False, True])
def test_phase_timers_and_model_bytes(fp32):
    """The per-phase device timers and the algorithmic byte count: a timed
    solve returns the same bits as an untimed one (the same kernels, launched
    one by one), its three phases are positive and sum to at most the wall
    time, and the byte count equals the kernel table's figures summed over
    the iterations (checked here in closed form for an FP64 and a mixed
    solve of fewer than 8 iterations on the padded grid)."""
    h, P, f = make("ico3_nz16", precond_fp32=fp32)
    fd = P.pack(f)
    a = P.device_vector()
    d0 = T.tpmg_solve_details(P.mg, fd, a, 1e-6, 7)
    b = P.device_vector()
    d1 = T.tpmg_solve_details(P.mg, fd, b, 1e-6, 7, phase_timers=True)
    assert torch.equal(a, b) and d0["iters"] == d1["iters"] and d0["model_bytes"] == d1["model_bytes"]
    ph = [d1["t_vcycle_ms"], d1["t_spmv_ms"], d1["t_blas_ms"]]
    assert all(t > 0 for t in ph) and sum(ph) <= d1["t_total_ms"]
    assert d0["t_vcycle_ms"] == 0.0
    # closed form: levels l = 0..L with n_l padded columns, nz levels
    k, nz = d0["iters"], P.nz
    ns = [T.tpmg_op_level_size(P.op, lvl) for lvl in range(P.n_levels)]
    npad = [(n + 63) // 64 * 64 * nz for n in ns]
    N = npad[-1]
    s = 4 if fp32 else 8
    L = len(npad) - 1
    vc = 0.0
    for lvl in range(L, -1, -1):
        n_l = npad[lvl]
        sweeps = 1 if lvl == 0 else 2
        for j in range(sweeps):
            zero = j == 0
            vc += ((0 if zero else s) + s + s) * n_l
        if lvl > 0:
            vc += 2.25 * s * n_l      # residual + restriction
    for lvl in range(1, L + 1):
        vc += 2.25 * s * npad[lvl]    # prolongation + correction
        vc += 2 * 3 * s * npad[lvl]   # two post-sweeps
    # finest-level adjustments: the first pre-sweep reads the right-hand side
    # as FP32 (copy of r) in mixed mode and as FP64 r otherwise; the last
    # post-sweep reads r (FP64) and q and writes z (FP32 in mixed mode)
    if fp32:
        vc += 0.0                     # first sweep: f from the FP32 copy (4 B) as counted
        vc += (8 - s) * N + 8 * N     # last sweep: FP64 r, plus q
    else:
        vc += 8 * N                   # last sweep: plus q
    per_it = [vc + ((4 if fp32 else 8) + (8 if it > 0 else 0) + 16) * N + (24 + (4 if fp32 else 0)) * N
              for it in range(k)]
    expect = (24 + (4 if fp32 else 0)) * N + sum(per_it) + 8 * (2 + k) * N
    assert abs(d0["model_bytes"] - expect) <= 1e-9 * expect, (d0["model_bytes"], expect)
