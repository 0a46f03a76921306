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
