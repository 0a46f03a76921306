"""The allocation-free entry point (tpmg_solve_noalloc: setup, solve and
teardown on the library's static device scratch) against the entry points
it stands for (tpmg_mg_setup on a caller workspace + tpmg_solve): the same
kernels in the same order, so the same bits, iteration counts and residual
histories; two calls in a row, the second on a smaller problem (the scratch
keeps the first call's contents and must be cleared where it matters), in
FP64 and mixed precision; and the size limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1408_2981_amd as T  # noqa: E402
import synth  # noqa: E402


def _problem(ref, nz, seed, fp32):
    r = synth.vertical_faces(nz, synth.H10KM, "quadratic")
    om2 = synth.omega_for(ref) ** 2
    prof = synth.profiles_random(nz, synth.n_cells(ref), seed=seed + 100)
    P = T.Problem(ref, r, om2, profiles=prof).setup(precond_fp32=fp32, use_graph=False, autotune=0)
    geo = P.geometry()
    f = synth.cell_integral(synth.uniform_noise(P.n, nz, seed), geo["areas"], P.vk())
    return P, P.pack(f)


@pytest.mark.parametrize("fp32", [False, True])
def test_noalloc_equals_setup_and_solve(fp32):
    for ref, nz, seed in ((4, 64, 31), (3, 16, 32)):      # the second call smaller than the first
        P, fd = _problem(ref, nz, seed, fp32)
        a = P.device_vector()
        d_ref = T.tpmg_solve_details(P.mg, fd, a, 1e-8, 100)
        p = T.tpmg_mg_params_default()
        p.precond_fp32 = int(fp32)
        b = P.device_vector()
        d = T.tpmg_solve_noalloc(P.op, p, P.stream, fd, b, 1e-8, 100)
        print(f"ref {ref} nz {nz} {'mixed' if fp32 else 'FP64'}: noalloc {d['iters']} iterations, "
              f"relres {d['relres']:.2e}; setup + solve {d_ref['iters']}")
        assert d["status"] == T.TPMG_OK == d_ref["status"]
        assert d["iters"] == d_ref["iters"] and d["relres"] == d_ref["relres"]
        assert np.array_equal(d["history"], d_ref["history"])
        assert torch.equal(a, b)
        assert d["model_bytes"] == d_ref["model_bytes"]
        P.close()


def test_noalloc_limits_and_arguments():
    P, fd = _problem(3, 16, 33, False)
    p = T.tpmg_mg_params_default()
    u = P.device_vector()
    p.use_graph = 1
    with pytest.raises(T.TpmgError) as e:
        T.tpmg_solve_noalloc(P.op, p, P.stream, fd, u, 1e-8, 100)
    assert e.value.status == T.TPMG_ERR_ARG
    p.use_graph = 0
    # a grid whose workspace exceeds the static scratch: rejected before any
    # device work
    big = T.Problem(7, synth.vertical_faces(128, synth.H10KM, "quadratic"), synth.omega_for(7) ** 2)
    need = T.tpmg_mg_workspace_size(big.op, p)
    assert need > T.NOALLOC_SCRATCH_BYTES
    with pytest.raises(T.TpmgError) as e:
        T.tpmg_solve_noalloc(big.op, p, P.stream, fd, u, 1e-8, 100)
    assert e.value.status == T.TPMG_ERR_NOMEM and "static scratch" in str(e.value)
    # maxit cap and a zero right-hand side, as tpmg_solve reports them
    d = T.tpmg_solve_noalloc(P.op, p, P.stream, fd, u, 1e-14, 3)
    assert d["status"] == T.TPMG_NOT_CONVERGED and d["iters"] == 3
    z = P.device_vector()
    d = T.tpmg_solve_noalloc(P.op, p, P.stream, P.device_vector(), z, 1e-8, 100)
    assert d["status"] == T.TPMG_OK and d["iters"] == 0 and not torch.any(z)
    big.close()
    P.close()
