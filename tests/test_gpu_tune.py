"""Launch tuning on the GPU. Every line-smoother kernel the setup can choose
(column in registers joined by block scans at 4, 8 or 16 levels per wave;
LDS-staged; global scratch) reproduces the oracle's V-cycle (Algorithm 1)
and flexible-CG solve within the FP64 bar, and its FP32 form stays within
the FP32 V-cycle bar; stencil chunks change no stencil output bit; the
autotuner's choices are admissible, cached and reused; a batch groups sweeps
of different levels per wave and still equals the single solves bitwise."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1408_2981_amd as T  # noqa: E402
import synth  # noqa: E402
from oracle import operator as opm, tpmg as otpmg  # noqa: E402
from gpu_common import make, rel  # noqa: E402

KINDS = {
    "scan4": dict(smoother=T.SMOOTHER_SCAN, scan_levels=4),
    "scan8": dict(smoother=T.SMOOTHER_SCAN, scan_levels=8),
    "scan16": dict(smoother=T.SMOOTHER_SCAN, scan_levels=16),
    "lds": dict(smoother=T.SMOOTHER_LDS),
    "global": dict(smoother=T.SMOOTHER_GLOBAL),
}


def _expect_tuning(P, cfg):
    for t in P.tuning():
        assert t["smoother"] == cfg["smoother"]
        if cfg["smoother"] == T.SMOOTHER_SCAN:
            assert t["scan_levels"] == cfg["scan_levels"]


@pytest.mark.parametrize("case", ["ico3_nz13_quad", "ico4_nz32_quad"])
@pytest.mark.parametrize("kind", list(KINDS))
def test_smoother_kinds_fp64(case, kind):
    h, P, f = make(case, use_graph=True, **KINDS[kind])
    _expect_tuning(P, KINDS[kind])
    zd = P.device_vector()
    P.vcycle(P.pack(f), zd)
    P.synchronize()
    z = P.unpack(zd)
    zref = otpmg.vcycle(h, f)
    ref = otpmg.solve(h, f, rtol=1e-8)
    ud = P.device_vector()
    st, iters, relres, hist, _ = P.solve(P.pack(f), ud, rtol=1e-8, maxit=100)
    u = P.unpack(ud)
    print(f"{case} {kind}: V-cycle {rel(z, zref):.2e}, solve iters {iters} (oracle {ref.iters}) err {rel(u, ref.x):.2e}")
    assert rel(z, zref) <= 1e-10
    assert st == T.TPMG_OK and iters == ref.iters
    assert rel(u, ref.x) <= 1e-10


@pytest.mark.parametrize("kind", list(KINDS))
def test_smoother_kinds_fp32(kind):
    """FP32 V-cycle bar (as for the default kernel): as close to the FP64
    V-cycle as the oracle's FP32 V-cycle is, within 10x plus 1e-7; the mixed
    solve converges within one iteration of the oracle's mixed solve."""
    case = "ico4_nz32_quad"
    h, P, f = make(case, precond_fp32=True, use_graph=True, **KINDS[kind])
    _expect_tuning(P, KINDS[kind])
    zd = P.device_vector()
    P.vcycle(P.pack(f), zd)
    P.synchronize()
    z = P.unpack(zd)
    z64 = otpmg.vcycle(h, f)
    z32 = otpmg.make_preconditioner(h, "fp32")(f)
    e_gpu = np.linalg.norm(z - z64) / np.linalg.norm(z64)
    e_orc = np.linalg.norm(z32 - z64) / np.linalg.norm(z64)
    ref32 = otpmg.solve(h, f, rtol=1e-8, precision="fp32")
    ud = P.device_vector()
    st, iters, relres, _, _ = P.solve(P.pack(f), ud, rtol=1e-8, maxit=100)
    print(f"{kind}: FP32 V-cycle error GPU {e_gpu:.2e} oracle {e_orc:.2e}; mixed iters {iters} (oracle {ref32.iters})")
    assert e_gpu <= 10 * e_orc + 1e-7
    assert st == T.TPMG_OK and abs(iters - ref32.iters) <= 1 and relres <= 1e-8


@pytest.mark.parametrize("nz", [200, 300])
def test_tall_columns(nz):
    """Columns beyond the 8-levels-per-wave scan: the default choice (scan at
    16 levels per wave up to nz 256 in FP32; LDS or global scratch otherwise)
    against the oracle, FP64 and mixed."""
    ref_level = 1
    r = synth.vertical_faces(nz, synth.H10KM, "quadratic")
    om2 = synth.omega_for(ref_level) ** 2
    prof = synth.profiles_random(nz, synth.n_cells(ref_level), seed=nz)
    h = otpmg.build(ref_level, r, om2, profiles=prof)
    fine = h.meshes[-1]
    f = synth.cell_integral(synth.uniform_noise(fine.n, nz, nz), fine.area, h.vert.vk)
    ref = otpmg.solve(h, f, rtol=1e-8)
    ref32 = otpmg.solve(h, f, rtol=1e-8, precision="fp32")
    for fp32 in (False, True):
        P = T.Problem(ref_level, r, om2, profiles=prof).setup(precond_fp32=fp32, use_graph=True)
        kinds = {t["smoother"] for t in P.tuning()}
        ud = P.device_vector()
        st, iters, relres, _, _ = P.solve(P.pack(f), ud, rtol=1e-8, maxit=100)
        u = P.unpack(ud)
        print(f"nz {nz} fp32={fp32}: smoother {kinds} iters {iters} (oracle {ref32.iters if fp32 else ref.iters}) "
              f"err {rel(u, ref.x):.2e}")
        assert st == T.TPMG_OK
        if fp32:
            # beyond 256 levels: LDS-staged where two FP32 [nz][64] arrays fit the
            # device's LDS per workgroup, else global scratch
            assert kinds == {T.SMOOTHER_SCAN} if nz <= 256 else len(kinds) == 1 and kinds <= {T.SMOOTHER_LDS, T.SMOOTHER_GLOBAL}
            assert abs(iters - ref32.iters) <= 1 and relres <= 1e-8
        else:
            assert kinds == {T.SMOOTHER_GLOBAL}    # two FP64 [nz][64] arrays exceed the LDS
            assert iters == ref.iters and rel(u, ref.x) <= 1e-10
        P.close()


@pytest.mark.parametrize("chunk", [1, 3, 16])
def test_stencil_chunks_change_no_output_bit(chunk):
    h, P0, f = make("ico4_nz32_quad")
    _, P1, _ = make("ico4_nz32_quad", stencil_chunk=chunk)
    assert all(t["chunk_restrict"] == chunk for t in P1.tuning()[1:])
    x = np.random.default_rng(5).standard_normal(f.shape)
    outs = []
    for P in (P0, P1):
        yd = P.device_vector()
        P.spmv(P.pack(x), yd)
        zd = P.device_vector()
        P.vcycle(P.pack(f), zd)
        P.synchronize()
        outs.append((P.unpack(yd), P.unpack(zd)))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    ref = otpmg.solve(h, f, rtol=1e-8)
    ud = P1.device_vector()
    st, iters, _, _, _ = P1.solve(P1.pack(f), ud, rtol=1e-8, maxit=100)
    assert st == T.TPMG_OK and iters == ref.iters and rel(P1.unpack(ud), ref.x) <= 1e-10


def test_autotune_choices_cached_and_reused(tmp_path):
    T.tpmg_tune_clear()
    h, P, f = make("ico4_nz32_quad", autotune=1, use_graph=True)
    trials, ms = T.tpmg_mg_autotune_stats(P.mg)
    tun = P.tuning()
    print(f"autotune: {trials} trials, {ms:.2f} ms; choices {tun}")
    assert trials > 0 and ms > 0
    nz = 32
    for lvl, t in enumerate(tun):
        assert t["smoother"] in (T.SMOOTHER_SCAN, T.SMOOTHER_LDS, T.SMOOTHER_GLOBAL)
        if t["smoother"] == T.SMOOTHER_SCAN:
            assert t["scan_levels"] in (4, 8, 16) and nz <= 16 * t["scan_levels"]
        if lvl > 0:
            assert t["chunk_restrict"] in (1, 2, 4, 8, 16) and t["chunk_prolong"] in (1, 2, 4, 8, 16)
    assert tun[-1]["chunk_spmv"] in (1, 2, 4, 8, 16)
    n_entries = T.tpmg_tune_entries()
    assert n_entries > 0
    # the autotuned solve keeps FP64 parity
    ref = otpmg.solve(h, f, rtol=1e-8)
    ud = P.device_vector()
    st, iters, _, _, _ = P.solve(P.pack(f), ud, rtol=1e-8, maxit=100)
    assert st == T.TPMG_OK and iters == ref.iters and rel(P.unpack(ud), ref.x) <= 1e-10
    # same shape again: served from the cache, no trials
    _, P2, _ = make("ico4_nz32_quad", autotune=1)
    assert T.tpmg_mg_autotune_stats(P2.mg)[0] == 0 and P2.tuning() == tun
    # through a file
    path = tmp_path / "tune.json"
    T.tpmg_tune_save(str(path))
    T.tpmg_tune_clear()
    T.tpmg_tune_load(str(path))
    assert T.tpmg_tune_entries() == n_entries
    _, P3, _ = make("ico4_nz32_quad", autotune=1)
    assert T.tpmg_mg_autotune_stats(P3.mg)[0] == 0 and P3.tuning() == tun
    # autotune=2 re-times
    _, P4, _ = make("ico4_nz32_quad", autotune=2)
    assert T.tpmg_mg_autotune_stats(P4.mg)[0] > 0
    # caller overrides win over the trials
    _, P5, _ = make("ico4_nz32_quad", autotune=1, smoother=T.SMOOTHER_SCAN, scan_levels=4)
    assert all(t["smoother"] == T.SMOOTHER_SCAN and t["scan_levels"] == 4 for t in P5.tuning())
    T.tpmg_tune_clear()


def test_batch_groups_levels_per_wave():
    """Problems whose scan sweeps use 4, 8 and 16 levels per wave in one batch:
    sweeps of one schedule position are split into one launch per kernel
    instance; every problem still equals its own single solve bitwise."""
    stream = torch.cuda.Stream()
    specs = [(2, 16, 4, 21), (3, 32, 8, 22), (3, 13, 16, 23), (2, 32, 4, 24)]
    probs = []
    for ref, nz, kb, seed in specs:
        r = synth.vertical_faces(nz, synth.H10KM, "quadratic")
        om2 = synth.omega_for(ref) ** 2
        prof = synth.profiles_random(nz, synth.n_cells(ref), seed=seed)
        P = T.Problem(ref, r, om2, profiles=prof).setup(precond_fp32=True, use_graph=True, stream=stream,
                                                        smoother=T.SMOOTHER_SCAN, scan_levels=kb)
        geo = P.geometry()
        f = synth.cell_integral(synth.uniform_noise(P.n, nz, seed), geo["areas"], P.vk())
        probs.append((P, f))
    fs = [P.pack(f) for P, f in probs]
    singles = []
    for (P, _), fd in zip(probs, fs):
        u = P.device_vector()
        st, iters, _, _, _ = P.solve(fd, u, rtol=1e-8, maxit=200)
        assert st == T.TPMG_OK
        singles.append((iters, P.unpack(u)))
    mgs = [P.mg for P, _ in probs]
    nbytes = T.tpmg_batch_workspace_size(mgs)
    ws = torch.zeros(nbytes + 256, dtype=torch.uint8, device="cuda")
    off = (-ws.data_ptr()) % 256
    torch.cuda.synchronize()
    batch = T.tpmg_batch_create(mgs, ws.data_ptr() + off, nbytes)
    us = [P.device_vector() for P, _ in probs]
    st, per, _ = T.tpmg_batch_solve(batch, fs, us, 1e-8, 200)
    assert st == T.TPMG_OK
    for (P, _), u, (iters, _, _), (it_s, u_s) in zip(probs, us, per, singles):
        assert iters == it_s
        assert np.array_equal(P.unpack(u), u_s)
    T.tpmg_batch_destroy(batch)
    # a problem with a non-scan smoother cannot join a batch
    r = synth.vertical_faces(16, synth.H10KM, "quadratic")
    Q = T.Problem(2, r, synth.omega_for(2) ** 2).setup(precond_fp32=True, use_graph=True, stream=stream,
                                                         smoother=T.SMOOTHER_LDS)
    with pytest.raises(T.TpmgError) as e:
        T.tpmg_batch_workspace_size([probs[0][0].mg, Q.mg])
    assert e.value.status == T.TPMG_ERR_ARG
