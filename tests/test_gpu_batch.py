"""Batched solves of uneven size (several problems advanced together by
grouped launches and one graph per FCG iteration) against the single solves
of the same problems: identical iteration counts and bitwise identical
solutions, because each problem keeps the block decomposition of its own
solve; and the oracle's solution within the FP64 bar."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1408_2981_amd as T  # noqa: E402
import synth  # noqa: E402
from oracle import tpmg as otpmg  # noqa: E402

PROBS = [(2, 8, "uniform", 11), (3, 13, "quadratic", 12), (3, 16, "quadratic", 13), (4, 32, "quadratic", 14),
         (2, 16, "uniform", 15)]


def _setup(fp32, stream):
    out = []
    for ref, nz, grading, seed in PROBS:
        r = synth.vertical_faces(nz, synth.H10KM, grading)
        om2 = synth.omega_for(ref) ** 2
        prof = synth.profiles_random(nz, synth.n_cells(ref), seed=seed + 100)
        P = T.Problem(ref, r, om2, profiles=prof).setup(precond_fp32=fp32, use_graph=True, stream=stream)
        geo = P.geometry()
        f = synth.cell_integral(synth.uniform_noise(P.n, nz, seed), geo["areas"], P.vk())
        out.append((P, f, (ref, r, om2, prof)))
    return out


@pytest.mark.parametrize("fp32", [False, True])
def test_batch_equals_single_solves(fp32):
    stream = torch.cuda.Stream()
    probs = _setup(fp32, stream)
    fs = [P.pack(f) for P, f, _ in probs]
    singles = []
    for (P, f, _), fd in zip(probs, fs):
        u = P.device_vector()
        st, iters, relres, hist, _ = P.solve(fd, u, rtol=1e-8, maxit=200)
        assert st == T.TPMG_OK
        singles.append((iters, P.unpack(u), hist))
    mgs = [P.mg for P, _, _ in probs]
    nbytes = T.tpmg_batch_workspace_size(mgs)
    ws = torch.zeros(nbytes + 256, dtype=torch.uint8, device="cuda")
    off = (-ws.data_ptr()) % 256
    torch.cuda.synchronize()
    batch = T.tpmg_batch_create(mgs, ws.data_ptr() + off, nbytes)
    for rep in range(2):   # second call replays the cached plan and graph
        us = [P.device_vector() for P, _, _ in probs]
        st, per, ms = T.tpmg_batch_solve(batch, fs, us, 1e-8, 200)
        assert st == T.TPMG_OK
        for (P, f, _), u, (iters, hist_b_unused, _h), (it_s, u_s, hist_s) in zip(probs, us, per, singles):
            assert iters == it_s
            assert np.array_equal(P.unpack(u), u_s)
    if not fp32:
        for (P, f, (ref, r, om2, prof)), (it_s, u_s, _) in zip(probs, singles):
            h = otpmg.build(ref, r, om2, profiles=prof)
            o = otpmg.solve(h, f, rtol=1e-8)
            assert o.iters == it_s
            assert np.linalg.norm(u_s - o.x) <= 1e-10 * np.linalg.norm(o.x)
    T.tpmg_batch_destroy(batch)


@pytest.mark.parametrize("fp32", [False, True])
def test_batch_converged_and_capped_problems(fp32):
    """A problem converged from the start stays untouched (0 iterations), and
    with maxit below convergence every problem stops after exactly maxit
    iterations, NOT_CONVERGED, with the solution, residual norm and history of
    its own single solve capped the same way (bit for bit): the iteration
    the host queues ahead changes nothing."""
    stream = torch.cuda.Stream()
    probs = _setup(fp32, stream)[:3]
    fs = [P.pack(f) for P, f, _ in probs]
    fs[1] = probs[1][0].pack(np.zeros_like(probs[1][1]))
    mgs = [P.mg for P, _, _ in probs]
    nbytes = T.tpmg_batch_workspace_size(mgs)
    ws = torch.zeros(nbytes + 256, dtype=torch.uint8, device="cuda")
    off = (-ws.data_ptr()) % 256
    torch.cuda.synchronize()
    batch = T.tpmg_batch_create(mgs, ws.data_ptr() + off, nbytes)
    for maxit in (200, 3):
        singles = []
        for (P, _, _), fd in zip(probs, fs):
            u = P.device_vector()
            st, iters, relres, hist, _ = P.solve(fd, u, rtol=1e-8, maxit=maxit)
            singles.append((st, iters, relres, hist, P.unpack(u)))
        us = [P.device_vector() for P, _, _ in probs]
        st, per, _ = T.tpmg_batch_solve(batch, fs, us, 1e-8, maxit)
        assert st == (T.TPMG_OK if maxit == 200 else T.TPMG_NOT_CONVERGED)
        for (P, _, _), u, (iters, relres, hist), (st_s, it_s, rr_s, hist_s, u_s) in zip(probs, us, per, singles):
            assert iters == it_s
            assert relres == rr_s
            assert np.array_equal(hist, hist_s[: iters + 1])
            assert np.array_equal(P.unpack(u), u_s)
        assert per[1][0] == 0 and not torch.any(us[1])
        if maxit == 3:
            assert per[0][0] == 3 and per[2][0] == 3
    T.tpmg_batch_destroy(batch)


def test_batch_rejects_mixed_parameters():
    stream = torch.cuda.Stream()
    a = _setup(False, stream)[:1]
    b = _setup(True, stream)[:1]
    with pytest.raises(T.TpmgError) as e:
        T.tpmg_batch_workspace_size([a[0][0].mg, b[0][0].mg])
    assert e.value.status == T.TPMG_ERR_ARG


def test_batch16_at_its_own_shape():
    """The sixteen-problem batch at its own shape (refinements 4, 5, 6 x nz
    32, 64, 128, quadratic grading, seeded uniform right-hand sides,
    35,061,760 unknowns, mixed precision, autotuned scan smoothers, as the
    batch report runs it): bitwise equal to the sixteen single solves, and
    for one problem of each (refinement, nz) pair the oracle's results
    stored in tests/golden/batch16_oracle.json by
    tests/golden/make_batch16.py: iteration count within one of the
    oracle's mixed solve, sampled solution within the mixed bar of the
    oracle's FP64 solution (1e-6 of the largest sample, or ten times the
    oracle's own mixed-vs-FP64 distance where that is larger)."""
    import json
    import os

    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "batch16_oracle.json")))
    stream = torch.cuda.Stream()
    ws = synth.batch_list()
    probs, fs = [], []
    for w in ws:
        P = T.Problem(w.refinement, w.r_faces(), w.omega2).setup(precond_fp32=True, use_graph=True, stream=stream,
                                                                 smoother=T.SMOOTHER_SCAN, autotune=1)
        geo = P.geometry()
        fs.append(P.pack(synth.make_rhs(w, geo["centres"], geo["areas"], P.vk())))
        probs.append(P)
    singles = []
    for P, fd in zip(probs, fs):
        u = P.device_vector()
        st, iters, *_ = P.solve(fd, u, rtol=1e-8, maxit=100)
        assert st == T.TPMG_OK
        singles.append((iters, u))
    mgs = [P.mg for P in probs]
    nbytes = T.tpmg_batch_workspace_size(mgs)
    wsp = torch.zeros(nbytes + 256, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    batch = T.tpmg_batch_create(mgs, wsp.data_ptr() + (-wsp.data_ptr()) % 256, nbytes)
    us = [P.device_vector() for P in probs]
    st, per, ms = T.tpmg_batch_solve(batch, fs, us, 1e-8, 100)
    assert st == T.TPMG_OK
    for i, ((it_b, _, _), (it_s, u_s), u_b) in enumerate(zip(per, singles, us)):
        assert it_b == it_s, i
        assert torch.equal(u_b, u_s), i
    for pg in g["problems"]:
        i = pg["index"]
        P = probs[i]
        assert (P.refinement, P.nz) == (pg["refinement"], pg["nz"])
        x = P.unpack(us[i])[np.array(pg["sample_cells"]), np.array(pg["sample_levels"])]
        ref = np.array(pg["fp64_x_samples"])
        err = np.max(np.abs(x - ref)) / np.max(np.abs(ref))
        bar = max(1e-6, 10 * pg["mixed_vs_fp64"])
        print(f"batch problem {i} (refinement {P.refinement}, nz {P.nz}): {per[i][0]} iterations (oracle mixed "
              f"{pg['mixed_iters']}), sampled solution vs oracle FP64 {err:.2e} (bar {bar:.1e})")
        assert abs(per[i][0] - pg["mixed_iters"]) <= 1
        assert err <= bar
    T.tpmg_batch_destroy(batch)
    for P in probs:
        P.close()


@pytest.mark.parametrize("fp32", [False, True])
def test_batch_with_block_sor(fp32):
    """Batched solves with the multicolour block-SOR smoother (colour passes
    of problems at the same schedule position grouped; refinement 1, whose
    grid takes four colours, has a pass the others lack): bitwise equal to
    the single SOR solves, and in FP64 the oracle's SOR solve (identical
    iteration counts, 1e-10)."""
    stream = torch.cuda.Stream()
    probs = []
    for ref, nz, grading, seed in PROBS[:4]:
        r = synth.vertical_faces(nz, synth.H10KM, grading)
        om2 = synth.omega_for(ref) ** 2
        prof = synth.profiles_random(nz, synth.n_cells(ref), seed=seed + 100)
        P = T.Problem(ref, r, om2, profiles=prof).setup(precond_fp32=fp32, use_graph=True, stream=stream,
                                                        smoother_order=T.SMOOTHER_ORDER_SOR, omega_relax=1.0)
        geo = P.geometry()
        f = synth.cell_integral(synth.uniform_noise(P.n, nz, seed), geo["areas"], P.vk())
        probs.append((P, f, (ref, r, om2, prof)))
    fs = [P.pack(f) for P, f, _ in probs]
    singles = []
    for (P, f, _), fd in zip(probs, fs):
        u = P.device_vector()
        st, iters, relres, hist, _ = P.solve(fd, u, rtol=1e-8, maxit=200)
        assert st == T.TPMG_OK
        singles.append((iters, relres, hist, P.unpack(u)))
    mgs = [P.mg for P, _, _ in probs]
    nbytes = T.tpmg_batch_workspace_size(mgs)
    ws = torch.zeros(nbytes + 256, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    batch = T.tpmg_batch_create(mgs, ws.data_ptr() + (-ws.data_ptr()) % 256, nbytes)
    us = [P.device_vector() for P, _, _ in probs]
    st, per, _ = T.tpmg_batch_solve(batch, fs, us, 1e-8, 200)
    assert st == T.TPMG_OK
    for (P, f, (ref, r, om2, prof)), u, (iters, relres, hist), (it_s, rr_s, hist_s, u_s) in zip(probs, us, per, singles):
        assert iters == it_s and relres == rr_s
        assert np.array_equal(P.unpack(u), u_s)
        if not fp32:
            h = otpmg.build(ref, r, om2, profiles=prof).with_sor(1.0)
            o = otpmg.solve(h, f, rtol=1e-8)
            assert o.iters == it_s
            assert np.linalg.norm(u_s - o.x) <= 1e-10 * np.linalg.norm(o.x)
    T.tpmg_batch_destroy(batch)
    # problems that disagree on the smoother are refused
    P0 = probs[0][0]
    Pj = T.Problem(PROBS[0][0], synth.vertical_faces(PROBS[0][1], synth.H10KM, PROBS[0][2]),
                   synth.omega_for(PROBS[0][0]) ** 2).setup(precond_fp32=fp32, stream=stream, omega_relax=1.0)
    with pytest.raises(T.TpmgError) as e:
        T.tpmg_batch_workspace_size([P0.mg, Pj.mg])
    assert e.value.status == T.TPMG_ERR_ARG


@pytest.mark.parametrize("count", [1, 2])
def test_small_batches_one_branch_per_problem(count):
    """A batch of one problem (a graph of one branch) and of two (two
    branches, one problem each) solve bit for bit as the single solves, also
    on a second call that replays the cached graph."""
    stream = torch.cuda.Stream()
    probs = _setup(True, stream)[1:1 + count]
    fs = [P.pack(f) for P, f, _ in probs]
    singles = []
    for (P, _, _), fd in zip(probs, fs):
        u = P.device_vector()
        st, iters, relres, hist, _ = P.solve(fd, u, rtol=1e-8, maxit=200)
        assert st == T.TPMG_OK
        singles.append((iters, relres, P.unpack(u)))
    mgs = [P.mg for P, _, _ in probs]
    nbytes = T.tpmg_batch_workspace_size(mgs)
    ws = torch.zeros(nbytes + 256, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    batch = T.tpmg_batch_create(mgs, ws.data_ptr() + (-ws.data_ptr()) % 256, nbytes)
    for rep in range(2):
        us = [P.device_vector() for P, _, _ in probs]
        st, per, _ = T.tpmg_batch_solve(batch, fs, us, 1e-8, 200)
        assert st == T.TPMG_OK
        for (P, _, _), u, (iters, relres, _h), (it_s, rr_s, u_s) in zip(probs, us, per, singles):
            assert iters == it_s and relres == rr_s
            assert np.array_equal(P.unpack(u), u_s)
    T.tpmg_batch_destroy(batch)


@pytest.mark.parametrize("fp32", [False, True])
def test_batch_with_profiles_that_do_not_factorise(fp32):
    """Problems whose operator has coefficients per (T, k), preconditioned by
    the V-cycle of the full operator (TPMG^(full)), of the approximate
    factorisation (TPMG^(x)) or of the partial one (TPMG^(partial)), batched
    with a factorising problem: each launch holds one profile mode, and every
    problem's iterates equal its single solve's bit for bit; in FP64 the
    TPMG^(full) problem also matches the oracle's solve (identical iteration
    count, 1e-10)."""
    from oracle import mesh, operator as opm

    stream = torch.cuda.Stream()
    cases = []
    for ref, nz, seed, code in ((3, 13, 42, T.PRECOND_FULL), (3, 13, 42, T.PRECOND_FACTORISED),
                                (3, 13, 42, T.PRECOND_PARTIAL), (2, 8, 52, T.PRECOND_FULL)):
        r = synth.vertical_faces(nz, synth.H10KM, "quadratic")
        om2 = synth.omega_for(ref) ** 2
        n = synth.n_cells(ref)
        rng = np.random.default_rng(seed)
        full = opm.FullProfiles(rng.uniform(0.5, 2.0, (n, nz + 1)), rng.uniform(0.5, 2.0, (n, nz)),
                                rng.uniform(0.5, 2.0, (n, nz)))
        prof = synth.profiles_random(nz, n, seed=seed + 1)
        P = T.Problem(ref, r, om2, profiles=prof, full=full).setup(precond_fp32=fp32, use_graph=True, stream=stream,
                                                                   precond_profiles=code)
        m = mesh.hierarchy(ref)[-1]
        f = synth.cell_integral(synth.uniform_noise(n, nz, seed + 2), m.area, opm.vertical(r).vk)
        cases.append((P, f, (ref, r, om2, prof, full, code)))
    ref, nz, grading, seed = PROBS[1]
    r = synth.vertical_faces(nz, synth.H10KM, grading)
    P = T.Problem(ref, r, synth.omega_for(ref) ** 2).setup(precond_fp32=fp32, use_graph=True, stream=stream)
    geo = P.geometry()
    cases.append((P, synth.cell_integral(synth.uniform_noise(P.n, nz, seed), geo["areas"], P.vk()), None))
    fs = [P.pack(f) for P, f, _ in cases]
    singles = []
    for (P, _, _), fd in zip(cases, fs):
        u = P.device_vector()
        st, iters, relres, hist, _ = P.solve(fd, u, rtol=1e-8, maxit=200)
        assert st == T.TPMG_OK
        singles.append((iters, relres, P.unpack(u)))
    mgs = [P.mg for P, _, _ in cases]
    nbytes = T.tpmg_batch_workspace_size(mgs)
    ws = torch.zeros(nbytes + 256, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    batch = T.tpmg_batch_create(mgs, ws.data_ptr() + (-ws.data_ptr()) % 256, nbytes)
    us = [P.device_vector() for P, _, _ in cases]
    st, per, _ = T.tpmg_batch_solve(batch, fs, us, 1e-8, 200)
    assert st == T.TPMG_OK
    for (P, _, _), u, (iters, relres, _h), (it_s, rr_s, u_s) in zip(cases, us, per, singles):
        assert iters == it_s and relres == rr_s
        assert np.array_equal(P.unpack(u), u_s)
    T.tpmg_batch_destroy(batch)
    if not fp32:
        P, f, (ref, r, om2, prof, full, code) = cases[0]
        A = otpmg.build(ref, r, om2, profiles=prof, full=full).finest
        h = otpmg.build(ref, r, om2, profiles=prof, full=full, full_terms=otpmg.FULL_TERMS)
        o = otpmg.solve(h, f, rtol=1e-8, maxit=200, outer=A)
        assert o.iters == singles[0][0]
        assert np.linalg.norm(singles[0][2] - o.x) <= 1e-10 * np.linalg.norm(o.x)
        # an operator with vertical advection is not symmetric: refused
        m = mesh.hierarchy(2)[-1]
        r2 = synth.vertical_faces(8, synth.H10KM, "quadratic")
        bf = synth.balanced_flow(0.5, m.centre, r2, synth.omega_for(2))
        Q = T.Problem(2, r2, synth.omega_for(2) ** 2, profiles=bf.factorised, full=bf, advection=True).setup(
            stream=stream)
        with pytest.raises(T.TpmgError) as e:
            T.tpmg_batch_workspace_size([Q.mg])
        assert e.value.status == T.TPMG_ERR_ARG
