"""Benchmark: time-to-1e-8 of the TPMG-preconditioned flexible-CG solve.

One step = one complete solve (zero initial guess, FCG until
||r|| <= 1e-8 ||f||) of the 10,485,760-unknown spherical-shell problem:
icosahedral grid refined 6 times (81,920 columns) x 128 quadratically graded
levels, H = 10 km, unit profiles, right-hand side = manufactured field plus
10% seeded uniform noise. The headline `value` is the mixed-precision solve
(FP64 CG, FP32 V-cycle); the FP64 solve is timed on the same grid and
reported alongside. Inputs are resident in HBM before timing starts.

Prints one JSON line. `--gpus N` with N > 1 is refused: the solver runs on
one GPU.
"""
from __future__ import annotations

import argparse
import gc
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "unknowns/s solved to 1e-8 rel. residual (TPMG-CG), HBM GB/s; mixed vs FP64"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(path: str, key: str, instance: str):
    """HBM bytes per dispatch of one kernel instance from a committed counter
    summary under profiles/ (lines "traffic_<key>_<instance>_bytes_per_dispatch:
    B"), or None when kernels.hip has changed since the counters were taken
    or the timed instance was not counted."""
    import hashlib

    src = os.path.join(ROOT, "paper_1408_2981_amd", "csrc", "kernels.hip")
    try:
        vals = dict(l.strip().split(": ", 1) for l in open(os.path.join(ROOT, "profiles", path))
                    if l.strip().startswith(("traffic_", "kernels_hip_")))
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if vals.get("kernels_hip_sha256") != digest:
        return None
    v = vals.get(f"traffic_{key}_{instance}_bytes_per_dispatch")
    return float(v) if v is not None else None


def cpu_baseline(w, iters_fp64: int, sample_iters: int = 2) -> dict:
    """The CPU oracle (NumPy, FP64, one thread) on a bounded sample of the same
    workload. Its FCG solve stopped by maxit = m runs the initial residual and
    V-cycle and m iterations of (q = A p, update, V-cycle): m + 1 operator
    applications and V-cycles. A converged solve of k iterations runs k
    V-cycles and k + 1 operator applications, so the sample's time is scaled
    by k / (m + 1) (k = the GPU FP64 count, which the parity tests pin to the
    oracle's own), leaving out one operator application. Also timed whole,
    on the 20,480-unknown workload: the oracle's FCG solve and a sparse
    direct solve of the assembled matrix (scipy spsolve)."""
    from threadpoolctl import threadpool_limits

    import synth
    from oracle import tpmg as otpmg

    with threadpool_limits(limits=1):
        h = otpmg.build(w.refinement, w.r_faces(), w.omega2)
        fine = h.meshes[-1]
        f = synth.make_rhs(w, fine.centre, fine.area, h.vert.vk)
        t0 = time.perf_counter()
        res = otpmg.solve(h, f, rtol=1e-8, maxit=sample_iters)
        t1 = time.perf_counter()
        del h, f
        w1 = synth.workload("ico3_nz16")
        h1 = otpmg.build(w1.refinement, w1.r_faces(), w1.omega2)
        f1 = synth.make_rhs(w1, h1.meshes[-1].centre, h1.meshes[-1].area, h1.vert.vk)
        t2 = time.perf_counter()
        s1 = otpmg.solve(h1, f1, rtol=1e-8)
        t3 = time.perf_counter()
        otpmg.direct_solve(h1.finest, f1)
        t4 = time.perf_counter()
    units = res.iters + 1 if res.status == "maxit" else res.iters
    t_solve = (t1 - t0) * iters_fp64 / max(units, 1)
    return {
        "value": w.unknowns / t_solve,
        "unit": "unknowns/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"oracle FP64 FCG on {w.name} stopped after {res.iters} iterations ({units} V-cycles and "
                  f"operator applications, {t1 - t0:.1f} s), scaled to the {iters_fp64} V-cycles of the full solve",
        "ico3_nz16_fcg_unknowns_per_s": w1.unknowns / (t3 - t2),
        "ico3_nz16_fcg_iters": s1.iters,
        "ico3_nz16_spsolve_unknowns_per_s": w1.unknowns / (t4 - t3),
    }


def roofline_workload(steps: int, reps: int) -> dict:
    """The HBM-bound workload (icosahedral refinement 7 x 128 quadratic levels,
    41,943,040 unknowns, H = 0.1 x the horizontal spacing, seeded uniform
    right-hand side; at refinement 6 the FP32 fields fit the 256 MB
    last-level cache): mixed and FP64 solve times with the solve's
    algorithmic bytes per second (tpmg_solve_info.model_bytes), and the two dominant
    kernels of the mixed solve timed alone with HIP events on the solver's
    stream (`reps` back-to-back launches each): the finest FP32 line-smoother
    sweep and q = A p with the direction update."""
    import numpy as np
    import torch

    import paper_1408_2981_amd as T
    import synth

    w = synth.workload("ico7_nz128_ar0.1")
    out = {"workload": f"{w.name}: icosahedral refinement 7 x nz 128 quadratic, H = 0.1 h_7, {w.unknowns} unknowns, "
                       f"uniform RHS, rtol 1e-8"}
    for name, fp32 in (("fp64", False), ("mixed", True)):
        P = T.Problem(w.refinement, w.r_faces(), w.omega2).setup(precond_fp32=fp32, use_graph=False, autotune=1)
        geo = P.geometry()
        f = P.pack(synth.make_rhs(w, geo["centres"], geo["areas"], P.vk()))
        u = P.device_vector()
        P.solve(f, u)
        times = []
        for _ in range(steps):
            u.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, it, rr, _, _ = P.solve(f, u)
            times.append(time.perf_counter() - t0)
            assert st == T.TPMG_OK, (name, st)
        ms = 1000.0 * float(np.median(times))
        u.zero_()
        torch.cuda.synchronize()
        model_bytes = T.tpmg_solve_details(P.mg, f, u, 1e-8, 100)["model_bytes"]   # (not timed)
        r = {"ms_per_solve": ms, "iters": it, "unknowns_per_s": w.unknowns / (ms / 1000.0),
             "model_GBs": model_bytes / (ms / 1000.0) / 1e9}
        if fp32:
            fine = P.tuning()[-1]
            sw_ms, sw_b = T.tpmg_mg_time_kernel(P.mg, T.KERNEL_SWEEP, reps)
            op_ms, op_b = T.tpmg_mg_time_kernel(P.mg, T.KERNEL_OPERATOR_PRING, reps)
            r.update(sweep_us=sw_ms * 1000.0, sweep_bytes=sw_b, operator_us=op_ms * 1000.0, operator_bytes=op_b,
                     sweep_instance=f"scan{fine['scan_levels']}", operator_instance=f"chunk{fine['chunk_spmv']}")
        out[name] = r
        P.close()
        del P, f, u
        torch.cuda.empty_cache()
    return out


# (scan levels per wave, stencil chunk) of the counter run: every sweep
# instance (8 or 16 levels per wave; 4 holds at most 64 levels) and every
# operator instance (1 .. 16 levels per wave) the autotuner chooses between
# on the refinement-7 x 128-level grid
PROFILE_INSTANCES = ((8, 4), (16, 16), (8, 8), (16, 2), (8, 1))


def profile_kernels(reps: int):
    """Counter run on the HBM-bound workload (refinement 7 x 128 levels,
    mixed): for each (levels per wave, stencil chunk) of PROFILE_INSTANCES a
    setup with that launch configuration, one solve, then `reps` + 1
    back-to-back finest-grid FP32 sweeps and `reps` + 1 launches of q = A p
    with the direction update; then one copy of 1 GiB (a plain copy kernel of
    known size, larger than the last-level cache, to calibrate FETCH_SIZE and
    WRITE_SIZE). A timed kernel is the only one launched that many times in a
    row, which identifies its dispatches in the trace."""
    import torch

    import paper_1408_2981_amd as T
    import synth

    w = synth.workload("ico7_nz128_ar0.1")
    for scan, chunk in PROFILE_INSTANCES:
        P = T.Problem(w.refinement, w.r_faces(), w.omega2).setup(precond_fp32=True, use_graph=False, autotune=0,
                                                                 smoother=T.SMOOTHER_SCAN, scan_levels=scan,
                                                                 stencil_chunk=chunk)
        geo = P.geometry()
        f = P.pack(synth.make_rhs(w, geo["centres"], geo["areas"], P.vk()))
        u = P.device_vector()
        st, it, rr, _, _ = P.solve(f, u)            # leaves realistic data in the buffers
        sw_ms, sw_b = T.tpmg_mg_time_kernel(P.mg, T.KERNEL_SWEEP, reps)
        op_ms, op_b = T.tpmg_mg_time_kernel(P.mg, T.KERNEL_OPERATOR_PRING, reps)
        fine = P.tuning()[-1]
        assert fine["scan_levels"] == scan and fine["chunk_spmv"] == chunk, fine
        print(json.dumps({"workload": w.name, "sweep_instance": f"scan{scan}", "operator_instance": f"chunk{chunk}",
                          "sweep_avg_us": sw_ms * 1000.0, "sweep_model_bytes": sw_b,
                          "operator_avg_us": op_ms * 1000.0, "operator_model_bytes": op_b,
                          "dispatches_each": reps + 1, "solve_iters": it}), flush=True)
        P.close()
        del P, f, u
        torch.cuda.empty_cache()
    src = torch.ones(1024 * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": 1024 * 1024 * 1024}), flush=True)


def anisotropy_report(steps: int = 3):
    """Refinement 7 x 128 quadratic levels (41,943,040 unknowns), H = ratio x h_7
    for ratio 1e-1, 1e-2, 1e-3, seeded uniform right-hand side: V-cycle rate
    (FP64 and mixed), mixed and FP64 solve time, finest-sweep bandwidth."""
    import numpy as np
    import torch

    import paper_1408_2981_amd as T
    import synth

    for ratio in ("0.1", "0.01", "0.001"):
        w = synth.workload(f"ico7_nz128_ar{ratio}")
        line = {"workload": w.name, "unknowns": w.unknowns, "thickness_km": w.thickness * synth.R_EARTH_M / 1e3}
        for name, fp32 in (("fp64", False), ("mixed", True)):
            P = T.Problem(w.refinement, w.r_faces(), w.omega2).setup(precond_fp32=fp32, use_graph=False,
                                                                      autotune=1)
            geo = P.geometry()
            f = P.pack(synth.make_rhs(w, geo["centres"], geo["areas"], P.vk()))
            u0 = P.pack(synth.uniform_noise(w.n, w.nz, 7))
            rate, _ = T.tpmg_richardson_rate(P.mg, u0, 12, 4)
            u = P.device_vector()
            P.solve(f, u)
            times = []
            for _ in range(steps):
                u.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, it, rr, _, _ = P.solve(f, u)
                times.append(time.perf_counter() - t0)
            ms = 1000.0 * float(np.median(times))
            sweep_ms, sweep_b = T.tpmg_mg_time_sweep(P.mg, 20)
            line[name] = {"vcycle_rate": rate, "iters": it, "status": int(st), "relres": rr, "ms_per_solve": ms,
                          "unknowns_per_s": w.unknowns / (ms / 1000.0), "finest_sweep_us": sweep_ms * 1000.0,
                          "finest_sweep_GBs": sweep_b / (sweep_ms / 1000.0) / 1e9}
            P.close()
            del P, f, u, u0
            torch.cuda.empty_cache()
        print(json.dumps(line), flush=True)


def sequence_report(epochs: int = 16, n_train: int = 150, n_total: int = 200):
    """Learned initial guess on the sequence f_t = f_0 + 0.05 t g (refinement 6
    x 64 quadratic levels, 5,242,880 unknowns, smooth seeded fields): solve
    t = 1..n_train from zero (mixed, rtol 1e-8) and train two per-column MLPs
    on those solutions (GPU, bf16 matrix cores, Adam, batch 4096): one on
    (f_t, u_t), one on the increments (f_t - f_{t-1}, u_t - u_{t-1}). Then
    solve t = n_train+1..n_total from each guess: zero; zero + one
    line-relaxation sweep; the previous solution, without and with the sweep;
    the two-step extrapolation 2 u_{t-1} - u_{t-2}; the network on f_t (+
    sweep); the previous solution + the increment network's output for
    f_t - f_{t-1} (+ sweep); and, for reference, the plain FP64 solve from
    zero. Times include producing the guess. The previous solutions are those
    of the zero-guess solves."""
    import numpy as np
    import torch

    import paper_1408_2981_amd as T
    import synth

    w = synth.workload("ico6_nz64_seq")
    P = T.Problem(w.refinement, w.r_faces(), w.omega2).setup(precond_fp32=True, use_graph=True, autotune=1)
    geo = P.geometry()
    vk = P.vk()
    f0 = P.pack(synth.sequence_rhs(w, geo["centres"], geo["areas"], vk, 0))
    g = P.pack(synth.sequence_rhs(w, geo["centres"], geo["areas"], vk, 1)) - f0   # 0.05 g as a cell integral
    torch.cuda.synchronize()

    def rhs(t):
        f = f0 + float(t) * g
        torch.cuda.synchronize()
        return f

    n_in, h = w.nz + 3, 256

    def new_net(seed):
        net = T.ColumnMLP(w.nz, h, max(4096, P.n), stream=P.stream)
        rng_params = np.random.default_rng(seed)
        he = lambda fan_in, shape: (rng_params.standard_normal(shape) * math.sqrt(2.0 / fan_in)).astype(np.float32)
        net.set_params(np.concatenate([he(n_in, (h, n_in)).ravel(), np.zeros(h, np.float32), he(h, (h, h)).ravel(),
                                       np.zeros(h, np.float32), he(h, (w.nz, h)).ravel(),
                                       np.zeros(w.nz, np.float32)]))
        return net

    net, net_inc = new_net(0), new_net(1)
    X = torch.empty((n_train * P.n, n_in), dtype=torch.float32, device="cuda")
    Y = torch.empty((n_train * P.n, w.nz), dtype=torch.float32, device="cuda")
    Xd = torch.empty(((n_train - 1) * P.n, n_in), dtype=torch.float32, device="cuda")
    Yd = torch.empty(((n_train - 1) * P.n, w.nz), dtype=torch.float32, device="cuda")
    sols = {}
    t0 = time.perf_counter()
    f_prev = u_prev = None
    for t in range(1, n_train + 1):
        f = rhs(t)
        u = P.device_vector()
        st, it, *_ = P.solve(f, u)
        net.features(P, f, X[(t - 1) * P.n:t * P.n])
        net.targets(P, u, Y[(t - 1) * P.n:t * P.n])
        if u_prev is not None:
            net_inc.features_increment(P, f, f_prev, Xd[(t - 2) * P.n:(t - 1) * P.n])
            net_inc.targets_increment(P, u, u_prev, Yd[(t - 2) * P.n:(t - 1) * P.n])
        net.synchronize()
        f_prev, u_prev = f, u
        if t >= n_train - 1:
            sols[t] = u
    t_data = time.perf_counter() - t0
    log(f"sequence: {n_train} training solves and features in {t_data:.1f} s")
    trained = {}
    for name, nn, xx, yy in (("network", net, X, Y), ("increment", net_inc, Xd, Yd)):
        nn.fit_scaling(xx, yy)
        t0 = time.perf_counter()
        losses = nn.train(xx, yy, epochs=epochs, batch=4096, lr=1e-3, seed=0)
        t_train = time.perf_counter() - t0
        log(f"sequence: {name} trained {epochs} epochs in {t_train:.1f} s, epoch losses {losses}")
        trained[name] = {"samples": xx.shape[0], "epochs": epochs, "steps": epochs * (xx.shape[0] // 4096),
                         "epoch_loss": losses, "seconds": t_train}
    flop_step = 6.0 * 4096 * (n_in * h + h * h + h * w.nz)
    for v in trained.values():
        v["TFLOPs_per_s"] = flop_step * v["steps"] / v["seconds"] / 1e12
    del X, Y, Xd, Yd
    torch.cuda.empty_cache()

    # inference timing (device events on the shared stream)
    f = rhs(n_train + 1)
    u = P.device_vector()
    infer_ms = {}
    for relax in (0, 1):
        for _ in range(3):
            net.infer(P, f, u, relax)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(P.stream)
        for _ in range(20):
            net.infer(P, f, u, relax)
        e1.record(P.stream)
        e1.synchronize()
        infer_ms[relax] = e0.elapsed_time(e1) / 20
    flop_inf = 2.0 * P.n * (n_in * h + h * h + h * w.nz)

    # the plain FP64 solve (FP64 V-cycle, zero guess) on the same grid and
    # right-hand sides: the reference the mixed + learned-guess form is to beat
    P64 = T.Problem(w.refinement, w.r_faces(), w.omega2).setup(precond_fp32=False, use_graph=True, autotune=1)
    kinds = ("zero", "zero_relax", "previous", "previous_relax", "extrapolation", "network", "network_increment",
             "fp64_zero")
    res = {k: {"iters": [], "ms": []} for k in kinds}
    for t in range(n_train + 1, n_total + 1):
        f = rhs(t)
        f_before = rhs(t - 1)
        for kind in res:
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if kind == "fp64_zero":
                u = P64.device_vector()
                torch.cuda.synchronize()
                st, it, *_ = P64.solve(f, u)
                res[kind]["ms"].append(1000.0 * (time.perf_counter() - t1))
                res[kind]["iters"].append(it)
                continue
            if kind == "zero":
                u = P.device_vector()
            elif kind == "zero_relax":
                z = P.device_vector()
                u = P.device_vector()
                P.relax(f, z, u)
            elif kind == "previous":
                u = sols[t - 1].clone()
            elif kind == "previous_relax":
                u = P.device_vector()
                P.relax(f, sols[t - 1], u)
            elif kind == "extrapolation":
                u = 2.0 * sols[t - 1] - sols[t - 2]
            elif kind == "network":
                u = P.device_vector()
                net.infer(P, f, u, 1)
            else:
                u = P.device_vector()
                net_inc.infer_increment(P, f, f_before, sols[t - 1], u, 1)
            torch.cuda.synchronize()
            st, it, *_ = P.solve(f, u)
            res[kind]["ms"].append(1000.0 * (time.perf_counter() - t1))
            res[kind]["iters"].append(it)
            if kind == "zero":
                sol = u
        sols[t] = sol
        sols.pop(t - 2, None)
    line = {"workload": f"{w.name}: f_t = f_0 + 0.05 t g, refinement 6 x nz 64 quadratic, {w.unknowns} unknowns, "
                        f"mixed, rtol 1e-8; train t=1..{n_train}, evaluate t={n_train + 1}..{n_total}",
            "train": trained,
            "inference": {"ms_network": infer_ms[0], "ms_with_relaxation": infer_ms[1], "GFLOP": flop_inf / 1e9,
                          "TFLOPs_per_s": flop_inf / (infer_ms[0] / 1000.0) / 1e12,
                          "mfma_bf16_peak_TFLOPs": 2500.0,
                          "frac": flop_inf / (infer_ms[0] / 1000.0) / 1e12 / 2500.0}}
    for kind, r in res.items():
        line[kind] = {"mean_iters": float(np.mean(r["iters"])), "max_iters": int(np.max(r["iters"])),
                      "mean_ms_incl_guess": float(np.mean(r["ms"]))}
    line["network_vs_fp64_zero_speedup"] = line["fp64_zero"]["mean_ms_incl_guess"] / line["network"]["mean_ms_incl_guess"]
    line["network_increment_vs_fp64_zero_speedup"] = (line["fp64_zero"]["mean_ms_incl_guess"]
                                                      / line["network_increment"]["mean_ms_incl_guess"])
    print(json.dumps(line), flush=True)
    P64.close()
    net.close()
    net_inc.close()
    P.close()


def profiles_report(refinement: int = 5, nz: int = 128, eps_list=(0.0, 0.25, 0.5, 0.75, 1.0, 1.23), steps: int = 3):
    """Balanced zonal flow (Section 5.2; profiles from constant buoyancy
    frequency N, eps = (N/N*)^2 - 1, approximate factorisation of the Exner
    pressure) on icosahedral refinement `refinement` x nz quadratically
    graded levels (refinement 5 x 128: the paper's 2.6 million unknowns),
    seeded uniform right-hand side: for each eps, precision and V-cycle
    kind (TPMG^(full), TPMG^(x), TPMG^(partial); the Krylov method always
    uses the full operator) the FCG iterations to 1e-8, the V-cycle's
    Richardson factor, the median solve time, time per iteration and the
    V-cycle's device time per iteration (phase timers)."""
    import numpy as np
    import torch

    import paper_1408_2981_amd as T
    import synth

    r = synth.vertical_faces(nz, synth.H10KM, "quadratic")
    om = synth.omega_for(refinement)
    base = T.Problem(refinement, r, om * om)
    geo = base.geometry()
    vk = base.vk()
    base.close()
    n = synth.n_cells(refinement)
    f_host = synth.cell_integral(synth.uniform_noise(n, nz, 60), geo["areas"], vk)
    u0_host = synth.uniform_noise(n, nz, 7)
    modes = (("full", T.PRECOND_FULL), ("factorised", T.PRECOND_FACTORISED), ("partial", T.PRECOND_PARTIAL))
    for eps in eps_list:
        bf = synth.balanced_flow(eps, geo["centres"], r, om)
        line = {"workload": f"balanced flow eps {eps}: icosahedral refinement {refinement} x nz {nz} quadratic, "
                            f"{n * nz} unknowns, uniform RHS, rtol 1e-8", "eps": eps, "lambda": bf.lam}
        for prec, fp32 in (("fp64", False), ("mixed", True)):
            for name, code in modes:
                P = T.Problem(refinement, r, om * om, profiles=bf.factorised, full=bf).setup(
                    precond_fp32=fp32, use_graph=False, autotune=1, precond_profiles=code)
                f = P.pack(f_host)
                rate, _ = T.tpmg_richardson_rate(P.mg, P.pack(u0_host), 12, 4)
                u = P.device_vector()
                P.solve(f, u)
                times = []
                for _ in range(steps):
                    u.zero_()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    st, it, rr, _, _ = P.solve(f, u, maxit=200)
                    times.append(time.perf_counter() - t0)
                ms = 1000.0 * float(np.median(times))
                u.zero_()
                torch.cuda.synchronize()
                d = T.tpmg_solve_details(P.mg, f, u, 1e-8, 200, phase_timers=True)
                line[f"{prec}_{name}"] = {
                    "status": int(st), "iters": it, "richardson_factor": rate, "ms_per_solve": ms,
                    "ms_per_iter": ms / max(it, 1), "vcycle_ms_per_iter": d["t_vcycle_ms"] / max(d["iters"], 1),
                    "model_GB_per_solve": d["model_bytes"] / 1e9}
                P.close()
                del P, f, u
                torch.cuda.empty_cache()
            # with the vertical advection: the paper's outer solvers
            for name, code in modes:
                P = T.Problem(refinement, r, om * om, profiles=bf.factorised, full=bf, advection=True).setup(
                    precond_fp32=fp32, use_graph=False, autotune=1, precond_profiles=code)
                f = P.pack(f_host)
                for method, fn in (("richardson", T.tpmg_solve_richardson), ("bicgstab", T.tpmg_solve_bicgstab)):
                    u = P.device_vector()
                    fn(P.mg, f, u, 1e-8, 200)
                    times = []
                    for _ in range(steps):
                        u.zero_()
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        d = fn(P.mg, f, u, 1e-8, 200)
                        times.append(time.perf_counter() - t0)
                    ms = 1000.0 * float(np.median(times))
                    line[f"{prec}_adv_{method}_{name}"] = {
                        "status": int(d["status"]), "iters": d["iters"], "ms_per_solve": ms,
                        "ms_per_iter": ms / max(d["iters"], 1), "model_GB_per_solve": d["model_bytes"] / 1e9}
                P.close()
                del P, f, u
                torch.cuda.empty_cache()
        print(json.dumps(line), flush=True)


def smoother_report(steps: int = 5):
    """Block-Jacobi against multicolour block-SOR (the paper's smoother,
    relaxation factor 1, colours ascending before the coarse-grid correction
    and descending after) on the benchmark workload and the refinement-7
    one: V-cycle Richardson factor, FCG iterations and solve time, FP64 and
    mixed."""
    import numpy as np
    import torch

    import paper_1408_2981_amd as T
    import synth

    for wname in ("ico6_nz128", "ico7_nz128_ar0.1"):
        w = synth.workload(wname)
        line = {"workload": f"{w.name}: {w.unknowns} unknowns, rtol 1e-8"}
        f_host = u0_host = None
        for prec, fp32 in (("fp64", False), ("mixed", True)):
            for name, order, omega in (("jacobi", T.SMOOTHER_ORDER_JACOBI, 2.0 / 3.0),
                                       ("sor", T.SMOOTHER_ORDER_SOR, 1.0)):
                P = T.Problem(w.refinement, w.r_faces(), w.omega2).setup(
                    precond_fp32=fp32, use_graph=False, autotune=1, smoother_order=order, omega_relax=omega)
                if f_host is None:
                    geo = P.geometry()
                    f_host = synth.make_rhs(w, geo["centres"], geo["areas"], P.vk())
                    u0_host = synth.uniform_noise(w.n, w.nz, 7)
                f = P.pack(f_host)
                rate, _ = T.tpmg_richardson_rate(P.mg, P.pack(u0_host), 12, 4)
                u = P.device_vector()
                P.solve(f, u)
                times = []
                for _ in range(steps):
                    u.zero_()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    st, it, *_ = P.solve(f, u)
                    times.append(time.perf_counter() - t0)
                ms = 1000.0 * float(np.median(times))
                line[f"{prec}_{name}"] = {"status": int(st), "iters": it, "richardson_factor": rate,
                                          "ms_per_solve": ms, "unknowns_per_s": w.unknowns / (ms / 1000.0)}
                P.close()
                del P, f, u
                torch.cuda.empty_cache()
        print(json.dumps(line), flush=True)


def batch_report(steps: int = 3):
    """Sixteen solves of uneven size (refinement 4/5/6 x nz 32/64/128,
    quadratic grading, seeded uniform right-hand sides, mixed precision):
    one batched solve vs a loop of the sixteen single solves."""
    import numpy as np
    import torch

    import paper_1408_2981_amd as T
    import synth

    stream = torch.cuda.Stream()
    ws = synth.batch_list()
    probs, fs = [], []
    for w in ws:
        P = T.Problem(w.refinement, w.r_faces(), w.omega2).setup(precond_fp32=True, use_graph=True, stream=stream,
                                                                 smoother=T.SMOOTHER_SCAN, autotune=1)
        geo = P.geometry()
        fs.append(P.pack(synth.make_rhs(w, geo["centres"], geo["areas"], P.vk())))
        probs.append(P)
    unknowns = sum(w.unknowns for w in ws)
    us = [P.device_vector() for P in probs]

    def sequential():
        its = []
        for P, f, u in zip(probs, fs, us):
            u.zero_()
            torch.cuda.synchronize()
            st, it, *_ = P.solve(f, u)
            its.append(it)
        return its

    sequential()
    t_seq = []
    for _ in range(steps):
        t0 = time.perf_counter()
        its_seq = sequential()
        t_seq.append(time.perf_counter() - t0)
    mgs = [P.mg for P in probs]
    nbytes = T.tpmg_batch_workspace_size(mgs)
    wsp = torch.zeros(nbytes + 256, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    batch = T.tpmg_batch_create(mgs, wsp.data_ptr() + (-wsp.data_ptr()) % 256, nbytes)
    t_bat = []
    for k in range(steps + 1):
        for u in us:
            u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, per, _ = T.tpmg_batch_solve(batch, fs, us, 1e-8, 100)
        if k:
            t_bat.append(time.perf_counter() - t0)
    its_bat = [p[0] for p in per]
    T.tpmg_batch_destroy(batch)
    chosen = {}
    for w, P in zip(ws, probs):
        fine = P.tuning()[-1]
        chosen[f"ref{w.refinement}_nz{w.nz}"] = {"scan_levels": fine["scan_levels"],
                                                "chunk_restrict": fine["chunk_restrict"],
                                                "chunk_spmv": fine["chunk_spmv"]}
    line = {"workload": "batch16: refinements 4/5/6 x nz 32/64/128 quadratic, mixed, rtol 1e-8",
            "unknowns": unknowns, "status": int(st),
            "batched_ms": 1000.0 * float(np.median(t_bat)), "sequential_ms": 1000.0 * float(np.median(t_seq)),
            "batched_unknowns_per_s": unknowns / float(np.median(t_bat)),
            "iters_batched": its_bat, "iters_single": its_seq, "tuned_finest_level": chosen}
    line["speedup"] = line["sequential_ms"] / line["batched_ms"]
    print(json.dumps(line), flush=True)
    for P in probs:
        P.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="ico6_nz128")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep-reps", type=int, default=50)
    ap.add_argument("--sequence", action="store_true",
                    help="only the learned-initial-guess sequence report (refinement 6 x nz 64, 200 solves)")
    ap.add_argument("--epochs", type=int, default=16)
    ap.add_argument("--autotune", type=int, default=1, choices=(0, 1),
                    help="choose kernels by timed trials at setup (excluded from the timed solves)")
    ap.add_argument("--graph", type=int, default=0, choices=(0, 1),
                    help="1: replay each FCG iteration as one HIP graph; 0 (default): launch the iteration's "
                         "kernels one by one, which on this workload leaves no gap between iterations "
                         "(a graph launch costs ~8 us at each boundary)")
    ap.add_argument("--profiles", action="store_true",
                    help="only the balanced-flow report: TPMG with full, factorised and partial profiles over eps")
    ap.add_argument("--smoothers", action="store_true",
                    help="only the smoother report: block-Jacobi against multicolour block-SOR")
    ap.add_argument("--batch", action="store_true",
                    help="only the batched-solve report (16 problems of uneven size, batched and one by one)")
    ap.add_argument("--report", action="store_true",
                    help="also measure the anisotropy sweep on the refinement-7 grid (one JSON line per ratio)")
    ap.add_argument("--profile-kernels", action="store_true",
                    help="only the kernel timing loops on the refinement-7 grid (finest FP32 sweep and the operator "
                         "with the direction update) and a 1 GiB calibration copy, for hardware-counter runs")
    ap.add_argument("--anisotropy", action="store_true",
                    help="only the anisotropy sweep on refinement 7 x 128 levels (H/h = 1e-1, 1e-2, 1e-3)")
    ap.add_argument("--no-roofline-workload", action="store_true",
                    help="skip the refinement-7 solves and kernel timings that the roofline is taken on")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU decomposition is not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1408_2981_amd as T
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    # The interpreter's cyclic garbage collector stays off for the run: a full
    # collection over torch's objects took ~40 ms, inside whichever timed
    # solve it happened to interrupt.
    gc.collect()
    gc.disable()

    w = synth.workload(args.workload)
    log(f"workload {w.name}: {w.unknowns} unknowns, refinement {w.refinement}, nz {w.nz}")
    if args.profile_kernels:
        profile_kernels(args.sweep_reps)
        return
    if args.sequence:
        sequence_report(epochs=args.epochs)
        return
    if args.batch:
        batch_report()
        return
    if args.anisotropy:
        anisotropy_report()
        return
    if args.profiles:
        profiles_report()
        return
    if args.smoothers:
        smoother_report()
        return
    results = {}
    P64 = T.Problem(w.refinement, w.r_faces(), w.omega2)
    geo = P64.geometry()
    f_host = synth.make_rhs(w, geo["centres"], geo["areas"], P64.vk())
    P32 = T.Problem(w.refinement, w.r_faces(), w.omega2)
    for name, P, fp32 in (("fp64", P64, False), ("mixed", P32, True)):
        P.setup(precond_fp32=fp32, use_graph=bool(args.graph), autotune=args.autotune)
        log(f"{name}: tuning (coarsest first) {P.tuning()}")
        f = P.pack(f_host)
        u = P.device_vector()
        for _ in range(args.warmup):
            u.zero_()
            torch.cuda.synchronize()
            P.solve(f, u)
        times, iters, relres = [], None, None
        for _ in range(args.steps):
            u.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, it, rr, hist, _ = P.solve(f, u)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            assert st == T.TPMG_OK, (name, st)
            iters, relres = it, rr
        ms = 1000.0 * sum(times) / len(times)
        avg_sweep_ms, sweep_bytes = T.tpmg_mg_time_sweep(P.mg, args.sweep_reps)
        # one more solve, untimed, with the per-phase device timers on (kernels
        # launched one by one with HIP events between the phases)
        u.zero_()
        torch.cuda.synchronize()
        d = T.tpmg_solve_details(P.mg, f, u, 1e-8, 100, phase_timers=True)
        results[name] = dict(ms=ms, iters=iters, relres=relres, sweep_ms=avg_sweep_ms, sweep_bytes=sweep_bytes,
                             value=w.unknowns / (ms / 1000.0), model_bytes=d["model_bytes"],
                             phases_ms={k: d[f"t_{k}_ms"] for k in ("vcycle", "spmv", "blas")})
        log(f"{name}: {ms:.3f} ms/solve, {iters} iterations, relres {relres:.2e}, "
            f"finest sweep {avg_sweep_ms * 1000:.1f} us ({sweep_bytes / avg_sweep_ms / 1e6:.0f} GB/s model), "
            f"phases {results[name]['phases_ms']}, model bytes {d['model_bytes'] / 1e9:.2f} GB")

    mixed, fp64 = results["mixed"], results["fp64"]
    tuning32 = P32.tuning()[-1]
    for P in (P64, P32):
        P.close()
    torch.cuda.empty_cache()
    out = {
        "metric": METRIC,
        "value": mixed["value"],
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {
            "workload": f"{w.name}: icosahedral refinement {w.refinement} x nz {w.nz} quadratic, "
                        f"H 10 km, {w.unknowns} unknowns, manufactured + 10% noise RHS, rtol 1e-8",
            "precond": "fp32 V-cycle in fp64 FCG",
            "iters": mixed["iters"],
            "relres": mixed["relres"],
            "model_GBs": mixed["model_bytes"] / (mixed["ms"] / 1000.0) / 1e9,
            "phases_ms": mixed["phases_ms"],
            "fp64_unknowns_per_s": fp64["value"],
            "fp64_ms_per_solve": fp64["ms"],
            "fp64_iters": fp64["iters"],
            "fp64_model_GBs": fp64["model_bytes"] / (fp64["ms"] / 1000.0) / 1e9,
            "fp64_phases_ms": fp64["phases_ms"],
            "mixed_speedup_vs_fp64": fp64["ms"] / mixed["ms"],
            "cache_resident_sweep_GBs": {
                "note": "finest sweep of this workload; its FP32 fields fit the 256 MB last-level cache",
                "mixed": mixed["sweep_bytes"] / (mixed["sweep_ms"] / 1000.0) / 1e9,
                "fp64": fp64["sweep_bytes"] / (fp64["sweep_ms"] / 1000.0) / 1e9},
            "autotune": args.autotune,
            "graph": args.graph,
            "finest_tuning_mixed": tuning32,
        },
    }
    if not args.no_roofline_workload:
        log("refinement-7 workload: solves and kernel timings ...")
        rw = roofline_workload(steps=3, reps=args.sweep_reps)
        m3 = rw["mixed"]
        out["config"]["roofline_workload"] = {
            "workload": rw["workload"],
            "mixed_unknowns_per_s": m3["unknowns_per_s"], "mixed_ms_per_solve": m3["ms_per_solve"],
            "mixed_iters": m3["iters"], "mixed_model_GBs": m3["model_GBs"],
            "fp64_unknowns_per_s": rw["fp64"]["unknowns_per_s"], "fp64_ms_per_solve": rw["fp64"]["ms_per_solve"],
            "fp64_iters": rw["fp64"]["iters"], "fp64_model_GBs": rw["fp64"]["model_GBs"]}
        achieved = m3["sweep_bytes"] / (m3["sweep_us"] / 1e6) / 1e9
        out["roofline"] = {
            "kernel": "finest-grid line-smoother sweep (FP32, mixed solve), refinement 7 x 128 levels",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic("kernels_ico7_nz128_counters.md", "sweep", m3["sweep_instance"]),
            "avg_launch_us": m3["sweep_us"],
            "bytes_per_launch": m3["sweep_bytes"],
        }
        achieved_op = m3["operator_bytes"] / (m3["operator_us"] / 1e6) / 1e9
        out["roofline_operator"] = {
            "kernel": "q = A p with the direction update (FP64), refinement 7 x 128 levels",
            "bound": "hbm",
            "achieved": achieved_op,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_op / HBM_PEAK_GBS,
            "traffic": measured_traffic("kernels_ico7_nz128_counters.md", "operator", m3["operator_instance"]),
            "avg_launch_us": m3["operator_us"],
            "bytes_per_launch": m3["operator_bytes"],
        }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample ...")
        out["cpu_baseline"] = cpu_baseline(w, fp64["iters"])
    print(json.dumps(out), flush=True)
    if args.report:
        batch_report()
        sequence_report()
        anisotropy_report()


if __name__ == "__main__":
    main()
