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


def measured_traffic(scan_levels: int):
    """HBM bytes per finest-sweep dispatch from the committed counter summary,
    or None when kernels.hip has changed since the counters were taken or the
    timed sweep uses another levels-per-wave instance than the one counted."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "smoother_ico6_nz128_counters.md")
    src = os.path.join(ROOT, "paper_1408_2981_amd", "csrc", "kernels.hip")
    try:
        vals = dict(l.strip().split(": ", 1) for l in open(path)
                    if l.strip().startswith(("traffic_", "kernels_hip_", "scan_levels")))
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if vals.get("kernels_hip_sha256") != digest or vals.get("scan_levels") != str(scan_levels):
        return None
    return float(vals["traffic_bytes_per_dispatch"])


def cpu_baseline(w, iters_fp64: int, sample_iters: int = 3) -> dict:
    """The CPU oracle (NumPy, FP64, one thread) on a bounded sample of the same
    workload: its FCG solve is run for `sample_iters` iterations (initial
    residual included) and timed, and the time is scaled to the iteration
    count the full solve needs (the GPU FP64 count, which the parity tests pin
    to the oracle's own)."""
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
    done = max(res.iters, 1)
    t_solve = (t1 - t0) * iters_fp64 / done
    return {
        "value": w.unknowns / t_solve,
        "unit": "unknowns/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"oracle FP64 FCG on {w.name}, first {done} iterations timed ({t1 - t0:.1f} s), "
                  f"scaled to the {iters_fp64} iterations of the full solve",
    }


def profile_sweep(w, reps: int):
    """Counter run: `reps` finest-grid FP32 sweeps, then one copy of 512 MiB
    (a plain copy kernel of known size, to calibrate FETCH_SIZE and
    WRITE_SIZE)."""
    import torch

    import paper_1408_2981_amd as T
    import synth

    P = T.Problem(w.refinement, w.r_faces(), w.omega2).setup(precond_fp32=True, use_graph=False, autotune=1)
    geo = P.geometry()
    f = P.pack(synth.make_rhs(w, geo["centres"], geo["areas"], P.vk()))
    u = P.device_vector()
    st, it, rr, _, _ = P.solve(f, u)            # leaves realistic data in the sweep buffers
    ms, nbytes = T.tpmg_mg_time_sweep(P.mg, reps)
    src = torch.ones(512 * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"sweep_avg_us": ms * 1000.0, "sweep_model_bytes": nbytes, "sweep_dispatches": reps,
                      "copy_bytes": 512 * 1024 * 1024, "solve_iters": it}), flush=True)


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


def sequence_report(epochs: int = 4, n_train: int = 150, n_total: int = 200):
    """Learned initial guess on the sequence f_t = f_0 + 0.05 t g (refinement 6
    x 64 quadratic levels, 5,242,880 unknowns, smooth seeded fields): solve
    t = 1..n_train from zero (mixed, rtol 1e-8), train the per-column MLP on
    those solutions (GPU, bf16 matrix cores, Adam, batch 4096), then solve
    t = n_train+1..n_total from four guesses: zero, the previous solution,
    the network (+ one line-relaxation sweep) and the two-step extrapolation
    2 u_{t-1} - u_{t-2}; and, for reference, the plain FP64 solve from zero.
    Times include producing the guess."""
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

    net = T.ColumnMLP(w.nz, 256, max(4096, P.n), stream=P.stream)
    rng_params = np.random.default_rng(0)
    n_in, h = w.nz + 3, 256
    he = lambda fan_in, shape: (rng_params.standard_normal(shape) * math.sqrt(2.0 / fan_in)).astype(np.float32)
    net.set_params(np.concatenate([he(n_in, (h, n_in)).ravel(), np.zeros(h, np.float32), he(h, (h, h)).ravel(),
                                   np.zeros(h, np.float32), he(h, (w.nz, h)).ravel(), np.zeros(w.nz, np.float32)]))
    X = torch.empty((n_train * P.n, n_in), dtype=torch.float32, device="cuda")
    Y = torch.empty((n_train * P.n, w.nz), dtype=torch.float32, device="cuda")
    sols = {}
    t0 = time.perf_counter()
    for t in range(1, n_train + 1):
        f = rhs(t)
        u = P.device_vector()
        st, it, *_ = P.solve(f, u)
        net.features(P, f, X[(t - 1) * P.n:t * P.n])
        net.targets(P, u, Y[(t - 1) * P.n:t * P.n])
        if t >= n_train - 1:
            sols[t] = u
    net.synchronize()
    t_data = time.perf_counter() - t0
    log(f"sequence: {n_train} training solves and features in {t_data:.1f} s")
    net.fit_scaling(X, Y)
    t0 = time.perf_counter()
    losses = net.train(X, Y, epochs=epochs, batch=4096, lr=1e-3, seed=0)
    t_train = time.perf_counter() - t0
    log(f"sequence: trained {epochs} epochs in {t_train:.1f} s, epoch losses {losses}")
    steps = epochs * (X.shape[0] // 4096)
    flop_step = 6.0 * 4096 * (n_in * h + h * h + h * w.nz)
    del X, Y
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
    res = {k: {"iters": [], "ms": []} for k in ("zero", "previous", "network", "extrapolation", "fp64_zero")}
    for t in range(n_train + 1, n_total + 1):
        f = rhs(t)
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
            elif kind == "previous":
                u = sols[t - 1].clone()
            elif kind == "extrapolation":
                u = 2.0 * sols[t - 1] - sols[t - 2]
            else:
                u = P.device_vector()
                net.infer(P, f, u, 1)
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
            "train": {"samples": n_train * P.n, "epochs": epochs, "steps": steps, "batch": 4096,
                      "epoch_loss": losses, "seconds": t_train, "data_seconds": t_data,
                      "TFLOPs_per_s": flop_step * steps / t_train / 1e12},
            "inference": {"ms_network": infer_ms[0], "ms_with_relaxation": infer_ms[1], "GFLOP": flop_inf / 1e9,
                          "TFLOPs_per_s": flop_inf / (infer_ms[0] / 1000.0) / 1e12,
                          "mfma_bf16_peak_TFLOPs": 2500.0,
                          "frac": flop_inf / (infer_ms[0] / 1000.0) / 1e12 / 2500.0}}
    for kind, r in res.items():
        line[kind] = {"mean_iters": float(np.mean(r["iters"])), "max_iters": int(np.max(r["iters"])),
                      "mean_ms_incl_guess": float(np.mean(r["ms"]))}
    line["network_vs_fp64_zero_speedup"] = line["fp64_zero"]["mean_ms_incl_guess"] / line["network"]["mean_ms_incl_guess"]
    print(json.dumps(line), flush=True)
    P64.close()
    net.close()
    P.close()


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
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--autotune", type=int, default=1, choices=(0, 1),
                    help="choose kernels by timed trials at setup (excluded from the timed solves)")
    ap.add_argument("--graph", type=int, default=0, choices=(0, 1),
                    help="1: replay each FCG iteration as one HIP graph; 0 (default): launch the iteration's "
                         "kernels one by one, which on this workload leaves no gap between iterations "
                         "(a graph launch costs ~8 us at each boundary)")
    ap.add_argument("--batch", action="store_true",
                    help="only the batched-solve report (16 problems of uneven size, batched and one by one)")
    ap.add_argument("--report", action="store_true",
                    help="also measure the anisotropy sweep on the refinement-7 grid (one JSON line per ratio)")
    ap.add_argument("--profile-sweep", action="store_true",
                    help="only the finest-grid sweep timing loop (mixed) and a 512 MiB calibration copy, "
                         "for hardware-counter runs")
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
    if args.profile_sweep:
        profile_sweep(w, args.sweep_reps)
        return
    if args.sequence:
        sequence_report(epochs=args.epochs)
        return
    if args.batch:
        batch_report()
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
        results[name] = dict(ms=ms, iters=iters, relres=relres, sweep_ms=avg_sweep_ms, sweep_bytes=sweep_bytes,
                             value=w.unknowns / (ms / 1000.0))
        log(f"{name}: {ms:.3f} ms/solve, {iters} iterations, relres {relres:.2e}, "
            f"finest sweep {avg_sweep_ms * 1000:.1f} us ({sweep_bytes / avg_sweep_ms / 1e6:.0f} GB/s model)")

    mixed, fp64 = results["mixed"], results["fp64"]
    achieved = mixed["sweep_bytes"] / (mixed["sweep_ms"] / 1000.0) / 1e9
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
            "fp64_unknowns_per_s": fp64["value"],
            "fp64_ms_per_solve": fp64["ms"],
            "fp64_iters": fp64["iters"],
            "mixed_speedup_vs_fp64": fp64["ms"] / mixed["ms"],
            "fp64_sweep_GBs": fp64["sweep_bytes"] / (fp64["sweep_ms"] / 1000.0) / 1e9,
            "autotune": args.autotune,
            "graph": args.graph,
            "finest_tuning_mixed": P32.tuning()[-1],
        },
        "roofline": {
            "kernel": "finest-grid line-smoother sweep (FP32, mixed solve)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(P32.tuning()[-1]["scan_levels"]) if args.workload == "ico6_nz128" else None,
            "avg_launch_us": mixed["sweep_ms"] * 1000.0,
            "bytes_per_launch": mixed["sweep_bytes"],
        },
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample ...")
        out["cpu_baseline"] = cpu_baseline(w, fp64["iters"])
    print(json.dumps(out), flush=True)
    if args.report:
        for P in (P64, P32):
            P.close()
        torch.cuda.empty_cache()
        batch_report()
        sequence_report()
        anisotropy_report()


if __name__ == "__main__":
    main()
