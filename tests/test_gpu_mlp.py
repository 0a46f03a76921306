"""GPU parity of the per-column MLP (learned initial guess) against the
oracle (oracle/mlp.py), through the C ABI: features and targets, the fitted
scaling, the forward pass, loss and gradients, Adam steps, inference into
the solver's layout, error paths; and the gain on a sequence of solves.

Bars (derived from the arithmetic). Both sides round the operands of every
product to bfloat16 (relative spacing 2^-8); the GPU sums in FP32, the
oracle in FP64, so a pre-activation within ~1e-6 of a bfloat16 rounding
boundary can round to the neighbouring value on one side only. Such flips
are rare and each moves an output by about 2^-8 of one term of a 256-term
sum: the outputs agree to 1e-3 of their rms on average and 1e-2 of their
largest magnitude everywhere. Gradients are sums over the batch of such
terms: 2e-2 in the relative 2-norm per tensor."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1408_2981_amd as T  # noqa: E402
import synth  # noqa: E402
from oracle import mlp as omlp, operator as opm, tpmg as otpmg  # noqa: E402

NZ, HIDDEN = 64, 256


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def _data(rows, nz=NZ, seed=0):
    rng = np.random.default_rng(seed)
    scale_x = 10.0 ** rng.uniform(-6, -3, nz + 3)      # cell integrals are small and graded
    x = (rng.standard_normal((rows, nz + 3)) * scale_x + 0.3 * scale_x).astype(np.float32)
    y = (rng.standard_normal((rows, nz)) * 1e-2 + 5e-3).astype(np.float32)
    return x, y


def _net(nz=NZ, hidden=HIDDEN, max_rows=4096, seed=1):
    net = T.ColumnMLP(nz, hidden, max_rows)
    p = omlp.init_params(nz + 3, hidden, nz, seed)
    rng = np.random.default_rng(seed + 1)
    for k in ("b1", "b2", "b3"):
        p[k] = omlp.fp32(rng.standard_normal(p[k].shape) * 0.05)
    net.set_params(omlp.pack(p).astype(np.float32))
    return net, p


def _cuda(a):
    t = torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    torch.cuda.synchronize()
    return t


def test_features_and_targets_match_oracle():
    w = synth.workload("seq_3_16")
    P = T.Problem(w.refinement, w.r_faces(), w.omega2).setup()
    h = otpmg.build(w.refinement, w.r_faces(), w.omega2)
    fine = h.meshes[-1]
    f = synth.sequence_rhs(w, fine.centre, fine.area, h.vert.vk, 3)
    u = np.random.default_rng(2).standard_normal(f.shape)
    net = T.ColumnMLP(w.nz, 64, 4096, stream=P.stream)
    fd, ud = P.pack(f), P.pack(u)
    x = net.features(P, fd)
    y = net.targets(P, ud)
    net.synchronize()
    xo = omlp.features(f, fine.nbr)
    assert x.shape == xo.shape
    assert np.all(np.abs(x.cpu().numpy() - xo) <= 1e-6 * np.abs(xo) + 1e-30)
    assert np.array_equal(y.cpu().numpy(), u.astype(np.float32))


def test_fit_scaling_matches_oracle():
    x, y = _data(10_000, seed=3)
    net = T.ColumnMLP(NZ, HIDDEN, 256)
    net.fit_scaling(_cuda(x), _cuda(y))
    s = omlp.fit_scaling(x.astype(np.float64), y.astype(np.float64))
    mx, sx, my, sy = net.get_scaling()
    for a, b in ((mx, s.mu_x), (sx, s.sd_x), (my, s.mu_y), (sy, s.sd_y)):
        assert np.allclose(a, b, rtol=1e-10, atol=0)


def _oracle_scaling(net):
    mx, sx, my, sy = net.get_scaling()
    return omlp.Scaling(mx.astype(np.float32).astype(np.float64), sx.astype(np.float32).astype(np.float64),
                        my.astype(np.float32).astype(np.float64), sy.astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("rows", [1000, 4096])
def test_forward_matches_oracle(rows):
    x, y = _data(rows, seed=4)
    net, p = _net()
    net.fit_scaling(_cuda(x), _cuda(y))
    s = _oracle_scaling(net)
    yg = net.forward(_cuda(x)).cpu().numpy().astype(np.float64)
    xs = omlp.standardise_x(s, x)
    yo, _ = omlp.forward(p, xs, act_bf16=True)
    yexact, _ = omlp.forward(p, xs, act_bf16=False, round_weights=False)
    d = yg - yo
    rms = float(np.sqrt(np.mean(yo ** 2)))
    print(f"rows {rows}: rms diff {np.sqrt(np.mean(d ** 2)) / rms:.2e}, max diff {np.max(np.abs(d)) / np.max(np.abs(yo)):.2e}, "
          f"vs unrounded network {_rel(yg, yexact):.2e}")
    assert np.sqrt(np.mean(d ** 2)) <= 1e-3 * rms
    assert np.max(np.abs(d)) <= 1e-2 * np.max(np.abs(yo))
    assert _rel(yg, yexact) <= 3e-2          # bfloat16 operands: percent-level against the unrounded network


def test_gradients_match_oracle():
    x, y = _data(20_000, seed=5)
    net, p = _net()
    xd, yd = _cuda(x), _cuda(y)
    net.fit_scaling(xd, yd)
    s = _oracle_scaling(net)
    rows = np.random.default_rng(6).choice(len(x), size=3000, replace=False).astype(np.int32)
    loss, g = net.gradients(xd, yd, _cuda(rows))
    lo, go = omlp.loss_and_grads(p, omlp.standardise_x(s, x[rows]), omlp.standardise_y(s, y[rows]))
    gg = omlp.unpack(g.astype(np.float64), NZ + 3, HIDDEN, NZ)
    print(f"loss GPU {loss:.6e} oracle {lo:.6e}; grads rel diff " +
          ", ".join(f"{k} {_rel(gg[k], go[k]):.1e}" for k in omlp.PARAM_NAMES))
    assert abs(loss - lo) <= 1e-3 * lo
    for k in omlp.PARAM_NAMES:
        assert _rel(gg[k], go[k]) <= 2e-2, k


def test_adam_steps_match_oracle():
    """Five steps with identical batches: the parameter updates agree (Adam
    normalises each update by the gradient's magnitude, so an update is
    about lr per entry; the bar is on the whole update vector)."""
    x, y = _data(16_384, seed=7)
    net, p = _net()
    xd, yd = _cuda(x), _cuda(y)
    net.fit_scaling(xd, yd)
    s = _oracle_scaling(net)
    xs, ys = omlp.standardise_x(s, x), omlp.standardise_y(s, y)
    p0 = omlp.pack(p)
    opt = omlp.Adam(lr=1e-3)
    rng = np.random.default_rng(8)
    for step in range(5):
        rows = rng.choice(len(x), size=2048, replace=False).astype(np.int32)
        net.train_step(xd, yd, _cuda(rows), 1e-3)
        _, g = omlp.loss_and_grads(p, xs[rows], ys[rows])
        p = opt.step(p, g)
    dg = net.get_params().astype(np.float64) - p0
    do = omlp.pack(p) - p0
    print(f"Adam: update rel diff {_rel(dg, do):.2e}, |update| {np.linalg.norm(do):.3e}")
    assert _rel(dg, do) <= 5e-2


def test_train_epoch_equals_train_steps():
    """tpmg_mlp_train_epoch runs the launches of its steps' train_step calls
    in the same order: the parameters after 7 steps (batch 1,000 of a
    seeded permutation of 7,500 rows) and the sampled losses (steps 0, 3, 6)
    are bit for bit those of seven train_step calls; an out-of-range row is
    reported and its flag cleared, and bad arguments are refused."""
    x, y = _data(7_500, seed=21)
    xd, yd = _cuda(x), _cuda(y)
    perm = np.random.default_rng(22).permutation(len(x)).astype(np.int32)
    pd = _cuda(perm)
    steps, batch = 7, 1000
    a, _ = _net(max_rows=batch, seed=3)
    a.fit_scaling(xd, yd)
    want = []
    for k in range(steps):
        loss = a.train_step(xd, yd, _cuda(perm[k * batch:(k + 1) * batch]), 2e-3, want_loss=True)
        if k % 3 == 0 or k == steps - 1:
            want.append(loss)
    b, _ = _net(max_rows=batch, seed=3)
    b.fit_scaling(xd, yd)
    b._ready(xd, yd, pd)
    losses = T.tpmg_mlp_train_epoch(b.h, xd, yd, len(x), pd, steps, batch, 2e-3, 3)
    assert np.array_equal(losses, np.array(want, dtype=np.float32))
    assert np.array_equal(a.get_params(), b.get_params())
    # loss_every 0 samples nothing; an index out of range is reported after the epoch
    bad = perm.copy()
    bad[1500] = len(x)
    assert len(T.tpmg_mlp_train_epoch(b.h, xd, yd, len(x), pd, 2, batch, 2e-3, 0)) == 0
    with pytest.raises(T.TpmgError) as e:
        T.tpmg_mlp_train_epoch(b.h, xd, yd, len(x), _cuda(bad), 2, batch, 2e-3, 0)
    assert e.value.status == T.TPMG_ERR_ARG
    T.tpmg_mlp_train_epoch(b.h, xd, yd, len(x), pd, 1, batch, 2e-3, 0)      # flag cleared
    for args in ((0, batch, 2e-3), (2, batch + 1, 2e-3), (2, batch, 0.0)):
        with pytest.raises(T.TpmgError):
            T.tpmg_mlp_train_epoch(b.h, xd, yd, len(x), pd, *args, 0)


def test_infer_into_solver_layout():
    w = synth.workload("seq_4_32")
    P = T.Problem(w.refinement, w.r_faces(), w.omega2).setup(precond_fp32=True)
    h = otpmg.build(w.refinement, w.r_faces(), w.omega2)
    fine = h.meshes[-1]
    f = synth.sequence_rhs(w, fine.centre, fine.area, h.vert.vk, 7)
    net = T.ColumnMLP(w.nz, 128, P.n, stream=P.stream)
    p = omlp.init_params(w.nz + 3, 128, w.nz, 11)
    net.set_params(omlp.pack(p).astype(np.float32))
    xo = omlp.features(f, fine.nbr)
    yo_raw = np.random.default_rng(12).standard_normal((P.n, w.nz)) * 1e-3
    s = omlp.fit_scaling(xo, yo_raw)
    net.set_scaling(s.mu_x, s.sd_x, s.mu_y, s.sd_y)
    s32 = _oracle_scaling(net)
    fd = P.pack(f)
    u0 = P.device_vector()
    net.infer(P, fd, u0, relax=0)
    net.synchronize()
    tiled = u0.cpu().numpy()
    got = P.unpack(u0)
    ref = omlp.predict(p, s32, f, fine.nbr)
    scale = np.sqrt(np.mean((ref - s32.mu_y) ** 2))
    d = got - ref
    print(f"infer: rms diff {np.sqrt(np.mean(d ** 2)) / scale:.2e}")
    assert np.sqrt(np.mean(d ** 2)) <= 1e-3 * scale
    assert np.count_nonzero(tiled) <= got.size       # padding columns untouched
    # with the line-relaxation sweep: the sweep is linear with a contraction
    # in u_hat, so the difference cannot grow beyond the raw one (x2 margin)
    u1 = P.device_vector()
    net.infer(P, fd, u1, relax=1)
    net.synchronize()
    got1 = P.unpack(u1)
    ref1 = omlp.guess(p, s32, f, fine.nbr, h.finest)
    d1 = got1 - ref1
    print(f"infer + relaxation: rms diff {np.sqrt(np.mean(d1 ** 2)) / scale:.2e}")
    assert np.sqrt(np.mean(d1 ** 2)) <= 2e-3 * scale
    assert np.count_nonzero(u1.cpu().numpy()) <= got1.size


@pytest.mark.parametrize("name", ["seq_4_32", "seq_4_64", "seq_3_128"])
def test_one_kernel_inference_equals_layer_by_layer(name):
    """Hidden width 256 runs the whole inference in one kernel. Its result
    equals the layer-by-layer products of forward() on the same features:
    same bf16 operands, same K order, so the same FP32 output, up to the
    rounding of the final de-standardisation (one fused multiply-add in the
    kernel, a multiply and an add here): bar 2 FP32 ulps of the larger of
    the two terms, |y sd| + |mu| (the result may cancel)."""
    w = synth.workload(name)
    P = T.Problem(w.refinement, w.r_faces(), w.omega2).setup(precond_fp32=True)
    h = otpmg.build(w.refinement, w.r_faces(), w.omega2)
    fine = h.meshes[-1]
    f = synth.sequence_rhs(w, fine.centre, fine.area, h.vert.vk, 5)
    net = T.ColumnMLP(w.nz, 256, P.n, stream=P.stream)
    p = omlp.init_params(w.nz + 3, 256, w.nz, 13)
    net.set_params(omlp.pack(p).astype(np.float32))
    fd = P.pack(f)
    x = net.features(P, fd)
    yo_raw = np.random.default_rng(14).standard_normal((P.n, w.nz)) * 1e-3
    xs = x.cpu().numpy().astype(np.float64)
    s = omlp.fit_scaling(xs, yo_raw)
    net.set_scaling(s.mu_x, s.sd_x, s.mu_y, s.sd_y)
    y = net.forward(x).cpu().numpy()                 # layer by layer, standardised output
    _, _, mu_y, sd_y = net.get_scaling()
    ref = y * np.asarray(sd_y, np.float32)[None, :] + np.asarray(mu_y, np.float32)[None, :]
    u0 = P.device_vector()
    net.infer(P, fd, u0, relax=0)
    net.synchronize()
    got = P.unpack(u0)
    tiled = u0.cpu().numpy()
    d = np.abs(got - ref.astype(np.float64))
    mag = (np.abs(y) * np.abs(np.asarray(sd_y, np.float32))[None, :]
           + np.abs(np.asarray(mu_y, np.float32))[None, :]).astype(np.float32)
    ulp = np.spacing(mag).astype(np.float64)
    tol = 2 * ulp
    print(f"{name}: one-kernel inference vs layer by layer: max diff {d.max():.2e}, "
          f"max diff in FP32 ulps of the terms {np.max(d / ulp):.2f}")
    assert np.all(d <= tol)
    assert np.count_nonzero(tiled) <= got.size       # padding columns untouched
    net.close()
    P.close()


def test_bad_rows_and_arguments():
    x, y = _data(100, seed=9)
    net, _ = _net(max_rows=256)
    xd, yd = _cuda(x), _cuda(y)
    bad = _cuda(np.array([0, 5, 100, 7], dtype=np.int32))       # 100 is out of range
    with pytest.raises(T.TpmgError) as e:
        net.gradients(xd, yd, bad)
    assert e.value.status == T.TPMG_ERR_ARG
    loss, _ = net.gradients(xd, yd, _cuda(np.array([0, 5, 99, 7], dtype=np.int32)))   # flag cleared
    assert np.isfinite(loss)
    with pytest.raises(T.TpmgError):
        net.train_step(xd, yd, _cuda(np.arange(300, dtype=np.int32) % 100), 1e-3)    # batch > max_rows
    with pytest.raises(T.TpmgError):
        T.tpmg_mlp_workspace_size(60, 256, 100)         # nz not a multiple of 8


def test_save_load_roundtrip(tmp_path):
    net, p = _net(nz=16, hidden=64, max_rows=64)
    net.set_scaling(np.arange(19.0), np.ones(19) * 2, np.zeros(16), np.ones(16) * 3)
    path = str(tmp_path / "net.bin")
    net.save(path)
    other = T.ColumnMLP(16, 64, 64)
    other.load(path)
    assert np.array_equal(other.get_params(), net.get_params())
    for a, b in zip(other.get_scaling(), net.get_scaling()):
        assert np.array_equal(a, b)
    wrong = T.ColumnMLP(24, 64, 64)
    with pytest.raises(T.TpmgError):
        wrong.load(path)


def test_learned_guess_saves_iterations():
    """Sequence f_t = f_0 + 0.05 t g on a refinement-4 grid with nz 32: train
    one network on (f_t, u_t) and one on the increments (f_t - f_{t-1},
    u_t - u_{t-1}) of the solutions of t = 1..40 (rtol 1e-10), then solve
    t = 41..50 (mixed precision, rtol 1e-8) from: zero; zero + one
    line-relaxation sweep (the sweep alone, tpmg_relax); the network on f_t
    without and with the sweep; the previous solution without and with the
    sweep; the previous solution + the increment network's output for
    f_t - f_{t-1} with the sweep. Controls separate what the network adds
    from what the sweep and the previous solution give. The network (+ sweep)
    must save iterations over the zero guess on every held-out step; the
    increment network (+ sweep) over the previous solution on every step,
    and over the previous solution + sweep in total, never needing more on
    any step. (Measured on MI355X: zero 15, zero + sweep 15, network 17-18,
    network + sweep 14, previous 12, previous + sweep 11-12, increment
    network + sweep 11 iterations: the network on f_t gains only over the
    zero guess, the increment network at most one iteration.)"""
    w = synth.workload("seq_4_32")
    P = T.Problem(w.refinement, w.r_faces(), w.omega2).setup(precond_fp32=True, use_graph=True)
    geo = P.geometry()
    vk = P.vk()
    ts_train, ts_test = range(1, 41), range(41, 51)
    net = T.ColumnMLP(w.nz, 256, max(4096, P.n), stream=P.stream)
    net.set_params(omlp.pack(omlp.init_params(w.nz + 3, 256, w.nz, 0)).astype(np.float32))
    net_inc = T.ColumnMLP(w.nz, 256, max(4096, P.n), stream=P.stream)
    net_inc.set_params(omlp.pack(omlp.init_params(w.nz + 3, 256, w.nz, 1)).astype(np.float32))
    X = torch.empty((len(ts_train) * P.n, w.nz + 3), dtype=torch.float32, device="cuda")
    Y = torch.empty((len(ts_train) * P.n, w.nz), dtype=torch.float32, device="cuda")
    Xd = torch.empty(((len(ts_train) - 1) * P.n, w.nz + 3), dtype=torch.float32, device="cuda")
    Yd = torch.empty(((len(ts_train) - 1) * P.n, w.nz), dtype=torch.float32, device="cuda")
    prev = None
    for i, t in enumerate(ts_train):
        fd = P.pack(synth.sequence_rhs(w, geo["centres"], geo["areas"], vk, t))
        u = P.device_vector()
        st, *_ = P.solve(fd, u, rtol=1e-10)
        assert st == T.TPMG_OK
        net.features(P, fd, X[i * P.n:(i + 1) * P.n])
        net.targets(P, u, Y[i * P.n:(i + 1) * P.n])
        if prev is not None:
            net_inc.features_increment(P, fd, prev[0], Xd[(i - 1) * P.n:i * P.n])
            net_inc.targets_increment(P, u, prev[1], Yd[(i - 1) * P.n:i * P.n])
        net.synchronize()
        prev = (fd, u)
    for nn, xx, yy, name in ((net, X, Y, "network"), (net_inc, Xd, Yd, "increment network")):
        nn.fit_scaling(xx, yy)
        losses = nn.train(xx, yy, epochs=30, batch=4096, lr=1e-3, seed=0)
        print(name, "epoch losses", [f"{v:.2e}" for v in losses[::5]], f"last {losses[-1]:.2e}")
        assert losses[-1] < 0.1 * losses[0]

    def resid_ratio(fd, u):
        au = P.device_vector()
        P.spmv(u, au)
        P.synchronize()
        return float(torch.linalg.norm(fd - au) / torch.linalg.norm(fd))

    kinds = ("zero", "zero_relax", "network", "network_relax", "previous", "previous_relax", "increment_relax")
    its = {k: [] for k in kinds}
    q = {k: [] for k in kinds}
    f_prev, u_prev = prev
    for t in ts_test:
        fd = P.pack(synth.sequence_rhs(w, geo["centres"], geo["areas"], vk, t))
        sol = None
        for kind in kinds:
            u = P.device_vector()
            if kind == "zero_relax":
                P.relax(fd, P.device_vector(), u)
            elif kind == "network":
                net.infer(P, fd, u, relax=0)
            elif kind == "network_relax":
                net.infer(P, fd, u, relax=1)
            elif kind == "previous":
                u.copy_(u_prev)
            elif kind == "previous_relax":
                P.relax(fd, u_prev, u)
            elif kind == "increment_relax":
                net_inc.infer_increment(P, fd, f_prev, u_prev, u, relax=1)
            P.synchronize()
            torch.cuda.synchronize()
            q[kind].append(resid_ratio(fd, u))
            st, it, *_ = P.solve(fd, u)
            assert st == T.TPMG_OK, kind
            its[kind].append(it)
            if kind == "zero":
                sol = u
        f_prev, u_prev = fd, sol
    for k in kinds:
        print(f"{k:16s} initial residual / |f| {np.mean(q[k]):.2e}, iterations {its[k]}")
    assert all(b < a for a, b in zip(its["zero"], its["network_relax"]))
    assert all(b < a for a, b in zip(its["previous"], its["increment_relax"]))
    assert all(b <= a for a, b in zip(its["previous_relax"], its["increment_relax"]))
    assert sum(its["increment_relax"]) < sum(its["previous_relax"])
    net.close()
    net_inc.close()


def test_relax_matches_oracle():
    """tpmg_relax (one undamped line-relaxation sweep in FP64) against the
    oracle's block-Jacobi sweep with damping 1 (eq. BlockJacobi), from a
    seeded guess and from zero, on a graded grid with random factorised
    profiles. Bar, entry by entry: the rounding floor of the sweep, (8 + nz)
    eps A_T^-1 (|f| + |A| |u_in|) for each side, twice: the residual
    f - A u_in is formed from stencil terms of size |A| |u_in| (|A| = 2 D - A
    for this M-matrix) and its rounding is carried through the column solve
    A_T^-1 (entrywise positive), and the margin-form Thomas solve adds a few
    roundings per level. (With the oracle in FP64 against the same sweep in
    80-bit arithmetic the error is 0.23 of eps A_T^-1 (2|f| + 2|A||u_in|) here,
    9e-11 of the result's largest magnitude: the graded columns amplify the
    rounding of the residual.)"""
    w = synth.workload("seq_4_32")
    prof = synth.profiles_random(w.nz, synth.n_cells(w.refinement), seed=5)
    P = T.Problem(w.refinement, w.r_faces(), w.omega2, profiles=prof).setup()
    h = otpmg.build(w.refinement, w.r_faces(), w.omega2, profiles=prof)
    fine = h.meshes[-1]
    op = h.finest
    l, m, e = opm.column_bands(op)
    f = synth.cell_integral(synth.uniform_noise(P.n, w.nz, 3), fine.area, h.vert.vk)
    u_in = synth.uniform_noise(P.n, w.nz, 4) * 1e-3
    eps = np.finfo(np.float64).eps
    for start in (u_in, np.zeros_like(u_in)):
        out = P.device_vector()
        P.relax(P.pack(f), P.pack(start), out)
        P.synchronize()
        got = P.unpack(out)
        ref = otpmg.smooth(op, f, start, 1.0)
        a = np.abs(start)
        abs_au = 2.0 * (e + l + m) * a - opm.apply(op, a)
        bound = 2 * (8 + w.nz) * eps * otpmg.thomas_margin(l, m, e, np.abs(f) + abs_au)
        ratio = float(np.max(np.abs(got - ref) / bound))
        print(f"relax vs oracle: {np.max(np.abs(got - ref)) / np.max(np.abs(ref)):.2e} of max |u|, "
              f"{ratio:.2e} of the rounding bar")
        assert ratio <= 1.0
    with pytest.raises(T.TpmgError):
        x = P.device_vector()
        P.relax(x, x, x)


def test_increment_features_targets_and_inference():
    """The increment forms against their definitions: features of f - f_prev
    equal the oracle's features of the difference (formed on the host; the
    bar of test_features_and_targets_match_oracle), targets equal u - u_prev
    rounded to FP32, and tpmg_mlp_infer_increment equals u_prev + the
    network's output for the difference (bit for bit, padding columns those
    of u_prev) and, with the sweep, tpmg_relax of that (bit for bit)."""
    w = synth.workload("seq_4_32")
    P = T.Problem(w.refinement, w.r_faces(), w.omega2).setup(precond_fp32=True)
    h = otpmg.build(w.refinement, w.r_faces(), w.omega2)
    fine = h.meshes[-1]
    f_prev = synth.sequence_rhs(w, fine.centre, fine.area, h.vert.vk, 7)
    f = synth.sequence_rhs(w, fine.centre, fine.area, h.vert.vk, 8) + 1e-9 * synth.uniform_noise(P.n, w.nz, 9)
    u_prev_h = synth.uniform_noise(P.n, w.nz, 10) * 1e-2
    u_h = u_prev_h + synth.uniform_noise(P.n, w.nz, 11) * 1e-4
    net = T.ColumnMLP(w.nz, 256, P.n, stream=P.stream)
    p = omlp.init_params(w.nz + 3, 256, w.nz, 13)
    net.set_params(omlp.pack(p).astype(np.float32))
    fd, fpd, ud, upd = P.pack(f), P.pack(f_prev), P.pack(u_h), P.pack(u_prev_h)
    x = net.features_increment(P, fd, fpd)
    y = net.targets_increment(P, ud, upd)
    net.synchronize()
    xo = omlp.features(f - f_prev, fine.nbr)
    assert _rel(x.cpu().numpy(), xo) <= 1e-6
    assert np.array_equal(y.cpu().numpy(), (u_h - u_prev_h).astype(np.float32))
    s = omlp.fit_scaling(xo, (u_h - u_prev_h))
    net.set_scaling(s.mu_x, s.sd_x, s.mu_y, s.sd_y)
    # reference: the plain inference on the difference vector, added to u_prev
    dfd = fd - fpd
    torch.cuda.synchronize()
    du = P.device_vector()
    net.infer(P, dfd, du, relax=0)
    net.synchronize()
    upd_t = upd.clone()
    real = P.pack(np.ones((P.n, w.nz))) != 0
    expect0 = torch.where(real, upd_t + du, upd_t)
    got0 = P.device_vector()
    net.infer_increment(P, fd, fpd, upd, got0, relax=0)
    net.synchronize()
    assert torch.equal(got0, expect0)
    expect1 = P.device_vector()
    P.relax(fd, expect0, expect1)
    got1 = P.device_vector()
    net.infer_increment(P, fd, fpd, upd, got1, relax=1)
    net.synchronize()
    P.synchronize()
    assert torch.equal(got1, expect1)
    with pytest.raises(T.TpmgError):
        net.infer_increment(P, fd, fpd, upd, upd, relax=1)
    net.close()


def test_features_and_inference_at_sequence_shape():
    """The learned guess at the sequence workload's own shape (icosahedral
    refinement 6 x 64 quadratic levels, 81,920 columns, hidden width 256,
    the one-kernel inference): features of every column against the
    oracle's (1e-6 relative), and the network's output on 2,048 seeded
    sample columns against the oracle's forward pass on the same columns
    (bars of the module header)."""
    w = synth.workload("ico6_nz64_seq")
    P = T.Problem(w.refinement, w.r_faces(), w.omega2).setup(precond_fp32=True)
    h = otpmg.build(w.refinement, w.r_faces(), w.omega2)
    fine = h.meshes[-1]
    f = synth.sequence_rhs(w, fine.centre, fine.area, h.vert.vk, 160)
    net = T.ColumnMLP(w.nz, 256, P.n, stream=P.stream)
    p = omlp.init_params(w.nz + 3, 256, w.nz, 17)
    rng = np.random.default_rng(18)
    for k in ("b1", "b2", "b3"):
        p[k] = omlp.fp32(rng.standard_normal(p[k].shape) * 0.05)
    net.set_params(omlp.pack(p).astype(np.float32))
    fd = P.pack(f)
    x = net.features(P, fd)
    net.synchronize()
    xo = omlp.features(f, fine.nbr)
    xg = x.cpu().numpy()
    assert xg.shape == xo.shape == (fine.n, w.nz + 3)
    assert np.all(np.abs(xg - xo) <= 1e-6 * np.abs(xo) + 1e-30)
    yo_raw = np.random.default_rng(19).standard_normal((P.n, w.nz)) * 1e-3
    s = omlp.fit_scaling(xo, yo_raw)
    net.set_scaling(s.mu_x, s.sd_x, s.mu_y, s.sd_y)
    s32 = _oracle_scaling(net)
    u0 = P.device_vector()
    net.infer(P, fd, u0, relax=0)
    net.synchronize()
    got = P.unpack(u0)
    cols = np.sort(np.random.default_rng(20).choice(fine.n, 2048, replace=False))
    yo, _ = omlp.forward(p, omlp.standardise_x(s32, xo[cols]), act_bf16=True)
    ref = yo * s32.sd_y + s32.mu_y
    scale = np.sqrt(np.mean((ref - s32.mu_y) ** 2))
    d = got[cols] - ref
    print(f"sequence shape: features max rel diff {np.max(np.abs(xg - xo) / (np.abs(xo) + 1e-300)):.2e}; "
          f"inference rms diff {np.sqrt(np.mean(d ** 2)) / scale:.2e}, max {np.max(np.abs(d)) / np.max(np.abs(ref - s32.mu_y)):.2e}")
    assert np.sqrt(np.mean(d ** 2)) <= 1e-3 * scale
    assert np.max(np.abs(d)) <= 1e-2 * np.max(np.abs(ref - s32.mu_y))
    net.close()
    P.close()
