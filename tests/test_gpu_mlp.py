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
from oracle import mlp as omlp, tpmg as otpmg  # noqa: E402

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
    on the solutions of t = 1..40, then solve t = 41..50 (mixed precision,
    rtol 1e-8) from the zero guess and from the network's guess. The learned
    guess must save iterations on every held-out step."""
    w = synth.workload("seq_4_32")
    P = T.Problem(w.refinement, w.r_faces(), w.omega2).setup(precond_fp32=True, use_graph=True)
    geo = P.geometry()
    vk = P.vk()
    ts_train, ts_test = range(1, 41), range(41, 51)
    net = T.ColumnMLP(w.nz, 256, max(4096, P.n), stream=P.stream)
    net.set_params(omlp.pack(omlp.init_params(w.nz + 3, 256, w.nz, 0)).astype(np.float32))
    X = torch.empty((len(ts_train) * P.n, w.nz + 3), dtype=torch.float32, device="cuda")
    Y = torch.empty((len(ts_train) * P.n, w.nz), dtype=torch.float32, device="cuda")
    for i, t in enumerate(ts_train):
        fd = P.pack(synth.sequence_rhs(w, geo["centres"], geo["areas"], vk, t))
        u = P.device_vector()
        st, *_ = P.solve(fd, u, rtol=1e-10)
        assert st == T.TPMG_OK
        net.features(P, fd, X[i * P.n:(i + 1) * P.n])
        net.targets(P, u, Y[i * P.n:(i + 1) * P.n])
    net.synchronize()
    net.fit_scaling(X, Y)
    losses = net.train(X, Y, epochs=30, batch=4096, lr=1e-3, seed=0)
    print("epoch losses", [f"{v:.2e}" for v in losses[::5]], f"last {losses[-1]:.2e}")
    assert losses[-1] < 0.1 * losses[0]
    def resid_ratio(fd, u):
        au = P.device_vector()
        P.spmv(u, au)
        P.synchronize()
        return float(torch.linalg.norm(fd - au) / torch.linalg.norm(fd))

    zero_it, mlp_it, raw_it, q_raw, q_rel = [], [], [], [], []
    for t in ts_test:
        fd = P.pack(synth.sequence_rhs(w, geo["centres"], geo["areas"], vk, t))
        u = P.device_vector()
        st, it0, *_ = P.solve(fd, u)
        ur = P.device_vector()
        net.infer(P, fd, ur, relax=0)
        net.synchronize()
        q_raw.append(resid_ratio(fd, ur))
        st1, itr, *_ = P.solve(fd, ur)
        u = P.device_vector()
        net.infer(P, fd, u, relax=1)
        net.synchronize()
        q_rel.append(resid_ratio(fd, u))
        st2, it1, *_ = P.solve(fd, u)
        assert st == T.TPMG_OK and st1 == T.TPMG_OK and st2 == T.TPMG_OK
        zero_it.append(it0)
        raw_it.append(itr)
        mlp_it.append(it1)
    print(f"t=41..50: initial residual / |f|: network {np.mean(q_raw):.2e}, with relaxation {np.mean(q_rel):.2e}")
    print(f"iterations: zero guess {zero_it}, network {raw_it}, network + relaxation {mlp_it}")
    assert all(b < a for a, b in zip(zero_it, mlp_it))


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
