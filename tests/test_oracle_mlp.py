"""Pins of the oracle's per-column MLP (learned initial guess): bfloat16
rounding against torch's conversion, the forward pass against a network
whose output is known in closed form, the hand-written backward pass against
central finite differences, Adam against its closed form for a constant
gradient, and the feature/scaling invariants."""
import numpy as np
import pytest

from oracle import mlp

torch = pytest.importorskip("torch")


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-20, 20, 20000),
                        [0.0, -0.0, 1.0, -1.0, 3.0e38, 1e-30]]).astype(np.float32)
    # exact ties: 8 significant bits plus a half unit
    ties = (np.arange(256, 512, dtype=np.float64) + 0.5) * 2.0 ** -8
    x = np.concatenate([x, ties.astype(np.float32), -ties.astype(np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x.astype(np.float64)), ref)


def _identity_net(n):
    """relu(x) - relu(-x) = x: W1 = [I; -I], W2 = I, W3 = [I, -I]."""
    eye = np.eye(n)
    return {"W1": np.vstack([eye, -eye]), "b1": np.zeros(2 * n), "W2": np.eye(2 * n), "b2": np.zeros(2 * n),
            "W3": np.hstack([eye, -eye]), "b3": np.arange(n, dtype=np.float64)}


def test_forward_closed_form():
    n = 6
    p = _identity_net(n)
    x = np.random.default_rng(1).standard_normal((50, n))
    y, _ = mlp.forward(p, x, act_bf16=False)
    assert np.allclose(y, x + np.arange(n), atol=1e-14, rtol=0)
    # with bfloat16 operands the input is rounded once; the weights are exact
    yb, _ = mlp.forward(p, x, act_bf16=True)
    assert np.allclose(yb, mlp.bf16_round(x) + np.arange(n), atol=1e-14, rtol=0)


def test_backward_matches_finite_differences():
    n_in, hidden, n_out = 7, 8, 4     # nz = 4 plus 3 neighbour means
    p = mlp.init_params(n_in, hidden, n_out, seed=3)
    rng = np.random.default_rng(4)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.standard_normal(p[k].shape) * 0.1
    x = rng.standard_normal((16, n_in))
    y = rng.standard_normal((16, n_out))
    loss, g = mlp.loss_and_grads(p, x, y, act_bf16=False, round_weights=False)
    h = 1e-6
    worst = 0.0
    for k in mlp.PARAM_NAMES:
        fd = np.zeros_like(p[k])
        it = np.nditer(p[k], flags=["multi_index"])
        for _ in it:
            i = it.multi_index
            pp = {kk: vv.copy() for kk, vv in p.items()}
            pm = {kk: vv.copy() for kk, vv in p.items()}
            pp[k][i] += h
            pm[k][i] -= h
            lp, _ = mlp.loss_and_grads(pp, x, y, act_bf16=False, round_weights=False)
            lm, _ = mlp.loss_and_grads(pm, x, y, act_bf16=False, round_weights=False)
            fd[i] = (lp - lm) / (2 * h)
        err = np.max(np.abs(fd - g[k])) / max(np.max(np.abs(g[k])), 1e-12)
        worst = max(worst, err)
        assert err < 1e-6, (k, err)
    assert loss > 0 and worst < 1e-6


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are exactly g and
    g^2, so every step moves by lr g / (|g| + eps)."""
    p = {k: np.zeros(s) for k, s in zip(mlp.PARAM_NAMES, [(2, 3), (2,), (2, 2), (2,), (1, 2), (1,)])}
    g = {k: np.full_like(v, 0.25) * (1 if i % 2 else -1) for i, (k, v) in enumerate(p.items())}
    opt = mlp.Adam(lr=1e-2)
    for step in range(1, 6):
        p = opt.step(p, g)
        for k in mlp.PARAM_NAMES:
            expect = -step * 1e-2 * g[k] / (np.abs(g[k]) + 1e-8)
            assert np.allclose(p[k], expect, rtol=1e-6, atol=0), (k, step)


def test_features_and_scaling_invariants():
    rng = np.random.default_rng(5)
    n, nz = 40, 5
    nbr = rng.integers(0, n, size=(n, 3))
    const = np.full((n, nz), 2.5)
    assert np.allclose(mlp.features(const, nbr), 2.5)
    levels = np.tile(np.arange(nz, dtype=np.float64), (n, 1))
    x = mlp.features(levels, nbr)
    assert np.array_equal(x[:, :nz], levels) and np.allclose(x[:, nz:], (nz - 1) / 2)
    xr = rng.standard_normal((1000, nz + 3)) * 3 + 1
    yr = rng.standard_normal((1000, nz)) * 0.5 - 2
    s = mlp.fit_scaling(xr, yr)
    xs, ys = mlp.standardise_x(s, xr), mlp.standardise_y(s, yr)
    assert np.allclose(xs.mean(0), 0, atol=1e-12) and np.allclose(xs.std(0), 1, atol=1e-12)
    assert np.allclose(ys.mean(0), 0, atol=1e-12) and np.allclose(ys.std(0), 1, atol=1e-12)
    s0 = mlp.fit_scaling(np.ones((10, 3)), np.zeros((10, 2)))
    assert np.all(s0.sd_x == 1) and np.all(s0.sd_y == 1)


def test_pack_roundtrip_and_count():
    p = mlp.init_params(67, 256, 64, seed=9)
    v = mlp.pack(p)
    assert v.size == mlp.param_count(67, 256, 64) == 99648
    q = mlp.unpack(v, 67, 256, 64)
    assert all(np.array_equal(p[k], q[k]) for k in mlp.PARAM_NAMES)
    assert all(np.array_equal(p[k], p[k].astype(np.float32)) for k in mlp.PARAM_NAMES)   # FP32 master values
