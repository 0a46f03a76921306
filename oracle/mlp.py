"""Learned initial guess: a per-column multilayer perceptron (test
infrastructure only, like the rest of oracle/).

The pressure-correction equation is solved once per time step of the
semi-implicit scheme (Section 1, Section 2.1), and each solve stops at a
residual tolerance, so a better first iterate saves iterations. The learned guess maps the right-hand side of one column (its
nz cell integrals) plus the vertical means of the right-hand sides of its
three horizontal neighbours to the nz values of the solution in that column:

    x = standardise([f_T,0 .. f_T,nz-1, mean_k f_N0,k, mean_k f_N1,k, mean_k f_N2,k])
    h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = W3 h2 + b3
    u0_T = y * sd_y + mu_y

trained by Adam on the mean squared error of standardised targets.

Precision reading (the network is not in the paper; these are the choices
the GPU path implements): master weights are FP32; every matrix product
takes its operands rounded to bfloat16 (round to nearest, ties to even) and
sums exactly (here in FP64; FP32 on the GPU); biases and the Adam update
stay FP32. `act_bf16=False` keeps the activations unrounded (the plain
definition), `round_weights=False` also keeps the weights unrounded (used
by the finite-difference pin, where rounding would make the loss piecewise
constant). Everything else is plain NumPy in FP64.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

PARAM_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def bf16_round(x) -> np.ndarray:
    """Round to the nearest bfloat16 value (8 significant bits, ties to even),
    returned as FP64. Exact for every finite input of bfloat16's range."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                    # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.round(m * 256.0), e - 8)   # np.round: ties to even


def fp32(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# features and targets
# ---------------------------------------------------------------------------

def features(f_cols: np.ndarray, nbr: np.ndarray) -> np.ndarray:
    """[n, nz + 3]: the column's right-hand side, then the vertical means of
    the right-hand sides of neighbours 0, 1, 2."""
    f_cols = np.asarray(f_cols, dtype=np.float64)
    nb_means = f_cols.mean(axis=1)[nbr]           # [n, 3]
    return np.concatenate([f_cols, nb_means], axis=1)


@dataclass
class Scaling:
    mu_x: np.ndarray
    sd_x: np.ndarray
    mu_y: np.ndarray
    sd_y: np.ndarray


def fit_scaling(x: np.ndarray, y: np.ndarray) -> Scaling:
    """Per-feature mean and (population) standard deviation over all training
    rows; a zero deviation is replaced by 1."""
    def ms(a):
        mu = a.mean(axis=0)
        sd = np.sqrt(np.mean((a - mu) ** 2, axis=0))
        return mu, np.where(sd > 0.0, sd, 1.0)
    mx, sx = ms(np.asarray(x, dtype=np.float64))
    my, sy = ms(np.asarray(y, dtype=np.float64))
    return Scaling(mx, sx, my, sy)


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------

def init_params(n_in: int, hidden: int, n_out: int, seed: int) -> dict:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, FP32 values."""
    rng = np.random.default_rng(seed)
    p = {
        "W1": rng.standard_normal((hidden, n_in)) * np.sqrt(2.0 / n_in),
        "b1": np.zeros(hidden),
        "W2": rng.standard_normal((hidden, hidden)) * np.sqrt(2.0 / hidden),
        "b2": np.zeros(hidden),
        "W3": rng.standard_normal((n_out, hidden)) * np.sqrt(2.0 / hidden),
        "b3": np.zeros(n_out),
    }
    return {k: fp32(v) for k, v in p.items()}


def param_count(n_in: int, hidden: int, n_out: int) -> int:
    return hidden * n_in + hidden + hidden * hidden + hidden + n_out * hidden + n_out


def pack(p: dict) -> np.ndarray:
    """Parameters in the order W1, b1, W2, b2, W3, b3, row-major."""
    return np.concatenate([np.asarray(p[k], dtype=np.float64).ravel() for k in PARAM_NAMES])


def unpack(v: np.ndarray, n_in: int, hidden: int, n_out: int) -> dict:
    shapes = {"W1": (hidden, n_in), "b1": (hidden,), "W2": (hidden, hidden), "b2": (hidden,),
              "W3": (n_out, hidden), "b3": (n_out,)}
    out, o = {}, 0
    for k in PARAM_NAMES:
        size = int(np.prod(shapes[k]))
        out[k] = np.asarray(v[o:o + size], dtype=np.float64).reshape(shapes[k])
        o += size
    assert o == len(v)
    return out


def forward(p: dict, xs: np.ndarray, act_bf16: bool = True, round_weights: bool = True):
    """Standardised inputs xs [rows, n_in] -> standardised outputs [rows, n_out],
    and the intermediate values the backward pass needs."""
    rw = bf16_round if round_weights else (lambda a: np.asarray(a, dtype=np.float64))
    ra = bf16_round if act_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    W1, W2, W3 = rw(p["W1"]), rw(p["W2"]), rw(p["W3"])
    a0 = ra(xs)
    z1 = a0 @ W1.T + p["b1"]
    a1 = ra(np.maximum(z1, 0.0))
    z2 = a1 @ W2.T + p["b2"]
    a2 = ra(np.maximum(z2, 0.0))
    y = a2 @ W3.T + p["b3"]
    return y, dict(a0=a0, z1=z1, a1=a1, z2=z2, a2=a2, W1=W1, W2=W2, W3=W3)


def loss_and_grads(p: dict, xs: np.ndarray, ys: np.ndarray, act_bf16: bool = True, round_weights: bool = True):
    """Mean squared error over all entries of the batch, and its gradients
    (backpropagation written out; the operands of every product are rounded
    like those of the forward pass; the weights' gradients are applied to
    the FP32 master weights)."""
    ra = bf16_round if act_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    y, c = forward(p, xs, act_bf16, round_weights)
    d = y - ys
    loss = float(np.mean(d * d))
    dy = ra(2.0 * d / d.size)
    g = {}
    g["W3"] = dy.T @ c["a2"]
    g["b3"] = dy.sum(axis=0)
    dz2 = ra((dy @ c["W3"]) * (c["z2"] > 0.0))
    g["W2"] = dz2.T @ c["a1"]
    g["b2"] = dz2.sum(axis=0)
    dz1 = ra((dz2 @ c["W2"]) * (c["z1"] > 0.0))
    g["W1"] = dz1.T @ c["a0"]
    g["b1"] = dz1.sum(axis=0)
    return loss, g


@dataclass
class Adam:
    """Adam (Kingma & Ba) with bias correction; moments in FP64, parameters
    stored back as FP32 master weights."""
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    t: int = 0
    m: dict = field(default_factory=dict)
    v: dict = field(default_factory=dict)

    def step(self, p: dict, g: dict) -> dict:
        self.t += 1
        out = {}
        for k in PARAM_NAMES:
            m = self.m.get(k, np.zeros_like(g[k]))
            v = self.v.get(k, np.zeros_like(g[k]))
            m = self.beta1 * m + (1.0 - self.beta1) * g[k]
            v = self.beta2 * v + (1.0 - self.beta2) * g[k] * g[k]
            self.m[k], self.v[k] = m, v
            mhat = m / (1.0 - self.beta1 ** self.t)
            vhat = v / (1.0 - self.beta2 ** self.t)
            out[k] = fp32(p[k] - self.lr * mhat / (np.sqrt(vhat) + self.eps))
        return out


def standardise_x(s: Scaling, x: np.ndarray) -> np.ndarray:
    return (np.asarray(x, dtype=np.float64) - s.mu_x) / s.sd_x


def standardise_y(s: Scaling, y: np.ndarray) -> np.ndarray:
    return (np.asarray(y, dtype=np.float64) - s.mu_y) / s.sd_y


def predict(p: dict, s: Scaling, f_cols: np.ndarray, nbr: np.ndarray, act_bf16: bool = True) -> np.ndarray:
    """Initial guess [n, nz] for the right-hand side f_cols [n, nz]."""
    y, _ = forward(p, standardise_x(s, features(f_cols, nbr)), act_bf16)
    return y * s.sd_y + s.mu_y


def guess(p: dict, s: Scaling, f_cols: np.ndarray, nbr: np.ndarray, op, act_bf16: bool = True) -> np.ndarray:
    """The network's prediction followed by one undamped line-relaxation
    sweep, u_hat + A_T^-1 (f - A u_hat) (the block-Jacobi column solve of
    Section 5 with damping 1), on the operator op of the grid."""
    from . import tpmg as tp

    return tp.smooth(op, f_cols, predict(p, s, f_cols, nbr, act_bf16), 1.0)
