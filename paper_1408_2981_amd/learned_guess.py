"""Per-column MLP initial guess on the GPU: a thin owner of the workspace
and handle of the tpmg_mlp_* calls (include/tpmg_mlp.h). Argument
marshalling and the epoch loop only; features, standardisation, products,
gradients, Adam and inference run in the library's kernels."""
from __future__ import annotations

import numpy as np

from . import (
    tpmg_mlp_create, tpmg_mlp_destroy, tpmg_mlp_features, tpmg_mlp_fit_scaling, tpmg_mlp_forward,
    tpmg_mlp_get_params, tpmg_mlp_get_scaling, tpmg_mlp_gradients, tpmg_mlp_infer, tpmg_mlp_load,
    tpmg_mlp_param_count, tpmg_mlp_save, tpmg_mlp_set_params, tpmg_mlp_set_scaling, tpmg_mlp_targets,
    tpmg_mlp_train_step, tpmg_mlp_train_epoch, tpmg_mlp_workspace_size, tpmg_mlp_features_increment,
    tpmg_mlp_targets_increment, tpmg_mlp_infer_increment,
)


class ColumnMLP:
    def __init__(self, nz: int, hidden: int = 256, max_rows: int = 4096, stream=None):
        import torch

        self.nz, self.hidden, self.n_in, self.max_rows = nz, hidden, nz + 3, max_rows
        self.n_params = tpmg_mlp_param_count(nz, hidden)
        nbytes = tpmg_mlp_workspace_size(nz, hidden, max_rows)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        off = (-self.workspace.data_ptr()) % 256
        self.stream = stream if stream is not None else torch.cuda.Stream()
        torch.cuda.current_stream().synchronize()
        self.h = tpmg_mlp_create(nz, hidden, max_rows, self.workspace.data_ptr() + off, nbytes, self.stream)

    # parameters and scaling ---------------------------------------------------
    def set_params(self, packed) -> None:
        tpmg_mlp_set_params(self.h, packed)

    def get_params(self) -> np.ndarray:
        return tpmg_mlp_get_params(self.h, self.n_params)

    def set_scaling(self, mu_x, sd_x, mu_y, sd_y) -> None:
        tpmg_mlp_set_scaling(self.h, mu_x, sd_x, mu_y, sd_y)

    def get_scaling(self):
        return tpmg_mlp_get_scaling(self.h, self.n_in, self.nz)

    def fit_scaling(self, x, y) -> None:
        self._ready(x, y)
        tpmg_mlp_fit_scaling(self.h, x, y, x.shape[0])

    # data ---------------------------------------------------------------------
    def _ready(self, *tensors) -> None:
        """Tensors made on torch's stream must be complete before the library's
        stream reads them, and must not be recycled by torch's allocator while
        the library's stream may still use them (record_stream)."""
        import torch

        torch.cuda.current_stream().synchronize()
        for t in tensors:
            if hasattr(t, "record_stream") and hasattr(self.stream, "cuda_stream"):
                t.record_stream(self.stream)

    def features(self, problem, f_tiled, out=None):
        import torch

        if out is None:
            out = torch.empty((problem.n, self.n_in), dtype=torch.float32, device="cuda")
        self._ready(f_tiled, out)
        tpmg_mlp_features(self.h, problem.mg, f_tiled, out)
        return out

    def targets(self, problem, u_tiled, out=None):
        import torch

        if out is None:
            out = torch.empty((problem.n, self.nz), dtype=torch.float32, device="cuda")
        self._ready(u_tiled, out)
        tpmg_mlp_targets(self.h, problem.mg, u_tiled, out)
        return out

    def features_increment(self, problem, f_tiled, f_prev_tiled, out=None):
        """Features of the increment f - f_prev of the right-hand side."""
        import torch

        if out is None:
            out = torch.empty((problem.n, self.n_in), dtype=torch.float32, device="cuda")
        self._ready(f_tiled, f_prev_tiled, out)
        tpmg_mlp_features_increment(self.h, problem.mg, f_tiled, f_prev_tiled, out)
        return out

    def targets_increment(self, problem, u_tiled, u_prev_tiled, out=None):
        """Targets: the increment u - u_prev of the solution."""
        import torch

        if out is None:
            out = torch.empty((problem.n, self.nz), dtype=torch.float32, device="cuda")
        self._ready(u_tiled, u_prev_tiled, out)
        tpmg_mlp_targets_increment(self.h, problem.mg, u_tiled, u_prev_tiled, out)
        return out

    def forward(self, x):
        import torch

        y = torch.empty((x.shape[0], self.nz), dtype=torch.float32, device="cuda")
        self._ready(x, y)
        tpmg_mlp_forward(self.h, x, x.shape[0], y)
        self.stream.synchronize()
        return y

    def gradients(self, x, y, rows):
        self._ready(x, y, rows)
        return tpmg_mlp_gradients(self.h, x, y, x.shape[0], rows, rows.shape[0], self.n_params)

    def train_step(self, x, y, rows, lr: float, want_loss: bool = False):
        self._ready(x, y, rows)
        return tpmg_mlp_train_step(self.h, x, y, x.shape[0], rows, rows.shape[0], lr, want_loss)

    def train(self, x, y, epochs: int, batch: int = 4096, lr: float = 1e-3, seed: int = 0, loss_every: int = 50):
        """Adam over shuffled mini-batches (a permutation per epoch, drawn on
        the GPU from a generator seeded with seed); returns the mean sampled
        batch loss per epoch."""
        import torch

        rows_total = x.shape[0]
        gen = torch.Generator(device="cuda")
        gen.manual_seed(seed)
        per_epoch = []
        self._ready(x, y)
        for _ in range(epochs):
            perm = torch.randperm(rows_total, generator=gen, device="cuda", dtype=torch.int32)
            self._ready(perm)
            nb = rows_total // batch
            # the epoch's steps in one call (the launches of nb train_step calls)
            losses = tpmg_mlp_train_epoch(self.h, x, y, rows_total, perm, nb, batch, lr, loss_every) if nb else []
            per_epoch.append(float(np.mean(losses)) if len(losses) else float("nan"))
        return per_epoch

    def infer(self, problem, f_tiled, u0_tiled, relax: int = 1) -> None:
        """u0_tiled (a zeroed tiled vector of problem) receives the guess, followed by
        one line-relaxation sweep when relax = 1; asynchronous on the shared stream."""
        self._ready(f_tiled, u0_tiled)
        tpmg_mlp_infer(self.h, problem.mg, f_tiled, u0_tiled, relax)

    def infer_increment(self, problem, f_tiled, f_prev_tiled, u_prev_tiled, u0_tiled, relax: int = 1) -> None:
        """u0_tiled = u_prev + the network's increment for f - f_prev, followed
        by one line-relaxation sweep when relax = 1; asynchronous."""
        self._ready(f_tiled, f_prev_tiled, u_prev_tiled, u0_tiled)
        tpmg_mlp_infer_increment(self.h, problem.mg, f_tiled, f_prev_tiled, u_prev_tiled, u0_tiled, relax)

    def save(self, path: str) -> None:
        tpmg_mlp_save(self.h, path)

    def load(self, path: str) -> None:
        tpmg_mlp_load(self.h, path)

    def synchronize(self) -> None:
        self.stream.synchronize()

    def close(self) -> None:
        if getattr(self, "h", None):
            tpmg_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
