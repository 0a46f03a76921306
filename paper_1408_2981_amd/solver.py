"""Convenience wrapper that owns the library handles of one solve setup.

Holds the grid, operator and multigrid handles and the device workspace (a
torch uint8 tensor on the GPU); every method is a direct call of the C ABI.
"""
from __future__ import annotations

import numpy as np

from . import (
    tpmg_grid_icosahedral, tpmg_grid_geometry, tpmg_grid_vertical, tpmg_op_create, tpmg_op_levels,
    tpmg_mg_params_default, tpmg_mg_workspace_size, tpmg_mg_setup, tpmg_mg_vector_length, tpmg_pack,
    tpmg_unpack, tpmg_spmv, tpmg_vcycle, tpmg_solve, tpmg_grid_destroy, tpmg_op_destroy, tpmg_mg_destroy,
    tpmg_mg_tuning, tpmg_op_set_full_profiles, tpmg_relax, tpmg_op_create_levels,
)


class Problem:
    """Grid + operator on the host; call setup() to place it on the GPU."""

    def __init__(self, refinement: int, r_faces, omega2: float, profiles=None, n_levels: int = 0, full=None,
                 advection: bool = False, level_factors=None):
        """profiles: factorised profile factors (None: unit profiles). full:
        an object with alpha_r [n, nz+1], alpha_s, beta [n, nz], samples of
        profiles that do not factorise on the finest grid; the factorised
        profiles then serve as their approximate factorisation. advection:
        also take full.xi_r [n, nz+1], the vertical advection. level_factors:
        {refinement level: (alpha_r_h, alpha_s_h, beta_h)}, horizontal
        factors sampled by the caller on those grids (entries may be None;
        tpmg_op_create_levels)."""
        r_faces = np.asarray(r_faces, dtype=np.float64)
        self.refinement = refinement
        self.nz = len(r_faces) - 1
        self.grid = tpmg_grid_icosahedral(refinement, self.nz, r_faces)
        if profiles is None:
            ar_v, as_v, b_v = np.ones(self.nz + 1), np.ones(self.nz), np.ones(self.nz)
            h = (None, None, None)
        else:
            ar_v, as_v, b_v = profiles.alpha_r_v, profiles.alpha_s_v, profiles.beta_v
            h = (profiles.alpha_r_h, profiles.alpha_s_h, profiles.beta_h)
        if level_factors:
            tables = [[None] * (refinement + 1) for _ in range(3)]
            for i in range(3):
                tables[i][refinement] = h[i]
                for r, planes in level_factors.items():
                    if planes[i] is not None:
                        tables[i][r] = planes[i]
            self.op = tpmg_op_create_levels(self.grid, n_levels, omega2, ar_v, as_v, b_v, *tables)
        else:
            self.op = tpmg_op_create(self.grid, n_levels, omega2, ar_v, as_v, b_v, *h)
        if full is not None:
            tpmg_op_set_full_profiles(self.op, self.grid, full.alpha_r, full.alpha_s, full.beta,
                                      getattr(full, "xi_r", None) if advection else None)
        self.n_levels = tpmg_op_levels(self.op)
        self.mg = None
        self.workspace = None
        self.stream = None

    # host queries -----------------------------------------------------------
    def geometry(self, refinement_level: int | None = None) -> dict:
        return tpmg_grid_geometry(self.grid, self.refinement if refinement_level is None else refinement_level)

    def vk(self) -> np.ndarray:
        return tpmg_grid_vertical(self.grid, self.nz)

    # device -------------------------------------------------------------------
    def setup(self, precond_fp32: bool = False, use_graph: bool = False, stream=None, **overrides):
        import torch

        if self.mg is not None:
            tpmg_mg_destroy(self.mg)
            self.mg = None
        p = tpmg_mg_params_default()
        p.precond_fp32 = int(precond_fp32)
        p.use_graph = int(use_graph)
        for k, v in overrides.items():
            setattr(p, k, v)
        nbytes = tpmg_mg_workspace_size(self.op, p)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        off = (-self.workspace.data_ptr()) % 256
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.mg = tpmg_mg_setup(self.op, p, self.workspace.data_ptr() + off, nbytes, self.stream)
        self.len, self.n, _ = tpmg_mg_vector_length(self.mg)
        return self

    def device_vector(self):
        """A zeroed tiled FP64 vector, ready for use on the library's stream."""
        import torch

        v = torch.zeros(self.len, dtype=torch.float64, device="cuda")
        torch.cuda.current_stream().synchronize()
        return v

    def pack(self, host_or_dev):
        """Cell-major [n, nz] (numpy or device tensor) -> tiled device vector."""
        import torch

        src = torch.as_tensor(np.ascontiguousarray(host_or_dev, dtype=np.float64)) if isinstance(host_or_dev, np.ndarray) else host_or_dev
        src = src.to("cuda").contiguous()
        out = self.device_vector()      # synchronises torch's stream, so src is ready too
        tpmg_pack(self.mg, src, out)
        self.stream.synchronize()
        return out

    def unpack(self, tiled) -> np.ndarray:
        import torch

        out = torch.empty(self.n * self.nz, dtype=torch.float64, device="cuda")
        torch.cuda.current_stream().synchronize()
        tpmg_unpack(self.mg, tiled, out)
        self.stream.synchronize()
        return out.cpu().numpy().reshape(self.n, self.nz)

    # The calls below run on the library's stream; their tensors must be
    # complete on torch's stream first (device_vector / pack guarantee that).
    def _uses(self, *tensors):
        """Keeps torch's allocator from recycling tensors the library's stream may still read or write."""
        for t in tensors:
            if hasattr(t, "record_stream") and hasattr(self.stream, "cuda_stream"):
                t.record_stream(self.stream)

    def spmv(self, x_tiled, y_tiled):
        self._uses(x_tiled, y_tiled)
        tpmg_spmv(self.mg, x_tiled, y_tiled)

    def vcycle(self, r_tiled, z_tiled):
        self._uses(r_tiled, z_tiled)
        tpmg_vcycle(self.mg, r_tiled, z_tiled)

    def relax(self, f_tiled, u_in_tiled, u_out_tiled):
        """One undamped FP64 line-relaxation sweep on the finest grid."""
        self._uses(f_tiled, u_in_tiled, u_out_tiled)
        tpmg_relax(self.mg, f_tiled, u_in_tiled, u_out_tiled)

    def solve(self, f_tiled, u_tiled, rtol: float = 1e-8, maxit: int = 100):
        """Synchronous; returns (status, iters, relres, history, t_total_ms)."""
        return tpmg_solve(self.mg, f_tiled, u_tiled, rtol, maxit)

    def tuning(self):
        """Launch configuration chosen at setup, one dict per level (0 = coarsest)."""
        return [tpmg_mg_tuning(self.mg, lvl) for lvl in range(tpmg_op_levels(self.op))]

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if self.mg is not None:
            tpmg_mg_destroy(self.mg)
            self.mg = None
        if self.op is not None:
            tpmg_op_destroy(self.op)
            self.op = None
        if self.grid is not None:
            tpmg_grid_destroy(self.grid)
            self.grid = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
