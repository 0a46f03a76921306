"""Python binding of libtpmg.so, the MI355X tensor-product multigrid solver.

Argument marshalling only: every step of the solve runs in the library's
HIP kernels. Functions carry the C ABI's names (include/tpmg.h); device
buffers are torch tensors on the GPU (their data_ptr() is passed), host
arrays are numpy arrays. The library must have been built
(paper_1408_2981_amd/build.py); importing without it raises ImportError, and
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtpmg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1408_2981_amd/build.py`")

# torch ships its own HIP and HSA runtimes under the same sonames as
# /opt/rocm's. Loading torch first makes libtpmg.so bind to those copies, so
# the process has a single runtime and both sides see the same device,
# memory and streams.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

TPMG_OK = 0
TPMG_NOT_CONVERGED = 1
TPMG_ERR_ARG = -1
TPMG_ERR_DEVICE = -2
TPMG_ERR_NOMEM = -3
TPMG_ERR_BREAKDOWN = -4
TPMG_ERR_STATE = -5

EXPORTED = [
    "tpmg_mg_params_default", "tpmg_grid_icosahedral", "tpmg_grid_level_size", "tpmg_grid_geometry",
    "tpmg_grid_vertical", "tpmg_grid_colouring", "tpmg_op_create", "tpmg_op_create_levels", "tpmg_op_set_full_profiles", "tpmg_op_coefficients_full", "tpmg_op_levels", "tpmg_op_level_size", "tpmg_op_coefficients",
    "tpmg_op_prolongation", "tpmg_mg_workspace_size", "tpmg_mg_setup", "tpmg_mg_vector_length", "tpmg_pack",
    "tpmg_unpack", "tpmg_spmv", "tpmg_vcycle", "tpmg_relax", "tpmg_solve", "tpmg_batch_workspace_size", "tpmg_batch_create", "tpmg_batch_solve", "tpmg_batch_destroy",
    "tpmg_richardson_rate", "tpmg_mg_time_sweep", "tpmg_mg_time_kernel", "tpmg_mg_tuning", "tpmg_mg_autotune_stats", "tpmg_tune_load",
    "tpmg_tune_save", "tpmg_tune_clear", "tpmg_tune_entries", "tpmg_grid_destroy", "tpmg_op_destroy",
    "tpmg_mlp_param_count", "tpmg_mlp_workspace_size", "tpmg_mlp_create", "tpmg_mlp_set_params", "tpmg_mlp_get_params",
    "tpmg_mlp_set_scaling", "tpmg_mlp_get_scaling", "tpmg_mlp_fit_scaling", "tpmg_mlp_features", "tpmg_mlp_targets",
    "tpmg_mlp_forward", "tpmg_mlp_gradients", "tpmg_mlp_train_step", "tpmg_mlp_train_epoch", "tpmg_mlp_infer", "tpmg_mlp_features_increment",
    "tpmg_mlp_targets_increment", "tpmg_mlp_infer_increment", "tpmg_mlp_save",
    "tpmg_mlp_load", "tpmg_mlp_destroy",
    "tpmg_mg_destroy", "tpmg_status_string", "tpmg_last_error", "tpmg_solve_noalloc", "tpmg_solve_richardson",
    "tpmg_solve_bicgstab",
]


class TpmgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{status_string(status)}: {message}")
        self.status = status


class MgParams(ctypes.Structure):
    _fields_ = [
        ("n_levels", ctypes.c_int), ("nu_pre", ctypes.c_int), ("nu_post", ctypes.c_int),
        ("nu_coarse", ctypes.c_int), ("omega_relax", ctypes.c_double), ("precond_fp32", ctypes.c_int),
        ("use_graph", ctypes.c_int), ("autotune", ctypes.c_int), ("smoother", ctypes.c_int),
        ("scan_levels", ctypes.c_int), ("stencil_chunk", ctypes.c_int), ("precond_profiles", ctypes.c_int),
        ("smoother_order", ctypes.c_int), ("tile_cols", ctypes.c_int),
    ]


# line-smoother kinds (tpmg_mg_params.smoother, tpmg_mg_tuning)
SMOOTHER_SCAN = 1
SMOOTHER_LDS = 2
SMOOTHER_GLOBAL = 3


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int), ("relres", ctypes.c_double), ("history", ctypes.POINTER(ctypes.c_double)),
        ("history_cap", ctypes.c_int), ("t_total_ms", ctypes.c_double), ("phase_timers", ctypes.c_int),
        ("div_tol", ctypes.c_double), ("t_vcycle_ms", ctypes.c_double), ("t_spmv_ms", ctypes.c_double),
        ("t_blas_ms", ctypes.c_double), ("model_bytes", ctypes.c_double),
    ]


_vp = ctypes.c_void_p
_ip = ctypes.c_int
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_i32p = ctypes.POINTER(ctypes.c_int32)

_sig = {
    "tpmg_mg_params_default": (None, [ctypes.POINTER(MgParams)]),
    "tpmg_grid_icosahedral": (_ip, [_ip, _ip, _dp, ctypes.POINTER(_vp)]),
    "tpmg_grid_level_size": (_ip, [_vp, _ip, ctypes.POINTER(_ip)]),
    "tpmg_grid_geometry": (_ip, [_vp, _ip, _dp, _dp, _i32p, _dp, _dp]),
    "tpmg_grid_vertical": (_ip, [_vp, _dp]),
    "tpmg_grid_colouring": (_ip, [_vp, _ip, _i32p, ctypes.POINTER(_ip)]),
    "tpmg_op_create": (_ip, [_vp, _ip, ctypes.c_double, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.POINTER(_vp)]),
    "tpmg_op_create_levels": (_ip, [_vp, _ip, ctypes.c_double, _dp, _dp, _dp, ctypes.POINTER(_dp),
                                    ctypes.POINTER(_dp), ctypes.POINTER(_dp), ctypes.POINTER(_vp)]),
    "tpmg_op_set_full_profiles": (_ip, [_vp, _vp, _dp, _dp, _dp, _dp]),
    "tpmg_op_coefficients_full": (_ip, [_vp, _ip, _dp, _dp, _dp, _dp, _dp]),
    "tpmg_op_levels": (_ip, [_vp, ctypes.POINTER(_ip)]),
    "tpmg_op_level_size": (_ip, [_vp, _ip, ctypes.POINTER(_ip)]),
    "tpmg_op_coefficients": (_ip, [_vp, _ip, _dp, _dp, _dp, _dp, _dp, _dp]),
    "tpmg_op_prolongation": (_ip, [_vp, _ip, _dp]),
    "tpmg_mg_workspace_size": (_ip, [_vp, ctypes.POINTER(MgParams), ctypes.POINTER(ctypes.c_size_t)]),
    "tpmg_mg_setup": (_ip, [_vp, ctypes.POINTER(MgParams), _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
    "tpmg_mg_vector_length": (_ip, [_vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(_ip), ctypes.POINTER(_ip)]),
    "tpmg_pack": (_ip, [_vp, _vp, _vp]),
    "tpmg_unpack": (_ip, [_vp, _vp, _vp]),
    "tpmg_spmv": (_ip, [_vp, _vp, _vp]),
    "tpmg_vcycle": (_ip, [_vp, _vp, _vp]),
    "tpmg_relax": (_ip, [_vp, _vp, _vp, _vp]),
    "tpmg_solve": (_ip, [_vp, _vp, _vp, ctypes.c_double, _ip, ctypes.POINTER(SolveInfo)]),
    "tpmg_solve_richardson": (_ip, [_vp, _vp, _vp, ctypes.c_double, _ip, ctypes.POINTER(SolveInfo)]),
    "tpmg_solve_bicgstab": (_ip, [_vp, _vp, _vp, ctypes.c_double, _ip, ctypes.POINTER(SolveInfo)]),
    "tpmg_batch_workspace_size": (_ip, [ctypes.POINTER(_vp), _ip, ctypes.POINTER(ctypes.c_size_t)]),
    "tpmg_batch_create": (_ip, [ctypes.POINTER(_vp), _ip, _vp, ctypes.c_size_t, ctypes.POINTER(_vp)]),
    "tpmg_batch_solve": (_ip, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_double, _ip,
                               ctypes.POINTER(SolveInfo)]),
    "tpmg_batch_destroy": (None, [_vp]),
    "tpmg_richardson_rate": (_ip, [_vp, _vp, _ip, _ip, _dp, _dp]),
    "tpmg_mg_time_sweep": (_ip, [_vp, _ip, _dp, _dp]),
    "tpmg_mg_time_kernel": (_ip, [_vp, _ip, _ip, _dp, _dp]),
    "tpmg_mg_tuning": (_ip, [_vp, _ip] + [ctypes.POINTER(_ip)] * 5),
    "tpmg_mg_autotune_stats": (_ip, [_vp, ctypes.POINTER(_ip), _dp]),
    "tpmg_tune_load": (_ip, [ctypes.c_char_p]),
    "tpmg_tune_save": (_ip, [ctypes.c_char_p]),
    "tpmg_tune_clear": (_ip, []),
    "tpmg_tune_entries": (_ip, [ctypes.POINTER(_ip)]),
    "tpmg_mlp_param_count": (_ip, [_ip, _ip, ctypes.POINTER(ctypes.c_size_t)]),
    "tpmg_mlp_workspace_size": (_ip, [_ip, _ip, _ip, ctypes.POINTER(ctypes.c_size_t)]),
    "tpmg_mlp_create": (_ip, [_ip, _ip, _ip, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
    "tpmg_mlp_set_params": (_ip, [_vp, _fp]),
    "tpmg_mlp_get_params": (_ip, [_vp, _fp]),
    "tpmg_mlp_set_scaling": (_ip, [_vp, _dp, _dp, _dp, _dp]),
    "tpmg_mlp_get_scaling": (_ip, [_vp, _dp, _dp, _dp, _dp]),
    "tpmg_mlp_fit_scaling": (_ip, [_vp, _vp, _vp, ctypes.c_size_t]),
    "tpmg_mlp_features": (_ip, [_vp, _vp, _vp, _vp]),
    "tpmg_mlp_targets": (_ip, [_vp, _vp, _vp, _vp]),
    "tpmg_mlp_forward": (_ip, [_vp, _vp, _ip, _vp]),
    "tpmg_mlp_gradients": (_ip, [_vp, _vp, _vp, ctypes.c_size_t, _vp, _ip, _fp, _fp]),
    "tpmg_mlp_train_step": (_ip, [_vp, _vp, _vp, ctypes.c_size_t, _vp, _ip, ctypes.c_float, _fp]),
    "tpmg_mlp_train_epoch": (_ip, [_vp, _vp, _vp, ctypes.c_size_t, _vp, _ip, _ip, ctypes.c_float, _ip, _fp]),
    "tpmg_mlp_infer": (_ip, [_vp, _vp, _vp, _ip, _vp]),
    "tpmg_mlp_features_increment": (_ip, [_vp, _vp, _vp, _vp, _vp]),
    "tpmg_mlp_targets_increment": (_ip, [_vp, _vp, _vp, _vp, _vp]),
    "tpmg_mlp_infer_increment": (_ip, [_vp, _vp, _vp, _vp, _vp, _ip, _vp]),
    "tpmg_mlp_save": (_ip, [_vp, ctypes.c_char_p]),
    "tpmg_mlp_load": (_ip, [_vp, ctypes.c_char_p]),
    "tpmg_mlp_destroy": (None, [_vp]),
    "tpmg_grid_destroy": (None, [_vp]),
    "tpmg_op_destroy": (None, [_vp]),
    "tpmg_mg_destroy": (None, [_vp]),
    "tpmg_solve_noalloc": (_ip, [_vp, ctypes.POINTER(MgParams), _vp, _vp, _vp, ctypes.c_double, _ip,
                                 ctypes.POINTER(SolveInfo)]),
    "tpmg_status_string": (ctypes.c_char_p, [_ip]),
    "tpmg_last_error": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def status_string(s: int) -> str:
    return _lib.tpmg_status_string(s).decode()


def tpmg_last_error() -> str:
    return _lib.tpmg_last_error().decode()


def _check(s: int, ok=(TPMG_OK,)) -> int:
    if s not in ok:
        raise TpmgError(s, tpmg_last_error())
    return s


def _dptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _dev(t) -> int:
    return t.data_ptr() if hasattr(t, "data_ptr") else int(t)


# ---------------------------------------------------------------- host ----

def tpmg_grid_icosahedral(refinement: int, nz: int, r_faces) -> int:
    r = np.ascontiguousarray(r_faces, dtype=np.float64)
    if r.shape != (nz + 1,):
        raise ValueError("r_faces must hold nz + 1 values")
    h = _vp()
    _check(_lib.tpmg_grid_icosahedral(refinement, nz, _dptr(r), ctypes.byref(h)))
    return h.value


def tpmg_grid_level_size(grid: int, level: int) -> int:
    n = _ip()
    _check(_lib.tpmg_grid_level_size(grid, level, ctypes.byref(n)))
    return n.value


def tpmg_grid_geometry(grid: int, level: int) -> dict:
    n = tpmg_grid_level_size(grid, level)
    out = dict(centres=np.zeros((n, 3)), areas=np.zeros(n), nbr=np.zeros((n, 3), dtype=np.int32),
               edge_len=np.zeros((n, 3)), edge_factor=np.zeros((n, 3)))
    _check(_lib.tpmg_grid_geometry(grid, level, _dptr(out["centres"]), _dptr(out["areas"]),
                                   out["nbr"].ctypes.data_as(_i32p), _dptr(out["edge_len"]),
                                   _dptr(out["edge_factor"])))
    return out


def tpmg_grid_colouring(grid: int, level: int):
    """Returns (colours[n] int32, number of colours) of a grid level."""
    n = tpmg_grid_level_size(grid, level)
    c = np.zeros(n, dtype=np.int32)
    k = _ip()
    _check(_lib.tpmg_grid_colouring(grid, level, c.ctypes.data_as(_i32p), ctypes.byref(k)))
    return c, k.value


# tpmg_mg_params.smoother_order
SMOOTHER_ORDER_JACOBI, SMOOTHER_ORDER_SOR = 0, 1


def tpmg_grid_vertical(grid: int, nz: int) -> np.ndarray:
    v = np.zeros(nz)
    _check(_lib.tpmg_grid_vertical(grid, _dptr(v)))
    return v


def tpmg_op_create(grid: int, n_levels: int, omega2: float, alpha_r_v, alpha_s_v, beta_v,
                   alpha_r_h=None, alpha_s_h=None, beta_h=None) -> int:
    arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64)
            for a in (alpha_r_v, alpha_s_v, beta_v, alpha_r_h, alpha_s_h, beta_h)]
    h = _vp()
    _check(_lib.tpmg_op_create(grid, n_levels, float(omega2), *[_dptr(a) for a in arrs], ctypes.byref(h)))
    return h.value


def tpmg_op_create_levels(grid: int, n_levels: int, omega2: float, alpha_r_v, alpha_s_v, beta_v,
                          alpha_r_levels=None, alpha_s_levels=None, beta_levels=None) -> int:
    """*_levels: None or a sequence indexed by refinement level (refinement + 1
    entries) of None or per-cell factors of that grid."""
    vert = [np.ascontiguousarray(a, dtype=np.float64) for a in (alpha_r_v, alpha_s_v, beta_v)]
    keep = []

    def table(levels):
        if levels is None:
            return None
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in levels]
        keep.append(arrs)
        return (_dp * len(arrs))(*[_dptr(a) for a in arrs])

    tables = [table(x) for x in (alpha_r_levels, alpha_s_levels, beta_levels)]
    h = _vp()
    _check(_lib.tpmg_op_create_levels(grid, n_levels, float(omega2), *[_dptr(a) for a in vert], *tables,
                                      ctypes.byref(h)))
    return h.value


def tpmg_op_set_full_profiles(op: int, grid: int, alpha_r, alpha_s, beta, xi_r=None) -> None:
    arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in (alpha_r, alpha_s, beta, xi_r)]
    _check(_lib.tpmg_op_set_full_profiles(op, grid, *[_dptr(a) for a in arrs]))


def tpmg_op_coefficients_full(op: int, level: int, nz: int) -> dict:
    n = tpmg_op_level_size(op, level)
    out = dict(beta=np.zeros((n, nz)), alpha_s=np.zeros((n, 3, nz)), alpha_r=np.zeros((n, nz + 1)),
               adv_lo=np.zeros((n, nz)), adv_up=np.zeros((n, nz)))
    _check(_lib.tpmg_op_coefficients_full(op, level, *[_dptr(out[k]) for k in
                                                       ("beta", "alpha_s", "alpha_r", "adv_lo", "adv_up")]))
    return out


# tpmg_mg_params.precond_profiles: the V-cycle of an operator with full profiles
PRECOND_FULL, PRECOND_FACTORISED, PRECOND_PARTIAL = 0, 1, 2


def tpmg_op_levels(op: int) -> int:
    n = _ip()
    _check(_lib.tpmg_op_levels(op, ctypes.byref(n)))
    return n.value


def tpmg_op_level_size(op: int, level: int) -> int:
    n = _ip()
    _check(_lib.tpmg_op_level_size(op, level, ctypes.byref(n)))
    return n.value


def tpmg_op_coefficients(op: int, level: int, nz: int) -> dict:
    n = tpmg_op_level_size(op, level)
    out = dict(beta_h=np.zeros(n), alpha_r_h=np.zeros(n), alpha_s_h=np.zeros((n, 3)), beta_v=np.zeros(nz),
               alpha_s_v=np.zeros(nz), alpha_r_v=np.zeros(nz + 1))
    _check(_lib.tpmg_op_coefficients(op, level, *[_dptr(out[k]) for k in
                                                  ("beta_h", "alpha_r_h", "alpha_s_h", "beta_v", "alpha_s_v", "alpha_r_v")]))
    return out


def tpmg_op_prolongation(op: int, level: int) -> np.ndarray:
    n = tpmg_op_level_size(op, level)
    w = np.zeros((n, 3))
    _check(_lib.tpmg_op_prolongation(op, level, _dptr(w)))
    return w


def tpmg_mg_params_default() -> MgParams:
    p = MgParams()
    _lib.tpmg_mg_params_default(ctypes.byref(p))
    return p


# -------------------------------------------------------------- device ----

def tpmg_mg_workspace_size(op: int, params: MgParams) -> int:
    b = ctypes.c_size_t()
    _check(_lib.tpmg_mg_workspace_size(op, ctypes.byref(params), ctypes.byref(b)))
    return b.value


def tpmg_mg_setup(op: int, params: MgParams, workspace, nbytes: int, stream) -> int:
    h = _vp()
    st = stream if isinstance(stream, int) or stream is None else stream.cuda_stream
    _check(_lib.tpmg_mg_setup(op, ctypes.byref(params), _dev(workspace), nbytes, st, ctypes.byref(h)))
    return h.value


def tpmg_mg_vector_length(mg: int):
    n = ctypes.c_size_t()
    c = _ip()
    z = _ip()
    _check(_lib.tpmg_mg_vector_length(mg, ctypes.byref(n), ctypes.byref(c), ctypes.byref(z)))
    return n.value, c.value, z.value


def tpmg_pack(mg: int, d_cellmajor, d_tiled):
    _check(_lib.tpmg_pack(mg, _dev(d_cellmajor), _dev(d_tiled)))


def tpmg_unpack(mg: int, d_tiled, d_cellmajor):
    _check(_lib.tpmg_unpack(mg, _dev(d_tiled), _dev(d_cellmajor)))


def tpmg_spmv(mg: int, d_x, d_y):
    _check(_lib.tpmg_spmv(mg, _dev(d_x), _dev(d_y)))


def tpmg_vcycle(mg: int, d_r, d_z):
    _check(_lib.tpmg_vcycle(mg, _dev(d_r), _dev(d_z)))


def tpmg_relax(mg: int, d_f, d_u_in, d_u_out):
    _check(_lib.tpmg_relax(mg, _dev(d_f), _dev(d_u_in), _dev(d_u_out)))


def tpmg_solve(mg: int, d_f, d_u, rtol: float, maxit: int, history_cap: int = 256):
    """Returns (status, iters, relres, history, t_total_ms)."""
    info = tpmg_solve_details(mg, d_f, d_u, rtol, maxit, history_cap)
    return info["status"], info["iters"], info["relres"], info["history"], info["t_total_ms"]


def tpmg_solve_details(mg: int, d_f, d_u, rtol: float, maxit: int, history_cap: int = 256, phase_timers: bool = False,
                    div_tol: float = 0.0) -> dict:
    """tpmg_solve with every field of tpmg_solve_info returned in a dict
    (status, iters, relres, history, t_total_ms, t_vcycle_ms, t_spmv_ms,
    t_blas_ms, model_bytes) and the message of a breakdown."""
    hist = np.zeros(history_cap)
    info = SolveInfo()
    info.history = hist.ctypes.data_as(_dp)
    info.history_cap = history_cap
    info.phase_timers = int(phase_timers)
    info.div_tol = float(div_tol)
    s = _lib.tpmg_solve(mg, _dev(d_f), _dev(d_u), float(rtol), int(maxit), ctypes.byref(info))
    _check(s, ok=(TPMG_OK, TPMG_NOT_CONVERGED, TPMG_ERR_BREAKDOWN))
    return dict(status=s, iters=info.iters, relres=info.relres, history=hist[: info.iters + 1].copy(),
                t_total_ms=info.t_total_ms, t_vcycle_ms=info.t_vcycle_ms, t_spmv_ms=info.t_spmv_ms,
                t_blas_ms=info.t_blas_ms, model_bytes=info.model_bytes,
                message=tpmg_last_error() if s == TPMG_ERR_BREAKDOWN else "")


def _solve_with(fn, mg: int, d_f, d_u, rtol: float, maxit: int, history_cap: int) -> dict:
    hist = np.zeros(history_cap)
    info = SolveInfo()
    info.history = hist.ctypes.data_as(_dp)
    info.history_cap = history_cap
    s = fn(mg, _dev(d_f), _dev(d_u), float(rtol), int(maxit), ctypes.byref(info))
    _check(s, ok=(TPMG_OK, TPMG_NOT_CONVERGED, TPMG_ERR_BREAKDOWN))
    return dict(status=s, iters=info.iters, relres=info.relres, history=hist[: info.iters + 1].copy(),
                t_total_ms=info.t_total_ms, model_bytes=info.model_bytes,
                message=tpmg_last_error() if s == TPMG_ERR_BREAKDOWN else "")


def tpmg_solve_richardson(mg: int, d_f, d_u, rtol: float, maxit: int, history_cap: int = 256) -> dict:
    """Preconditioned Richardson; returns the fields of tpmg_solve_details."""
    return _solve_with(_lib.tpmg_solve_richardson, mg, d_f, d_u, rtol, maxit, history_cap)


def tpmg_solve_bicgstab(mg: int, d_f, d_u, rtol: float, maxit: int, history_cap: int = 256) -> dict:
    """Preconditioned BiCGStab; returns the fields of tpmg_solve_details."""
    return _solve_with(_lib.tpmg_solve_bicgstab, mg, d_f, d_u, rtol, maxit, history_cap)


NOALLOC_SCRATCH_BYTES = 256 << 20


def tpmg_solve_noalloc(op: int, params: MgParams, stream, d_f, d_u, rtol: float, maxit: int,
                       history_cap: int = 256) -> dict:
    """The allocation-free solve (setup, solve and teardown in one call on the
    library's static scratch); returns the fields of tpmg_solve_details."""
    hist = np.zeros(history_cap)
    info = SolveInfo()
    info.history = hist.ctypes.data_as(_dp)
    info.history_cap = history_cap
    st = stream if isinstance(stream, int) or stream is None else stream.cuda_stream
    s = _lib.tpmg_solve_noalloc(op, ctypes.byref(params), st, _dev(d_f), _dev(d_u), float(rtol), int(maxit),
                                ctypes.byref(info))
    _check(s, ok=(TPMG_OK, TPMG_NOT_CONVERGED, TPMG_ERR_BREAKDOWN))
    return dict(status=s, iters=info.iters, relres=info.relres, history=hist[: info.iters + 1].copy(),
                t_total_ms=info.t_total_ms, model_bytes=info.model_bytes,
                message=tpmg_last_error() if s == TPMG_ERR_BREAKDOWN else "")


def _ptrs(handles):
    return (_vp * len(handles))(*[_dev(h) for h in handles])


def tpmg_batch_workspace_size(mgs) -> int:
    b = ctypes.c_size_t()
    _check(_lib.tpmg_batch_workspace_size(_ptrs(mgs), len(mgs), ctypes.byref(b)))
    return b.value


def tpmg_batch_create(mgs, workspace, nbytes: int) -> int:
    h = _vp()
    _check(_lib.tpmg_batch_create(_ptrs(mgs), len(mgs), _dev(workspace), nbytes, ctypes.byref(h)))
    return h.value


def tpmg_batch_solve(batch: int, fs, us, rtol: float, maxit: int, history_cap: int = 256):
    """Returns (status, [(iters, relres, history)], t_total_ms)."""
    n = len(fs)
    hists = [np.zeros(history_cap) for _ in range(n)]
    infos = (SolveInfo * n)()
    for i in range(n):
        infos[i].history = hists[i].ctypes.data_as(_dp)
        infos[i].history_cap = history_cap
    s = _lib.tpmg_batch_solve(batch, _ptrs(fs), _ptrs(us), float(rtol), int(maxit), infos)
    _check(s, ok=(TPMG_OK, TPMG_NOT_CONVERGED, TPMG_ERR_BREAKDOWN))
    per = [(infos[i].iters, infos[i].relres, hists[i][: infos[i].iters + 1].copy()) for i in range(n)]
    return s, per, infos[0].t_total_ms if n else 0.0


def tpmg_batch_destroy(h):
    _lib.tpmg_batch_destroy(h)


def tpmg_richardson_rate(mg: int, d_u, cycles: int = 12, skip: int = 4):
    """Returns (rate, norms[cycles + 1]); d_u is overwritten."""
    rate = ctypes.c_double()
    norms = np.zeros(cycles + 1)
    _check(_lib.tpmg_richardson_rate(mg, _dev(d_u), cycles, skip, ctypes.byref(rate), _dptr(norms)))
    return rate.value, norms


def tpmg_mg_time_sweep(mg: int, reps: int):
    """Returns (avg_ms, model_bytes) of one finest-grid smoother sweep."""
    ms = ctypes.c_double()
    b = ctypes.c_double()
    _check(_lib.tpmg_mg_time_sweep(mg, reps, ctypes.byref(ms), ctypes.byref(b)))
    return ms.value, b.value


# kernels of tpmg_mg_time_kernel
KERNEL_SWEEP, KERNEL_OPERATOR_PRING, KERNEL_OPERATOR, KERNEL_RESTRICT, KERNEL_PROLONG = range(5)


def tpmg_mg_time_kernel(mg: int, kernel: int, reps: int):
    """Returns (avg_ms, model_bytes) of one launch of a finest-grid kernel."""
    ms = ctypes.c_double()
    b = ctypes.c_double()
    _check(_lib.tpmg_mg_time_kernel(mg, kernel, reps, ctypes.byref(ms), ctypes.byref(b)))
    return ms.value, b.value


def tpmg_mg_tuning(mg: int, level: int) -> dict:
    """Launch configuration of a level: smoother kind, scan levels per wave
    and the stencil chunks (0 where a kernel does not run on the level)."""
    v = [ctypes.c_int() for _ in range(5)]
    _check(_lib.tpmg_mg_tuning(mg, level, *[ctypes.byref(x) for x in v]))
    keys = ("smoother", "scan_levels", "chunk_restrict", "chunk_prolong", "chunk_spmv")
    return {k: x.value for k, x in zip(keys, v)}


def tpmg_mg_autotune_stats(mg: int):
    """Returns (timed trials, their device milliseconds) of mg's setup."""
    n = ctypes.c_int()
    ms = ctypes.c_double()
    _check(_lib.tpmg_mg_autotune_stats(mg, ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def tpmg_tune_load(path: str) -> None:
    _check(_lib.tpmg_tune_load(os.fsencode(path)))


def tpmg_tune_save(path: str) -> None:
    _check(_lib.tpmg_tune_save(os.fsencode(path)))


def tpmg_tune_clear() -> None:
    _check(_lib.tpmg_tune_clear())


def tpmg_tune_entries() -> int:
    n = ctypes.c_int()
    _check(_lib.tpmg_tune_entries(ctypes.byref(n)))
    return n.value


def tpmg_grid_destroy(h):
    _lib.tpmg_grid_destroy(h)


def tpmg_op_destroy(h):
    _lib.tpmg_op_destroy(h)


def tpmg_mg_destroy(h):
    _lib.tpmg_mg_destroy(h)


# ------------------------------------------------------ learned guess ----

def tpmg_mlp_param_count(nz: int, hidden: int) -> int:
    n = ctypes.c_size_t()
    _check(_lib.tpmg_mlp_param_count(nz, hidden, ctypes.byref(n)))
    return n.value


def tpmg_mlp_workspace_size(nz: int, hidden: int, max_rows: int) -> int:
    n = ctypes.c_size_t()
    _check(_lib.tpmg_mlp_workspace_size(nz, hidden, max_rows, ctypes.byref(n)))
    return n.value


def tpmg_mlp_create(nz: int, hidden: int, max_rows: int, workspace, nbytes: int, stream) -> int:
    h = _vp()
    s = stream.cuda_stream if hasattr(stream, "cuda_stream") else stream
    _check(_lib.tpmg_mlp_create(nz, hidden, max_rows, _dev(workspace), nbytes, s, ctypes.byref(h)))
    return h.value


def _fptr(a):
    assert a.dtype == np.float32 and a.flags.c_contiguous
    return a.ctypes.data_as(_fp)


def tpmg_mlp_set_params(m: int, params) -> None:
    p = np.ascontiguousarray(params, dtype=np.float32)
    _check(_lib.tpmg_mlp_set_params(m, _fptr(p)))


def tpmg_mlp_get_params(m: int, n: int) -> np.ndarray:
    p = np.zeros(n, dtype=np.float32)
    _check(_lib.tpmg_mlp_get_params(m, _fptr(p)))
    return p


def tpmg_mlp_set_scaling(m: int, mu_x, sd_x, mu_y, sd_y) -> None:
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (mu_x, sd_x, mu_y, sd_y)]
    _check(_lib.tpmg_mlp_set_scaling(m, *[_dptr(a) for a in arrs]))


def tpmg_mlp_get_scaling(m: int, n_in: int, nz: int):
    out = [np.zeros(n_in), np.zeros(n_in), np.zeros(nz), np.zeros(nz)]
    _check(_lib.tpmg_mlp_get_scaling(m, *[_dptr(a) for a in out]))
    return out


def tpmg_mlp_fit_scaling(m: int, d_x, d_y, rows: int) -> None:
    _check(_lib.tpmg_mlp_fit_scaling(m, _dev(d_x), _dev(d_y), rows))


def tpmg_mlp_features(m: int, mg: int, d_f, d_x) -> None:
    _check(_lib.tpmg_mlp_features(m, mg, _dev(d_f), _dev(d_x)))


def tpmg_mlp_targets(m: int, mg: int, d_u, d_y) -> None:
    _check(_lib.tpmg_mlp_targets(m, mg, _dev(d_u), _dev(d_y)))


def tpmg_mlp_forward(m: int, d_x, rows: int, d_y) -> None:
    _check(_lib.tpmg_mlp_forward(m, _dev(d_x), rows, _dev(d_y)))


def tpmg_mlp_gradients(m: int, d_x, d_y, rows_total: int, d_rows, batch: int, n_params: int):
    """Returns (loss, grads[n_params]) of the batch; synchronous."""
    loss = ctypes.c_float()
    g = np.zeros(n_params, dtype=np.float32)
    _check(_lib.tpmg_mlp_gradients(m, _dev(d_x), _dev(d_y), rows_total, _dev(d_rows), batch, ctypes.byref(loss),
                                   _fptr(g)))
    return loss.value, g


def tpmg_mlp_train_step(m: int, d_x, d_y, rows_total: int, d_rows, batch: int, lr: float, want_loss: bool = False):
    loss = ctypes.c_float()
    _check(_lib.tpmg_mlp_train_step(m, _dev(d_x), _dev(d_y), rows_total, _dev(d_rows), batch, lr,
                                    ctypes.byref(loss) if want_loss else None))
    return loss.value if want_loss else None


def tpmg_mlp_train_epoch(m: int, d_x, d_y, rows_total: int, d_perm, steps: int, batch: int, lr: float,
                         loss_every: int = 0) -> np.ndarray:
    n = (steps - 1) // loss_every + 2 if loss_every > 0 else 0
    losses = np.zeros(max(n, 1), dtype=np.float32)
    ptr = losses.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if loss_every > 0 else None
    _check(_lib.tpmg_mlp_train_epoch(m, _dev(d_x), _dev(d_y), rows_total, _dev(d_perm), steps, batch, lr, loss_every,
                                     ptr))
    k = len(range(0, steps, loss_every)) + (1 if (steps - 1) % loss_every else 0) if loss_every > 0 else 0
    return losses[:k]


def tpmg_mlp_infer(m: int, mg: int, d_f, d_u0, relax: int = 1) -> None:
    _check(_lib.tpmg_mlp_infer(m, mg, _dev(d_f), relax, _dev(d_u0)))


def tpmg_mlp_features_increment(m: int, mg: int, d_f, d_f_prev, d_x) -> None:
    _check(_lib.tpmg_mlp_features_increment(m, mg, _dev(d_f), _dev(d_f_prev), _dev(d_x)))


def tpmg_mlp_targets_increment(m: int, mg: int, d_u, d_u_prev, d_y) -> None:
    _check(_lib.tpmg_mlp_targets_increment(m, mg, _dev(d_u), _dev(d_u_prev), _dev(d_y)))


def tpmg_mlp_infer_increment(m: int, mg: int, d_f, d_f_prev, d_u_prev, d_u0, relax: int = 1) -> None:
    _check(_lib.tpmg_mlp_infer_increment(m, mg, _dev(d_f), _dev(d_f_prev), _dev(d_u_prev), relax, _dev(d_u0)))


def tpmg_mlp_save(m: int, path: str) -> None:
    _check(_lib.tpmg_mlp_save(m, os.fsencode(path)))


def tpmg_mlp_load(m: int, path: str) -> None:
    _check(_lib.tpmg_mlp_load(m, os.fsencode(path)))


def tpmg_mlp_destroy(m: int) -> None:
    _lib.tpmg_mlp_destroy(m)


from .solver import Problem  # noqa: E402  (convenience wrapper over the calls above)
from .learned_guess import ColumnMLP  # noqa: E402
