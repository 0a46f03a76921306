"""Finite-volume operator of the pressure-correction equation (oracle).

The operator is L u = -omega^2 div(alpha grad u) + beta u on the shell
S x [1, 1+H] without the advection term (Section 3.2.1), discretised with
cell-centred finite volumes (Appendix A). For cell E = (T, k):

  (A u)_{T,k} = beta^_{T,k} u_{T,k}
              + sum_{T'} alphaS^_{TT',k} (u_{T,k} - u_{T',k})
              + alphar^_{T,k+1} (u_{T,k} - u_{T,k+1})
              + alphar^_{T,k}   (u_{T,k} - u_{T,k-1})

with the coefficients of Appendix A (eq. hatFunctionsNonFac):
  beta^_{T,k}      = |T| v_k beta_{T,k},   v_k = (r_{k+1}^3 - r_k^3)/3
  alphaS^_{TT',k}  = omega^2 (r_{k+1}-r_k) |S_TT'| n.(r_T'-r_T)/|r_T'-r_T|^2 alpha_S
  alphar^_{T,k}    = omega^2 sigma_k |T| 2 r_k^2 / (r_{k+1}-r_{k-1}) alpha_r
and sigma_0 = sigma_nz = 0 (homogeneous Neumann top and bottom).

This is the block form of eq. ColumnEquation: A_T is tridiagonal (vertical
couplings alphar^), A_TT' diagonal (horizontal couplings alphaS^). It is
written in flux form (sum of couplings times differences) rather than as a
diagonal minus off-diagonals; the two are equal in exact arithmetic, and the
flux form keeps the small column excess beta^ + sum alphaS^ exact when the
vertical couplings are many orders of magnitude larger.

Readings: v_k is evaluated as (r_{k+1}-r_k)(r_{k+1}^2 + r_{k+1} r_k + r_k^2)/3,
the same number without the cancellation of the cubic difference; the
horizontal profile factor on an edge is the mean of the two cells' values;
on coarse grids the horizontal factors are area-weighted means of the four
children and the operator is rediscretised on the coarse geometry.

Pins (tests/test_oracle_operator.py): exact symmetry and positive
definiteness of the assembled matrix, matrix-free apply == explicit sparse
matrix, A 1 = beta^, second-order decay of the error for manufactured
solutions, agreement with a direct sparse solve.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .mesh import Mesh


@dataclass
class Vertical:
    r: np.ndarray            # [nz+1] faces
    vk: np.ndarray           # [nz]  (r_{k+1}^3 - r_k^3)/3
    dr: np.ndarray           # [nz]  r_{k+1} - r_k
    face_factor: np.ndarray  # [nz+1] sigma_k 2 r_k^2 / (r_{k+1} - r_{k-1})
    # vertical advection of cell k through its lower and upper face
    # (Appendix A): sigma_k r_k^2 (r_{k+1}-r_k)/(r_{k+1}-r_{k-1}) and
    # sigma_{k+1} r_{k+1}^2 (r_{k+1}-r_k)/(r_{k+2}-r_k), [nz] each
    adv_lo_factor: np.ndarray | None = None
    adv_up_factor: np.ndarray | None = None

    @property
    def nz(self) -> int:
        return len(self.vk)


def vertical(r: np.ndarray) -> Vertical:
    r = np.asarray(r, dtype=np.float64)
    nz = len(r) - 1
    lo, hi = r[:-1], r[1:]
    dr = hi - lo
    vk = dr * (hi * hi + hi * lo + lo * lo) / 3.0
    ff = np.zeros(nz + 1)
    for k in range(1, nz):
        ff[k] = 2.0 * r[k] * r[k] / (r[k + 1] - r[k - 1])
    lo = np.zeros(nz)
    up = np.zeros(nz)
    for k in range(nz):
        if k > 0:
            lo[k] = r[k] * r[k] * (r[k + 1] - r[k]) / (r[k + 1] - r[k - 1])
        if k + 1 < nz:
            up[k] = r[k + 1] * r[k + 1] * (r[k + 1] - r[k]) / (r[k + 2] - r[k])
    return Vertical(r, vk, dr, ff, lo, up)


@dataclass
class LevelOperator:
    """Coefficients of one grid level, all of shape [n, nz] / [n, 3, nz] / [n, nz+1]."""

    nbr: np.ndarray
    beta: np.ndarray      # beta^_{T,k}
    alpha_s: np.ndarray   # alphaS^_{T,j,k}, coupling to nbr[T, j]
    alpha_r: np.ndarray   # alphar^_{T,k} on radial face k (0 and nz are zero)
    # vertical advection (None: absent): omega^2 times the coefficients of
    # the cell's lower and upper face, [n, nz]
    adv_lo: np.ndarray | None = None
    adv_up: np.ndarray | None = None

    @property
    def n(self) -> int:
        return self.beta.shape[0]

    @property
    def nz(self) -> int:
        return self.beta.shape[1]

    def astype(self, dtype) -> "LevelOperator":
        cast = (lambda a: None if a is None else a.astype(dtype))
        return LevelOperator(self.nbr, self.beta.astype(dtype), self.alpha_s.astype(dtype), self.alpha_r.astype(dtype),
                             cast(self.adv_lo), cast(self.adv_up))


def assemble(mesh: Mesh, vert: Vertical, omega2: float, alpha_r_v, alpha_s_v, beta_v,
             alpha_r_h, alpha_s_h, beta_h) -> LevelOperator:
    """Coefficients from point samples of factorised profiles.

    alpha_r_v [nz+1] at the faces, alpha_s_v, beta_v [nz] at the layer
    midpoints; alpha_r_h, alpha_s_h, beta_h [n] per horizontal cell of this
    mesh. The full profile value is the product of the two factors.
    """
    n, nz = mesh.n, vert.nz
    alpha_r = alpha_r_h[:, None] * np.asarray(alpha_r_v)[None, :]             # [n, nz+1]
    beta = beta_h[:, None] * np.asarray(beta_v)[None, :]                      # [n, nz]
    edge_h = 0.5 * (alpha_s_h[:, None] + alpha_s_h[mesh.nbr])               # [n, 3]
    alpha_s = edge_h[:, :, None] * np.asarray(alpha_s_v)[None, None, :]       # [n, 3, nz]

    beta_hat = mesh.area[:, None] * vert.vk[None, :] * beta
    alpha_s_hat = omega2 * vert.dr[None, None, :] * mesh.g[:, :, None] * alpha_s
    alpha_r_hat = omega2 * vert.face_factor[None, :] * mesh.area[:, None] * alpha_r
    assert beta_hat.shape == (n, nz) and alpha_r_hat.shape == (n, nz + 1)
    return LevelOperator(mesh.nbr, beta_hat, alpha_s_hat, alpha_r_hat)


def restrict_cell_factor(fine_values: np.ndarray, fine_area: np.ndarray) -> np.ndarray:
    """Area-weighted mean of the four children 4P..4P+3."""
    w = (fine_values * fine_area).reshape(-1, 4).sum(axis=1)
    return w / fine_area.reshape(-1, 4).sum(axis=1)


@dataclass
class FullProfiles:
    """Point samples of profiles that need not factorise (Section 4.2: the
    non-factorising case; Appendix A, eq. hatFunctionsNonFac), one value per
    cell and level of a grid, cell-major:
      alpha_r [n, nz+1] at the radial faces (r_k, centre of T),
      alpha_s [n, nz]   at the layer midpoints (r_{k+1/2}, centre of T),
      beta    [n, nz]   at the layer midpoints (r_{k+1/2}, centre of T),
      xi_r    [n, nz+1] at the radial faces, or None (no vertical advection)."""

    alpha_r: np.ndarray
    alpha_s: np.ndarray
    beta: np.ndarray
    xi_r: np.ndarray | None = None


def restrict_cell_profile(fine_values: np.ndarray, fine_area: np.ndarray) -> np.ndarray:
    """Area-weighted mean of the four children 4P..4P+3 of every column
    entry of a per-cell profile [n, m] (the coarse-grid reading of the
    factorised case, applied level by level)."""
    n, m = fine_values.shape
    w = (fine_values * fine_area[:, None]).reshape(n // 4, 4, m).sum(axis=1)
    return w / fine_area.reshape(-1, 4).sum(axis=1)[:, None]


def assemble_full(mesh: Mesh, vert: Vertical, omega2: float, alpha_r: np.ndarray, alpha_s: np.ndarray,
                  beta: np.ndarray, xi_r: np.ndarray | None = None) -> LevelOperator:
    """Coefficients of eq. hatFunctionsNonFac from point samples of profiles
    that need not factorise (FullProfiles layout on this mesh). As in the
    factorised case, the horizontal profile on an edge is the mean of its two
    cells' values (here level by level).

    Vertical advection (xi_r given, Appendix A "Vertical advection"): the
    cell integral of xi_r d_r u over cell k is taken as the appendix writes
    it, |T| (r_{k+1}-r_k) times the mean of the two face terms
    r_f^2 xi_{T,f} (u across face f) / (centre distance across f), f = k,
    k+1; the operator term is -omega^2 times it:
      -omega^2 adv_k = adv_up_k (u_k - u_{k+1}) - adv_lo_k (u_k - u_{k-1}),
      adv_lo_k = omega^2 sigma_k |T| r_k^2 (r_{k+1}-r_k)/(r_{k+1}-r_{k-1}) xi_{T,k},
      adv_up_k = omega^2 sigma_{k+1} |T| r_{k+1}^2 (r_{k+1}-r_k)/(r_{k+2}-r_k) xi_{T,k+1}."""
    n, nz = mesh.n, vert.nz
    assert alpha_r.shape == (n, nz + 1) and alpha_s.shape == (n, nz) and beta.shape == (n, nz)
    edge = 0.5 * (alpha_s[:, None, :] + alpha_s[mesh.nbr])                    # [n, 3, nz]
    beta_hat = mesh.area[:, None] * vert.vk[None, :] * beta
    alpha_s_hat = omega2 * vert.dr[None, None, :] * mesh.g[:, :, None] * edge
    alpha_r_hat = omega2 * vert.face_factor[None, :] * mesh.area[:, None] * alpha_r
    adv_lo = adv_up = None
    if xi_r is not None:
        assert xi_r.shape == (n, nz + 1)
        adv_lo = omega2 * mesh.area[:, None] * vert.adv_lo_factor[None, :] * xi_r[:, :-1]
        adv_up = omega2 * mesh.area[:, None] * vert.adv_up_factor[None, :] * xi_r[:, 1:]
    return LevelOperator(mesh.nbr, beta_hat, alpha_s_hat, alpha_r_hat, adv_lo, adv_up)


def apply(op: LevelOperator, u: np.ndarray) -> np.ndarray:
    """y = A u in flux form; u is [n, nz] (cell-major)."""
    y = op.beta * u
    for j in range(3):
        y = y + op.alpha_s[:, j, :] * (u - u[op.nbr[:, j], :])
    flux = op.alpha_r[:, 1:-1] * (u[:, :-1] - u[:, 1:])   # face k = 1..nz-1
    y[:, :-1] += flux
    y[:, 1:] -= flux
    if op.adv_lo is not None:
        d = u[:, :-1] - u[:, 1:]                           # u_k - u_{k+1} across face k+1
        y[:, :-1] += op.adv_up[:, :-1] * d
        y[:, 1:] += op.adv_lo[:, 1:] * d                   # -adv_lo (u_k - u_{k-1})
    return y


def column_bands(op: LevelOperator):
    """The tridiagonal blocks A_T of eq. TridiagonalSystem in margin form.

    Row k of A_T: diagonal e_k + l_k + m_k, sub-diagonal -l_k, super-diagonal
    -m_k, where l_k = alphar^_{T,k} (face below), m_k = alphar^_{T,k+1} (face
    above) and the excess e_k = beta^_{T,k} + sum_T' alphaS^_{TT',k}.
    """
    l = op.alpha_r[:, :-1]
    m = op.alpha_r[:, 1:]
    if op.adv_lo is not None:
        # vertical advection: the couplings differ below and above
        l = l - op.adv_lo
        m = m + op.adv_up
    e = op.beta + op.alpha_s.sum(axis=1)
    return l, m, e


def to_sparse(op: LevelOperator) -> sp.csr_matrix:
    """Explicit sparse matrix, cell-major index T*nz + k."""
    n, nz = op.n, op.nz
    idx = np.arange(n * nz).reshape(n, nz)
    rows, cols, vals = [], [], []
    l, m, e = column_bands(op)
    diag = e + l + m
    rows.append(idx.ravel()); cols.append(idx.ravel()); vals.append(diag.ravel())
    for j in range(3):
        rows.append(idx.ravel()); cols.append(idx[op.nbr[:, j], :].ravel()); vals.append(-op.alpha_s[:, j, :].ravel())
    rows.append(idx[:, 1:].ravel()); cols.append(idx[:, :-1].ravel()); vals.append(-l[:, 1:].ravel())
    rows.append(idx[:, :-1].ravel()); cols.append(idx[:, 1:].ravel()); vals.append(-m[:, :-1].ravel())
    a = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n * nz, n * nz))
    return a.tocsr()
