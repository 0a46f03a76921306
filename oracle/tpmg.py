"""Tensor-product multigrid preconditioned flexible CG (oracle).

Paper: Section 3 (Algorithm 1, the TPMG V-cycle: pre-smoothing, residual,
restriction, recursion from a zero guess, coarse-grid correction,
post-smoothing), Section 4.1 (eq. BlockJacobi: vertical line relaxation with
a tridiagonal solve per column by the Thomas algorithm), Section 5 (nu_pre =
nu_post = 2, one smoother step on the coarsest grid, restriction of the
cell-integral residual by summing the four children, linear interpolation
for the prolongation, 4 - 7 levels).

Readings (where the paper is silent or its implementation and theory differ):
  * smoother: damped block-Jacobi with omega_J = 2/3 (the theory's weighted
    block-Jacobi, Section 3.2.1) rather than sequential block-SOR, so the
    sweep is order independent;
  * Thomas algorithm tracked through the diagonal-dominance margin
    s_k = p_k - m_k (p_k the pivot), so every addition is of positive terms;
  * prolongation: least-squares linear reconstruction in the tangent plane
    at the parent centre from the parent and its three neighbours, the same
    gradient for all four children;
  * coarsest grid: one damped sweep from a zero guess;
  * outer solver: flexible CG with one-term orthogonalisation,
    alpha = <r,z>/<p,q>, beta = -<z',q>/<p,q>, stopping when
    ||r||_2 <= rtol ||f||_2 (the operator is SPD without advection,
    Section 3.2.1);
  * V-cycle rate: Richardson u <- u + M(f - A u) with f = 0, 12 cycles from
    seeded U[-1,1], rate (||r_12|| / ||r_4||)^(1/8).

Pins (tests/test_oracle_tpmg.py): Thomas vs dense LU; the smoother vs dense
block inverses; conservation of the restriction; exactness of the
prolongation on constants and O(h^2) on linear fields; the tensor-decoupling
of the V-cycle spectrum (Section 3.2.1, eq. EigenvalueEquation); a V-cycle
rate bounded in h and anisotropy; FCG == textbook CG (scipy) for M = I,
one step for M = A^-1, == PCG (scipy) for a symmetric M; the solve ==
scipy.sparse.linalg.spsolve; the V-cycle of Algorithm 1 == its dense
composition from explicit matrices; the FP32 V-cycle (make_preconditioner)
a float32 rounding of the FP64 one; the block-SOR sweep == the dense block
SOR formula in colour order; Richardson and BiCGStab against their
definitions (tests/test_oracle_sor.py, tests/test_oracle_advection.py).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse.linalg as spla

from . import mesh as mesh_mod
from . import operator as opmod


# ---------------------------------------------------------------------------
# column (Thomas) solve and the line smoother
# ---------------------------------------------------------------------------


def thomas_margin(l: np.ndarray, m: np.ndarray, e: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Solve A_T x = b for every column at once.

    Row k of A_T: (e_k + l_k + m_k) x_k - l_k x_{k-1} - m_k x_{k+1} = b_k,
    with l_0 = m_{nz-1} = 0 and e_k > 0 (arrays [n, nz]). Forward
    elimination keeps the margin s_k = pivot_k - m_k:
      s_0 = e_0,  s_k = e_k + l_k s_{k-1} / p_{k-1},  p_k = s_k + m_k,
      d_k = (b_k + l_k d_{k-1}) / p_k;
    back substitution x_{nz-1} = d_{nz-1}, x_k = d_k + (m_k / p_k) x_{k+1}.
    """
    n, nz = b.shape
    p = np.empty_like(b)
    d = np.empty_like(b)
    s = e[:, 0]
    p[:, 0] = s + m[:, 0]
    d[:, 0] = b[:, 0] / p[:, 0]
    for k in range(1, nz):
        s = e[:, k] + l[:, k] * s / p[:, k - 1]
        p[:, k] = s + m[:, k]
        d[:, k] = (b[:, k] + l[:, k] * d[:, k - 1]) / p[:, k]
    x = np.empty_like(b)
    x[:, nz - 1] = d[:, nz - 1]
    for k in range(nz - 2, -1, -1):
        x[:, k] = d[:, k] + (m[:, k] / p[:, k]) * x[:, k + 1]
    return x


def smooth(op: opmod.LevelOperator, f: np.ndarray, u: np.ndarray, omega: float) -> np.ndarray:
    """One damped block-Jacobi sweep u + omega A_T^-1 (f - A u)_T (eq. BlockJacobi)."""
    l, m, e = opmod.column_bands(op)
    r = f - opmod.apply(op, u)
    return u + omega * thomas_margin(l, m, e, r)


def greedy_colouring(nbr: np.ndarray) -> np.ndarray:
    """Colours of the cells such that neighbours differ: cells in index
    order, each taking the smallest colour none of its already coloured
    neighbours has (at most 4 colours on a graph of degree 3)."""
    n = len(nbr)
    col = np.full(n, -1, dtype=np.int64)
    for t in range(n):
        used = {int(col[j]) for j in nbr[t] if col[j] >= 0}
        c = 0
        while c in used:
            c += 1
        col[t] = c
    return col


def smooth_sor(op: opmod.LevelOperator, f: np.ndarray, u: np.ndarray, omega: float, colours: np.ndarray,
               reverse: bool = False) -> np.ndarray:
    """One multicolour block-SOR sweep (eq. BlockJacobi with the cells of one
    colour relaxed at a time, each colour seeing the updates of the colours
    before it): for c in colour order, u_T += omega A_T^-1 (f - A u)_T for
    every cell T of colour c. reverse: colours in descending order."""
    l, m, e = opmod.column_bands(op)
    order = range(int(colours.max()) + 1)
    for c in (reversed(order) if reverse else order):
        sel = colours == c
        r = f - opmod.apply(op, u)
        u = u.copy()
        u[sel] += omega * thomas_margin(l[sel], m[sel], e[sel], r[sel])
    return u


# ---------------------------------------------------------------------------
# grid transfers
# ---------------------------------------------------------------------------


def restrict(r_fine: np.ndarray) -> np.ndarray:
    """Sum of the four children 4P..4P+3 (cell integrals, Section 5)."""
    n, nz = r_fine.shape
    return r_fine.reshape(n // 4, 4, nz).sum(axis=1)


def prolongation_weights(coarse: mesh_mod.Mesh, fine: mesh_mod.Mesh) -> np.ndarray:
    """w[c, j] with e_c = e_P + sum_j w[c, j] (e_{N_j(P)} - e_P), P = c // 4.

    Least-squares gradient G in the tangent plane at r_P from the offsets
    d_j = Pi(r_{N_j} - r_P): G = argmin sum_j (d_j . G - (e_{N_j} - e_P))^2,
    then e_c = e_P + G . delta_c with delta_c = Pi(r_c - r_P), Pi the
    tangent-plane projection. Written in 2-D coordinates of the plane.
    """
    rp = coarse.centre                                        # [nc, 3]
    nc = len(rp)

    def proj(v):
        return v - np.sum(v * rp, axis=-1, keepdims=True) * rp

    # an orthonormal tangent basis (t1, t2) at each parent centre
    helper = np.where(np.abs(rp[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]))
    t1 = proj(helper)
    t1 = t1 / np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(rp, t1)
    D = np.zeros((nc, 3, 2))
    for j in range(3):
        d = proj(coarse.centre[coarse.nbr[:, j]] - rp)
        D[:, j, 0] = np.sum(d * t1, axis=1)
        D[:, j, 1] = np.sum(d * t2, axis=1)
    normal = np.einsum("nji,njk->nik", D, D)                 # D^T D, [nc, 2, 2]
    pinv = np.linalg.solve(normal, np.transpose(D, (0, 2, 1)))  # (D^T D)^-1 D^T, [nc, 2, 3]
    w = np.zeros((fine.n, 3))
    for i in range(4):
        c = 4 * np.arange(nc) + i
        delta = proj(fine.centre[c] - rp)
        dl = np.stack([np.sum(delta * t1, axis=1), np.sum(delta * t2, axis=1)], axis=1)   # [nc, 2]
        w[c] = np.einsum("ni,nij->nj", dl, pinv)
    return w


def prolong(e_coarse: np.ndarray, coarse_nbr: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Linear interpolation of a coarse correction to the fine grid."""
    nf = w.shape[0]
    parent = np.arange(nf) // 4
    ep = e_coarse[parent]
    out = ep.copy()
    for j in range(3):
        out = out + w[:, j:j + 1] * (e_coarse[coarse_nbr[parent, j]] - ep)
    return out


# ---------------------------------------------------------------------------
# hierarchy and V-cycle
# ---------------------------------------------------------------------------


@dataclass
class Hierarchy:
    ops: list          # LevelOperator per level, 0 = coarsest
    weights: list      # weights[l] prolongs level l-1 -> l (weights[0] unused)
    meshes: list
    vert: opmod.Vertical
    nu_pre: int = 2
    nu_post: int = 2
    nu_coarse: int = 1
    omega: float = 2.0 / 3.0
    dtype: type = np.float64
    colours: list | None = None   # multicolour block-SOR: colours per level (None: block-Jacobi)

    @property
    def finest(self) -> opmod.LevelOperator:
        return self.ops[-1]

    def astype(self, dtype) -> "Hierarchy":
        return Hierarchy([o.astype(dtype) for o in self.ops], [None if w is None else w.astype(dtype) for w in self.weights],
                         self.meshes, self.vert, self.nu_pre, self.nu_post, self.nu_coarse, self.omega, dtype,
                         self.colours)

    def with_sor(self, omega: float = 1.0) -> "Hierarchy":
        """The same hierarchy with the multicolour block-SOR smoother (the
        paper's implementation, Section 5: block-SOR with relaxation factor
        1, here in colour order), colours from greedy_colouring."""
        return Hierarchy(self.ops, self.weights, self.meshes, self.vert, self.nu_pre, self.nu_post, self.nu_coarse,
                         omega, self.dtype, [greedy_colouring(o.nbr) for o in self.ops])


FULL_TERMS = ("alpha_r", "alpha_s", "beta")
# the full operator with vertical advection (FullProfiles.xi_r given)
FULL_TERMS_ADV = FULL_TERMS + ("xi_r",)


def build(refinement: int, r_faces, omega2: float, profiles=None, n_levels: int = 0,
          meshes: list | None = None, vert: opmod.Vertical | None = None,
          full: opmod.FullProfiles | None = None, full_terms=FULL_TERMS,
          level_factors: dict | None = None) -> Hierarchy:
    """Meshes, coefficients and transfer weights for TPMG on refinement `refinement`.

    profiles: object with alpha_r_v, alpha_s_v, beta_v and optional per-cell
    finest-grid alpha_r_h, alpha_s_h, beta_h (None = 1). vert replaces the
    radial factors derived from r_faces (used to pose the 2-D problems of the
    tensor decoupling).

    level_factors: {refinement level: (alpha_r_h, alpha_s_h, beta_h)}, the
    horizontal factors of that grid sampled by the caller (entries may be
    None); where none is given, a coarse grid takes the area-weighted means
    of its children's factors (the coarse operator is rediscretised on each
    grid, Section 3.2.1).

    full: profiles that need not factorise, sampled on the finest grid
    (Section 4.2). The coefficients named in full_terms are then taken from
    them on every level (coarse grids: area-weighted means of the four
    children, level by level), the others from the factorised `profiles`:
    all three terms give the operator of TPMG^(full), alpha_r alone that of
    TPMG^(partial) (Section 5.3), none (full = None) that of TPMG^(x).
    """
    if n_levels <= 0:
        n_levels = min(6, refinement + 1)
    if n_levels > refinement + 1:
        raise ValueError("more levels than refinements")
    if meshes is None:
        meshes = mesh_mod.hierarchy(refinement)
    if vert is None:
        vert = opmod.vertical(r_faces)
    nz = vert.nz
    if profiles is None:
        ar_v, as_v, b_v = np.ones(nz + 1), np.ones(nz), np.ones(nz)
        ar_h = as_h = b_h = None
    else:
        ar_v, as_v, b_v = profiles.alpha_r_v, profiles.alpha_s_v, profiles.beta_v
        ar_h, as_h, b_h = profiles.alpha_r_h, profiles.alpha_s_h, profiles.beta_h
    nf = meshes[refinement].n
    given = level_factors or {}

    def sampled(ref, i):
        v = given.get(ref, (None, None, None))[i]
        return None if v is None else np.asarray(v, dtype=np.float64)

    h = [np.ones(nf) if x is None else np.asarray(x, dtype=np.float64) for x in (ar_h, as_h, b_h)]
    h = [h[i] if sampled(refinement, i) is None else sampled(refinement, i) for i in range(3)]
    levels = list(range(refinement - n_levels + 1, refinement + 1))
    per_level = {refinement: h}
    for ref in range(refinement, levels[0], -1):
        fine_area = meshes[ref].area
        per_level[ref - 1] = [opmod.restrict_cell_factor(x, fine_area) if sampled(ref - 1, i) is None
                              else sampled(ref - 1, i) for i, x in enumerate(per_level[ref])]
    full_level = {}
    if full is not None and full_terms:
        if "xi_r" in full_terms and getattr(full, "xi_r", None) is None:
            full_terms = tuple(k for k in full_terms if k != "xi_r")
        full_level[refinement] = {k: np.asarray(getattr(full, k), dtype=np.float64) for k in full_terms}
        for ref in range(refinement, levels[0], -1):
            full_level[ref - 1] = {k: opmod.restrict_cell_profile(v, meshes[ref].area)
                                   for k, v in full_level[ref].items()}
    ops, weights, used = [], [None], []
    for ref in levels:
        ar, as_, b = per_level[ref]
        op = opmod.assemble(meshes[ref], vert, omega2, ar_v, as_v, b_v, ar, as_, b)
        if ref in full_level:
            fl = full_level[ref]
            n = meshes[ref].n
            # the factorised samples of the other terms, as [n, *] arrays
            fac = {"alpha_r": ar[:, None] * np.asarray(ar_v)[None, :], "alpha_s": as_[:, None] * np.asarray(as_v)[None, :],
                   "beta": b[:, None] * np.asarray(b_v)[None, :]}
            fac.update(fl)
            assert fac["alpha_r"].shape == (n, nz + 1)
            op = opmod.assemble_full(meshes[ref], vert, omega2, fac["alpha_r"], fac["alpha_s"], fac["beta"],
                                     fl.get("xi_r"))
        ops.append(op)
        used.append(meshes[ref])
    for i in range(1, len(levels)):
        weights.append(prolongation_weights(used[i - 1], used[i]))
    return Hierarchy(ops, weights, used, vert)


def vcycle(h: Hierarchy, f: np.ndarray, level: int | None = None) -> np.ndarray:
    """Algorithm 1 applied to f from a zero initial guess; returns u."""
    if level is None:
        level = len(h.ops) - 1
    op = h.ops[level]
    u = np.zeros_like(f)

    def sweep(u, post=False):
        if h.colours is None:
            return smooth(op, f, u, h.omega)
        # colours ascending before the coarse-grid correction, descending after
        return smooth_sor(op, f, u, h.omega, h.colours[level], reverse=post)

    if level == 0:
        for _ in range(h.nu_coarse):
            u = sweep(u)
        return u
    for _ in range(h.nu_pre):
        u = sweep(u)
    r = f - opmod.apply(op, u)
    fc = restrict(r)
    uc = vcycle(h, fc, level - 1)
    u = u + prolong(uc, h.ops[level - 1].nbr, h.weights[level])
    for _ in range(h.nu_post):
        u = sweep(u, post=True)
    return u


def make_preconditioner(h: Hierarchy, precision: str = "fp64"):
    """One V-cycle as a preconditioner r -> z. "fp32": the whole V-cycle
    (coefficients, smoother, Thomas, transfers) in float32; the input is
    rounded to float32 and the output widened back to float64."""
    if precision == "fp64":
        return lambda r: vcycle(h, r)
    h32 = h.astype(np.float32)
    return lambda r: vcycle(h32, r.astype(np.float32)).astype(np.float64)


# ---------------------------------------------------------------------------
# flexible CG
# ---------------------------------------------------------------------------


@dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    status: str                        # "converged", "maxit", "breakdown"
    history: list = field(default_factory=list)   # ||r_k|| / ||f|| after each iteration (index 0: initial)


def fcg(apply_a, precond, f: np.ndarray, x0: np.ndarray | None = None, rtol: float = 1e-8,
        maxit: int = 100) -> SolveResult:
    """Flexible CG with one-term orthogonalisation (FCG(1)).

    r0 = f - A x0, z0 = M r0, p0 = z0; per iteration: q = A p,
    alpha = <r,z>/<p,q>, x += alpha p, r -= alpha q, stop if
    ||r|| <= rtol ||f||, z' = M r, beta = -<z',q>/<p,q>, p = z' + beta p.
    """
    x = np.zeros_like(f) if x0 is None else x0.astype(np.float64).copy()
    fnorm = math.sqrt(float(np.sum(f * f)))
    r = f - apply_a(x)
    rnorm = math.sqrt(float(np.sum(r * r)))
    hist = [rnorm / fnorm if fnorm > 0 else 0.0]
    if rnorm <= rtol * fnorm:
        return SolveResult(x, 0, "converged", hist)
    z = precond(r)
    p = z.copy()
    rz = float(np.sum(r * z))
    for it in range(maxit):
        q = apply_a(p)
        pq = float(np.sum(p * q))
        if not (pq > 0.0) or not math.isfinite(pq) or not math.isfinite(rz):
            return SolveResult(x, it, "breakdown", hist)
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        rnorm = math.sqrt(float(np.sum(r * r)))
        hist.append(rnorm / fnorm)
        if not math.isfinite(rnorm):
            return SolveResult(x, it + 1, "breakdown", hist)
        if rnorm <= rtol * fnorm:
            return SolveResult(x, it + 1, "converged", hist)
        z = precond(r)
        zq = float(np.sum(z * q))
        rz = float(np.sum(z * r))
        beta = -zq / pq
        p = z + beta * p
    return SolveResult(x, maxit, "maxit", hist)


def richardson(apply_a, precond, f: np.ndarray, x0: np.ndarray | None = None, rtol: float = 1e-8,
               maxit: int = 100) -> SolveResult:
    """Preconditioned Richardson iteration (Section 3.2.2, Section 5.2):
    x_{k+1} = x_k + M (f - A x_k), stopping when ||f - A x_k|| <= rtol ||f||
    (k corrections applied)."""
    x = np.zeros_like(f) if x0 is None else x0.astype(np.float64).copy()
    fnorm = math.sqrt(float(np.sum(f * f)))
    hist = []
    for it in range(maxit + 1):
        r = f - apply_a(x)
        rnorm = math.sqrt(float(np.sum(r * r)))
        hist.append(rnorm / fnorm if fnorm > 0 else 0.0)
        if not math.isfinite(rnorm):
            return SolveResult(x, it, "breakdown", hist)
        if rnorm <= rtol * fnorm:
            return SolveResult(x, it, "converged", hist)
        if it == maxit:
            break
        x = x + precond(r)
    return SolveResult(x, maxit, "maxit", hist)


def bicgstab(apply_a, precond, f: np.ndarray, x0: np.ndarray | None = None, rtol: float = 1e-8,
             maxit: int = 100) -> SolveResult:
    """Right-preconditioned BiCGStab (van der Vorst; the paper's second outer
    solver, Section 5.2: two operator applications and two preconditioner
    applications per iteration). r0 = f - A x0, shadow residual r^ = r0;
    per iteration: rho = <r^, r>, beta = (rho / rho_prev)(alpha / w),
    p = r + beta (p - w v), y = M p, v = A y, alpha = rho / <r^, v>,
    s = r - alpha v, z = M s, t = A z, w = <t, s> / <t, t>,
    x += alpha y + w z, r = s - w t; stop when ||r|| <= rtol ||f||
    (tested once per iteration)."""
    x = np.zeros_like(f) if x0 is None else x0.astype(np.float64).copy()
    fnorm = math.sqrt(float(np.sum(f * f)))
    r = f - apply_a(x)
    rnorm = math.sqrt(float(np.sum(r * r)))
    hist = [rnorm / fnorm if fnorm > 0 else 0.0]
    if rnorm <= rtol * fnorm:
        return SolveResult(x, 0, "converged", hist)
    rh = r.copy()
    rho_prev = alpha = w = 1.0
    p = np.zeros_like(f)
    v = np.zeros_like(f)
    for it in range(maxit):
        rho = float(np.sum(rh * r))
        if rho == 0.0 or not math.isfinite(rho):
            return SolveResult(x, it, "breakdown", hist)
        beta = (rho / rho_prev) * (alpha / w)
        p = r + beta * (p - w * v)
        y = precond(p)
        v = apply_a(y)
        alpha = rho / float(np.sum(rh * v))
        s = r - alpha * v
        z = precond(s)
        t = apply_a(z)
        tt = float(np.sum(t * t))
        w = float(np.sum(t * s)) / tt if tt > 0 else 0.0
        x = x + alpha * y + w * z
        r = s - w * t
        rnorm = math.sqrt(float(np.sum(r * r)))
        hist.append(rnorm / fnorm)
        if not math.isfinite(rnorm) or w == 0.0:
            return SolveResult(x, it + 1, "breakdown", hist)
        if rnorm <= rtol * fnorm:
            return SolveResult(x, it + 1, "converged", hist)
        rho_prev = rho
    return SolveResult(x, maxit, "maxit", hist)


def solve(h: Hierarchy, f: np.ndarray, x0=None, rtol=1e-8, maxit=100, precision="fp64",
          outer: opmod.LevelOperator | None = None, method: str = "fcg") -> SolveResult:
    """TPMG-preconditioned FCG (or "bicgstab", "richardson") on the finest
    level of h. outer: the operator of the equation when it differs from the
    one the V-cycle is built on (TPMG^(x) or TPMG^(partial) for
    non-factorising profiles, Section 3.2.2)."""
    op = h.finest if outer is None else outer
    solver = {"fcg": fcg, "bicgstab": bicgstab, "richardson": richardson}[method]
    return solver(lambda v: opmod.apply(op, v), make_preconditioner(h, precision), f, x0, rtol, maxit)


def richardson_rate(h: Hierarchy, seed: int = 7, cycles: int = 12, skip: int = 4, precision="fp64",
                    outer: opmod.LevelOperator | None = None) -> float:
    """Asymptotic V-cycle factor of u <- u + M(f - A u) with f = 0 (A: the
    finest operator of h, or `outer`, Section 3.2.2)."""
    op = h.finest if outer is None else outer
    m = make_preconditioner(h, precision)
    u = np.random.default_rng(seed).uniform(-1.0, 1.0, size=(op.n, op.nz))
    norms = []
    for _ in range(cycles + 1):
        r = -opmod.apply(op, u)
        norms.append(math.sqrt(float(np.sum(r * r))))
        u = u + m(r)
    return (norms[cycles] / norms[skip]) ** (1.0 / (cycles - skip))


def direct_solve(op: opmod.LevelOperator, f: np.ndarray) -> np.ndarray:
    """u = A^-1 f with a sparse direct solver (the plain definition)."""
    a = opmod.to_sparse(op).tocsc()
    return spla.spsolve(a, f.ravel()).reshape(f.shape)
