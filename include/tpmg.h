/*
 * tpmg.h -- C ABI of the MI355X (gfx950) tensor-product multigrid solver for
 * the anisotropic pressure-correction equation in a thin spherical shell.
 *
 * Problem (Dedner, Mueller & Scheichl, Section 2.1 and Appendix A): find u
 * with A u = f, where A is the cell-centred finite-volume discretisation of
 *     L u = -omega^2 div(alpha grad u) + beta u
 * on the shell S x [1, 1+H] (lengths in Earth radii), without the vertical
 * advection term (Section 3.2.1: this operator is symmetric positive
 * definite). The horizontal grid is an icosahedral grid refined
 * `refinement` times; each horizontal cell T carries a column of nz cells
 * between radial faces r_0 = 1 < ... < r_nz = 1 + H (Section 4.1). Profiles
 * factorise: alpha_r = alpha_r^r(r) alpha_r^S(x), likewise alpha_S and beta
 * (Appendix A, eq. hatFunctionsFac), homogeneous Neumann top and bottom.
 *
 * The solve is flexible CG (FP64) preconditioned by one tensor-product
 * multigrid V-cycle (Algorithm 1): horizontal-only coarsening, vertical line
 * relaxation (eq. BlockJacobi, damped block-Jacobi with a Thomas solve per
 * column), restriction by summing the four children and linear
 * interpolation (Section 5).
 *
 * Conventions for every entry point:
 *  - Return value: a tpmg_status. Arguments are checked before any device
 *    work; on error nothing is enqueued and tpmg_last_error() (thread-local)
 *    holds a message. TPMG_NOT_CONVERGED is not an error: the solution
 *    buffer holds the last iterate.
 *  - Ownership: the caller owns every device buffer (right-hand sides,
 *    solutions, workspace). The library never allocates device memory; it
 *    carves the workspace given to tpmg_mg_setup. The library owns its host
 *    handles; a handle must outlive the device work it enqueued.
 *  - Streams: all device work of a tpmg_mg runs on the HIP stream given to
 *    tpmg_mg_setup (a non-default stream if graphs are enabled).
 *  - Layouts: host arrays are cell-major, value (T, k) at T * nz + k (the
 *    column-contiguous storage of Section 4.1). Device vectors passed to
 *    tpmg_spmv / tpmg_vcycle / tpmg_solve use the library's tiled layout of
 *    64 columns per tile, value (T, k) at (T / 64) * 64 * nz + k * 64 +
 *    T % 64, with the column count padded up to a multiple of 64 (padding
 *    entries are zero on input and stay zero); tpmg_pack / tpmg_unpack
 *    convert between the two.
 */
#ifndef TPMG_H
#define TPMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TPMG_OK = 0,
  TPMG_NOT_CONVERGED = 1,   /* maxit reached; u holds the last iterate      */
  TPMG_ERR_ARG = -1,        /* invalid or mis-sized argument                */
  TPMG_ERR_DEVICE = -2,     /* a HIP call failed                            */
  TPMG_ERR_NOMEM = -3,      /* workspace smaller than tpmg_mg_workspace_size */
  TPMG_ERR_BREAKDOWN = -4,  /* NaN/Inf, <p, A p> <= 0, or divergence        */
  TPMG_ERR_STATE = -5       /* call out of order for this handle            */
} tpmg_status;

typedef struct tpmg_grid tpmg_grid;
typedef struct tpmg_op tpmg_op;
typedef struct tpmg_mg tpmg_mg;
typedef struct tpmg_batch tpmg_batch;

/* Multigrid parameters (Section 5: nu_pre = nu_post = 2, one coarse sweep). */
typedef struct {
  int n_levels;        /* multigrid levels; 0 = min(6, refinement + 1)      */
  int nu_pre;          /* pre-smoothing sweeps per level (default 2)        */
  int nu_post;         /* post-smoothing sweeps per level (default 2)       */
  int nu_coarse;       /* sweeps on the coarsest level (default 1)          */
  double omega_relax;  /* block-Jacobi damping (default 2/3)                */
  int precond_fp32;    /* 1: V-cycle in FP32 inside the FP64 CG (default 0) */
  int use_graph;       /* 1: replay the FCG iteration as a HIP graph        */
  /* Launch configuration (see "Launch tuning" below). 0 in any field keeps
   * the built-in choice or, with autotune, lets the trials decide it. */
  int autotune;        /* 0: built-in choices; 1: timed trials at setup,
                          reusing the process-wide tuning cache; 2: timed
                          trials that replace the cached entries          */
  int smoother;        /* line-smoother kernel on every level: 1 = column in
                          registers, solved by block scans over the waves
                          (nz <= 16 * scan_levels, required for batches);
                          2 = LDS-staged; 3 = global scratch (any nz)     */
  int scan_levels;     /* levels per wave of the scan smoother: 4, 8, 16   */
  int stencil_chunk;   /* levels per wave of the transfer kernels and the
                          operator: 1 .. 256                              */
  int precond_profiles; /* for an operator with profiles that do not
                          factorise (tpmg_op_set_full_profiles), the
                          operator the V-cycle is built on (Section 4.2,
                          Section 5.3): 0 = the full profiles
                          (TPMG^(full)); 1 = the factorised profiles given
                          to tpmg_op_create, the approximate factorisation
                          (TPMG^(x)); 2 = the full alpha_r with the
                          factorised alpha_S and beta (TPMG^(partial)).
                          The Krylov method always uses the full operator.
                          1 and 2 need full profiles.                     */
  int smoother_order;  /* 0 = block-Jacobi: every column relaxed from the
                          old values, damped by omega_relax (default);
                          1 = multicolour block-SOR (Section 5: block-SOR
                          with relaxation factor omega_relax, the paper's
                          1): cells coloured greedily in index order so
                          that neighbours differ (tpmg_grid_colouring),
                          the colours relaxed one after another, ascending
                          before the coarse-grid correction and descending
                          after; one pass over the grid per colour. The
                          problems of a batch share it.                   */
  int tile_cols;       /* columns per tile of the device layout: 0 (auto)
                          or 64, the only width: one lane per column and
                          one 64-lane wavefront per tile, so that every
                          level of a tile is one coalesced row and the
                          neighbour exchange stays inside a wave; other
                          values are TPMG_ERR_ARG. (Work per block is tuned
                          through levels per wave and stencil chunks.)   */
} tpmg_mg_params;

/* Result of a solve. Inputs: history (optional, caller-owned, history_cap
 * entries) receives ||r_k|| / ||f|| for k = 0 .. iters; phase_timers = 1
 * times the phases of every iteration with HIP events on the solve's stream
 * (the iteration's kernels are then launched one by one, never as a graph);
 * div_tol (0 = 1e3) stops the solve with TPMG_ERR_BREAKDOWN once
 * ||r_k|| > div_tol ||r_0||. Outputs: the rest. */
typedef struct {
  int iters;
  double relres;       /* ||r|| / ||f|| of the recursively updated residual */
  double* history;
  int history_cap;
  double t_total_ms;   /* wall time of tpmg_solve, first kernel to return   */
  int phase_timers;    /* in: 1 = fill t_vcycle_ms, t_spmv_ms, t_blas_ms    */
  double div_tol;      /* in: divergence bound on ||r_k|| / ||r_0||; 0 = 1e3 */
  double t_vcycle_ms;  /* device time in the V-cycles (smoother sweeps,
                          transfers, the dots formed by the last sweep)     */
  double t_spmv_ms;    /* device time in q = A p (with the direction update
                          formed inside it) and the initial residual        */
  double t_blas_ms;    /* device time in the other vector updates and
                          reductions (r -= alpha q, x += alpha p)           */
  double model_bytes;  /* algorithmic HBM bytes the solve moved: every
                          field read or written once per kernel that touches
                          it (the per-kernel figures of the kernel table),
                          summed over the kernels the solve ran             */
} tpmg_solve_info;

/* Fills p with the defaults above. */
void tpmg_mg_params_default(tpmg_mg_params* p);

/* ---------------------------------------------------------------- host -- */

/* Icosahedral grid hierarchy (Section 4.2: icosahedral grid projected onto
 * the sphere, each coarse triangle the union of four fine ones) for
 * refinements 0..refinement, with the radial faces r_faces[0..nz]
 * (strictly increasing, r_faces[0] = 1; copied). Base icosahedron: poles
 * plus two rings of five vertices at latitude +-atan(1/2), longitudes 72 i
 * and 36 + 72 i; child i of cell P on the next finer grid is cell 4P + i;
 * neighbour j of a cell lies across its edge j. Host only.
 * Errors: TPMG_ERR_ARG for refinement outside [0, 10], nz < 1, NULL
 * pointers or non-increasing faces. */
tpmg_status tpmg_grid_icosahedral(int refinement, int nz, const double* r_faces, tpmg_grid** out);

/* Number of cells n_T = 20 * 4^refinement_level of grid level
 * refinement_level (0..refinement). */
tpmg_status tpmg_grid_level_size(const tpmg_grid* g, int refinement_level, int* n_cells);

/* Geometry of grid level refinement_level (Appendix A): spherical
 * circumcentres (3 n), spherical areas |T| (n), neighbours (3 n, int32),
 * great-circle edge lengths |S_TT'| (3 n) and two-point flux factors
 * |S_TT'| n_TT'.(r_T' - r_T) / |r_T' - r_T|^2 (3 n), all cell-major
 * ([T][j]). Any output may be NULL. Host arrays, caller-owned. */
tpmg_status tpmg_grid_geometry(const tpmg_grid* g, int refinement_level, double* centres, double* areas,
                               int32_t* nbr, double* edge_len, double* edge_factor);

/* The colouring of grid level refinement_level used by the multicolour
 * block-SOR smoother: cells in index order, each taking the smallest colour
 * (0, 1, ...) that none of its already coloured neighbours has, so that no
 * two neighbours share a colour (at most 4 colours). colours: n int32
 * (host, caller-owned); n_colours may be NULL. Host only. */
tpmg_status tpmg_grid_colouring(const tpmg_grid* g, int refinement_level, int32_t* colours, int* n_colours);

/* Radial cell volume factors v_k = (r_{k+1}^3 - r_k^3) / 3 (Appendix A),
 * nz values. */
tpmg_status tpmg_grid_vertical(const tpmg_grid* g, double* vk);

/* Tensor-stencil operator on the n_levels finest grids (0 = min(6,
 * refinement + 1)), Appendix A eq. hatFunctionsFac with the vertical
 * advection dropped. Vertical profile factors: alpha_r_v at the nz+1
 * faces, alpha_s_v and beta_v at the nz layer midpoints. Horizontal
 * factors: one value per finest-grid cell (n_T values) or NULL for 1; the
 * value on an edge is the mean of its two cells; coarse grids use
 * area-weighted means of the four children and are rediscretised on their
 * own geometry. omega2 = omega^2 > 0. All factors must be > 0.
 * Errors: TPMG_ERR_ARG. */
tpmg_status tpmg_op_create(const tpmg_grid* g, int n_levels, double omega2, const double* alpha_r_v,
                           const double* alpha_s_v, const double* beta_v, const double* alpha_r_h,
                           const double* alpha_s_h, const double* beta_h, tpmg_op** out);

/* As tpmg_op_create, with the horizontal factors of coarse grids sampled by
 * the caller (the coarse-grid operator is rediscretised on each grid,
 * Section 3.2.1; the profiles can be evaluated at its cells). alpha_r_h,
 * alpha_s_h, beta_h: NULL or arrays of refinement + 1 pointers indexed by
 * refinement level, entry r NULL or n_r values (tpmg_grid_level_size) for
 * the cells of that grid, all > 0 and finite. Where an entry is NULL the
 * finest grid takes the factor 1 and a coarse grid the area-weighted means
 * of its four children's factors on the next finer grid, as tpmg_op_create
 * does. Entries of grids outside the hierarchy are not read. Host arrays,
 * caller-owned, read during the call. Errors: TPMG_ERR_ARG. */
tpmg_status tpmg_op_create_levels(const tpmg_grid* g, int n_levels, double omega2, const double* alpha_r_v,
                                  const double* alpha_s_v, const double* beta_v, const double* const* alpha_r_h,
                                  const double* const* alpha_s_h, const double* const* beta_h, tpmg_op** out);

/* Profiles that do not factorise (Section 4.2: the general case of
 * Appendix A, eq. hatFunctionsNonFac, with the vertical advection dropped):
 * point samples on the finest grid of g (the grid op was created on),
 * cell-major: alpha_r [n][nz+1] at the radial faces (r_k, centre of T),
 * alpha_s and beta [n][nz] at the layer midpoints (r_{k+1/2}, centre of T);
 * all positive (alpha_r at the top and bottom faces is not used). The
 * coefficients per (T, k) are formed on every level (coarse grids:
 * area-weighted means of the four children's samples, level by level; on an
 * edge the mean of its two cells, as in the factorised case). The operator
 * of the equation then uses them (tpmg_spmv, the Krylov method of
 * tpmg_solve); the factorised profiles given to tpmg_op_create stay as the
 * approximate factorisation a V-cycle may be built on
 * (tpmg_mg_params.precond_profiles). Host arrays, copied. Such operators run
 * the scan smoother at 8 or 16 levels per wave and no batched solves.
 *
 * xi_r (NULL = none) adds the vertical advection -omega^2 xi_r d_r u
 * (Section 2.1, eq. HelmholtzVector; samples [n][nz+1] at the radial faces),
 * discretised as Appendix A writes the cell integral of cell k: |T|
 * (r_{k+1} - r_k) times the mean of r_f^2 xi_{T,f} (u across face f) /
 * (centre distance across f) over its faces f = k, k+1. The operator is
 * then not symmetric: solve it with tpmg_solve_bicgstab or
 * tpmg_solve_richardson (tpmg_solve refuses it). The V-cycle of the full
 * profiles includes the advection, those of the factorised and partial
 * profiles do not. The advection must leave both radial couplings of every
 * row positive (alphar^_k - adv_lo_k, alphar^_{k+1} + adv_up_k).
 * Errors: TPMG_ERR_ARG. */
tpmg_status tpmg_op_set_full_profiles(tpmg_op* op, const tpmg_grid* g, const double* alpha_r, const double* alpha_s,
                                      const double* beta, const double* xi_r);

/* The coefficients per (T, k) of level (0 = coarsest) of an operator with
 * full profiles, cell-major: beta^_{T,k} [n][nz], alphaS^_{TT'_j,k}
 * [n][3][nz] (coupling to neighbour j), alphar^_{T,k} [n][nz+1] (radial
 * face k), and with vertical advection omega^2 times the coefficients of
 * cell k's lower and upper face [n][nz] (zeros without advection). Any
 * output may be NULL. TPMG_ERR_STATE without full profiles. */
tpmg_status tpmg_op_coefficients_full(const tpmg_op* op, int level, double* beta, double* alpha_s, double* alpha_r,
                                      double* adv_lo, double* adv_up);

/* Number of multigrid levels of op, and the cell count of level (0 =
 * coarsest). */
tpmg_status tpmg_op_levels(const tpmg_op* op, int* n_levels);
tpmg_status tpmg_op_level_size(const tpmg_op* op, int level, int* n_cells);

/* Factorised coefficients of level (0 = coarsest), for parity checks:
 * horizontal beta^S_T = |T| beta^S (n), alphar^S_T = omega^2 |T| alpha_r^S
 * (n), alphaS^S_TT' = omega^2 g_TT' alpha_S^S (3 n, [T][j]); vertical
 * beta^r_k = v_k beta^r (nz), alphaS^r_k = (r_{k+1} - r_k) alpha_S^r (nz),
 * alphar^r_k = sigma_k 2 r_k^2 / (r_{k+1} - r_{k-1}) alpha_r^r (nz+1).
 * The full coefficient is the product of a horizontal and a vertical
 * factor. Any output may be NULL. */
tpmg_status tpmg_op_coefficients(const tpmg_op* op, int level, double* beta_h, double* alpha_r_h,
                                 double* alpha_s_h, double* beta_v, double* alpha_s_v, double* alpha_r_v);

/* Prolongation weights into level (1..n_levels-1) from level-1: 3 per fine
 * cell c ([c][j]), e_c = e_P + sum_j w[c][j] (e_{N_j(P)} - e_P), P = c / 4
 * (least-squares linear reconstruction in the tangent plane at r_P). */
tpmg_status tpmg_op_prolongation(const tpmg_op* op, int level, double* w);

/* -------------------------------------------------------------- device -- */

/* Device workspace bytes that tpmg_mg_setup needs for (op, params). */
tpmg_status tpmg_mg_workspace_size(const tpmg_op* op, const tpmg_mg_params* params, size_t* bytes);

/* Carves d_workspace (device, >= tpmg_mg_workspace_size bytes, 256-byte
 * aligned), uploads the coefficients on hip_stream (a hipStream_t; NULL =
 * default stream, which disables graphs) and synchronises it. op may be
 * destroyed afterwards. Errors: TPMG_ERR_ARG, TPMG_ERR_NOMEM (workspace too
 * small), TPMG_ERR_DEVICE. */
tpmg_status tpmg_mg_setup(const tpmg_op* op, const tpmg_mg_params* params, void* d_workspace, size_t bytes,
                          void* hip_stream, tpmg_mg** out);

/* Length in doubles of a device vector in the tiled layout (padded columns
 * times nz), and the real cell count of the finest grid. */
tpmg_status tpmg_mg_vector_length(const tpmg_mg* mg, size_t* n_doubles, int* n_cells, int* nz);

/* Cell-major <-> tiled conversion of a finest-grid FP64 vector (device
 * pointers, asynchronous on the setup stream). d_cellmajor holds
 * n_cells * nz doubles, d_tiled tpmg_mg_vector_length doubles. */
tpmg_status tpmg_pack(tpmg_mg* mg, const double* d_cellmajor, double* d_tiled);
tpmg_status tpmg_unpack(tpmg_mg* mg, const double* d_tiled, double* d_cellmajor);

/* y = A x on the finest grid, matrix-free tensor stencil (eq. ColumnEquation),
 * FP64, tiled layout, asynchronous. x and y must not alias. */
tpmg_status tpmg_spmv(tpmg_mg* mg, const double* d_x, double* d_y);

/* z = one V-cycle (Algorithm 1) applied to r from a zero initial guess, in
 * the precision chosen at setup; FP64 tiled vectors in and out,
 * asynchronous. r and z must not alias. */
tpmg_status tpmg_vcycle(tpmg_mg* mg, const double* d_r, double* d_z);

/* One undamped line-relaxation sweep on the finest grid in FP64 (the
 * smoother's column solves, eq. BlockJacobi, with damping 1, on the
 * operator the V-cycle is built on): u_out = u_in + A_T^-1 (f - A u_in),
 * A_T the vertical part of each column's block. Tiled FP64 vectors;
 * u_out must not alias f or u_in; every entry of u_out is written (padding
 * entries zero when those of f are). Asynchronous. nz <= 128 always fits;
 * a larger nz needs the LDS-staged smoother (two [nz][64] FP64 arrays in
 * LDS; factorised profiles only), else TPMG_ERR_ARG. It is the relaxation that
 * follows the learned initial guess (tpmg_mlp.h), and from a zero u_in it
 * is the column solves alone. */
tpmg_status tpmg_relax(tpmg_mg* mg, const double* d_f, const double* d_u_in, double* d_u_out);

/* Solves A u = f by V-cycle-preconditioned flexible CG, starting from the
 * guess in d_u (tiled FP64), until ||r|| <= rtol ||f|| (2-norms of the
 * cell-integral residual) or maxit iterations. The host reads each
 * iteration's residual norm from a record the device writes to pinned
 * memory, with the next iteration usually queued already; the call returns
 * after the stream has drained. A guess that already meets the tolerance,
 * or maxit = 0, returns u unchanged with 0 iterations. Returns TPMG_OK,
 * TPMG_NOT_CONVERGED, or TPMG_ERR_BREAKDOWN (u then holds the last finite
 * iterate). info may be NULL. */
tpmg_status tpmg_solve(tpmg_mg* mg, const double* d_f, double* d_u, double rtol, int maxit,
                       tpmg_solve_info* info);

/* The paper's outer solvers (Section 5.2), preconditioned by one V-cycle of
 * the handle (right preconditioning), for any operator, the non-symmetric
 * one with vertical advection included:
 *  - Richardson: u <- u + M (f - A u) until ||f - A u|| <= rtol ||f||
 *    (iters = corrections applied, history[k] = ||f - A u_k|| / ||f||);
 *  - BiCGStab (van der Vorst): r^ = r_0; per iteration rho = <r^, r>,
 *    beta = (rho / rho_prev)(alpha / w), p = r + beta (p - w v), y = M p,
 *    v = A y, alpha = rho / <r^, v>, s = r - alpha v, z = M s, t = A z,
 *    w = <t, s> / <t, t>, u += alpha y + w z, r = s - w t; the residual
 *    norm is tested once per iteration.
 * Vectors as tpmg_solve (tiled FP64); both synchronise the stream once per
 * iteration to read the residual norm. Returns TPMG_OK, TPMG_NOT_CONVERGED
 * or TPMG_ERR_BREAKDOWN (a zero or non-finite scalar). info as tpmg_solve
 * (no phase timers). */
tpmg_status tpmg_solve_richardson(tpmg_mg* mg, const double* d_f, double* d_u, double rtol, int maxit,
                                  tpmg_solve_info* info);
tpmg_status tpmg_solve_bicgstab(tpmg_mg* mg, const double* d_f, double* d_u, double rtol, int maxit,
                                tpmg_solve_info* info);

/* ----------------------------------------------------------- batched -- */

/* Several independent solves of uneven size advanced together. The problems
 * fall into up to four groups (longest vectors first, each to the group
 * with the least work so far); in each group every step of the FCG
 * iteration (each smoother sweep, transfer and BLAS-1 operation of the
 * V-cycle of Algorithm 1, taken level by level from the finest grid down)
 * is one grouped launch over the group's problems. The whole iteration is
 * replayed as one HIP graph whose branches, one per group, run
 * concurrently, and each problem stops when its own relative residual
 * meets rtol (tested on the device; a finished problem's work is skipped).
 * Each problem is computed with the block decomposition of its own
 * tpmg_solve, so its iterates and iteration count equal those of a single
 * solve. tpmg_batch_create creates the streams and events that capture the
 * branches (up to three of each, default priority; released by
 * tpmg_batch_destroy). The problems must share one non-default stream, the
 * precision and the smoother parameters (block-Jacobi or multicolour
 * block-SOR, damping, sweep counts), have at least two levels, a symmetric
 * operator (no vertical advection; profiles that factorise or not, with any
 * of the three V-cycles) and the scan smoother on every level (the default
 * for nz <= 256). The batch workspace (device, 256-byte aligned) holds the
 * per-problem scalars and the launch tables; problems must outlive the
 * batch. Errors: TPMG_ERR_ARG, TPMG_ERR_NOMEM. */
tpmg_status tpmg_batch_workspace_size(tpmg_mg* const* problems, int n, size_t* bytes);
tpmg_status tpmg_batch_create(tpmg_mg* const* problems, int n, void* d_workspace, size_t bytes, tpmg_batch** out);

/* Solves problem p from the guess in d_u[p] with right-hand side d_f[p]
 * (tiled FP64, as tpmg_solve). infos (optional) holds n entries; of their
 * inputs only history and history_cap are read (no phase timers; the
 * divergence bound is 1e3), and each receives its problem's iters, relres,
 * model_bytes and the batch's t_total_ms. Returns
 * TPMG_OK when all converged, TPMG_NOT_CONVERGED if one reached maxit,
 * TPMG_ERR_BREAKDOWN if one broke down (its u holds its last finite
 * iterate). The host waits for each iteration's scalars (an event after
 * their copy) with the next iteration usually queued already; the call
 * returns after the stream has drained. */
tpmg_status tpmg_batch_solve(tpmg_batch* b, const double* const* d_f, double* const* d_u, double rtol, int maxit,
                             tpmg_solve_info* infos);
void tpmg_batch_destroy(tpmg_batch* b);

/* Asymptotic V-cycle convergence factor (Section 5.2: the rate of the
 * V-cycle in the Richardson iteration): runs u <- u + M(f - A u) with f = 0
 * from the start vector in d_u (tiled FP64, overwritten by the last
 * iterate), records ||r_i|| = ||A u_i|| for i = 0..cycles in norms
 * (optional, cycles + 1 values) and returns
 * rate = (||r_cycles|| / ||r_skip||)^(1 / (cycles - skip)).
 * Requires 0 <= skip < cycles. Synchronises the stream. */
tpmg_status tpmg_richardson_rate(tpmg_mg* mg, double* d_u, int cycles, int skip, double* rate, double* norms);

/* Diagnostics: times `reps` back-to-back launches of one finest-grid
 * line-smoother sweep (the general form, reading u and f and writing u, in
 * the precision chosen at setup) between two HIP events on the setup
 * stream, using workspace buffers only (their contents are overwritten).
 * avg_ms: mean duration per launch; model_bytes: the algorithmic HBM bytes
 * of one sweep (read u and f, write u: 3 values per unknown of the
 * finest grid, counting padding columns). Synchronises the stream. */
tpmg_status tpmg_mg_time_sweep(tpmg_mg* mg, int reps, double* avg_ms, double* model_bytes);

/* Diagnostics: times `reps` back-to-back launches (after one untimed launch)
 * of one finest-grid kernel of the solve, alone (no finalize kernel), between
 * two HIP events on the setup stream, on workspace buffers (overwritten):
 *   0  the line-smoother sweep, as tpmg_mg_time_sweep (3 s B per unknown,
 *      s the V-cycle precision's bytes);
 *   1  q = A p with the direction update p = z + beta p_prev formed inside
 *      it, as in an iteration of tpmg_solve (z in the V-cycle's output
 *      precision, p_prev, p and q FP64: 4 or 8 + 24 B per unknown);
 *   2  q = A p (FP64, 16 B per unknown);
 *   3  residual + restriction from the finest grid (2.25 s B per unknown);
 *   4  prolongation + correction into the finest grid (2.25 s B).
 * With coefficients per (T, k) (tpmg_op_set_full_profiles) the stencil
 * kernels also read 5 values per unknown (beta^, three alphaS^, one radial
 * face; 1 for the partial form): 0, 3 + 5 s (or + s) and the operators
 * + 40 B. The counts are per unknown of the padded finest grid. avg_ms: mean
 * duration per launch; model_bytes: the algorithmic HBM bytes of one launch.
 * Kernel 1 overwrites the solver's scalars (the next solve resets them).
 * Synchronises the stream. Errors: TPMG_ERR_ARG (kernel 1 without a fused
 * operator instance, 3 and 4 on a single level). */
tpmg_status tpmg_mg_time_kernel(tpmg_mg* mg, int kernel, int reps, double* avg_ms, double* model_bytes);

/* ------------------------------------------------------ launch tuning -- */

/* The line-smoother kernel (how a column is held while its tridiagonal
 * system is solved), the levels per wave of the scan smoother and the
 * levels per wave of the stencil kernels (residual + restriction,
 * prolongation + correction, the FP64 operator) are chosen per level and
 * per precision at tpmg_mg_setup. With params->autotune the setup times
 * each admissible candidate on the workspace (a few launches each) and
 * keeps the fastest (the built-in choice unless another is 5% faster); the
 * choice is stored in a process-wide cache keyed by
 * device (architecture and compute-unit count), kernel, precision, padded
 * column count and nz, so that later setups of the same shape run no trials.
 * The smoother choice changes the rounding order of the column solve (the
 * result stays within the FP64 parity bar of the same algorithm); the
 * stencil chunks change no stencil output bit, only the summation order of
 * the dot product fused into the operator. */

/* Chosen configuration of level (0 = coarsest): smoother kind (1, 2, 3 as in
 * tpmg_mg_params), scan levels per wave, and the stencil chunks of
 * residual + restriction from this level, prolongation into this level and
 * (finest level only) the FP64 operator. Any output may be NULL. */
tpmg_status tpmg_mg_tuning(const tpmg_mg* mg, int level, int* smoother, int* scan_levels, int* chunk_restrict,
                           int* chunk_prolong, int* chunk_spmv);

/* Timed trials run by the setup of mg and their total device time. */
tpmg_status tpmg_mg_autotune_stats(const tpmg_mg* mg, int* trials, double* trial_ms);

/* Process-wide tuning cache, JSON text: one object whose keys name
 * "device|kernel|precision|padded columns|nz" and whose values are
 * [choice, scan levels] arrays. load merges a file into the cache
 * (TPMG_ERR_ARG if it cannot be read or parsed; the cache is then
 * unchanged), save writes the whole cache, clear empties it, entries counts
 * it. Host only; thread-safe. */
tpmg_status tpmg_tune_load(const char* path);
tpmg_status tpmg_tune_save(const char* path);
tpmg_status tpmg_tune_clear(void);
tpmg_status tpmg_tune_entries(int* n);

/* ------------------------------------------------- allocation-free -- */

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): tpmg_solve with its
 * device setup and teardown in one call that allocates nothing, neither
 * device memory nor pinned host memory. Its workspace is a static array in
 * device memory of TPMG_NOALLOC_SCRATCH_BYTES per GPU, part of the library's
 * code object (each GPU the library runs on holds its copy until the process
 * ends). The call uploads op's coefficients into it (clearing what it uses
 * first), solves A u = f from the guess in d_u exactly as tpmg_solve does
 * (the same kernels in the same order, so the same results, iteration
 * counts and histories), and reads the iteration records by device-to-host
 * copies a few iterations at a time instead of from pinned memory. d_f, d_u:
 * tiled device vectors of op's finest grid (padded cell count times nz
 * doubles, the layout of tpmg_pack), on hip_stream. params->autotune and
 * use_graph must be 0 (built-in launch choices), info->phase_timers 0.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (other threads, other streams) race and must be serialised by the
 * caller. Synchronises hip_stream. Errors: TPMG_ERR_NOMEM when the problem's
 * workspace (tpmg_mg_workspace_size) exceeds the array, TPMG_ERR_ARG, and
 * tpmg_solve's statuses. */
#define TPMG_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
tpmg_status tpmg_solve_noalloc(const tpmg_op* op, const tpmg_mg_params* params, void* hip_stream, const double* d_f,
                               double* d_u, double rtol, int maxit, tpmg_solve_info* info);

void tpmg_grid_destroy(tpmg_grid* g);
void tpmg_op_destroy(tpmg_op* op);
void tpmg_mg_destroy(tpmg_mg* mg);

const char* tpmg_status_string(tpmg_status s);
const char* tpmg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TPMG_H */
