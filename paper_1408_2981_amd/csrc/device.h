// Device-side views and kernel launchers of the TPMG library (gfx950).
//
// Vector layout on the device: tiles of 64 columns; value (T, k) lives at
// (T / 64) * 64 * nz + k * 64 + T % 64. One wave of 64 lanes owns one tile,
// one lane one column, so every level of a tile is one contiguous,
// coalesced 64-element row, and each tile is one contiguous chunk of HBM.
// Per-column data (coefficients, neighbours, weights) is stored SoA with
// the column count padded to a multiple of 64; padding columns are inert
// (beta = 1, no couplings, neighbour = self) and their vector entries stay
// zero.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace tpmg {

constexpr int kTile = 64;
// waves per block of the stencil kernels (SpMV, residual + restriction)
constexpr int kStencilWaves = 4;
// LDS of a scan-smoother block of `waves` waves in precision prec: eight
// summary slots and a two-tile neighbour exchange slice per wave
constexpr size_t scan_lds_bytes(int waves, int prec) {
  return static_cast<size_t>(waves) * (8 + 2) * kTile * static_cast<size_t>(prec);
}

// Where the line smoother keeps a column while it solves it.
enum SmootherKind {
  kSmScan = 0,    // registers, the column split over the waves of a workgroup and joined by block scans
  kSmLds = 1,     // residual and Thomas factors staged in LDS, one wave runs the recurrence
  kSmGlobal = 2,  // Thomas factors in global scratch (any nz)
};

// Launch configuration of one level, chosen at setup (defaults, caller
// overrides or timed trials). The smoother choice changes the rounding of the
// column solve; the stencil chunks only change how work is dealt to waves.
struct LevelTune {
  int smoother = kSmScan;
  int scan_levels = 8;   // levels per wave of the scan smoother: 4, 8 or 16 (nz <= 16 * scan_levels)
  int chunk_rr = 0;      // levels per wave of residual + restriction from this level (0: heuristic)
  int chunk_pr = 0;      // levels per wave of prolongation + correction into this level
  int chunk_spmv = 0;    // levels per wave of the FP64 operator (finest level)
};

// One grid level as the kernels see it. Pointers are of the precision the
// launcher is called with (double or float).
struct LevelView {
  int n = 0;       // real columns
  int npad = 0;    // padded to a multiple of 64
  int nz = 0;
  const int32_t* nbr = nullptr;   // [3][npad]
  // where a stencil kernel finds neighbour j of a column at the level its
  // wave holds: byte j of code[col] is the neighbour's lane in the column's
  // own tile (< 64), or 64 + its slot in the tile's halo, the list of
  // out-of-tile neighbour columns halo[64 t + slot] (unused slots: the slot's
  // own column)
  const int32_t* code = nullptr;  // [npad]
  const int32_t* halo = nullptr;  // [npad]
  const void* beta_h = nullptr;   // [npad]
  const void* ar_h = nullptr;     // [npad]
  const void* as_h = nullptr;     // [3][npad]
  const void* pw = nullptr;       // [3][npad] prolongation weights into this level
  const void* beta_v = nullptr;   // [nz]
  const void* as_v = nullptr;     // [nz]
  const void* ar_v = nullptr;     // [nz+1]
  // tiled [npad * nz]: the margin s_k of every column's Thomas factorisation
  // (fixed by the operator, factorised once at setup); nullptr: the scan
  // smoother forms the margins it needs itself
  const void* margin = nullptr;
  // profiles that do not factorise (Section 4.2): pm = 0 factorised (the
  // column scalars and vertical vectors above); 1 radial couplings per (T, k)
  // from far, the rest factorised (TPMG^(partial)); 2 every coefficient per
  // (T, k): fb (beta^, tiled like a vector), fas (alphaS^, three such planes,
  // one per neighbour j), far (alphar^ at the nz + 1 radial faces, tiled with
  // nz + 1 rows per tile). pm > 0 runs the scan smoother with 8 or 16 levels
  // per wave only, and no batched kernels.
  int pm = 0;
  const void* fb = nullptr;
  const void* far = nullptr;
  const void* fas = nullptr;
  // pm 3: pm 2 plus the vertical advection, omega^2 times the coefficients
  // of every cell's lower (fxl) and upper (fxu) face, tiled like a vector;
  // row k then couples to the cell below by alphar^_k - fxl_k and to the
  // cell above by alphar^_{k+1} + fxu_k
  const void* fxl = nullptr;
  const void* fxu = nullptr;
  // multicolour block-SOR (Section 5: block-SOR; colours relaxed one after
  // another): the colour of every column ([npad], padding -1) and the colour
  // a smoother pass relaxes; pass < 0 relaxes every column (block-Jacobi).
  // Columns a pass does not relax are copied from u_in (0 from a zero guess).
  const int8_t* colour = nullptr;
  int pass = -1;
  LevelTune tune;
};

// Device scalars of the flexible CG recurrence.
// Single solves keep the last kDirSlots search directions and their step
// lengths, and add them to x every kDirSlots iterations and at the end.
constexpr int kDirSlots = 8;

struct FcgScalars {
  double alpha_hist[kDirSlots];   // alpha of iteration i at i % kDirSlots (single solves)
  double rz;      // <r, z>
  double pq;      // <p, A p>
  double alpha;
  double beta;
  double rr;      // <r, r>
  double ff;      // <f, f>
  double rtol;    // stopping tolerance (set at kFinInit)
  double rr0;     // <r_0, r_0> (set at kFinInit)
  double div2;    // divergence bound on <r, r> / <r_0, r_0> (set at kFinInit)
  double w;       // BiCGStab: the stabilising step omega (rz holds rho)
  int status;     // 0 ok, 1 breakdown, 2 divergence
  int done;       // converged or broken down: batched launches skip the problem
  int iters;      // completed iterations (maintained on the device)
  int seq;        // records published so far (single solves)
  int flushed;    // iterations whose alpha p is in x (single solves)
};

// What a single solve's host loop needs of one FCG iteration, published by
// the iteration's last kernel into pinned host memory (a ring of kRecords
// slots, slot seq % kRecords), so that the host can wait for iteration k while
// iteration k+1 is already queued.
struct FcgRecord {
  double rr;
  int status;
  int done;
  int iters;
  int seq;        // written last: the host sets -1 before a solve
  double ff;      // ||f||^2 (the record of kFinInit, seq 0)
};
constexpr int kRecords = 4;
// A solve stops as diverged once ||r_k|| > 1e3 ||r_0|| unless told otherwise.
constexpr double kDefaultDiv2 = 1e6;

// Operations of one FCG iteration, as grouped by the batched executor.
enum OpKind { kOpSmooth = 0, kOpRestrict, kOpProlong, kOpSpmv, kOpPupdate, kOpUpdate, kOpFinalize, kOpPupdateRing,
              kOpSpmvRing, kOpRupdate, kOpSpmvPRing };

// One problem's part of a grouped launch (device memory, sorted by start).
struct Seg {
  int start;        // first block of this segment in the grouped grid (multiple of 8)
  int nblocks;      // blocks of the problem's own launch (reduction width for finalize)
  int chunk;        // levels per wave of the stencil kernels
  int site;         // finalize site
  LevelView L;      // level (the fine level for restriction and prolongation)
  LevelView C;      // coarse level (restriction, prolongation)
  const void* in0;  // smoother: f; restriction: f; prolongation: e; spmv: x; pupdate: z; update: p
  const void* in1;  // smoother: u_in; restriction: u; update: q
  void* out0;       // smoother: u_out; restriction: f_coarse; prolongation, spmv: y; pupdate: p; update: x
  void* out1;       // smoother: fcopy; update: r
  const double* q;  // smoother with fused dots
  double* partials;
  FcgScalars* sc;
  size_t len;       // BLAS-1 vector length
  double* aux;      // direction update inside the operator: the direction ring
};

// A grouped launch over the segments of several problems.
struct BatchLaunch {
  int kind;         // OpKind
  int prec;         // 8 or 4 (V-cycle precision)
  int scan_levels;  // smoother: levels per wave (the same for every segment of the launch)
  int chunk;        // residual + restriction, operator: the levels-per-wave instance of every
                    // segment (1, 2, 4, 8, 16), or 0 for the per-segment runtime chunk
  bool f_double, out_double, zero, fcopy, dots;   // smoother variant
  int pm;           // profile mode of every segment's level (0, 1, 2; LevelView::pm)
  double omega;
  unsigned grid, block;
  size_t lds;
  const Seg* segs;  // device
  int nseg;
};
hipError_t launch_batched(const BatchLaunch& b, hipStream_t s);

constexpr int kRedBlocks = 1024;   // fixed grid of the BLAS-1 reductions
constexpr int kRedThreads = 256;
constexpr int kFinThreads = 1024;  // one-block finalisation of the partial sums

// Where a reduction's last block applies its sums to the FCG scalars.
enum FinalizeSite { kFinInit = 0, kFinAlpha = 1, kFinRR = 2, kFinBeta = 3, kFinNone = 4 };

int stencil_chunk(int npad, int nz);   // heuristic levels per wave of the stencil kernels
int effective_chunk(int tuned, int npad, int nz);   // tuned if set, else the heuristic
size_t stencil_blocks(int npad, int nz, int chunk);  // blocks of 256 threads of a stencil kernel
constexpr int kScanWavesMax = 16;
int scan_waves(int nz, int scan_levels);   // waves per tile of the scan smoother
// whether the smoother kind (with scan_levels for kSmScan) can run a level of nz
// levels in precision prec (LDS limits included)
bool smoother_fits(int kind, int scan_levels, int nz, int prec);
LevelTune default_tune(int nz, int prec);
unsigned pupdate_blocks(size_t len);      // blocks of the p-update kernel

// All launchers enqueue on `s` and return hipGetLastError().
// prec: 8 = double, 4 = float (the V-cycle precision of the level data).
// Reductions write two partial sums per block to `partials`; a one-block
// finalize kernel then sums them in a fixed order and applies them to the
// FCG scalars at `site`.

// mode 0: y = A x (partials <x, y>, e.g. site kFinAlpha). mode 1: y = b - A x
// (partials <y, y>, <b, b>; site kFinInit), with y32 non-NULL also its FP32
// rounding. FP64; x and y must not alias.
// div2 (kFinInit): the squared divergence bound, see FcgScalars::div2.
hipError_t launch_spmv64(const LevelView& L, int mode, const double* x, const double* b, double* y,
                         double* partials, int site, FcgScalars* sc, hipStream_t s, double rtol = 0.0,
                         float* y32 = nullptr, FcgRecord* ring = nullptr, double div2 = kDefaultDiv2);
// one-block finalisation of nblocks partials at `site` (rtol used at kFinInit)
hipError_t launch_finalize(int site, const double* partials, int nblocks, FcgScalars* sc, double rtol, hipStream_t s);

// One damped block-Jacobi sweep with the Thomas solve per column:
// u_out = u_in + omega A_T^-1 (f - A u_in), with the kernel L.tune selects.
// zero_guess: u_in taken as 0 (not read). f_double: f is FP64 (else of
// precision prec); out_double: u_out is FP64. fcopy (optional): receives f
// rounded to prec. sd, sc: scratch vectors of the level size (used only by
// the global-scratch kernel). q non-NULL (FP64 f and output and the scan
// kernel required): also reduces <u_out, q> and <u_out, f> and applies them
// at site kFinBeta. hipErrorInvalidValue if the tuned kernel cannot run.
hipError_t launch_smooth(const LevelView& L, int prec, const void* f, bool f_double, const void* u_in,
                         bool zero_guess, void* u_out, bool out_double, void* fcopy, void* sd, void* sc,
                         double omega, hipStream_t s, const double* q = nullptr, double* partials = nullptr,
                         FcgScalars* scal = nullptr);

// Largest dynamic LDS a workgroup may use (set once from the device
// properties); bounds the LDS-staged smoother.
hipError_t set_max_lds(size_t bytes);

// f_coarse[P] = sum_{i<4} (f - A u)[4P + i] on the fine level L.
hipError_t launch_residual_restrict(const LevelView& L, const LevelView& C, int prec, const void* f,
                                    const void* u, void* f_coarse, hipStream_t s);

// u_fine += P e_coarse (linear interpolation), in place.
hipError_t launch_prolong_add(const LevelView& F, const LevelView& C, int prec, const void* e_coarse,
                              void* u_fine, hipStream_t s);

// Single solves with the direction ring (kDirSlots vectors of len at
// ring); iteration k = iters, each launch skipped once done:
//   pupdate_ring: p_k = z + beta p_{k-1} into slot k % kDirSlots; when k is a
//     positive multiple of kDirSlots, first x += alpha p of the kDirSlots
//     iterations before k (in order, the slots about to be reused);
//   spmv_ring: q = A p_k (site kFinAlpha, which also records alpha_k);
//   rupdate: r -= alpha q (site kFinRR); with r32 non-NULL also r32 = the
//   FP32 rounding of the new r;
// flush, after the last iteration: x += alpha p of the iterations not yet
// added.
hipError_t launch_pupdate_ring(const void* z, bool z_double, double* ring, double* x, FcgScalars* sc, size_t len,
                               hipStream_t s);
hipError_t launch_spmv_ring(const LevelView& L, const double* ring, size_t len, double* q, double* partials,
                            FcgScalars* sc, hipStream_t s);
hipError_t launch_rupdate(double* r, const double* q, FcgScalars* sc, size_t len, double* partials, FcgRecord* ring,
                          hipStream_t s, float* r32 = nullptr);

// pupdate_ring and spmv_ring in one launch (the same bits), for the operator
// chunks that have an instance (spmv_pring_fits).
bool spmv_pring_fits(const LevelView& L);
// (site kFinNone: the operator kernel alone, no finalize; for timing)
hipError_t launch_spmv_pring(const LevelView& L, const void* z, bool z_double, double* ring, size_t len, double* x,
                             double* q, double* partials, FcgScalars* sc, hipStream_t s, int site = kFinAlpha);
hipError_t launch_flush(double* x, const double* ring, const FcgScalars* sc, size_t len, hipStream_t s);

// margin[k] = s_k of every column of level L64 (FP64 view): s_0 = e_0,
// s_k = e_k + l_k s_{k-1} / (s_{k-1} + l_k), computed in FP64 and stored in
// precision prec (tiled like the level's vectors).
hipError_t launch_margins(const LevelView& L64, int prec, void* margin, hipStream_t s);

// x += alpha p, r -= alpha q (site kFinRR: <r, r>), FP64, padded length len.
// Skipped once the scalars say done (an iteration queued after convergence
// leaves x, r and the scalars alone); with ring != nullptr the finalize then
// publishes the iteration's record.
hipError_t launch_fcg_update(double* x, double* r, const double* p, const double* q, FcgScalars* sc, size_t len,
                             double* partials, FcgRecord* ring, hipStream_t s);
// <z, q>, <z, r> (site kFinBeta), for nz beyond the fused smoother's range.
hipError_t launch_dots(const double* z, const double* q, const double* r, size_t len, double* partials,
                       FcgScalars* sc, hipStream_t s);
// BiCGStab (the outer solver for operators with vertical advection): the
// scalar stages applied by launch_krylov_finalize to the sums of the
// preceding reduction (s0, s1):
//   kKInit  (no sums): rho = rr (the shadow residual is r_0), alpha = w = 1,
//           beta = 0;
//   kKAlpha s0 = <r^, v>: alpha = rho / s0;
//   kKOmega s0 = <t, s>, s1 = <t, t>: w = s0 / s1;
//   kKRho   s0 = <r^, r>, s1 = <r, r>: beta = (s0 / rho)(alpha / w), rho = s0,
//           rr = s1;
// each sets status 1 on a zero or non-finite divisor.
enum KrylovStage { kKInit = 10, kKAlpha = 11, kKOmega = 12, kKRho = 13 };
// partials <a, b>, <c, d> over len (fixed grid, deterministic)
hipError_t launch_dots2(const double* a, const double* b, const double* c, const double* d, size_t len,
                        double* partials, hipStream_t s);
hipError_t launch_krylov_finalize(int stage, const double* partials, FcgScalars* sc, hipStream_t s);
// p = r + beta (p - w v)
hipError_t launch_bicg_p(const double* r, double* p, const double* v, const FcgScalars* sc, size_t len,
                         hipStream_t s);
// r -= alpha v (r then holds s)
hipError_t launch_bicg_s(double* r, const double* v, const FcgScalars* sc, size_t len, hipStream_t s);
// x += alpha y + w z, r = s - w t (r holds s on entry); partials <rh, r>, <r, r>
hipError_t launch_bicg_x(double* x, double* r, const double* y, const double* z, const double* t, const double* rh,
                         const FcgScalars* sc, size_t len, double* partials, hipStream_t s);

// p = z + beta p (beta from the scalars), in place; z FP64 or FP32.
hipError_t launch_pupdate(const void* z, bool z_double, double* p, const FcgScalars* sc, size_t len, hipStream_t s);
hipError_t launch_add(double* x, const double* y, size_t len, hipStream_t s);   // x += y
hipError_t launch_fill(void* p, size_t bytes, hipStream_t s);   // zero fill (graph-safe)

// Finest grid of a set-up solver, for the kernels that read its vectors
// directly (the learned initial guess).
struct FineGrid {
  int n = 0, npad = 0, nz = 0;
  const int32_t* nbr = nullptr;   // [3][npad]
  // where a stencil kernel finds neighbour j of a column at the level its
  // wave holds: byte j of code[col] is the neighbour's lane in the column's
  // own tile (< 64), or 64 + its slot in the tile's halo, the list of
  // out-of-tile neighbour columns halo[64 t + slot] (unused slots: the slot's
  // own column)
  const int32_t* code = nullptr;  // [npad]
  const int32_t* halo = nullptr;  // [npad]
  hipStream_t stream = nullptr;
};

// layout conversion of a finest-grid FP64 vector
hipError_t launch_pack(const double* cm, double* tiled, int n, int npad, int nz, hipStream_t s);
hipError_t launch_unpack(const double* tiled, double* cm, int n, int npad, int nz, hipStream_t s);

}  // namespace tpmg

struct tpmg_mg;
// Finest grid of mg (defined next to the solver's handle).
bool tpmg_fine_grid(const tpmg_mg* mg, tpmg::FineGrid* out);
// Sets the thread's message returned by tpmg_last_error().
void tpmg_set_last_error(const char* msg);
// One line-relaxation sweep on mg's finest grid in FP64, u_out = u_in +
// omega A_T^-1 (f - A u_in) (tiled vectors, u_in and u_out distinct; sd, sc:
// FP64 scratch vectors of the finest length), enqueued on s.
hipError_t tpmg_relax_finest(const tpmg_mg* mg, const double* f, const double* u_in, double* u_out, double* sd,
                             double* sc, double omega, hipStream_t s);
