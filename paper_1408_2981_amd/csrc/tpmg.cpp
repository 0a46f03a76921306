// C ABI of the TPMG library: argument checking, host handles, device
// setup (workspace carving and coefficient upload), the V-cycle schedule
// (Algorithm 1) and the flexible-CG driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cctype>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <fstream>
#include <functional>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/tpmg.h"
#include "device.h"
#include "host.h"

struct tpmg_grid {
  tpmg::Grid g;
};
struct tpmg_op {
  tpmg::Operator op;
};

namespace {

thread_local std::string g_last_error;

tpmg_status fail(tpmg_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

#define TPMG_HIP(call)                                                                              \
  do {                                                                                              \
    hipError_t e_ = (call);                                                                         \
    if (e_ != hipSuccess)                                                                           \
      return fail(TPMG_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));              \
  } while (0)

int pad64(int n) { return (n + tpmg::kTile - 1) / tpmg::kTile * tpmg::kTile; }

// Bump allocator over the caller's workspace; with base == nullptr it only
// measures.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  void* take(size_t bytes) {
    off = (off + 255) / 256 * 256;
    void* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
};

struct DevLevel {
  int n = 0, npad = 0;
  int32_t* nbr = nullptr;
  int32_t* code = nullptr;             // neighbour location codes (LevelView::code)
  int32_t* halo = nullptr;             // per-tile out-of-tile neighbour lists
  void* bh[2] = {nullptr, nullptr};   // [0] double, [1] float
  void* arh[2] = {nullptr, nullptr};
  void* ash[2] = {nullptr, nullptr};
  void* pw[2] = {nullptr, nullptr};
  void* f = nullptr;                   // right-hand side (coarse levels; precision of the V-cycle)
  void* u[2] = {nullptr, nullptr};     // ping-pong iterates
  void* margin[2] = {nullptr, nullptr};   // Thomas margins, [0] double, [1] float (tiled)
  // coefficients of profiles that do not factorise ([0] double, [1] float):
  // beta^ and the three alphaS^ planes tiled like a vector, alphar^ with
  // nz + 1 rows per tile
  void* fb[2] = {nullptr, nullptr};
  void* far[2] = {nullptr, nullptr};
  void* fas[2] = {nullptr, nullptr};
  // vertical advection: omega^2 times the coefficients of a cell's lower and
  // upper face, tiled like a vector
  void* fxl[2] = {nullptr, nullptr};
  void* fxu[2] = {nullptr, nullptr};
  // multicolour block-SOR: the colour of every column (padding -1) and the
  // number of colours
  int8_t* colour = nullptr;
  int ncol = 0;
};

}  // namespace

struct tpmg_mg {
  int nlev = 0, nz = 0, n_fine = 0, npad_fine = 0;
  int nu_pre = 2, nu_post = 2, nu_coarse = 1;
  double omega = 2.0 / 3.0;
  bool fp32 = false, use_graph = false;
  // profile mode of the V-cycle's levels (tpmg::LevelView::pm) and whether
  // the operator of the equation has profiles that do not factorise
  int pm = 0;
  bool full_outer = false;
  bool adv = false;                      // the operator has vertical advection (not symmetric)
  bool sor = false;                      // multicolour block-SOR smoother (else block-Jacobi)
  hipStream_t stream = nullptr;
  std::vector<DevLevel> lv;
  void* bv[2] = {nullptr, nullptr};
  void* asv[2] = {nullptr, nullptr};
  void* arv[2] = {nullptr, nullptr};
  void* fcopy = nullptr;                 // FP32 copy of the finest right-hand side
  void* sd = nullptr;                    // Thomas scratch
  void* sc = nullptr;
  double *r = nullptr, *p = nullptr, *q = nullptr, *z = nullptr;   // FCG vectors (tiled, FP64)
  double* dirs = nullptr;                // single solves: the last kDirSlots directions
  double* partials = nullptr;
  tpmg::FcgScalars* scal = nullptr;
  tpmg::FcgScalars* h_scal = nullptr;    // pinned host mirror
  tpmg::FcgRecord* ring = nullptr;       // pinned ring of iteration records (host address)
  tpmg::FcgRecord* ring_dev = nullptr;   // the same memory as the device addresses it
  tpmg::FcgRecord* ring_ws = nullptr;    // a device-memory ring in the workspace (handles without pinned memory)
  bool pinned = true;                    // ring and h_scal in pinned host memory
  size_t len = 0;                        // padded finest vector length
  int max_partial_blocks = 0;
  // events of the per-phase timers (created on first use, reused)
  std::vector<hipEvent_t> tev;
  // graph of one FCG iteration for the solution vector graph_x
  hipGraphExec_t graph = nullptr;
  double* graph_x = nullptr;
  // launch configuration per level, and the cost of choosing it
  std::vector<tpmg::LevelTune> tune;
  int tune_trials = 0;
  double tune_ms = 0.0;

  tpmg::LevelView view(int l) const {
    const DevLevel& d = lv[l];
    const int i = fp32 ? 1 : 0;
    tpmg::LevelView v;
    v.n = d.n;
    v.npad = d.npad;
    v.nz = nz;
    v.nbr = d.nbr;
    v.code = d.code;
    v.halo = d.halo;
    v.beta_h = d.bh[i];
    v.ar_h = d.arh[i];
    v.as_h = d.ash[i];
    v.pw = d.pw[i];
    v.beta_v = bv[i];
    v.as_v = asv[i];
    v.ar_v = arv[i];
    v.margin = d.margin[i];
    v.pm = pm;
    v.fb = d.fb[i];
    v.far = d.far[i];
    v.fas = d.fas[i];
    v.fxl = d.fxl[i];
    v.fxu = d.fxu[i];
    v.colour = d.colour;
    if (!tune.empty()) v.tune = tune[l];
    return v;
  }
  // the finest grid's FP64 operator of the equation itself (the outer
  // Krylov method's), every coefficient per (T, k) when the profiles do not
  // factorise
  tpmg::LevelView view_outer() const {
    tpmg::LevelView v = view64(nlev - 1);
    v.pm = adv ? 3 : full_outer ? 2 : 0;
    return v;
  }
  tpmg::LevelView view64(int l) const {
    const DevLevel& d = lv[l];
    tpmg::LevelView v;
    v.n = d.n;
    v.npad = d.npad;
    v.nz = nz;
    v.nbr = d.nbr;
    v.code = d.code;
    v.halo = d.halo;
    v.beta_h = d.bh[0];
    v.ar_h = d.arh[0];
    v.as_h = d.ash[0];
    v.pw = d.pw[0];
    v.beta_v = bv[0];
    v.as_v = asv[0];
    v.ar_v = arv[0];
    v.margin = d.margin[0];
    v.pm = pm;
    v.fb = d.fb[0];
    v.far = d.far[0];
    v.fas = d.fas[0];
    v.fxl = d.fxl[0];
    v.fxu = d.fxu[0];
    v.colour = d.colour;
    if (!tune.empty()) v.tune = tune[l];
    return v;
  }
};

namespace {

// Lays out every device buffer of (op, params) on the carver.
void carve(tpmg_mg& m, const tpmg::Operator& op, Carver& cv) {
  const int nz = op.nz;
  const size_t s = m.fp32 ? 4 : 8;
  m.lv.assign(op.levels.size(), DevLevel());
  for (size_t l = 0; l < op.levels.size(); ++l) {
    DevLevel& d = m.lv[l];
    d.n = op.levels[l].n;
    d.npad = pad64(d.n);
    const size_t np = d.npad;
    d.nbr = static_cast<int32_t*>(cv.take(3 * np * sizeof(int32_t)));
    d.code = static_cast<int32_t*>(cv.take(np * sizeof(int32_t)));
    d.halo = static_cast<int32_t*>(cv.take(np * sizeof(int32_t)));
    for (int i = 0; i < 2; ++i) {
      const size_t es = i == 0 ? 8 : 4;
      d.bh[i] = cv.take(np * es);
      d.arh[i] = cv.take(np * es);
      d.ash[i] = cv.take(3 * np * es);
      d.pw[i] = l > 0 ? cv.take(3 * np * es) : nullptr;
    }
    const size_t vec = np * nz * s;
    const bool finest = l + 1 == op.levels.size();
    d.f = finest ? nullptr : cv.take(vec);
    d.u[0] = cv.take(vec);
    d.u[1] = cv.take(vec);
    // margins in the V-cycle's precision; FP64 ones also on the finest level,
    // whose FP64 view serves the relaxation after a learned guess
    d.margin[1] = m.fp32 ? cv.take(np * nz * 4) : nullptr;
    d.margin[0] = (!m.fp32 || finest) ? cv.take(np * nz * 8) : nullptr;
    if (m.sor) d.colour = static_cast<int8_t*>(cv.take(np));
    if (op.full)
      for (int i = 0; i < (m.fp32 ? 2 : 1); ++i) {
        const size_t es = i == 0 ? 8 : 4;
        d.fb[i] = cv.take(np * nz * es);
        d.far[i] = cv.take(np * (nz + 1) * es);
        d.fas[i] = cv.take(3 * np * nz * es);
        if (op.adv) {
          d.fxl[i] = cv.take(np * nz * es);
          d.fxu[i] = cv.take(np * nz * es);
        }
      }
  }
  for (int i = 0; i < 2; ++i) {
    const size_t es = i == 0 ? 8 : 4;
    m.bv[i] = cv.take(nz * es);
    m.asv[i] = cv.take(nz * es);
    m.arv[i] = cv.take((nz + 1) * es);
  }
  const size_t fine_len = static_cast<size_t>(pad64(op.levels.back().n)) * nz;
  m.fcopy = m.fp32 ? cv.take(fine_len * 4) : nullptr;
  m.sd = cv.take(fine_len * s);
  m.sc = cv.take(fine_len * s);
  m.r = static_cast<double*>(cv.take(fine_len * 8));
  m.p = static_cast<double*>(cv.take(fine_len * 8));
  m.dirs = static_cast<double*>(cv.take(fine_len * 8 * tpmg::kDirSlots));
  m.q = static_cast<double*>(cv.take(fine_len * 8));
  m.z = static_cast<double*>(cv.take(fine_len * 8));
  // reductions: stencil blocks of the finest grid (at most: one level per
  // wave), the BLAS grid, or one block per tile (the smoother with fused dots)
  const size_t fine_npad = pad64(op.levels.back().n);
  m.max_partial_blocks = static_cast<int>(std::max(
      {static_cast<size_t>(tpmg::kRedBlocks), tpmg::stencil_blocks(static_cast<int>(fine_npad), nz, 1), fine_npad / 64}));
  m.partials = static_cast<double*>(cv.take(2 * static_cast<size_t>(m.max_partial_blocks) * 8));
  m.scal = static_cast<tpmg::FcgScalars*>(cv.take(sizeof(tpmg::FcgScalars)));
  m.ring_ws = static_cast<tpmg::FcgRecord*>(cv.take(tpmg::kRecords * sizeof(tpmg::FcgRecord)));
  m.len = fine_len;
}

// Neighbour location codes and tile halos (see LevelView::code) from the
// padded [3][npad] neighbour table. A tile's halo lists its distinct
// out-of-tile neighbour columns in order of first use; false if a tile has
// more than 64 (the cell ordering keeps a tile a compact patch: a refined
// icosahedron's tile of 64 cells is the patch of one cell three refinements
// coarser).
bool tile_halos(const std::vector<int32_t>& nb, int npad, std::vector<int32_t>& code, std::vector<int32_t>& halo) {
  code.assign(static_cast<size_t>(npad), 0);
  halo.assign(static_cast<size_t>(npad), 0);
  for (int t = 0; t < npad / tpmg::kTile; ++t) {
    std::vector<int32_t> h;
    for (int lane = 0; lane < tpmg::kTile; ++lane) {
      const int col = t * tpmg::kTile + lane;
      uint32_t packed = 0;
      for (int j = 0; j < 3; ++j) {
        const int32_t n = nb[static_cast<size_t>(j) * npad + col];
        uint32_t cj;
        if (n / tpmg::kTile == t) {
          cj = static_cast<uint32_t>(n % tpmg::kTile);
        } else {
          auto it = std::find(h.begin(), h.end(), n);
          if (it == h.end()) {
            if (h.size() == static_cast<size_t>(tpmg::kTile)) return false;
            h.push_back(n);
            it = h.end() - 1;
          }
          cj = static_cast<uint32_t>(tpmg::kTile + (it - h.begin()));
        }
        packed |= cj << (8 * j);
      }
      code[col] = static_cast<int32_t>(packed);
    }
    for (int slot = 0; slot < tpmg::kTile; ++slot)
      halo[t * tpmg::kTile + slot] = slot < static_cast<int>(h.size()) ? h[slot] : t * tpmg::kTile + slot;
  }
  return true;
}

tpmg_status check_params(const tpmg_mg_params* p) {
  if (!p) return fail(TPMG_ERR_ARG, "params is NULL");
  if (p->nu_pre < 1 || p->nu_post < 1 || p->nu_coarse < 1)
    return fail(TPMG_ERR_ARG, "nu_pre, nu_post and nu_coarse must be >= 1");
  if (!(p->omega_relax > 0.0) || !(p->omega_relax < 2.0)) return fail(TPMG_ERR_ARG, "omega_relax must be in (0, 2)");
  if (p->n_levels < 0) return fail(TPMG_ERR_ARG, "n_levels must be >= 0");
  if (p->autotune < 0 || p->autotune > 2) return fail(TPMG_ERR_ARG, "autotune must be 0, 1 or 2");
  if (p->smoother < 0 || p->smoother > 3) return fail(TPMG_ERR_ARG, "smoother must be 0 (auto), 1, 2 or 3");
  if (p->scan_levels != 0 && p->scan_levels != 4 && p->scan_levels != 8 && p->scan_levels != 16)
    return fail(TPMG_ERR_ARG, "scan_levels must be 0, 4, 8 or 16");
  if (p->scan_levels != 0 && p->smoother > 1)
    return fail(TPMG_ERR_ARG, "scan_levels applies to the scan smoother only");
  if (p->stencil_chunk < 0 || p->stencil_chunk > 256) return fail(TPMG_ERR_ARG, "stencil_chunk must be in 0..256");
  if (p->precond_profiles < 0 || p->precond_profiles > 2)
    return fail(TPMG_ERR_ARG, "precond_profiles must be 0, 1 or 2");
  if (p->smoother_order < 0 || p->smoother_order > 1) return fail(TPMG_ERR_ARG, "smoother_order must be 0 or 1");
  if (p->tile_cols != 0 && p->tile_cols != tpmg::kTile)
    return fail(TPMG_ERR_ARG, "tile_cols must be 0 or 64 (one lane per column, one wavefront per tile)");
  return TPMG_OK;
}

template <typename T>
std::vector<T> padded(const std::vector<double>& src, int n, int npad, int comps, double fill) {
  // src is [n][comps] cell-major; result is [comps][npad] SoA
  std::vector<T> out(static_cast<size_t>(npad) * comps, static_cast<T>(fill));
  for (int c = 0; c < comps; ++c)
    for (int t = 0; t < n; ++t) out[static_cast<size_t>(c) * npad + t] = static_cast<T>(src[static_cast<size_t>(t) * comps + c]);
  return out;
}

// cell-major [n][comps][rows] -> comps tiled planes (value (T, k) of plane
// c at c npad rows + (T / 64) 64 rows + k 64 + T % 64); padding columns fill
template <typename T>
std::vector<T> tiled(const std::vector<double>& cm, int n, int npad, int comps, int rows, double fill) {
  std::vector<T> out(static_cast<size_t>(comps) * npad * rows, static_cast<T>(fill));
  for (int c = 0; c < comps; ++c)
    for (int t = 0; t < n; ++t)
      for (int k = 0; k < rows; ++k)
        out[static_cast<size_t>(c) * npad * rows + static_cast<size_t>(t / tpmg::kTile) * tpmg::kTile * rows +
            static_cast<size_t>(k) * tpmg::kTile + t % tpmg::kTile] =
            static_cast<T>(cm[(static_cast<size_t>(t) * comps + c) * rows + k]);
  return out;
}

template <typename T>
hipError_t upload(void* dst, const std::vector<T>& v, hipStream_t s) {
  return hipMemcpyAsync(dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

// ---- V-cycle (Algorithm 1) and the FCG iteration as lists of operations -----
//
// Each operation carries its place in the lockstep schedule (order), so the
// same list serves a single solve (executed in program order) and a batch of
// solves (operations of all problems with the same order become one grouped
// launch).
struct Op {
  int order[4] = {0, 0, 0, 0};
  int kind = tpmg::kOpSmooth;
  int prec = 8;
  bool f_double = false, zero = false, out_double = false, fcopy = false, dots = false;
  double omega = 0.0;
  tpmg::LevelView L, C;
  const void* in0 = nullptr;
  const void* in1 = nullptr;
  void* out0 = nullptr;
  void* out1 = nullptr;
  const double* q = nullptr;
  double* partials = nullptr;
  tpmg::FcgScalars* sc = nullptr;
  int site = tpmg::kFinNone;
  size_t len = 0;
  void* scratch_d = nullptr;   // fallback smoother only
  void* scratch_c = nullptr;
  tpmg::FcgRecord* ring = nullptr;   // update of a single solve: record ring
  double* aux = nullptr;             // single solves: the direction ring
};

bool order_less(const Op& a, const Op& b) {
  for (int i = 0; i < 4; ++i)
    if (a.order[i] != b.order[i]) return a.order[i] < b.order[i];
  return false;
}

// Level l > 0: nu_pre sweeps (the first from a zero guess), residual +
// restriction to level l-1, recursion from a zero guess, prolongation +
// correction, nu_post sweeps. Level 0: nu_coarse sweeps from zero. In the
// mixed mode every level is FP32: the first finest sweep reads the FP64
// residual and keeps an FP32 copy of it, the last writes FP64 z (and, when
// q_dots is given, also forms <z, q> and <z, r>, applied at kFinBeta).
// With r32_ready (mixed single solves) the FP32 rounding of r_in is already
// in the copy (written by the r update): the first finest sweep reads it.
void vcycle_ops(tpmg_mg& m, const double* r_in, void* z_out, const double* q_dots, tpmg::FcgScalars* sc,
                std::vector<Op>& ops, bool z_float = false, bool r32_ready = false) {
  const int L = m.nlev - 1;
  const int prec = m.fp32 ? 4 : 8;
  std::vector<int> cur(m.nlev, 0);
  auto rhs = [&](int l) -> const void* {
    if (l < L) return m.lv[l].f;
    return m.fp32 ? static_cast<const void*>(m.fcopy) : static_cast<const void*>(r_in);
  };
  auto sweep = [&](int o0, int o1, int o2, int o3, int l, const void* f, bool f_double, bool zero, void* out,
                   bool out_double, bool fcopy, bool dots, int pass = -1, const void* u_in = nullptr) {
    Op op;
    op.order[0] = o0;
    op.order[1] = o1;
    op.order[2] = o2;
    op.order[3] = o3;
    op.kind = tpmg::kOpSmooth;
    op.prec = prec;
    op.f_double = f_double;
    op.zero = zero;
    op.out_double = out_double;
    op.fcopy = fcopy;
    op.dots = dots;
    op.omega = m.omega;
    op.L = m.view(l);
    op.L.pass = pass;
    op.in0 = f;
    op.in1 = u_in ? u_in : m.lv[l].u[cur[l]];
    op.out0 = out;
    op.out1 = fcopy ? m.fcopy : nullptr;
    op.q = dots ? q_dots : nullptr;
    op.partials = m.partials;
    op.sc = sc;
    op.site = dots ? tpmg::kFinBeta : tpmg::kFinNone;
    op.scratch_d = m.sd;
    op.scratch_c = m.sc;
    ops.push_back(op);
  };
  // A smoother sweep of level l: block-Jacobi in one pass; multicolour
  // block-SOR in one pass per colour (ascending before the coarse-grid
  // correction, descending after), each pass reading the previous one's
  // output. final_out (or the level's other buffer) receives the sweep's
  // result; the level's current buffer index follows it.
  auto smooth_sweep = [&](int o0, int o1, int o2, int k, int l, const void* f, bool f_double, bool zero,
                          void* final_out, bool out_double, bool fcopy, bool dots, bool post) {
    if (!m.sor) {
      void* out = final_out ? final_out : m.lv[l].u[zero ? cur[l] : 1 - cur[l]];
      sweep(o0, o1, o2, k, l, f, f_double, zero, out, out_double, fcopy, dots);
      if (!zero && !final_out) cur[l] = 1 - cur[l];
      return;
    }
    const int nc = m.lv[l].ncol;
    int src = cur[l];
    for (int j = 0; j < nc; ++j) {
      const bool first_pass = j == 0, last_pass = j + 1 == nc;
      const int colour = post ? nc - 1 - j : j;
      const int dst = (first_pass && zero) ? src : 1 - src;
      void* out = (last_pass && final_out) ? final_out : m.lv[l].u[dst];
      sweep(o0, o1, o2, k * 8 + j, l, f, f_double, zero && first_pass, out, last_pass && out_double,
            fcopy && first_pass, dots && last_pass, colour, m.lv[l].u[src]);
      src = dst;
    }
    if (!final_out) cur[l] = src;
  };
  for (int l = L; l >= 0; --l) {
    const int j = L - l;
    const int sweeps = l == 0 ? m.nu_coarse : m.nu_pre;
    for (int k = 0; k < sweeps; ++k) {
      const bool first = k == 0;
      const bool finest_first = first && l == L;
      const bool last_of_cycle = (l == 0 && L == 0 && k + 1 == sweeps);
      const bool dots = last_of_cycle && q_dots;
      const bool from32 = finest_first && m.fp32 && r32_ready && !dots;
      const void* f = from32 ? m.fcopy : (finest_first || dots) ? static_cast<const void*>(r_in) : rhs(l);
      const bool f_double = !from32 && (dots || ((l == L) && (finest_first || !m.fp32)));
      smooth_sweep(0, j, 0, k, l, f, f_double, first, last_of_cycle ? z_out : nullptr, last_of_cycle && !z_float,
                   finest_first && m.fp32 && !from32, dots, false);
    }
    if (l > 0) {
      Op op;
      op.order[0] = 0;
      op.order[1] = j;
      op.order[2] = 1;
      op.kind = tpmg::kOpRestrict;
      op.prec = prec;
      op.L = m.view(l);
      op.C = m.view(l - 1);
      op.in0 = rhs(l);
      op.in1 = m.lv[l].u[cur[l]];
      op.out0 = m.lv[l - 1].f;
      op.sc = sc;   // (a batch skips a finished problem's operations)
      ops.push_back(op);
    }
  }
  for (int l = 1; l <= L; ++l) {
    const int j = L - l;
    Op op;
    op.order[0] = 1;
    op.order[1] = -j;
    op.kind = tpmg::kOpProlong;
    op.prec = prec;
    op.L = m.view(l);
    op.C = m.view(l - 1);
    op.in0 = m.lv[l - 1].u[cur[l - 1]];
    op.out0 = m.lv[l].u[cur[l]];
    op.sc = sc;
    ops.push_back(op);
    for (int k = 0; k < m.nu_post; ++k) {
      const bool last = l == L && k + 1 == m.nu_post;
      // the last sweep reads the FP64 residual when it also forms <z, q>, <z, r>
      const bool dots = last && q_dots;
      smooth_sweep(1, -j, 1, k, l, dots ? static_cast<const void*>(r_in) : rhs(l), dots || (l == L && !m.fp32), false,
                   last ? z_out : nullptr, last && !z_float, false, dots, true);
    }
  }
}

// One FCG iteration after the convergence test of the previous one:
//   z = M r, with beta = -<z,q>/<p,q> and rz = <z,r> formed by the last sweep;
//   p = z + beta p; q = A p, alpha = rz/<p,q>;
//   x += alpha p, r -= alpha q, rr = <r,r>.
// With nz beyond the fused smoother's range the dots are a separate op
// (kind -1, single solves only).
// batch_ring: a batch whose problems all have the fused operator instance
// runs the single solves' direction-ring form too.
void fcg_ops(tpmg_mg& m, double* x, tpmg::FcgScalars* sc, std::vector<Op>& ops, bool single = true,
             bool batch_ring = false) {
  const bool fused = m.tune.back().smoother == tpmg::kSmScan;
  // z of an FP32 V-cycle is an FP32 value: kept in FP32 when the last sweep
  // also forms the dots (nothing else reads it in FP64)
  const bool z_float = fused && m.fp32;
  const bool pring = single ? tpmg::spmv_pring_fits(m.view_outer()) : batch_ring;
  // (the ring form ends each iteration with the r update, which then also
  // writes the FP32 copy of r; the solve's start makes the first one)
  vcycle_ops(m, m.r, m.z, fused ? m.q : nullptr, sc, ops, z_float, (single || pring) && m.fp32);
  if (!fused) {
    Op d;
    d.order[0] = 2;
    d.kind = -1;
    d.in0 = m.z;
    d.in1 = m.q;
    d.out0 = m.r;
    d.partials = m.partials;
    d.sc = sc;
    d.len = m.len;
    ops.push_back(d);
  }
  if (pring) {
    // the directions stay in a ring and alpha p is added to x when the ring
    // is full (and after the last iteration), not in every update; the
    // direction update runs inside q = A p
    Op sp;
    sp.order[0] = 2;
    sp.order[1] = 1;
    sp.site = tpmg::kFinAlpha;
    sp.kind = tpmg::kOpSpmvPRing;
    sp.L = m.view_outer();
    sp.f_double = !z_float;
    sp.in0 = m.z;
    sp.out0 = m.q;
    sp.out1 = x;
    sp.aux = m.dirs;
    sp.partials = m.partials;
    sp.sc = sc;
    sp.len = m.len;
    ops.push_back(sp);
    Op ru;
    ru.order[0] = 2;
    ru.order[1] = 2;
    ru.site = tpmg::kFinRR;
    ru.kind = tpmg::kOpRupdate;
    ru.in1 = m.q;
    ru.out0 = m.fp32 ? m.fcopy : nullptr;
    ru.out1 = m.r;
    ru.partials = m.partials;
    ru.sc = sc;
    ru.len = m.len;
    ru.ring = single ? m.ring_dev : nullptr;
    ops.push_back(ru);
    return;
  }
  if (single) {
    // the same with the direction update apart (operator chunks without a
    // fused instance)
    Op pr;
    pr.kind = tpmg::kOpPupdateRing;
    pr.f_double = !z_float;
    pr.in0 = m.z;
    pr.out0 = m.dirs;
    pr.out1 = x;
    pr.sc = sc;
    pr.len = m.len;
    ops.push_back(pr);
    Op sr;
    sr.kind = tpmg::kOpSpmvRing;
    sr.L = m.view_outer();
    sr.in0 = m.dirs;
    sr.out0 = m.q;
    sr.partials = m.partials;
    sr.sc = sc;
    sr.len = m.len;
    ops.push_back(sr);
    Op ru;
    ru.kind = tpmg::kOpRupdate;
    ru.in1 = m.q;
    ru.out0 = m.fp32 ? m.fcopy : nullptr;
    ru.out1 = m.r;
    ru.partials = m.partials;
    ru.sc = sc;
    ru.len = m.len;
    ru.ring = m.ring_dev;
    ops.push_back(ru);
    return;
  }
  Op pu;
  pu.order[0] = 2;
  pu.order[1] = 1;
  pu.kind = tpmg::kOpPupdate;
  pu.f_double = !z_float;
  pu.in0 = m.z;
  pu.out0 = m.p;
  pu.sc = sc;
  pu.len = m.len;
  ops.push_back(pu);
  Op sp;
  sp.order[0] = 2;
  sp.order[1] = 2;
  sp.kind = tpmg::kOpSpmv;
  sp.L = m.view_outer();
  sp.in0 = m.p;
  sp.out0 = m.q;
  sp.partials = m.partials;
  sp.sc = sc;
  sp.site = tpmg::kFinAlpha;
  ops.push_back(sp);
  Op up;
  up.order[0] = 2;
  up.order[1] = 3;
  up.kind = tpmg::kOpUpdate;
  up.in0 = m.p;
  up.in1 = m.q;
  up.out0 = x;
  up.out1 = m.r;
  up.partials = m.partials;
  up.sc = sc;
  up.site = tpmg::kFinRR;
  up.len = m.len;
  up.ring = m.ring_dev;
  ops.push_back(up);
}

// executes one operation with the single-problem launchers (which also run
// the finalize kernel of a reducing operation)
hipError_t exec_op(const Op& op, hipStream_t s) {
  switch (op.kind) {
    case tpmg::kOpSmooth:
      return tpmg::launch_smooth(op.L, op.prec, op.in0, op.f_double, op.in1, op.zero, op.out0, op.out_double, op.out1,
                                 op.scratch_d, op.scratch_c, op.omega, s, op.q, op.partials, op.sc);
    case tpmg::kOpPupdateRing:
      return tpmg::launch_pupdate_ring(op.in0, op.f_double, static_cast<double*>(op.out0),
                                       static_cast<double*>(op.out1), op.sc, op.len, s);
    case tpmg::kOpSpmvPRing:
      return tpmg::launch_spmv_pring(op.L, op.in0, op.f_double, op.aux, op.len, static_cast<double*>(op.out1),
                                     static_cast<double*>(op.out0), op.partials, op.sc, s);
    case tpmg::kOpSpmvRing:
      return tpmg::launch_spmv_ring(op.L, static_cast<const double*>(op.in0), op.len, static_cast<double*>(op.out0),
                                    op.partials, op.sc, s);
    case tpmg::kOpRupdate:
      return tpmg::launch_rupdate(static_cast<double*>(op.out1), static_cast<const double*>(op.in1), op.sc, op.len,
                                  op.partials, op.ring, s, static_cast<float*>(op.out0));
    case tpmg::kOpRestrict:
      return tpmg::launch_residual_restrict(op.L, op.C, op.prec, op.in0, op.in1, op.out0, s);
    case tpmg::kOpProlong:
      return tpmg::launch_prolong_add(op.L, op.C, op.prec, op.in0, op.out0, s);
    case tpmg::kOpPupdate:
      return tpmg::launch_pupdate(op.in0, op.f_double, static_cast<double*>(op.out0), op.sc, op.len, s);
    case tpmg::kOpSpmv:
      return tpmg::launch_spmv64(op.L, 0, static_cast<const double*>(op.in0), nullptr, static_cast<double*>(op.out0),
                                 op.partials, op.site, op.sc, s);
    case tpmg::kOpUpdate:
      return tpmg::launch_fcg_update(static_cast<double*>(op.out0), static_cast<double*>(op.out1),
                                     static_cast<const double*>(op.in0), static_cast<const double*>(op.in1), op.sc,
                                     op.len, op.partials, op.ring, s);
    case -1:
      return tpmg::launch_dots(static_cast<const double*>(op.in0), static_cast<const double*>(op.in1),
                               static_cast<const double*>(op.out0), op.len, op.partials, op.sc, s);
    default:
      return hipErrorInvalidValue;
  }
}

// Phase of an operation for the per-phase timers of a solve: 0 V-cycle,
// 1 operator, 2 other vector updates and reductions.
int op_phase(const Op& op) {
  switch (op.kind) {
    case tpmg::kOpSmooth:
    case tpmg::kOpRestrict:
    case tpmg::kOpProlong:
      return 0;
    case tpmg::kOpSpmv:
    case tpmg::kOpSpmvRing:
    case tpmg::kOpSpmvPRing:
      return 1;
    default:
      return 2;
  }
}

// Algorithmic HBM bytes of one operation: every field it reads or writes
// counted once (per-column coefficients, halo rows and the scalars are
// O(1/nz) per unknown and left out). it: the iteration the operation belongs
// to (the first takes p = z; every kDirSlots-th direction update also adds
// the ring's kDirSlots directions to x).
double op_model_bytes(const Op& op, int it) {
  const double s = op.prec;
  const double n = static_cast<double>(op.L.npad) * op.L.nz;
  const double len = static_cast<double>(op.len);
  const double zb = op.f_double ? 8.0 : 4.0;
  const bool flush = it > 0 && it % tpmg::kDirSlots == 0;
  // coefficients per (T, k) of profiles that do not factorise, read by every
  // stencil kernel: beta^, three alphaS^ and one new radial face per unknown
  // (all of them), or the radial face alone (the partial form)
  const double coef = op.L.pm == 3 ? 7.0 : op.L.pm == 2 ? 5.0 : op.L.pm == 1 ? 1.0 : 0.0;
  const double ring_x = flush ? 8.0 * (tpmg::kDirSlots + 2) : 0.0;
  switch (op.kind) {
    case tpmg::kOpSmooth: {
      double b = (op.zero ? 0.0 : s) + (op.f_double ? 8.0 : s) + (op.out_double ? 8.0 : s);
      if (op.fcopy) b += 4.0;
      if (op.dots) b += 8.0;   // q (the residual is the right-hand side)
      return (b + coef * s) * n;
    }
    case tpmg::kOpRestrict:
      return (2.0 * s + s / 4.0 + coef * s) * n;
    case tpmg::kOpProlong:
      return (2.0 * s + s / 4.0) * n;
    case tpmg::kOpSpmvPRing:
      return (zb + (it > 0 ? 8.0 : 0.0) + 16.0 + ring_x + coef * 8.0) * len;
    case tpmg::kOpPupdateRing:
      return (zb + (it > 0 ? 8.0 : 0.0) + 8.0 + ring_x) * len;
    case tpmg::kOpSpmvRing:
      return (16.0 + coef * 8.0) * len;
    case tpmg::kOpRupdate:
      return (24.0 + (op.out0 ? 4.0 : 0.0)) * len;
    case tpmg::kOpPupdate:
      return (zb + 16.0) * len;
    case tpmg::kOpSpmv:
      return (16.0 + coef * 8.0) * n;
    case tpmg::kOpUpdate:
      return 48.0 * len;
    case -1:
      return 24.0 * len;
    default:
      return 0.0;
  }
}

// Model bytes of a solve of `iters` iterations: the initial residual
// (reads u and f, writes r and, for an FP32 V-cycle, its FP32 copy), the
// iterations, and the final x update of a single solve's direction ring.
double solve_model_bytes(const std::vector<Op>& ops, int iters, size_t len, bool fp32, bool ring, bool full = false) {
  double b = (24.0 + (fp32 ? 4.0 : 0.0) + (full ? 40.0 : 0.0)) * static_cast<double>(len);
  for (int it = 0; it < iters; ++it)
    for (const Op& op : ops) b += op_model_bytes(op, it);
  if (ring && iters > 0) {
    const int flushed = (iters - 1) / tpmg::kDirSlots * tpmg::kDirSlots;
    b += 8.0 * (2 + iters - flushed) * static_cast<double>(len);
  }
  return b;
}

hipError_t vcycle(tpmg_mg& m, const double* r_in, double* z_out) {
  std::vector<Op> ops;
  vcycle_ops(m, r_in, z_out, nullptr, m.scal, ops);
  for (const Op& op : ops) {
    hipError_t e = exec_op(op, m.stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t fcg_iteration(tpmg_mg& m, double* x) {
  std::vector<Op> ops;
  fcg_ops(m, x, m.scal, ops);
  for (const Op& op : ops) {
    hipError_t e = exec_op(op, m.stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

// Branches of a batched iteration's graph: groups of problems whose grouped
// launches form chains of their own, forked from the batch's stream and
// joined before the scalars are copied, so that one group's latency-bound
// coarse levels run beside another's bandwidth-bound fine ones. (Four: the
// hardware queues a process gets by default.)
constexpr int kBatchBranches = 4;

struct tpmg_batch {
  std::vector<tpmg_mg*> probs;
  hipStream_t stream = nullptr;
  tpmg::FcgScalars* scal = nullptr;     // device, one per problem
  tpmg::FcgScalars* h_scal = nullptr;   // pinned host mirrors: the initial scalars, then two per iteration in turn
  hipEvent_t ev[2] = {nullptr, nullptr};   // each iteration's copy of the scalars has arrived
  tpmg::Seg* segs = nullptr;            // device segment tables
  size_t max_segs = 0;
  std::vector<std::vector<tpmg::BatchLaunch>> plans;   // one launch chain per branch
  hipStream_t aux[kBatchBranches - 1] = {};            // capture streams of branches 1, 2, ...
  hipEvent_t fork = nullptr, join[kBatchBranches - 1] = {};
  std::vector<double*> plan_u;          // solution vectors the plan was built for
  hipGraphExec_t graph = nullptr;
};

namespace {

// whether every problem of the batch has the fused operator instance
bool batch_ring(const tpmg_batch& b) {
  for (const tpmg_mg* m : b.probs)
    if (!tpmg::spmv_pring_fits(m->view64(m->nlev - 1))) return false;
  return true;
}

// The problems of each branch: longest vectors first, each to the branch with
// the least work so far (ties to the lower index), as many branches as
// problems up to kBatchBranches.
std::vector<std::vector<int>> batch_groups(const tpmg_batch& b) {
  const int n = static_cast<int>(b.probs.size());
  const int ng = std::min(n, kBatchBranches);
  std::vector<int> order(n);
  for (int p = 0; p < n; ++p) order[p] = p;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b.probs[x]->len > b.probs[y]->len; });
  std::vector<std::vector<int>> groups(ng);
  std::vector<size_t> load(ng, 0);
  for (int p : order) {
    int g = 0;
    for (int k = 1; k < ng; ++k)
      if (load[k] < load[g]) g = k;
    groups[g].push_back(p);
    load[g] += b.probs[p]->len;
  }
  for (auto& gr : groups) std::sort(gr.begin(), gr.end());
  return groups;
}

// Groups the FCG-iteration operations of a branch's problems by schedule
// position: one grouped launch per position, followed by a grouped finalize
// where the operation reduces. Appends the segments to host and the launches
// (with the offsets of their segments) to plan.
hipError_t plan_branch(tpmg_batch& b, const std::vector<int>& group, double* const* d_u, std::vector<tpmg::Seg>& host,
                       std::vector<tpmg::BatchLaunch>& plan, std::vector<size_t>& seg_offset) {
  struct Item {
    Op op;
    int prob;
  };
  std::vector<Item> items;
  const bool ring = batch_ring(b);
  for (int p : group) {
    std::vector<Op> ops;
    // (with the direction ring, as single solves; otherwise x and p are
    // updated in place in every iteration, with the same bits)
    fcg_ops(*b.probs[p], d_u ? d_u[p] : nullptr, b.scal ? b.scal + p : nullptr, ops, false, ring);
    for (const Op& op : ops) items.push_back({op, p});
  }
  // smoother sweeps of one position are grouped by levels per wave (one
  // kernel instance per launch)
  auto kb_of = [](const Op& o) { return o.kind == tpmg::kOpSmooth ? o.L.tune.scan_levels : 0; };
  // residual + restriction and the operator: problems whose chunk has an
  // instance of its own launch it apart from the rest (runtime chunk, 0)
  auto ch_of = [](const Op& o) {
    if (o.kind != tpmg::kOpRestrict && o.kind != tpmg::kOpSpmv && o.kind != tpmg::kOpSpmvPRing) return 0;
    const int c = tpmg::effective_chunk(o.kind == tpmg::kOpRestrict ? o.L.tune.chunk_rr : o.L.tune.chunk_spmv,
                                        o.L.npad, o.L.nz);
    return (c == 1 || c == 2 || c == 4 || c == 8 || c == 16) ? c : 0;
  };
  // (a launch holds one profile mode: problems whose V-cycle or outer operator
  // rebuilds coefficients differently launch apart)
  auto group_less = [&](const Op& a, const Op& c) {
    if (order_less(a, c)) return true;
    if (order_less(c, a)) return false;
    if (a.L.pm != c.L.pm) return a.L.pm < c.L.pm;
    if (kb_of(a) != kb_of(c)) return kb_of(a) < kb_of(c);
    return ch_of(a) < ch_of(c);
  };
  std::stable_sort(items.begin(), items.end(),
                   [&](const Item& a, const Item& c) { return group_less(a.op, c.op); });
  size_t i = 0;
  while (i < items.size()) {
    size_t j = i;
    while (j < items.size() && !group_less(items[i].op, items[j].op) && !group_less(items[j].op, items[i].op)) ++j;
    const Op& o = items[i].op;
    tpmg::BatchLaunch L{};
    L.kind = o.kind;
    L.prec = o.prec;
    L.scan_levels = kb_of(o);
    L.chunk = ch_of(o);
    L.f_double = o.f_double;
    L.out_double = o.out_double;
    L.zero = o.zero;
    L.fcopy = o.fcopy;
    L.dots = o.dots;
    L.omega = o.omega;
    L.pm = o.L.pm;
    L.block = 256;
    tpmg::BatchLaunch F{};
    F.kind = tpmg::kOpFinalize;
    const bool reduces = o.site != tpmg::kFinNone;
    const size_t first = host.size();
    std::vector<tpmg::Seg> fin;
    unsigned start = 0;
    // a grouped sweep's blocks hold the waves of the deepest problem's tile
    if (o.kind == tpmg::kOpSmooth)
      for (size_t k = i; k < j; ++k)
        L.block = std::max(L.block,
                           static_cast<unsigned>(64 * tpmg::scan_waves(items[k].op.L.nz, items[k].op.L.tune.scan_levels)));
    for (size_t k = i; k < j; ++k) {
      const Op& a = items[k].op;
      if (a.kind != o.kind || a.prec != o.prec || a.f_double != o.f_double || a.out_double != o.out_double ||
          a.zero != o.zero || a.fcopy != o.fcopy || a.dots != o.dots)
        return hipErrorInvalidValue;   // problems disagree on the schedule
      tpmg::Seg g{};
      g.site = a.site;
      g.L = a.L;
      g.C = a.C;
      g.in0 = a.in0;
      g.in1 = a.in1;
      g.out0 = a.out0;
      g.out1 = a.out1;
      g.q = a.q;
      g.partials = a.partials;
      g.sc = a.sc;
      g.len = a.len;
      g.aux = a.aux;
      int nb = 0;
      switch (a.kind) {
        case tpmg::kOpSmooth: {
          if (a.L.tune.smoother != tpmg::kSmScan) return hipErrorInvalidValue;
          // tiles per block: as many as the block's waves hold, one in the
          // sweep that forms the dot products (its partial sums are per tile)
          const int waves = tpmg::scan_waves(a.L.nz, a.L.tune.scan_levels);
          const int tpb = a.dots ? 1 : std::max(1, static_cast<int>(L.block / 64) / waves);
          const int ntiles = a.L.npad / tpmg::kTile;
          nb = (ntiles + tpb - 1) / tpb;
          break;
        }
        case tpmg::kOpRestrict:
        case tpmg::kOpProlong:
        case tpmg::kOpSpmv:
        case tpmg::kOpSpmvPRing: {
          const int tuned = a.kind == tpmg::kOpRestrict  ? a.L.tune.chunk_rr
                            : a.kind == tpmg::kOpProlong ? a.L.tune.chunk_pr
                                                         : a.L.tune.chunk_spmv;
          g.chunk = tpmg::effective_chunk(tuned, a.L.npad, a.L.nz);
          nb = static_cast<int>(tpmg::stencil_blocks(a.L.npad, a.L.nz, g.chunk));
          break;
        }
        case tpmg::kOpPupdate:
          nb = static_cast<int>(tpmg::pupdate_blocks(a.len));
          break;
        case tpmg::kOpUpdate:
        case tpmg::kOpRupdate:
          nb = tpmg::kRedBlocks;
          break;
        default:
          return hipErrorInvalidValue;   // unfused dots: nz beyond the scan smoother
      }
      g.start = static_cast<int>(start);
      g.nblocks = nb;
      start += (static_cast<unsigned>(nb) + 7u) / 8u * 8u;
      host.push_back(g);
      if (reduces) {
        tpmg::Seg f = g;
        f.start = static_cast<int>(fin.size());
        fin.push_back(f);
      }
    }
    L.grid = start;
    L.nseg = static_cast<int>(j - i);
    // every wave of the block, idle or not, publishes its 8 summaries
    if (o.kind == tpmg::kOpSmooth) L.lds = tpmg::scan_lds_bytes(L.block / 64, o.prec);
    seg_offset.push_back(first);
    plan.push_back(L);
    if (reduces) {
      F.nseg = static_cast<int>(fin.size());
      F.grid = static_cast<unsigned>(fin.size());
      F.block = tpmg::kFinThreads;
      seg_offset.push_back(host.size());
      host.insert(host.end(), fin.begin(), fin.end());
      plan.push_back(F);
    }
    i = j;
  }
  return hipSuccess;
}

// The launch chains of all branches over one segment table. Returns the
// number of segments; with upload == false it only counts them.
hipError_t build_plan(tpmg_batch& b, double* const* d_u, bool upload, size_t* nsegs_out) {
  std::vector<tpmg::Seg> host;
  std::vector<std::vector<tpmg::BatchLaunch>> plans;
  std::vector<std::vector<size_t>> offsets;   // first segment of each launch
  for (const std::vector<int>& group : batch_groups(b)) {
    plans.emplace_back();
    offsets.emplace_back();
    hipError_t e = plan_branch(b, group, d_u, host, plans.back(), offsets.back());
    if (e != hipSuccess) return e;
  }
  if (nsegs_out) *nsegs_out = host.size();
  if (!upload) return hipSuccess;
  if (host.size() > b.max_segs) return hipErrorInvalidValue;
  for (size_t g = 0; g < plans.size(); ++g)
    for (size_t k = 0; k < plans[g].size(); ++k) plans[g][k].segs = b.segs + offsets[g][k];
  hipError_t e = hipMemcpyAsync(b.segs, host.data(), host.size() * sizeof(tpmg::Seg), hipMemcpyHostToDevice, b.stream);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(b.stream);
  if (e != hipSuccess) return e;
  b.plans = std::move(plans);
  return hipSuccess;
}

tpmg_status check_batch(tpmg_mg* const* problems, int n) {
  if (!problems || n < 1) return fail(TPMG_ERR_ARG, "need at least one problem");
  const tpmg_mg* a = problems[0];
  for (int i = 0; i < n; ++i) {
    const tpmg_mg* m = problems[i];
    if (!m) return fail(TPMG_ERR_ARG, "NULL problem");
    if (m->nlev < 2) return fail(TPMG_ERR_ARG, "batched problems need at least 2 multigrid levels");
    if (m->adv) return fail(TPMG_ERR_ARG, "batched problems need a symmetric operator (no vertical advection)");
    for (const tpmg::LevelTune& t : m->tune)
      if (t.smoother != tpmg::kSmScan)
        return fail(TPMG_ERR_ARG, "batched problems need the scan smoother on every level (params.smoother = 1)");
    if (m->fp32 != a->fp32 || m->nu_pre != a->nu_pre || m->nu_post != a->nu_post || m->nu_coarse != a->nu_coarse ||
        m->omega != a->omega || m->sor != a->sor)
      return fail(TPMG_ERR_ARG, "batched problems must share precision and smoother parameters");
    if (m->stream != a->stream || m->stream == nullptr)
      return fail(TPMG_ERR_ARG, "batched problems must share one non-default stream");
    for (int j = 0; j < i; ++j)
      if (problems[j] == m) return fail(TPMG_ERR_ARG, "a problem appears twice in the batch");
  }
  return TPMG_OK;
}

void drop_graph(tpmg_mg& m) {
  if (m.graph) (void)hipGraphExecDestroy(m.graph);
  m.graph = nullptr;
  m.graph_x = nullptr;
}

tpmg_status check_mg(const tpmg_mg* mg) {
  if (!mg) return fail(TPMG_ERR_ARG, "mg handle is NULL");
  return TPMG_OK;
}

// ---- launch tuning -----------------------------------------------------------

// Process-wide cache of tuned choices: key "device|kernel|precision|npad|nz",
// value {choice, scan levels}.
struct TuneCache {
  std::mutex mu;
  std::map<std::string, std::array<int, 2>> map;
};

TuneCache& tune_cache() {
  static TuneCache c;
  return c;
}

std::string tune_key(const std::string& dev, const char* kernel, int prec, int npad, int nz) {
  return dev + "|" + kernel + "|" + std::to_string(prec) + "|" + std::to_string(npad) + "|" + std::to_string(nz);
}

// Parses the cache format: {"key": [int, int], ...} (keys without quotes or
// backslashes). Returns false on any deviation.
bool parse_tune_json(const std::string& text, std::map<std::string, std::array<int, 2>>& out) {
  size_t i = 0;
  auto ws = [&]() {
    while (i < text.size() && std::isspace(static_cast<unsigned char>(text[i]))) ++i;
  };
  auto eat = [&](char ch) {
    ws();
    if (i < text.size() && text[i] == ch) {
      ++i;
      return true;
    }
    return false;
  };
  auto integer = [&](int& v) {
    ws();
    const size_t b = i;
    if (i < text.size() && text[i] == '-') ++i;
    while (i < text.size() && std::isdigit(static_cast<unsigned char>(text[i]))) ++i;
    if (i == b || (i == b + 1 && text[b] == '-') || i - b > 10) return false;
    const long long x = std::stoll(text.substr(b, i - b));
    if (x < -1000000 || x > 1000000) return false;
    v = static_cast<int>(x);
    return true;
  };
  if (!eat('{')) return false;
  if (eat('}')) {
    ws();
    return i == text.size();
  }
  for (;;) {
    if (!eat('"')) return false;
    const size_t b = i;
    while (i < text.size() && text[i] != '"' && text[i] != '\\') ++i;
    if (i >= text.size() || text[i] != '"' || i == b) return false;
    const std::string key = text.substr(b, i - b);
    ++i;
    std::array<int, 2> v{};
    if (!eat(':') || !eat('[') || !integer(v[0]) || !eat(',') || !integer(v[1]) || !eat(']')) return false;
    out[key] = v;
    if (eat(',')) continue;
    if (!eat('}')) return false;
    ws();
    return i == text.size();
  }
}

std::string device_tag() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string arch(prop.gcnArchName);
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch.resize(colon);
  return arch + ":" + std::to_string(prop.multiProcessorCount);
}

// Mean device time per launch of `launch`: two warm-up launches, then the
// better of two timed groups of `reps` launches between events.
hipError_t time_launches(hipStream_t s, int reps, const std::function<hipError_t()>& launch, double* ms) {
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  for (int w = 0; w < 2 && e == hipSuccess; ++w) e = launch();
  double best = 1e300;
  for (int g = 0; g < 2 && e == hipSuccess; ++g) {
    e = hipEventRecord(a, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    if (e == hipSuccess) best = std::min(best, static_cast<double>(t) / reps);
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  *ms = best;
  return e;
}

// Picks, among candidates, the one with the smallest time; the first
// candidate (the built-in choice) is kept unless another is 5% faster, so
// that near-ties (run-to-run noise) do not change the kernel.
template <typename C>
hipError_t pick(tpmg_mg& m, const std::vector<C>& cands, const std::function<hipError_t(const C&)>& launch,
                size_t* best_index) {
  double best_t = 0.0;
  *best_index = 0;
  for (size_t i = 0; i < cands.size(); ++i) {
    double t = 0.0;
    hipError_t e = time_launches(m.stream, 8, [&]() { return launch(cands[i]); }, &t);
    if (e != hipSuccess) return e;
    m.tune_trials += 1;
    m.tune_ms += t * (8 * 2 + 2);
    if (i == 0 || t < 0.95 * best_t) {
      best_t = t;
      *best_index = i;
    }
  }
  return hipSuccess;
}

tpmg_status autotune(tpmg_mg& m, const tpmg_mg_params& p);

// Sets m.tune from the defaults and the caller's overrides (trials ==
// false, before any device work), or refines it by timed trials on the
// workspace (trials == true), whose vectors hold zeros at that point and
// still hold zeros afterwards (every trial maps zero data to zero data).
tpmg_status choose_tuning(tpmg_mg& m, const tpmg_mg_params& p, bool trials) {
  const int prec = m.fp32 ? 4 : 8;
  const int L = m.nlev - 1;
  if (trials) {
    if (p.autotune == 0) return TPMG_OK;
    return autotune(m, p);
  }
  m.tune.assign(m.nlev, tpmg::default_tune(m.nz, prec));
  for (int l = 0; l <= L; ++l) {
    tpmg::LevelTune& t = m.tune[l];
    if (p.smoother != 0) {
      t.smoother = p.smoother - 1;
      if (t.smoother == tpmg::kSmScan && !tpmg::smoother_fits(tpmg::kSmScan, t.scan_levels, m.nz, prec))
        t.scan_levels = 16;
    }
    if (p.scan_levels != 0) {
      t.smoother = tpmg::kSmScan;
      t.scan_levels = p.scan_levels;
    }
    if (p.stencil_chunk != 0) t.chunk_rr = t.chunk_pr = t.chunk_spmv = p.stencil_chunk;
    if (m.pm != 0) {
      // coefficients per (T, k): the scan smoother at 8 or 16 levels per wave
      if (p.smoother > 1 || p.scan_levels == 4)
        return fail(TPMG_ERR_ARG, "profiles that do not factorise run the scan smoother at 8 or 16 levels per wave");
      t.smoother = tpmg::kSmScan;
      if (t.scan_levels == 4) t.scan_levels = 8;
      if (!tpmg::smoother_fits(tpmg::kSmScan, t.scan_levels, m.nz, prec)) t.scan_levels = 16;
    }
    if (!tpmg::smoother_fits(t.smoother, t.scan_levels, m.nz, prec))
      return fail(TPMG_ERR_ARG, "the requested line smoother cannot run nz = " + std::to_string(m.nz) +
                                    " (scan form: nz <= 16 * scan_levels; LDS form: two [nz][64] arrays in LDS)");
  }
  return TPMG_OK;
}

tpmg_status autotune(tpmg_mg& m, const tpmg_mg_params& p) {
  const int prec = m.fp32 ? 4 : 8;
  const int L = m.nlev - 1;
  const std::string dev = device_tag();
  TuneCache& cache = tune_cache();
  auto lookup = [&](const std::string& key, std::array<int, 2>* v) {
    if (p.autotune == 2) return false;
    std::lock_guard<std::mutex> lk(cache.mu);
    auto it = cache.map.find(key);
    if (it == cache.map.end()) return false;
    *v = it->second;
    return true;
  };
  auto store = [&](const std::string& key, std::array<int, 2> v) {
    std::lock_guard<std::mutex> lk(cache.mu);
    cache.map[key] = v;
  };
  const bool tune_smoother = p.smoother == 0 && p.scan_levels == 0;
  const bool tune_scan_levels = p.smoother == 1 && p.scan_levels == 0;
  const bool tune_chunks = p.stencil_chunk == 0;
  std::vector<int> chunks;
  for (int c = 1; c <= 16; c *= 2)
    if (c <= m.nz) chunks.push_back(c);
  auto chunk_cands = [&](int npad) {
    // the heuristic first
    std::vector<int> v{tpmg::stencil_chunk(npad, m.nz)};
    for (int c : chunks)
      if (c != v[0]) v.push_back(c);
    return v;
  };

  for (int l = 0; l <= L; ++l) {
    tpmg::LevelTune& t = m.tune[l];
    const int npad = m.lv[l].npad;
    const void* f = l < L ? m.lv[l].f : (m.fp32 ? static_cast<const void*>(m.fcopy) : static_cast<const void*>(m.r));
    // (the profile mode changes what the kernels load: its own cache entries)
    const std::string pm_tag = m.pm == 0 ? "" : (m.pm == 1 ? "_partial" : "_full");
    if (tune_smoother || tune_scan_levels) {
      const std::string key =
          tune_key(dev, (std::string(tune_smoother ? "smooth" : "smooth_scan") + pm_tag).c_str(), prec, npad, m.nz);
      std::array<int, 2> v{};
      if (lookup(key, &v) && tpmg::smoother_fits(v[0], v[1], m.nz, prec)) {
        t.smoother = v[0];
        t.scan_levels = v[1];
      } else {
        std::vector<std::array<int, 2>> cands{{t.smoother, t.scan_levels}};
        for (int kb : {4, 8, 16})
          if (tpmg::smoother_fits(tpmg::kSmScan, kb, m.nz, prec) && !(t.smoother == tpmg::kSmScan && t.scan_levels == kb) &&
              !(m.pm != 0 && kb == 4))
            cands.push_back({tpmg::kSmScan, kb});
        if (tune_smoother && m.pm == 0)
          for (int kind : {tpmg::kSmLds, tpmg::kSmGlobal})
            if (tpmg::smoother_fits(kind, 8, m.nz, prec) && t.smoother != kind) cands.push_back({kind, 8});
        size_t best = 0;
        std::function<hipError_t(const std::array<int, 2>&)> run = [&](const std::array<int, 2>& c) {
          tpmg::LevelView v = m.view(l);
          v.tune.smoother = c[0];
          v.tune.scan_levels = c[1];
          return tpmg::launch_smooth(v, prec, f, prec == 8, m.lv[l].u[0], false, m.lv[l].u[1], prec == 8, nullptr,
                                     m.sd, m.sc, m.omega, m.stream);
        };
        hipError_t e = pick(m, cands, run, &best);
        if (e != hipSuccess) return fail(TPMG_ERR_DEVICE, std::string("autotune (smoother): ") + hipGetErrorString(e));
        t.smoother = cands[best][0];
        t.scan_levels = cands[best][1];
        store(key, cands[best]);
      }
    }
    if (!tune_chunks) continue;
    const std::vector<int> cc = chunk_cands(npad);
    auto tune_chunk = [&](const char* kernel, int kprec, int* field,
                          const std::function<hipError_t(int)>& launch) -> tpmg_status {
      const bool outer = std::string(kernel) == "spmv_p";
      const std::string tag = outer ? (m.full_outer ? "_full" : "") : pm_tag;
      const std::string key = tune_key(dev, (std::string(kernel) + tag).c_str(), kprec, npad, m.nz);
      std::array<int, 2> v{};
      if (lookup(key, &v) && v[0] >= 1 && v[0] <= 256) {
        *field = v[0];
        return TPMG_OK;
      }
      size_t best = 0;
      std::function<hipError_t(const int&)> run = [&](const int& c) { return launch(c); };
      hipError_t e = pick(m, cc, run, &best);
      if (e != hipSuccess) return fail(TPMG_ERR_DEVICE, std::string("autotune (") + kernel + "): " + hipGetErrorString(e));
      *field = cc[best];
      store(key, {cc[best], 0});
      return TPMG_OK;
    };
    tpmg_status st = TPMG_OK;
    if (l > 0) {
      st = tune_chunk("restrict", prec, &t.chunk_rr, [&](int c) {
        tpmg::LevelView F = m.view(l);
        F.tune.chunk_rr = c;
        return tpmg::launch_residual_restrict(F, m.view(l - 1), prec, f, m.lv[l].u[0], m.lv[l - 1].f, m.stream);
      });
      if (st == TPMG_OK)
        st = tune_chunk("prolong", prec, &t.chunk_pr, [&](int c) {
          tpmg::LevelView F = m.view(l);
          F.tune.chunk_pr = c;
          return tpmg::launch_prolong_add(F, m.view(l - 1), prec, m.lv[l - 1].u[0], m.lv[l].u[0], m.stream);
        });
    }
    if (st == TPMG_OK && l == L)
      // timed as single solves run it: the direction update inside the
      // operator (on the zeroed workspace: iteration 0, no flush), with a
      // finalize that changes no scalar
      st = tune_chunk("spmv_p", 8, &t.chunk_spmv, [&](int c) {
        tpmg::LevelView V = m.view_outer();
        V.tune.chunk_spmv = c;
        if (tpmg::spmv_pring_fits(V))
          return tpmg::launch_spmv_pring(V, m.z, !m.fp32, m.dirs, m.len, m.r, m.q, m.partials, m.scal, m.stream,
                                         tpmg::kFinNone);
        hipError_t e = tpmg::launch_spmv64(V, 0, m.p, nullptr, m.q, m.partials, tpmg::kFinNone, m.scal, m.stream);
        if (e != hipSuccess) return e;
        return tpmg::launch_finalize(tpmg::kFinNone, m.partials,
                                     static_cast<int>(tpmg::stencil_blocks(V.npad, V.nz, c)), m.scal, 0.0, m.stream);
      });
    if (st != TPMG_OK) return st;
  }
  return TPMG_OK;
}

}  // namespace

extern "C" {

void tpmg_mg_params_default(tpmg_mg_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->n_levels = 0;
  p->nu_pre = 2;
  p->nu_post = 2;
  p->nu_coarse = 1;
  p->omega_relax = 2.0 / 3.0;
  p->precond_fp32 = 0;
  p->use_graph = 0;
}

const char* tpmg_status_string(tpmg_status s) {
  switch (s) {
    case TPMG_OK: return "TPMG_OK";
    case TPMG_NOT_CONVERGED: return "TPMG_NOT_CONVERGED";
    case TPMG_ERR_ARG: return "TPMG_ERR_ARG";
    case TPMG_ERR_DEVICE: return "TPMG_ERR_DEVICE";
    case TPMG_ERR_NOMEM: return "TPMG_ERR_NOMEM";
    case TPMG_ERR_BREAKDOWN: return "TPMG_ERR_BREAKDOWN";
    case TPMG_ERR_STATE: return "TPMG_ERR_STATE";
  }
  return "unknown status";
}

const char* tpmg_last_error(void) { return g_last_error.c_str(); }

tpmg_status tpmg_grid_icosahedral(int refinement, int nz, const double* r_faces, tpmg_grid** out) {
  if (!out) return fail(TPMG_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (refinement < 0 || refinement > 10) return fail(TPMG_ERR_ARG, "refinement must be in [0, 10]");
  if (nz < 1 || nz > 4096) return fail(TPMG_ERR_ARG, "nz must be in [1, 4096]");
  if (!r_faces) return fail(TPMG_ERR_ARG, "r_faces is NULL");
  for (int k = 0; k < nz; ++k)
    if (!(r_faces[k + 1] > r_faces[k]) || !std::isfinite(r_faces[k + 1]))
      return fail(TPMG_ERR_ARG, "r_faces must be finite and strictly increasing");
  if (!(r_faces[0] > 0.0)) return fail(TPMG_ERR_ARG, "r_faces[0] must be positive");
  try {
    auto* g = new tpmg_grid();
    tpmg::build_grid(g->g, refinement, nz, r_faces);
    *out = g;
  } catch (const std::exception& ex) {
    return fail(TPMG_ERR_ARG, ex.what());
  }
  return TPMG_OK;
}

tpmg_status tpmg_grid_level_size(const tpmg_grid* g, int level, int* n_cells) {
  if (!g || !n_cells) return fail(TPMG_ERR_ARG, "NULL argument");
  if (level < 0 || level > g->g.refinement) return fail(TPMG_ERR_ARG, "level out of range");
  *n_cells = g->g.levels[level].n;
  return TPMG_OK;
}

tpmg_status tpmg_grid_geometry(const tpmg_grid* g, int level, double* centres, double* areas, int32_t* nbr,
                               double* edge_len, double* edge_factor) {
  if (!g) return fail(TPMG_ERR_ARG, "grid is NULL");
  if (level < 0 || level > g->g.refinement) return fail(TPMG_ERR_ARG, "level out of range");
  const tpmg::MeshLevel& L = g->g.levels[level];
  if (centres) std::copy(L.centre.begin(), L.centre.end(), centres);
  if (areas) std::copy(L.area.begin(), L.area.end(), areas);
  if (nbr) std::copy(L.nbr.begin(), L.nbr.end(), nbr);
  if (edge_len) std::copy(L.arc.begin(), L.arc.end(), edge_len);
  if (edge_factor) std::copy(L.g.begin(), L.g.end(), edge_factor);
  return TPMG_OK;
}

tpmg_status tpmg_grid_colouring(const tpmg_grid* g, int level, int32_t* colours, int* n_colours) {
  if (!g || !colours) return fail(TPMG_ERR_ARG, "NULL argument");
  if (level < 0 || level > g->g.refinement) return fail(TPMG_ERR_ARG, "level out of range");
  const tpmg::MeshLevel& M = g->g.levels[level];
  const std::vector<int8_t> c = tpmg::greedy_colouring(M.nbr, M.n);
  int nc = 0;
  for (int t = 0; t < M.n; ++t) {
    colours[t] = c[t];
    nc = std::max(nc, c[t] + 1);
  }
  if (n_colours) *n_colours = nc;
  return TPMG_OK;
}

tpmg_status tpmg_grid_vertical(const tpmg_grid* g, double* vk) {
  if (!g || !vk) return fail(TPMG_ERR_ARG, "NULL argument");
  std::copy(g->g.vk.begin(), g->g.vk.end(), vk);
  return TPMG_OK;
}

tpmg_status tpmg_op_create_levels(const tpmg_grid* g, int n_levels, double omega2, const double* alpha_r_v,
                                  const double* alpha_s_v, const double* beta_v, const double* const* alpha_r_h,
                                  const double* const* alpha_s_h, const double* const* beta_h, tpmg_op** out) {
  if (!out) return fail(TPMG_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!g) return fail(TPMG_ERR_ARG, "grid is NULL");
  if (!alpha_r_v || !alpha_s_v || !beta_v) return fail(TPMG_ERR_ARG, "vertical profile factors are required");
  if (!(omega2 > 0.0) || !std::isfinite(omega2)) return fail(TPMG_ERR_ARG, "omega2 must be positive");
  const int ref = g->g.refinement, nz = g->g.nz;
  if (n_levels == 0) n_levels = std::min(6, ref + 1);
  if (n_levels < 1 || n_levels > ref + 1) return fail(TPMG_ERR_ARG, "n_levels must be in [1, refinement + 1]");
  auto positive = [](const double* v, size_t n) {
    for (size_t i = 0; i < n; ++i)
      if (!(v[i] > 0.0) || !std::isfinite(v[i])) return false;
    return true;
  };
  if (!positive(alpha_r_v + 1, nz > 1 ? nz - 1 : 0) || !positive(alpha_s_v, nz) || !positive(beta_v, nz))
    return fail(TPMG_ERR_ARG, "vertical profile factors must be positive and finite");
  for (const double* const* lv : {alpha_r_h, alpha_s_h, beta_h}) {
    if (!lv) continue;
    for (int r = ref - n_levels + 1; r <= ref; ++r)
      if (lv[r] && !positive(lv[r], g->g.levels[r].n))
        return fail(TPMG_ERR_ARG, "horizontal profile factors of refinement level " + std::to_string(r) +
                                      " must be positive and finite");
  }
  try {
    auto* o = new tpmg_op();
    // (the finest grid's factors are entry ref of the tables)
    tpmg::build_operator(o->op, g->g, n_levels, omega2, alpha_r_v, alpha_s_v, beta_v, nullptr, nullptr, nullptr,
                         alpha_r_h, alpha_s_h, beta_h);
    *out = o;
  } catch (const std::exception& ex) {
    return fail(TPMG_ERR_ARG, ex.what());
  }
  return TPMG_OK;
}

tpmg_status tpmg_op_create(const tpmg_grid* g, int n_levels, double omega2, const double* alpha_r_v,
                           const double* alpha_s_v, const double* beta_v, const double* alpha_r_h,
                           const double* alpha_s_h, const double* beta_h, tpmg_op** out) {
  // the finest grid's factors as the only entries of the per-grid tables
  if (!g) return tpmg_op_create_levels(g, n_levels, omega2, alpha_r_v, alpha_s_v, beta_v, nullptr, nullptr, nullptr,
                                       out);
  std::vector<const double*> tr(g->g.refinement + 1, nullptr), ts(tr), tb(tr);
  tr.back() = alpha_r_h;
  ts.back() = alpha_s_h;
  tb.back() = beta_h;
  return tpmg_op_create_levels(g, n_levels, omega2, alpha_r_v, alpha_s_v, beta_v, tr.data(), ts.data(), tb.data(),
                               out);
}

tpmg_status tpmg_op_set_full_profiles(tpmg_op* op, const tpmg_grid* g, const double* alpha_r, const double* alpha_s,
                                      const double* beta, const double* xi_r) {
  if (!op || !g || !alpha_r || !alpha_s || !beta) return fail(TPMG_ERR_ARG, "NULL argument");
  const int ref = g->g.refinement, nz = g->g.nz;
  if (ref != op->op.refinement || nz != op->op.nz) return fail(TPMG_ERR_ARG, "op was not created on this grid");
  const size_t n = g->g.levels[ref].n;
  auto positive = [](const double* v, size_t count, size_t stride, size_t skip_lo, size_t skip_hi) {
    for (size_t i = 0; i < count; ++i) {
      const size_t k = i % stride;
      if (k < skip_lo || k + skip_hi >= stride) continue;
      if (!(v[i] > 0.0) || !std::isfinite(v[i])) return false;
    }
    return true;
  };
  if (!positive(alpha_r, n * (nz + 1), nz + 1, 1, 1) || !positive(alpha_s, n * nz, nz, 0, 0) ||
      !positive(beta, n * nz, nz, 0, 0))
    return fail(TPMG_ERR_ARG, "full profiles must be positive and finite");
  if (xi_r)
    for (size_t i = 0; i < n * (nz + 1); ++i)
      if (!std::isfinite(xi_r[i])) return fail(TPMG_ERR_ARG, "xi_r must be finite");
  try {
    tpmg::build_full(op->op, g->g, alpha_r, alpha_s, beta, xi_r);
  } catch (const std::exception& ex) {
    return fail(TPMG_ERR_ARG, ex.what());
  }
  return TPMG_OK;
}

tpmg_status tpmg_op_coefficients_full(const tpmg_op* op, int level, double* beta, double* alpha_s, double* alpha_r,
                                      double* adv_lo, double* adv_up) {
  if (!op) return fail(TPMG_ERR_ARG, "op is NULL");
  if (level < 0 || level >= static_cast<int>(op->op.levels.size())) return fail(TPMG_ERR_ARG, "level out of range");
  if (!op->op.full) return fail(TPMG_ERR_STATE, "the operator has no full profiles");
  const tpmg::LevelCoeffs& C = op->op.levels[level];
  if (beta) std::copy(C.fb.begin(), C.fb.end(), beta);
  if (alpha_s) std::copy(C.fas.begin(), C.fas.end(), alpha_s);
  if (alpha_r) std::copy(C.far.begin(), C.far.end(), alpha_r);
  const size_t nn = static_cast<size_t>(C.n) * op->op.nz;
  if (adv_lo) {
    if (op->op.adv) std::copy(C.fxl.begin(), C.fxl.end(), adv_lo);
    else std::fill(adv_lo, adv_lo + nn, 0.0);
  }
  if (adv_up) {
    if (op->op.adv) std::copy(C.fxu.begin(), C.fxu.end(), adv_up);
    else std::fill(adv_up, adv_up + nn, 0.0);
  }
  return TPMG_OK;
}

tpmg_status tpmg_op_levels(const tpmg_op* op, int* n_levels) {
  if (!op || !n_levels) return fail(TPMG_ERR_ARG, "NULL argument");
  *n_levels = static_cast<int>(op->op.levels.size());
  return TPMG_OK;
}

tpmg_status tpmg_op_level_size(const tpmg_op* op, int level, int* n_cells) {
  if (!op || !n_cells) return fail(TPMG_ERR_ARG, "NULL argument");
  if (level < 0 || level >= static_cast<int>(op->op.levels.size())) return fail(TPMG_ERR_ARG, "level out of range");
  *n_cells = op->op.levels[level].n;
  return TPMG_OK;
}

tpmg_status tpmg_op_coefficients(const tpmg_op* op, int level, double* beta_h, double* alpha_r_h, double* alpha_s_h,
                                 double* beta_v, double* alpha_s_v, double* alpha_r_v) {
  if (!op) return fail(TPMG_ERR_ARG, "op is NULL");
  if (level < 0 || level >= static_cast<int>(op->op.levels.size())) return fail(TPMG_ERR_ARG, "level out of range");
  const tpmg::LevelCoeffs& C = op->op.levels[level];
  if (beta_h) std::copy(C.beta_h.begin(), C.beta_h.end(), beta_h);
  if (alpha_r_h) std::copy(C.ar_h.begin(), C.ar_h.end(), alpha_r_h);
  if (alpha_s_h) std::copy(C.as_h.begin(), C.as_h.end(), alpha_s_h);
  if (beta_v) std::copy(op->op.beta_v.begin(), op->op.beta_v.end(), beta_v);
  if (alpha_s_v) std::copy(op->op.as_v.begin(), op->op.as_v.end(), alpha_s_v);
  if (alpha_r_v) std::copy(op->op.ar_v.begin(), op->op.ar_v.end(), alpha_r_v);
  return TPMG_OK;
}

tpmg_status tpmg_op_prolongation(const tpmg_op* op, int level, double* w) {
  if (!op || !w) return fail(TPMG_ERR_ARG, "NULL argument");
  if (level < 1 || level >= static_cast<int>(op->op.levels.size())) return fail(TPMG_ERR_ARG, "level out of range");
  const auto& pw = op->op.levels[level].pw;
  std::copy(pw.begin(), pw.end(), w);
  return TPMG_OK;
}

tpmg_status tpmg_mg_workspace_size(const tpmg_op* op, const tpmg_mg_params* params, size_t* bytes) {
  if (!op || !bytes) return fail(TPMG_ERR_ARG, "NULL argument");
  tpmg_status st = check_params(params);
  if (st != TPMG_OK) return st;
  tpmg_mg m;
  m.fp32 = params->precond_fp32 != 0;
  m.sor = params->smoother_order == 1;
  Carver cv(nullptr);
  carve(m, op->op, cv);
  *bytes = cv.off + 256;
  return TPMG_OK;
}

}  // extern "C"

namespace {

// tpmg_mg_setup; with pinned = false the handle keeps its iteration records
// in the workspace (device memory) and allocates no pinned host memory.
tpmg_status setup_impl(const tpmg_op* op, const tpmg_mg_params* params, void* d_workspace, size_t bytes,
                       void* hip_stream, bool pinned, tpmg_mg** out) {
  if (!out) return fail(TPMG_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!op) return fail(TPMG_ERR_ARG, "op is NULL");
  tpmg_status st = check_params(params);
  if (st != TPMG_OK) return st;
  if (!d_workspace) return fail(TPMG_ERR_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(d_workspace) % 256 != 0) return fail(TPMG_ERR_ARG, "workspace must be 256-byte aligned");
  if (params->n_levels != 0 && params->n_levels != static_cast<int>(op->op.levels.size()))
    return fail(TPMG_ERR_ARG, "params->n_levels differs from the operator's level count");
  size_t need = 0;
  if ((st = tpmg_mg_workspace_size(op, params, &need)) != TPMG_OK) return st;
  if (bytes < need) return fail(TPMG_ERR_NOMEM, "workspace too small: need " + std::to_string(need) + " bytes");

  auto* m = new tpmg_mg();
  m->nlev = static_cast<int>(op->op.levels.size());
  m->nz = op->op.nz;
  m->n_fine = op->op.levels.back().n;
  m->npad_fine = pad64(m->n_fine);
  m->nu_pre = params->nu_pre;
  m->nu_post = params->nu_post;
  m->nu_coarse = params->nu_coarse;
  m->omega = params->omega_relax;
  m->fp32 = params->precond_fp32 != 0;
  m->sor = params->smoother_order == 1;
  m->full_outer = op->op.full;
  if (params->precond_profiles != 0 && !op->op.full) {
    delete m;
    return fail(TPMG_ERR_ARG, "precond_profiles 1 and 2 need an operator with full profiles (tpmg_op_set_full_profiles)");
  }
  m->adv = op->op.adv;
  // (the V-cycle of the full profiles includes the advection; the factorised
  // and partial ones are built without it)
  m->pm = !op->op.full ? 0 : params->precond_profiles == 0 ? (op->op.adv ? 3 : 2) : params->precond_profiles == 1 ? 0 : 1;
  m->stream = static_cast<hipStream_t>(hip_stream);
  m->use_graph = params->use_graph != 0 && m->stream != nullptr;
  Carver cv(d_workspace);
  carve(*m, op->op, cv);

  auto cleanup_fail = [&](tpmg_status s, const std::string& msg) {
    if (m->h_scal) (void)hipHostFree(m->h_scal);
    if (m->ring) (void)hipHostFree(m->ring);
    delete m;
    return fail(s, msg);
  };
  int dev = 0, max_lds = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) {
    delete m;
    return fail(TPMG_ERR_DEVICE, std::string("device query: ") + hipGetErrorString(e));
  }
  tpmg::set_max_lds(static_cast<size_t>(max_lds));
  if ((st = choose_tuning(*m, *params, false)) != TPMG_OK) {
    delete m;
    return st;
  }
  m->pinned = pinned;
  if (pinned) {
    e = hipHostMalloc(reinterpret_cast<void**>(&m->h_scal), sizeof(tpmg::FcgScalars), hipHostMallocDefault);
    if (e != hipSuccess) {
      m->h_scal = nullptr;
      return cleanup_fail(TPMG_ERR_DEVICE, std::string("hipHostMalloc: ") + hipGetErrorString(e));
    }
    e = hipHostMalloc(reinterpret_cast<void**>(&m->ring), tpmg::kRecords * sizeof(tpmg::FcgRecord),
                      hipHostMallocDefault);
    if (e != hipSuccess) {
      m->ring = nullptr;
      return cleanup_fail(TPMG_ERR_DEVICE, std::string("hipHostMalloc: ") + hipGetErrorString(e));
    }
    std::memset(m->ring, 0, tpmg::kRecords * sizeof(tpmg::FcgRecord));
    e = hipHostGetDevicePointer(reinterpret_cast<void**>(&m->ring_dev), m->ring, 0);
    if (e != hipSuccess)
      return cleanup_fail(TPMG_ERR_DEVICE, std::string("hipHostGetDevicePointer: ") + hipGetErrorString(e));
  } else {
    m->ring_dev = m->ring_ws;   // zeroed with the workspace below
  }
  // zero the whole workspace once: padding entries of every vector stay zero
  e = tpmg::launch_fill(d_workspace, (cv.off + 3) / 4 * 4, m->stream);
  std::vector<std::vector<double>> keep64;
  std::vector<std::vector<float>> keep32;
  std::vector<std::vector<int32_t>> keepi;
  std::vector<std::vector<int8_t>> keepc;
  const int nz = m->nz;
  for (int l = 0; l < m->nlev && e == hipSuccess; ++l) {
    const tpmg::LevelCoeffs& C = op->op.levels[l];
    DevLevel& d = m->lv[l];
    std::vector<int32_t> nb(3 * static_cast<size_t>(d.npad));
    for (int j = 0; j < 3; ++j)
      for (int t = 0; t < d.npad; ++t) nb[static_cast<size_t>(j) * d.npad + t] = t < d.n ? C.nbr[3 * static_cast<size_t>(t) + j] : t;
    std::vector<int32_t> code, halo;
    if (!tile_halos(nb, d.npad, code, halo)) {
      (void)hipStreamSynchronize(m->stream);
      return cleanup_fail(TPMG_ERR_ARG, "a 64-column tile has more than 64 distinct out-of-tile neighbours");
    }
    if (m->sor) {
      std::vector<int8_t> col = tpmg::greedy_colouring(C.nbr, d.n);
      d.ncol = 1 + *std::max_element(col.begin(), col.end());
      col.resize(static_cast<size_t>(d.npad), static_cast<int8_t>(-1));
      keepc.push_back(std::move(col));
      if (e == hipSuccess) e = upload(d.colour, keepc.back(), m->stream);
    }
    keepi.push_back(std::move(nb));
    if (e == hipSuccess) e = upload(d.nbr, keepi.back(), m->stream);
    keepi.push_back(std::move(code));
    if (e == hipSuccess) e = upload(d.code, keepi.back(), m->stream);
    keepi.push_back(std::move(halo));
    if (e == hipSuccess) e = upload(d.halo, keepi.back(), m->stream);
    // inert padding columns: beta = 1, no couplings
    keep64.push_back(padded<double>(C.beta_h, d.n, d.npad, 1, 1.0));
    keep32.push_back(padded<float>(C.beta_h, d.n, d.npad, 1, 1.0));
    if (e == hipSuccess) e = upload(d.bh[0], keep64.back(), m->stream);
    if (e == hipSuccess) e = upload(d.bh[1], keep32.back(), m->stream);
    keep64.push_back(padded<double>(C.ar_h, d.n, d.npad, 1, 0.0));
    keep32.push_back(padded<float>(C.ar_h, d.n, d.npad, 1, 0.0));
    if (e == hipSuccess) e = upload(d.arh[0], keep64.back(), m->stream);
    if (e == hipSuccess) e = upload(d.arh[1], keep32.back(), m->stream);
    keep64.push_back(padded<double>(C.as_h, d.n, d.npad, 3, 0.0));
    keep32.push_back(padded<float>(C.as_h, d.n, d.npad, 3, 0.0));
    if (e == hipSuccess) e = upload(d.ash[0], keep64.back(), m->stream);
    if (e == hipSuccess) e = upload(d.ash[1], keep32.back(), m->stream);
    if (l > 0) {
      keep64.push_back(padded<double>(C.pw, d.n, d.npad, 3, 0.0));
      keep32.push_back(padded<float>(C.pw, d.n, d.npad, 3, 0.0));
      if (e == hipSuccess) e = upload(d.pw[0], keep64.back(), m->stream);
      if (e == hipSuccess) e = upload(d.pw[1], keep32.back(), m->stream);
    }
    if (op->op.full) {
      // (padding columns: unit mass, no couplings)
      const std::vector<double>* src[5] = {&C.fb, &C.far, &C.fas, &C.fxl, &C.fxu};
      void* const* dst[5] = {d.fb, d.far, d.fas, d.fxl, d.fxu};
      const int comps[5] = {1, 1, 3, 1, 1}, rows[5] = {nz, nz + 1, nz, nz, nz};
      const double fill[5] = {1.0, 0.0, 0.0, 0.0, 0.0};
      for (int a = 0; a < (op->op.adv ? 5 : 3) && e == hipSuccess; ++a) {
        keep64.push_back(tiled<double>(*src[a], d.n, d.npad, comps[a], rows[a], fill[a]));
        e = upload(dst[a][0], keep64.back(), m->stream);
        if (e == hipSuccess && dst[a][1]) {
          keep32.push_back(tiled<float>(*src[a], d.n, d.npad, comps[a], rows[a], fill[a]));
          e = upload(dst[a][1], keep32.back(), m->stream);
        }
      }
    }
  }
  const std::vector<double>* vv[3] = {&op->op.beta_v, &op->op.as_v, &op->op.ar_v};
  void** dst[3] = {m->bv, m->asv, m->arv};
  for (int i = 0; i < 3 && e == hipSuccess; ++i) {
    keep64.push_back(*vv[i]);
    keep32.push_back(std::vector<float>(vv[i]->begin(), vv[i]->end()));
    e = upload(dst[i][0], keep64.back(), m->stream);
    if (e == hipSuccess) e = upload(dst[i][1], keep32.back(), m->stream);
  }
  // the operator's Thomas margins, before the autotuner times the smoothers
  for (int l = 0; l < m->nlev && e == hipSuccess; ++l) {
    const tpmg::LevelView v64 = m->view64(l);
    for (int i = 0; i < 2 && e == hipSuccess; ++i)
      if (m->lv[l].margin[i]) e = tpmg::launch_margins(v64, i == 0 ? 8 : 4, m->lv[l].margin[i], m->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  (void)nz;
  if (e != hipSuccess) return cleanup_fail(TPMG_ERR_DEVICE, std::string("setup upload: ") + hipGetErrorString(e));
  if ((st = choose_tuning(*m, *params, true)) != TPMG_OK) {
    const std::string msg = g_last_error;
    return cleanup_fail(st, msg);
  }
  *out = m;
  return TPMG_OK;
}

}  // namespace

extern "C" {

tpmg_status tpmg_mg_setup(const tpmg_op* op, const tpmg_mg_params* params, void* d_workspace, size_t bytes,
                          void* hip_stream, tpmg_mg** out) {
  return setup_impl(op, params, d_workspace, bytes, hip_stream, true, out);
}

tpmg_status tpmg_mg_tuning(const tpmg_mg* mg, int level, int* smoother, int* scan_levels, int* chunk_restrict,
                           int* chunk_prolong, int* chunk_spmv) {
  tpmg_status st = check_mg(mg);
  if (st != TPMG_OK) return st;
  if (level < 0 || level >= mg->nlev) return fail(TPMG_ERR_ARG, "level out of range");
  const tpmg::LevelTune& t = mg->tune[level];
  const int npad = mg->lv[level].npad;
  if (smoother) *smoother = t.smoother + 1;
  if (scan_levels) *scan_levels = t.scan_levels;
  if (chunk_restrict) *chunk_restrict = level > 0 ? tpmg::effective_chunk(t.chunk_rr, npad, mg->nz) : 0;
  if (chunk_prolong) *chunk_prolong = level > 0 ? tpmg::effective_chunk(t.chunk_pr, npad, mg->nz) : 0;
  if (chunk_spmv) *chunk_spmv = level + 1 == mg->nlev ? tpmg::effective_chunk(t.chunk_spmv, npad, mg->nz) : 0;
  return TPMG_OK;
}

tpmg_status tpmg_mg_autotune_stats(const tpmg_mg* mg, int* trials, double* trial_ms) {
  tpmg_status st = check_mg(mg);
  if (st != TPMG_OK) return st;
  if (trials) *trials = mg->tune_trials;
  if (trial_ms) *trial_ms = mg->tune_ms;
  return TPMG_OK;
}

tpmg_status tpmg_tune_load(const char* path) {
  if (!path) return fail(TPMG_ERR_ARG, "path is NULL");
  std::ifstream in(path, std::ios::binary);
  if (!in) return fail(TPMG_ERR_ARG, std::string("cannot read ") + path);
  std::stringstream ss;
  ss << in.rdbuf();
  std::map<std::string, std::array<int, 2>> parsed;
  if (!parse_tune_json(ss.str(), parsed)) return fail(TPMG_ERR_ARG, std::string("malformed tuning file ") + path);
  TuneCache& c = tune_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  for (const auto& kv : parsed) c.map[kv.first] = kv.second;
  return TPMG_OK;
}

tpmg_status tpmg_tune_save(const char* path) {
  if (!path) return fail(TPMG_ERR_ARG, "path is NULL");
  std::string text = "{\n";
  {
    TuneCache& c = tune_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    size_t i = 0;
    for (const auto& kv : c.map) {
      text += "  \"" + kv.first + "\": [" + std::to_string(kv.second[0]) + ", " + std::to_string(kv.second[1]) + "]";
      text += ++i < c.map.size() ? ",\n" : "\n";
    }
  }
  text += "}\n";
  std::ofstream out(path, std::ios::binary | std::ios::trunc);
  if (!out) return fail(TPMG_ERR_ARG, std::string("cannot write ") + path);
  out << text;
  out.close();
  if (!out) return fail(TPMG_ERR_ARG, std::string("write failed: ") + path);
  return TPMG_OK;
}

tpmg_status tpmg_tune_clear(void) {
  TuneCache& c = tune_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  c.map.clear();
  return TPMG_OK;
}

tpmg_status tpmg_tune_entries(int* n) {
  if (!n) return fail(TPMG_ERR_ARG, "n is NULL");
  TuneCache& c = tune_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  *n = static_cast<int>(c.map.size());
  return TPMG_OK;
}

tpmg_status tpmg_mg_vector_length(const tpmg_mg* mg, size_t* n_doubles, int* n_cells, int* nz) {
  tpmg_status st = check_mg(mg);
  if (st != TPMG_OK) return st;
  if (n_doubles) *n_doubles = mg->len;
  if (n_cells) *n_cells = mg->n_fine;
  if (nz) *nz = mg->nz;
  return TPMG_OK;
}

tpmg_status tpmg_pack(tpmg_mg* mg, const double* d_cellmajor, double* d_tiled) {
  tpmg_status st = check_mg(mg);
  if (st != TPMG_OK) return st;
  if (!d_cellmajor || !d_tiled) return fail(TPMG_ERR_ARG, "NULL vector");
  TPMG_HIP(tpmg::launch_pack(d_cellmajor, d_tiled, mg->n_fine, mg->npad_fine, mg->nz, mg->stream));
  return TPMG_OK;
}

tpmg_status tpmg_unpack(tpmg_mg* mg, const double* d_tiled, double* d_cellmajor) {
  tpmg_status st = check_mg(mg);
  if (st != TPMG_OK) return st;
  if (!d_cellmajor || !d_tiled) return fail(TPMG_ERR_ARG, "NULL vector");
  TPMG_HIP(tpmg::launch_unpack(d_tiled, d_cellmajor, mg->n_fine, mg->npad_fine, mg->nz, mg->stream));
  return TPMG_OK;
}

tpmg_status tpmg_spmv(tpmg_mg* mg, const double* d_x, double* d_y) {
  tpmg_status st = check_mg(mg);
  if (st != TPMG_OK) return st;
  if (!d_x || !d_y) return fail(TPMG_ERR_ARG, "NULL vector");
  if (d_x == d_y) return fail(TPMG_ERR_ARG, "x and y must not alias");
  TPMG_HIP(tpmg::launch_spmv64(mg->view_outer(), 0, d_x, nullptr, d_y, mg->partials, tpmg::kFinNone, mg->scal,
                                mg->stream));
  return TPMG_OK;
}

tpmg_status tpmg_vcycle(tpmg_mg* mg, const double* d_r, double* d_z) {
  tpmg_status st = check_mg(mg);
  if (st != TPMG_OK) return st;
  if (!d_r || !d_z) return fail(TPMG_ERR_ARG, "NULL vector");
  if (d_r == d_z) return fail(TPMG_ERR_ARG, "r and z must not alias");
  TPMG_HIP(vcycle(*mg, d_r, d_z));
  return TPMG_OK;
}

namespace {

// Waits until the record with sequence number seq is in the ring (spinning on
// the pinned slot; the stream is asked from time to time whether it failed or
// went idle without publishing it).
hipError_t wait_record(const tpmg::FcgRecord* ring, int seq, hipStream_t s, tpmg::FcgRecord* out) {
  const tpmg::FcgRecord* slot = ring + (seq % tpmg::kRecords);
  for (unsigned spin = 1;; ++spin) {
    if (__atomic_load_n(&slot->seq, __ATOMIC_ACQUIRE) == seq) break;
    if ((spin & 1023u) == 0) {
      const hipError_t q = hipStreamQuery(s);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) return q;
      if (__atomic_load_n(&slot->seq, __ATOMIC_ACQUIRE) == seq) break;
      return hipErrorUnknown;   // idle stream, record never published
    }
  }
  out->rr = slot->rr;
  out->ff = slot->ff;
  out->status = slot->status;
  out->done = slot->done;
  out->iters = slot->iters;
  out->seq = seq;
  return hipSuccess;
}

}  // namespace

tpmg_status tpmg_solve(tpmg_mg* mg, const double* d_f, double* d_u, double rtol, int maxit, tpmg_solve_info* info) {
  tpmg_status st = check_mg(mg);
  if (st != TPMG_OK) return st;
  if (!d_f || !d_u) return fail(TPMG_ERR_ARG, "NULL vector");
  if (d_f == d_u) return fail(TPMG_ERR_ARG, "f and u must not alias");
  if (!(rtol >= 0.0) || maxit < 0) return fail(TPMG_ERR_ARG, "rtol must be >= 0 and maxit >= 0");
  if (info && info->history_cap > 0 && !info->history) return fail(TPMG_ERR_ARG, "history_cap > 0 with NULL history");
  if (info && !(info->div_tol >= 0.0)) return fail(TPMG_ERR_ARG, "div_tol must be >= 0");
  if (mg->adv)
    return fail(TPMG_ERR_ARG, "the operator with vertical advection is not symmetric: use tpmg_solve_bicgstab or "
                              "tpmg_solve_richardson");
  const bool timers = info && info->phase_timers != 0;
  const double div2 = info && info->div_tol > 0.0 ? info->div_tol * info->div_tol : tpmg::kDefaultDiv2;
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = mg->stream;
  const tpmg::LevelView F = mg->view_outer();
  // one FCG iteration as a list of operations (also the basis of the byte
  // count and of the per-phase timers)
  std::vector<Op> iter_ops;
  fcg_ops(*mg, d_u, mg->scal, iter_ops);
  const bool graph = mg->use_graph && !timers;
  // the iteration as a graph, captured once per solution vector (on an idle
  // stream, before this solve's work is queued)
  if (maxit > 0 && graph && (mg->graph_x != d_u || mg->graph == nullptr)) {
    TPMG_HIP(hipStreamSynchronize(s));
    drop_graph(*mg);
    hipGraph_t g = nullptr;
    TPMG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t ce = fcg_iteration(*mg, d_u);
    hipError_t ee = hipStreamEndCapture(s, &g);
    if (ce != hipSuccess || ee != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(TPMG_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(ce != hipSuccess ? ce : ee));
    }
    hipError_t ie = hipGraphInstantiate(&mg->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
      mg->graph = nullptr;
      return fail(TPMG_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    }
    mg->graph_x = d_u;
  }
  // per-phase timers: an event where a phase starts (its phase) and where a
  // timed stretch ends (-1); the gaps between iterations are not counted
  std::vector<std::pair<hipEvent_t, int>> marks;
  auto mark = [&](int phase) -> hipError_t {
    if (marks.size() == mg->tev.size()) {
      hipEvent_t ev = nullptr;
      const hipError_t ce = hipEventCreate(&ev);
      if (ce != hipSuccess) return ce;
      mg->tev.push_back(ev);
    }
    const hipEvent_t ev = mg->tev[marks.size()];
    marks.emplace_back(ev, phase);
    return hipEventRecord(ev, s);
  };
  auto run_ops = [&](const std::vector<Op>& ops) -> hipError_t {
    int cur = -1;
    for (const Op& op : ops) {
      if (timers && op_phase(op) != cur) {
        cur = op_phase(op);
        const hipError_t me = mark(cur);
        if (me != hipSuccess) return me;
      }
      const hipError_t e = exec_op(op, s);
      if (e != hipSuccess) return e;
    }
    return timers ? mark(-1) : hipSuccess;
  };
  // no slot holds a record of this solve yet (the previous solve ended with
  // its stream drained)
  for (int i = 0; i < tpmg::kRecords; ++i) mg->ring[i].seq = -1;
  // r = f - A u, rr, ff (published as record 0), and for an FP32 V-cycle its
  // first right-hand side, the FP32 rounding of r (later ones come with the r
  // update). The first iteration takes beta = 0 and p = z, reading neither
  // q nor the ring's previous slot.
  if (timers) TPMG_HIP(mark(1));
  TPMG_HIP(tpmg::launch_spmv64(F, 1, d_u, d_f, mg->r, mg->partials, tpmg::kFinInit, mg->scal, s, rtol,
                               mg->fp32 ? static_cast<float*>(mg->fcopy) : nullptr, mg->ring_dev, div2));
  if (timers) TPMG_HIP(mark(-1));
  int launched = 0;
  auto launch_next = [&]() -> hipError_t {
    ++launched;
    return graph ? hipGraphLaunch(mg->graph, s) : run_ops(iter_ops);
  };
  // The first iteration is queued before the host reads record 0: when the
  // initial residual already meets the tolerance (or is not finite) the
  // device flag is set and the iteration leaves everything as it was.
  hipError_t werr = hipSuccess;
  if (maxit > 0) werr = launch_next();
  tpmg::FcgRecord rec0;
  if (werr == hipSuccess) werr = wait_record(mg->ring, 0, s, &rec0);
  if (werr != hipSuccess) {
    (void)hipStreamSynchronize(s);
    return fail(TPMG_ERR_DEVICE, std::string("solve: ") + hipGetErrorString(werr));
  }
  const double ff = rec0.ff;
  const double fnorm = std::sqrt(ff);
  double rnorm = std::sqrt(rec0.rr);
  int iters = 0;
  bool diverged = false;
  auto record = [&](int k, double v) {
    if (info && info->history && k < info->history_cap) info->history[k] = v;
  };
  record(0, fnorm > 0 ? rnorm / fnorm : 0.0);
  tpmg_status result = TPMG_NOT_CONVERGED;
  if (!std::isfinite(rnorm) || !std::isfinite(fnorm)) {
    result = TPMG_ERR_BREAKDOWN;
  } else if (rnorm <= rtol * fnorm) {
    result = TPMG_OK;
  } else {
    // Iteration it+1 is queued before the host waits for iteration it's
    // record unless the residual norms so far suggest that iteration it may
    // converge: a queued iteration after convergence is left without effect
    // (the update and the scalars skip once done) but costs its time.
    const double target = rtol * fnorm;
    double prev = rnorm;   // norm before the last known one (ratio estimate)
    for (int it = 0; it < maxit; ++it) {
      if (launched == it) TPMG_HIP(launch_next());
      const double ratio = prev > 0.0 ? std::min(1.0, rnorm / prev) : 1.0;
      const bool ahead = it + 1 < maxit && rnorm * ratio > 3.0 * target;
      if (ahead && launched == it + 1) TPMG_HIP(launch_next());
      tpmg::FcgRecord rec;
      if ((werr = wait_record(mg->ring, it + 1, s, &rec)) != hipSuccess) break;
      iters = it + 1;
      if (rec.status == 2) {
        // ||r|| > div_tol ||r_0||: the iterate is finite and kept
        rnorm = std::sqrt(rec.rr);
        record(iters, fnorm > 0 ? rnorm / fnorm : 0.0);
        diverged = true;
        result = TPMG_ERR_BREAKDOWN;
        break;
      }
      if (rec.status != 0) {
        iters = it;
        result = TPMG_ERR_BREAKDOWN;
        break;
      }
      prev = rnorm;
      rnorm = std::sqrt(rec.rr);
      record(iters, fnorm > 0 ? rnorm / fnorm : 0.0);
      if (!std::isfinite(rnorm)) {
        result = TPMG_ERR_BREAKDOWN;
        break;
      }
      if (rnorm <= target) {
        result = TPMG_OK;
        break;
      }
    }
  }
  // x += alpha p of the iterations not yet added (after an iteration queued
  // ahead, which changes neither iters nor the ring's counted slots)
  if (timers && werr == hipSuccess) werr = mark(2);
  hipError_t fe = tpmg::launch_flush(d_u, mg->dirs, mg->scal, mg->len, s);
  if (werr == hipSuccess) werr = fe;
  if (timers && werr == hipSuccess) werr = mark(-1);
  // drains an iteration queued ahead; reports the first device error
  const hipError_t se = hipStreamSynchronize(s);
  if (werr != hipSuccess || se != hipSuccess)
    return fail(TPMG_ERR_DEVICE, std::string("solve: ") + hipGetErrorString(werr != hipSuccess ? werr : se));
  const auto t1 = std::chrono::steady_clock::now();
  if (info) {
    info->iters = iters;
    info->relres = fnorm > 0 ? rnorm / fnorm : 0.0;
    info->t_total_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    info->t_vcycle_ms = info->t_spmv_ms = info->t_blas_ms = 0.0;
    double* tp[3] = {&info->t_vcycle_ms, &info->t_spmv_ms, &info->t_blas_ms};
    for (size_t i = 0; i + 1 < marks.size(); ++i) {
      if (marks[i].second < 0) continue;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, marks[i].first, marks[i + 1].first) == hipSuccess) *tp[marks[i].second] += ms;
    }
    // the device ran the iterations it counted (one queued after the last
    // returned at once)
    info->model_bytes = solve_model_bytes(iter_ops, iters, mg->len, mg->fp32, true, mg->full_outer);
  }
  if (diverged) return fail(TPMG_ERR_BREAKDOWN, "divergence: ||r|| exceeded div_tol ||r_0||");
  if (result == TPMG_ERR_BREAKDOWN) return fail(result, "breakdown: non-finite value or <p, A p> <= 0");
  return result;
}

tpmg_status tpmg_relax(tpmg_mg* mg, const double* d_f, const double* d_u_in, double* d_u_out) {
  tpmg_status st = check_mg(mg);
  if (st != TPMG_OK) return st;
  if (!d_f || !d_u_in || !d_u_out) return fail(TPMG_ERR_ARG, "NULL vector");
  if (d_u_in == d_u_out || d_f == d_u_out) return fail(TPMG_ERR_ARG, "u_out must not alias f or u_in");
  const tpmg::LevelTune t = tpmg::default_tune(mg->nz, 8);
  if (t.smoother == tpmg::kSmGlobal || (mg->pm != 0 && t.smoother != tpmg::kSmScan))
    return fail(TPMG_ERR_ARG, "tpmg_relax: nz = " + std::to_string(mg->nz) +
                                  " is beyond the FP64 line smoothers that need no scratch");
  TPMG_HIP(tpmg_relax_finest(mg, d_f, d_u_in, d_u_out, nullptr, nullptr, 1.0, mg->stream));
  return TPMG_OK;
}

namespace {

// The two outer solvers of the paper (Section 5.2), for any operator of the
// handle (with vertical advection the only ones it accepts): the host reads
// the residual norm after each iteration (one copy of the scalars).
tpmg_status krylov_check(tpmg_mg* mg, const double* d_f, double* d_u, double rtol, int maxit,
                         const tpmg_solve_info* info) {
  tpmg_status st = check_mg(mg);
  if (st != TPMG_OK) return st;
  if (!d_f || !d_u) return fail(TPMG_ERR_ARG, "NULL vector");
  if (d_f == d_u) return fail(TPMG_ERR_ARG, "f and u must not alias");
  if (!(rtol >= 0.0) || maxit < 0) return fail(TPMG_ERR_ARG, "rtol must be >= 0 and maxit >= 0");
  if (info && info->history_cap > 0 && !info->history) return fail(TPMG_ERR_ARG, "history_cap > 0 with NULL history");
  if (info && info->phase_timers) return fail(TPMG_ERR_ARG, "phase timers are available with tpmg_solve only");
  if (!mg->pinned) return fail(TPMG_ERR_STATE, "handle without pinned scalars");
  return TPMG_OK;
}

hipError_t read_scalars(tpmg_mg& m) {
  hipError_t e = hipMemcpyAsync(m.h_scal, m.scal, sizeof(tpmg::FcgScalars), hipMemcpyDeviceToHost, m.stream);
  return e == hipSuccess ? hipStreamSynchronize(m.stream) : e;
}

}  // namespace

tpmg_status tpmg_solve_richardson(tpmg_mg* mg, const double* d_f, double* d_u, double rtol, int maxit,
                                  tpmg_solve_info* info) {
  tpmg_status st = krylov_check(mg, d_f, d_u, rtol, maxit, info);
  if (st != TPMG_OK) return st;
  const auto t0 = std::chrono::steady_clock::now();
  tpmg_mg& m = *mg;
  hipStream_t s = m.stream;
  const tpmg::LevelView F = m.view_outer();
  double fnorm = 0.0, rnorm = 0.0;
  int it = 0;
  tpmg_status result = TPMG_NOT_CONVERGED;
  for (;; ++it) {
    // r = f - A u, ||r||^2 and ||f||^2
    TPMG_HIP(tpmg::launch_spmv64(F, 1, d_u, d_f, m.r, m.partials, tpmg::kFinInit, m.scal, s, rtol));
    TPMG_HIP(read_scalars(m));
    fnorm = std::sqrt(m.h_scal->ff);
    rnorm = std::sqrt(m.h_scal->rr);
    if (info && info->history && it < info->history_cap) info->history[it] = fnorm > 0 ? rnorm / fnorm : 0.0;
    if (!std::isfinite(rnorm)) {
      result = TPMG_ERR_BREAKDOWN;
      break;
    }
    if (rnorm <= rtol * fnorm) {
      result = TPMG_OK;
      break;
    }
    if (it == maxit) break;
    // u += M r
    TPMG_HIP(vcycle(m, m.r, m.z));
    TPMG_HIP(tpmg::launch_add(d_u, m.z, m.len, s));
  }
  TPMG_HIP(hipStreamSynchronize(s));
  if (info) {
    info->iters = it;
    info->relres = fnorm > 0 ? rnorm / fnorm : 0.0;
    info->t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    info->t_vcycle_ms = info->t_spmv_ms = info->t_blas_ms = 0.0;
    std::vector<Op> vc;
    vcycle_ops(m, m.r, m.z, nullptr, m.scal, vc);
    double vb = 0.0;
    for (const Op& op : vc) vb += op_model_bytes(op, 1);
    const double n = static_cast<double>(m.len);
    const double ab = (24.0 + (m.adv ? 56.0 : m.full_outer ? 40.0 : 0.0)) * n;   // r = f - A u
    info->model_bytes = (it + 1) * ab + it * (vb + 24.0 * n);
  }
  if (result == TPMG_ERR_BREAKDOWN) return fail(result, "breakdown: non-finite residual");
  return result;
}

tpmg_status tpmg_solve_bicgstab(tpmg_mg* mg, const double* d_f, double* d_u, double rtol, int maxit,
                                tpmg_solve_info* info) {
  tpmg_status st = krylov_check(mg, d_f, d_u, rtol, maxit, info);
  if (st != TPMG_OK) return st;
  const auto t0 = std::chrono::steady_clock::now();
  tpmg_mg& m = *mg;
  hipStream_t s = m.stream;
  const tpmg::LevelView F = m.view_outer();
  const size_t len = m.len;
  // vectors: r (then s) in r, p in p, v in q, y = M p in z, the shadow
  // residual, z = M s and t in three slots of the direction ring
  double* r = m.r;
  double* p = m.p;
  double* v = m.q;
  double* y = m.z;
  double* rh = m.dirs;
  double* zs = m.dirs + len;
  double* t = m.dirs + 2 * len;
  TPMG_HIP(tpmg::launch_spmv64(F, 1, d_u, d_f, r, m.partials, tpmg::kFinInit, m.scal, s, rtol));
  TPMG_HIP(hipMemcpyAsync(rh, r, len * sizeof(double), hipMemcpyDeviceToDevice, s));
  TPMG_HIP(tpmg::launch_fill(p, len * sizeof(double), s));
  TPMG_HIP(tpmg::launch_fill(v, len * sizeof(double), s));
  TPMG_HIP(tpmg::launch_krylov_finalize(tpmg::kKInit, m.partials, m.scal, s));
  TPMG_HIP(read_scalars(m));
  const double fnorm = std::sqrt(m.h_scal->ff);
  double rnorm = std::sqrt(m.h_scal->rr);
  auto record = [&](int k) {
    if (info && info->history && k < info->history_cap) info->history[k] = fnorm > 0 ? rnorm / fnorm : 0.0;
  };
  record(0);
  int it = 0;
  tpmg_status result = TPMG_NOT_CONVERGED;
  if (!std::isfinite(rnorm)) {
    result = TPMG_ERR_BREAKDOWN;
  } else if (rnorm <= rtol * fnorm) {
    result = TPMG_OK;
  } else {
    for (; it < maxit;) {
      TPMG_HIP(tpmg::launch_bicg_p(r, p, v, m.scal, len, s));
      TPMG_HIP(vcycle(m, p, y));
      TPMG_HIP(tpmg::launch_spmv64(F, 0, y, nullptr, v, m.partials, tpmg::kFinNone, m.scal, s));
      TPMG_HIP(tpmg::launch_dots2(rh, v, rh, v, len, m.partials, s));
      TPMG_HIP(tpmg::launch_krylov_finalize(tpmg::kKAlpha, m.partials, m.scal, s));
      TPMG_HIP(tpmg::launch_bicg_s(r, v, m.scal, len, s));
      TPMG_HIP(vcycle(m, r, zs));
      TPMG_HIP(tpmg::launch_spmv64(F, 0, zs, nullptr, t, m.partials, tpmg::kFinNone, m.scal, s));
      TPMG_HIP(tpmg::launch_dots2(t, r, t, t, len, m.partials, s));
      TPMG_HIP(tpmg::launch_krylov_finalize(tpmg::kKOmega, m.partials, m.scal, s));
      TPMG_HIP(tpmg::launch_bicg_x(d_u, r, y, zs, t, rh, m.scal, len, m.partials, s));
      TPMG_HIP(tpmg::launch_krylov_finalize(tpmg::kKRho, m.partials, m.scal, s));
      TPMG_HIP(read_scalars(m));
      ++it;
      rnorm = std::sqrt(m.h_scal->rr);
      record(it);
      if (m.h_scal->status != 0 || !std::isfinite(rnorm)) {
        result = TPMG_ERR_BREAKDOWN;
        break;
      }
      if (rnorm <= rtol * fnorm) {
        result = TPMG_OK;
        break;
      }
    }
  }
  TPMG_HIP(hipStreamSynchronize(s));
  if (info) {
    info->iters = it;
    info->relres = fnorm > 0 ? rnorm / fnorm : 0.0;
    info->t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    info->t_vcycle_ms = info->t_spmv_ms = info->t_blas_ms = 0.0;
    std::vector<Op> vc;
    vcycle_ops(m, r, zs, nullptr, m.scal, vc);
    double vb = 0.0;
    for (const Op& op : vc) vb += op_model_bytes(op, 1);
    const double n = static_cast<double>(len);
    const double ab = (16.0 + (m.adv ? 56.0 : m.full_outer ? 40.0 : 0.0)) * n;   // v = A y, t = A z
    // per iteration: p update 24, two V-cycles, two operators, dots 16 + 24,
    // s update 24, x/r update 64
    info->model_bytes = (32.0 + (m.adv ? 56.0 : m.full_outer ? 40.0 : 0.0)) * n +
                        it * (2.0 * vb + 2.0 * ab + (24.0 + 16.0 + 24.0 + 24.0 + 64.0) * n);
  }
  if (result == TPMG_ERR_BREAKDOWN) return fail(result, "breakdown: zero or non-finite BiCGStab scalar");
  return result;
}

tpmg_status tpmg_richardson_rate(tpmg_mg* mg, double* d_u, int cycles, int skip, double* rate, double* norms) {
  tpmg_status st = check_mg(mg);
  if (st != TPMG_OK) return st;
  if (!d_u || !rate) return fail(TPMG_ERR_ARG, "NULL argument");
  if (skip < 0 || cycles <= skip) return fail(TPMG_ERR_ARG, "need 0 <= skip < cycles");
  hipStream_t s = mg->stream;
  const tpmg::LevelView F = mg->view_outer();
  // p holds the zero right-hand side, r the residual -A u, z the correction
  TPMG_HIP(tpmg::launch_fill(mg->p, mg->len * 8, s));
  std::vector<double> nrm(cycles + 1);
  for (int i = 0; i <= cycles; ++i) {
    TPMG_HIP(tpmg::launch_spmv64(F, 1, d_u, mg->p, mg->r, mg->partials, tpmg::kFinInit, mg->scal, s));
    TPMG_HIP(hipMemcpyAsync(mg->h_scal, mg->scal, sizeof(tpmg::FcgScalars), hipMemcpyDeviceToHost, s));
    TPMG_HIP(hipStreamSynchronize(s));
    nrm[i] = std::sqrt(mg->h_scal->rr);
    if (i == cycles) break;
    TPMG_HIP(vcycle(*mg, mg->r, mg->z));
    TPMG_HIP(tpmg::launch_add(d_u, mg->z, mg->len, s));
  }
  if (norms) std::copy(nrm.begin(), nrm.end(), norms);
  if (!(nrm[skip] > 0.0) || !std::isfinite(nrm[cycles]))
    return fail(TPMG_ERR_BREAKDOWN, "residual norms not positive and finite");
  *rate = std::pow(nrm[cycles] / nrm[skip], 1.0 / (cycles - skip));
  return TPMG_OK;
}

tpmg_status tpmg_mg_time_sweep(tpmg_mg* mg, int reps, double* avg_ms, double* model_bytes) {
  tpmg_status st = check_mg(mg);
  if (st != TPMG_OK) return st;
  if (reps < 1 || !avg_ms) return fail(TPMG_ERR_ARG, "reps must be >= 1 and avg_ms non-NULL");
  const int L = mg->nlev - 1;
  const int prec = mg->fp32 ? 4 : 8;
  const tpmg::LevelView V = mg->view(L);
  // f: the FP32 copy (mixed) or the FCG residual buffer (FP64); u: the
  // finest ping-pong pair
  const void* f = mg->fp32 ? static_cast<const void*>(mg->fcopy) : static_cast<const void*>(mg->r);
  hipEvent_t e0, e1;
  TPMG_HIP(hipEventCreate(&e0));
  TPMG_HIP(hipEventCreate(&e1));
  hipError_t e = hipEventRecord(e0, mg->stream);
  for (int i = 0; i < reps && e == hipSuccess; ++i)
    e = tpmg::launch_smooth(V, prec, f, false, mg->lv[L].u[i & 1], false, mg->lv[L].u[1 - (i & 1)], false, nullptr,
                            mg->sd, mg->sc, mg->omega, mg->stream);
  if (e == hipSuccess) e = hipEventRecord(e1, mg->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(TPMG_ERR_DEVICE, std::string("time sweep: ") + hipGetErrorString(e));
  *avg_ms = static_cast<double>(ms) / reps;
  if (model_bytes) *model_bytes = 3.0 * (mg->fp32 ? 4.0 : 8.0) * static_cast<double>(mg->len);
  return TPMG_OK;
}

tpmg_status tpmg_mg_time_kernel(tpmg_mg* mg, int kernel, int reps, double* avg_ms, double* model_bytes) {
  tpmg_status st = check_mg(mg);
  if (st != TPMG_OK) return st;
  if (reps < 1 || !avg_ms) return fail(TPMG_ERR_ARG, "reps must be >= 1 and avg_ms non-NULL");
  if (kernel < 0 || kernel > 4) return fail(TPMG_ERR_ARG, "kernel must be 0 .. 4");
  if (kernel >= 3 && mg->nlev < 2) return fail(TPMG_ERR_ARG, "the transfer kernels need two levels");
  const int L = mg->nlev - 1;
  const int prec = mg->fp32 ? 4 : 8;
  const tpmg::LevelView V = mg->view(L);
  const tpmg::LevelView F = mg->view_outer();
  hipStream_t s = mg->stream;
  const bool z_float = mg->tune.back().smoother == tpmg::kSmScan && mg->fp32;
  if (kernel == 1 && !tpmg::spmv_pring_fits(F))
    return fail(TPMG_ERR_ARG, "the operator chunk of this grid has no direction-update instance");
  if (kernel == 1) {
    // scalars of an iteration in the middle of a solve (not done, iteration 1:
    // p_1 = z + beta p_0, no x update); the next solve's start resets them
    std::memset(mg->h_scal, 0, sizeof(tpmg::FcgScalars));
    mg->h_scal->iters = 1;
    mg->h_scal->beta = 0.5;
    TPMG_HIP(hipMemcpyAsync(mg->scal, mg->h_scal, sizeof(tpmg::FcgScalars), hipMemcpyHostToDevice, s));
  }
  const void* f = mg->fp32 ? static_cast<const void*>(mg->fcopy) : static_cast<const void*>(mg->r);
  const int Lc = L > 0 ? L - 1 : 0;
  auto launch = [&](int i) -> hipError_t {
    switch (kernel) {
      case 0:
        return tpmg::launch_smooth(V, prec, f, false, mg->lv[L].u[i & 1], false, mg->lv[L].u[1 - (i & 1)], false,
                                   nullptr, mg->sd, mg->sc, mg->omega, s);
      case 1:
        return tpmg::launch_spmv_pring(F, mg->z, !z_float, mg->dirs, mg->len, mg->p, mg->q, mg->partials, mg->scal, s,
                                       tpmg::kFinNone);
      case 2:
        return tpmg::launch_spmv64(F, 0, mg->p, nullptr, mg->q, mg->partials, tpmg::kFinNone, mg->scal, s);
      case 3:
        return tpmg::launch_residual_restrict(V, mg->view(Lc), prec, f, mg->lv[L].u[0], mg->lv[Lc].f, s);
      default:
        return tpmg::launch_prolong_add(V, mg->view(Lc), prec, mg->lv[Lc].u[0], mg->lv[L].u[0], s);
    }
  };
  hipEvent_t e0, e1;
  TPMG_HIP(hipEventCreate(&e0));
  TPMG_HIP(hipEventCreate(&e1));
  hipError_t e = launch(0);   // one untimed launch
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  for (int i = 0; i < reps && e == hipSuccess; ++i) e = launch(i + 1);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(TPMG_ERR_DEVICE, std::string("time kernel: ") + hipGetErrorString(e));
  *avg_ms = static_cast<double>(ms) / reps;
  if (model_bytes) {
    const double n = static_cast<double>(mg->len);
    const double s_b = prec;
    // (coefficients per (T, k): five values per unknown, or the radial one)
    const double cv = mg->pm == 3 ? 7.0 : mg->pm == 2 ? 5.0 : mg->pm == 1 ? 1.0 : 0.0;
    const double co = mg->adv ? 56.0 : mg->full_outer ? 40.0 : 0.0;
    switch (kernel) {
      case 0: *model_bytes = (3.0 + cv) * s_b * n; break;
      case 1: *model_bytes = ((z_float ? 4.0 : 8.0) + 24.0 + co) * n; break;
      case 2: *model_bytes = (16.0 + co) * n; break;
      case 3: *model_bytes = (2.0 * s_b + s_b / 4.0 + cv * s_b) * n; break;
      default: *model_bytes = (2.0 * s_b + s_b / 4.0) * n; break;
    }
  }
  return TPMG_OK;
}

tpmg_status tpmg_batch_workspace_size(tpmg_mg* const* problems, int n, size_t* bytes) {
  if (!bytes) return fail(TPMG_ERR_ARG, "bytes is NULL");
  tpmg_status st = check_batch(problems, n);
  if (st != TPMG_OK) return st;
  tpmg_batch b;
  b.probs.assign(problems, problems + n);
  size_t nseg = 0;
  if (build_plan(b, nullptr, false, &nseg) != hipSuccess) return fail(TPMG_ERR_ARG, "problems disagree on the schedule");
  Carver cv(nullptr);
  cv.take(static_cast<size_t>(n) * sizeof(tpmg::FcgScalars));
  cv.take(nseg * sizeof(tpmg::Seg));
  *bytes = cv.off + 256;
  return TPMG_OK;
}

tpmg_status tpmg_batch_create(tpmg_mg* const* problems, int n, void* d_workspace, size_t bytes, tpmg_batch** out) {
  if (!out) return fail(TPMG_ERR_ARG, "out is NULL");
  *out = nullptr;
  size_t need = 0;
  tpmg_status st = tpmg_batch_workspace_size(problems, n, &need);
  if (st != TPMG_OK) return st;
  if (!d_workspace || reinterpret_cast<uintptr_t>(d_workspace) % 256 != 0)
    return fail(TPMG_ERR_ARG, "workspace must be non-NULL and 256-byte aligned");
  if (bytes < need) return fail(TPMG_ERR_NOMEM, "batch workspace too small: need " + std::to_string(need) + " bytes");
  auto* b = new tpmg_batch();
  b->probs.assign(problems, problems + n);
  b->stream = problems[0]->stream;
  Carver cv(d_workspace);
  b->scal = static_cast<tpmg::FcgScalars*>(cv.take(static_cast<size_t>(n) * sizeof(tpmg::FcgScalars)));
  b->max_segs = (need - 256 - (static_cast<size_t>(n) * sizeof(tpmg::FcgScalars) + 255) / 256 * 256) / sizeof(tpmg::Seg);
  b->segs = static_cast<tpmg::Seg*>(cv.take(b->max_segs * sizeof(tpmg::Seg)));
  hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&b->h_scal), 3 * static_cast<size_t>(n) * sizeof(tpmg::FcgScalars),
                               hipHostMallocDefault);
  for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&b->ev[i], hipEventDisableTiming);
  // (the streams that capture the graph's branches; default priority)
  const int nbr = std::min(n, kBatchBranches);
  if (e == hipSuccess && nbr > 1) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  for (int k = 0; k + 1 < nbr && e == hipSuccess; ++k) {
    e = hipStreamCreateWithFlags(&b->aux[k], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    tpmg_batch_destroy(b);
    return fail(TPMG_ERR_DEVICE, std::string("batch host buffers: ") + hipGetErrorString(e));
  }
  *out = b;
  return TPMG_OK;
}

tpmg_status tpmg_batch_solve(tpmg_batch* b, const double* const* d_f, double* const* d_u, double rtol, int maxit,
                             tpmg_solve_info* infos) {
  if (!b || !d_f || !d_u) return fail(TPMG_ERR_ARG, "NULL argument");
  if (!(rtol >= 0.0) || maxit < 0) return fail(TPMG_ERR_ARG, "rtol must be >= 0 and maxit >= 0");
  const int n = static_cast<int>(b->probs.size());
  for (int p = 0; p < n; ++p) {
    if (!d_f[p] || !d_u[p] || d_f[p] == d_u[p]) return fail(TPMG_ERR_ARG, "NULL or aliasing f/u");
    if (infos && infos[p].history_cap > 0 && !infos[p].history)
      return fail(TPMG_ERR_ARG, "history_cap > 0 with NULL history");
  }
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = b->stream;
  // per problem: r = f - A u, rr, ff (kFinInit also marks already-converged
  // problems done), with the ring form the FP32 copy of r for an FP32
  // V-cycle; the first iteration takes beta = 0 (p = 0 for the in-place
  // form, whose update reads it)
  const bool ring = batch_ring(*b);
  // (each problem's start and end run on its branch's stream, forked from
  // the batch's stream and joined back, so that they overlap as the
  // iterations do)
  const std::vector<std::vector<int>> groups = batch_groups(*b);
  auto fork = [&]() -> hipError_t {
    if (groups.size() < 2) return hipSuccess;
    hipError_t e = hipEventRecord(b->fork, s);
    for (size_t k = 1; k < groups.size() && e == hipSuccess; ++k) e = hipStreamWaitEvent(b->aux[k - 1], b->fork, 0);
    return e;
  };
  auto join = [&]() -> hipError_t {
    hipError_t e = hipSuccess;
    for (size_t k = 1; k < groups.size() && e == hipSuccess; ++k) {
      e = hipEventRecord(b->join[k - 1], b->aux[k - 1]);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, b->join[k - 1], 0);
    }
    return e;
  };
  TPMG_HIP(fork());
  for (size_t k = 0; k < groups.size(); ++k) {
    hipStream_t sk = k == 0 ? s : b->aux[k - 1];
    for (int p : groups[k]) {
      tpmg_mg& m = *b->probs[p];
      TPMG_HIP(tpmg::launch_spmv64(m.view_outer(), 1, d_u[p], d_f[p], m.r, m.partials, tpmg::kFinInit, b->scal + p,
                                    sk, rtol, ring && m.fp32 ? static_cast<float*>(m.fcopy) : nullptr));
      if (!ring) TPMG_HIP(tpmg::launch_fill(m.p, m.len * 8, sk));
    }
  }
  TPMG_HIP(join());
  const bool rebuild = b->plan_u.size() != static_cast<size_t>(n) || !std::equal(b->plan_u.begin(), b->plan_u.end(), d_u);
  if (rebuild || b->graph == nullptr) {
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
    b->plan_u.clear();
    hipError_t e = build_plan(*b, d_u, true, nullptr);
    if (e != hipSuccess) return fail(TPMG_ERR_DEVICE, std::string("batch plan: ") + hipGetErrorString(e));
    hipGraph_t g = nullptr;
    TPMG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    // branch 0 on the batch's stream, the others forked from it and joined
    // back (every branch is joined, also after a failed launch, so that the
    // capture ends)
    const int nbr = static_cast<int>(b->plans.size());
    hipError_t ce = nbr > 1 ? hipEventRecord(b->fork, s) : hipSuccess;
    int forked = 1;
    for (; forked < nbr && ce == hipSuccess; ++forked) ce = hipStreamWaitEvent(b->aux[forked - 1], b->fork, 0);
    if (ce != hipSuccess) --forked;
    for (int k = 0; k < nbr && ce == hipSuccess; ++k) {
      hipStream_t sk = k == 0 ? s : b->aux[k - 1];
      for (const tpmg::BatchLaunch& L : b->plans[k])
        if ((ce = tpmg::launch_batched(L, sk)) != hipSuccess) break;
    }
    for (int k = 1; k < forked; ++k) {
      hipError_t je = hipEventRecord(b->join[k - 1], b->aux[k - 1]);
      if (je == hipSuccess) je = hipStreamWaitEvent(s, b->join[k - 1], 0);
      if (ce == hipSuccess) ce = je;
    }
    hipError_t ee = hipStreamEndCapture(s, &g);
    if (ce != hipSuccess || ee != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(TPMG_ERR_DEVICE, std::string("batch graph capture: ") + hipGetErrorString(ce != hipSuccess ? ce : ee));
    }
    hipError_t ie = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
      b->graph = nullptr;
      return fail(TPMG_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    }
    b->plan_u.assign(d_u, d_u + n);
  }
  const size_t sbytes = static_cast<size_t>(n) * sizeof(tpmg::FcgScalars);
  TPMG_HIP(hipMemcpyAsync(b->h_scal, b->scal, sbytes, hipMemcpyDeviceToHost, s));
  TPMG_HIP(hipStreamSynchronize(s));
  const tpmg::FcgScalars* cur = b->h_scal;   // the latest scalars the host has
  std::vector<double> fnorm(n), rn(n), prev(n);
  for (int p = 0; p < n; ++p) {
    fnorm[p] = std::sqrt(cur[p].ff);
    rn[p] = prev[p] = std::sqrt(cur[p].rr);
    if (infos && infos[p].history && infos[p].history_cap > 0)
      infos[p].history[0] = fnorm[p] > 0 ? rn[p] / fnorm[p] : 0.0;
  }
  auto all_done = [&]() {
    for (int p = 0; p < n; ++p)
      if (!cur[p].done) return false;
    return true;
  };
  // Iteration it+1 is queued before the host waits for iteration it's
  // scalars unless every unfinished problem may converge in it; a queued
  // iteration after all have converged does nothing (every operation of a
  // finished problem is skipped on the device) and costs only its launches.
  int launched = 0;
  auto launch_next = [&]() -> hipError_t {
    const int slot = launched % 2;
    hipError_t e = hipGraphLaunch(b->graph, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b->h_scal + static_cast<size_t>(1 + slot) * n, b->scal, sbytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipEventRecord(b->ev[slot], s);
    ++launched;
    return e;
  };
  hipError_t werr = hipSuccess;
  for (int it = 0; it < maxit && !all_done(); ++it) {
    if (launched == it && (werr = launch_next()) != hipSuccess) break;
    bool ahead = false;
    for (int p = 0; p < n; ++p) {
      if (cur[p].done) continue;
      const double ratio = prev[p] > 0.0 ? std::min(1.0, rn[p] / prev[p]) : 1.0;
      if (rn[p] * ratio > 3.0 * rtol * fnorm[p]) ahead = true;
    }
    if (ahead && it + 1 < maxit && launched == it + 1 && (werr = launch_next()) != hipSuccess) break;
    if ((werr = hipEventSynchronize(b->ev[it % 2])) != hipSuccess) break;
    cur = b->h_scal + static_cast<size_t>(1 + it % 2) * n;
    for (int p = 0; p < n; ++p) {
      const tpmg::FcgScalars& c = cur[p];
      if (c.status == 0 && c.iters == it + 1) {
        prev[p] = rn[p];
        rn[p] = std::sqrt(c.rr);
        if (infos && infos[p].history && c.iters < infos[p].history_cap)
          infos[p].history[c.iters] = fnorm[p] > 0 ? rn[p] / fnorm[p] : 0.0;
      }
    }
  }
  if (werr != hipSuccess) {
    (void)hipStreamSynchronize(s);
    return fail(TPMG_ERR_DEVICE, std::string("batch solve: ") + hipGetErrorString(werr));
  }
  // x += alpha p of each problem's iterations not yet added (after an
  // iteration queued ahead, which changes neither); drains the stream
  if (ring) {
    TPMG_HIP(fork());
    for (size_t k = 0; k < groups.size(); ++k) {
      hipStream_t sk = k == 0 ? s : b->aux[k - 1];
      for (int p : groups[k])
        TPMG_HIP(tpmg::launch_flush(d_u[p], b->probs[p]->dirs, b->scal + p, b->probs[p]->len, sk));
    }
    TPMG_HIP(join());
  }
  TPMG_HIP(hipStreamSynchronize(s));
  const auto t1 = std::chrono::steady_clock::now();
  tpmg_status worst = TPMG_OK;
  for (int p = 0; p < n; ++p) {
    const tpmg::FcgScalars& c = cur[p];
    tpmg_status st = c.status ? TPMG_ERR_BREAKDOWN : (c.done ? TPMG_OK : TPMG_NOT_CONVERGED);
    if (infos) {
      infos[p].iters = c.iters;
      infos[p].relres = fnorm[p] > 0 ? std::sqrt(c.rr) / fnorm[p] : 0.0;
      infos[p].t_total_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
      infos[p].t_vcycle_ms = infos[p].t_spmv_ms = infos[p].t_blas_ms = 0.0;
      std::vector<Op> ops;
      fcg_ops(*b->probs[p], d_u[p], b->scal + p, ops, false, ring);
      infos[p].model_bytes =
          solve_model_bytes(ops, c.iters, b->probs[p]->len, b->probs[p]->fp32, ring, b->probs[p]->full_outer);
    }
    if (st == TPMG_ERR_BREAKDOWN) worst = st;
    else if (st == TPMG_NOT_CONVERGED && worst == TPMG_OK) worst = st;
  }
  if (worst == TPMG_ERR_BREAKDOWN) return fail(worst, "breakdown in at least one problem of the batch");
  return worst;
}

void tpmg_batch_destroy(tpmg_batch* b) {
  if (!b) return;
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  if (b->h_scal) (void)hipHostFree(b->h_scal);
  for (hipEvent_t ev : b->ev)
    if (ev) (void)hipEventDestroy(ev);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (int k = 0; k + 1 < kBatchBranches; ++k) {
    if (b->join[k]) (void)hipEventDestroy(b->join[k]);
    if (b->aux[k]) (void)hipStreamDestroy(b->aux[k]);
  }
  delete b;
}

void tpmg_grid_destroy(tpmg_grid* g) { delete g; }
void tpmg_op_destroy(tpmg_op* op) { delete op; }
void tpmg_mg_destroy(tpmg_mg* mg) {
  if (!mg) return;
  drop_graph(*mg);
  for (hipEvent_t ev : mg->tev) (void)hipEventDestroy(ev);
  if (mg->h_scal) (void)hipHostFree(mg->h_scal);
  if (mg->ring) (void)hipHostFree(mg->ring);
  delete mg;
}

}  // extern "C"

namespace {

// The flexible-CG solve of tpmg_solve on a handle whose iteration records
// are in device memory: the host queues kRecords iterations at a time (each
// skipped on the device once the solve is done), then copies the ring and
// reads the records of those iterations in order. The kernels and their
// order are those of tpmg_solve, so the results are the same bits.
tpmg_status solve_device_records(tpmg_mg& m, const double* d_f, double* d_u, double rtol, int maxit,
                                 tpmg_solve_info* info) {
  if (!d_f || !d_u) return fail(TPMG_ERR_ARG, "NULL vector");
  if (d_f == d_u) return fail(TPMG_ERR_ARG, "f and u must not alias");
  if (!(rtol >= 0.0) || maxit < 0) return fail(TPMG_ERR_ARG, "rtol must be >= 0 and maxit >= 0");
  if (info && info->history_cap > 0 && !info->history) return fail(TPMG_ERR_ARG, "history_cap > 0 with NULL history");
  if (info && !(info->div_tol >= 0.0)) return fail(TPMG_ERR_ARG, "div_tol must be >= 0");
  if (info && info->phase_timers) return fail(TPMG_ERR_ARG, "phase timers are not available here");
  const double div2 = info && info->div_tol > 0.0 ? info->div_tol * info->div_tol : tpmg::kDefaultDiv2;
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = m.stream;
  std::vector<Op> ops;
  fcg_ops(m, d_u, m.scal, ops);
  tpmg::FcgRecord recs[tpmg::kRecords];
  auto read_ring = [&]() -> hipError_t {
    hipError_t e = hipMemcpyAsync(recs, m.ring_dev, sizeof(recs), hipMemcpyDeviceToHost, s);
    return e == hipSuccess ? hipStreamSynchronize(s) : e;
  };
  TPMG_HIP(tpmg::launch_spmv64(m.view_outer(), 1, d_u, d_f, m.r, m.partials, tpmg::kFinInit, m.scal, s, rtol,
                               m.fp32 ? static_cast<float*>(m.fcopy) : nullptr, m.ring_dev, div2));
  TPMG_HIP(read_ring());
  if (recs[0].seq != 0) return fail(TPMG_ERR_DEVICE, "initial residual record missing");
  const double fnorm = std::sqrt(recs[0].ff);
  double rnorm = std::sqrt(recs[0].rr);
  int iters = 0;
  bool diverged = false;
  auto record = [&](int k, double v) {
    if (info && info->history && k < info->history_cap) info->history[k] = v;
  };
  record(0, fnorm > 0 ? rnorm / fnorm : 0.0);
  tpmg_status result = TPMG_NOT_CONVERGED;
  hipError_t werr = hipSuccess;
  if (!std::isfinite(rnorm) || !std::isfinite(fnorm)) {
    result = TPMG_ERR_BREAKDOWN;
  } else if (rnorm <= rtol * fnorm) {
    result = TPMG_OK;
  } else {
    bool stop = false;
    for (int it = 0; it < maxit && !stop;) {
      const int n = std::min(tpmg::kRecords, maxit - it);
      for (int j = 0; j < n && werr == hipSuccess; ++j)
        for (const Op& op : ops)
          if ((werr = exec_op(op, s)) != hipSuccess) break;
      if (werr == hipSuccess) werr = read_ring();
      if (werr != hipSuccess) break;
      for (int j = 0; j < n && !stop; ++j) {
        const int seq = it + j + 1;
        const tpmg::FcgRecord& rec = recs[seq % tpmg::kRecords];
        if (rec.seq != seq) {
          werr = hipErrorUnknown;   // a queued iteration published no record
          stop = true;
          break;
        }
        iters = seq;
        if (rec.status == 2) {
          rnorm = std::sqrt(rec.rr);
          record(iters, fnorm > 0 ? rnorm / fnorm : 0.0);
          diverged = true;
          result = TPMG_ERR_BREAKDOWN;
          stop = true;
        } else if (rec.status != 0) {
          iters = seq - 1;
          result = TPMG_ERR_BREAKDOWN;
          stop = true;
        } else {
          rnorm = std::sqrt(rec.rr);
          record(iters, fnorm > 0 ? rnorm / fnorm : 0.0);
          if (!std::isfinite(rnorm)) {
            result = TPMG_ERR_BREAKDOWN;
            stop = true;
          } else if (rnorm <= rtol * fnorm) {
            result = TPMG_OK;
            stop = true;
          }
        }
      }
      it += n;
    }
  }
  const hipError_t fe = tpmg::launch_flush(d_u, m.dirs, m.scal, m.len, s);
  if (werr == hipSuccess) werr = fe;
  const hipError_t se = hipStreamSynchronize(s);
  if (werr != hipSuccess || se != hipSuccess)
    return fail(TPMG_ERR_DEVICE, std::string("solve: ") + hipGetErrorString(werr != hipSuccess ? werr : se));
  const auto t1 = std::chrono::steady_clock::now();
  if (info) {
    info->iters = iters;
    info->relres = fnorm > 0 ? rnorm / fnorm : 0.0;
    info->t_total_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    info->t_vcycle_ms = info->t_spmv_ms = info->t_blas_ms = 0.0;
    info->model_bytes = solve_model_bytes(ops, iters, m.len, m.fp32, true, m.full_outer);
  }
  if (diverged) return fail(TPMG_ERR_BREAKDOWN, "divergence: ||r|| exceeded div_tol ||r_0||");
  if (result == TPMG_ERR_BREAKDOWN) return fail(result, "breakdown: non-finite value or <p, A p> <= 0");
  return result;
}

}  // namespace

tpmg_status tpmg_solve_on_workspace(const tpmg_op* op, const tpmg_mg_params* params, void* d_workspace,
                                    size_t bytes, void* hip_stream, const double* d_f, double* d_u, double rtol,
                                    int maxit, tpmg_solve_info* info) {
  if (!params) return fail(TPMG_ERR_ARG, "params is NULL");
  if (params->autotune != 0 || params->use_graph != 0)
    return fail(TPMG_ERR_ARG, "autotune and use_graph must be 0 (trials and graphs need allocations)");
  tpmg_mg* m = nullptr;
  tpmg_status st = setup_impl(op, params, d_workspace, bytes, hip_stream, false, &m);
  if (st != TPMG_OK) return st;
  st = solve_device_records(*m, d_f, d_u, rtol, maxit, info);
  delete m;
  return st;
}

bool tpmg_fine_grid(const tpmg_mg* mg, tpmg::FineGrid* out) {
  if (!mg || !out) return false;
  const DevLevel& d = mg->lv[mg->nlev - 1];
  out->n = d.n;
  out->npad = d.npad;
  out->nz = mg->nz;
  out->nbr = d.nbr;
  out->stream = mg->stream;
  return true;
}

void tpmg_set_last_error(const char* msg) { g_last_error = msg ? msg : ""; }

hipError_t tpmg_relax_finest(const tpmg_mg* mg, const double* f, const double* u_in, double* u_out, double* sd,
                             double* sc, double omega, hipStream_t s) {
  if (!mg || !f || !u_in || !u_out || u_in == u_out) return hipErrorInvalidValue;
  tpmg::LevelView v = mg->view64(mg->nlev - 1);
  v.tune = tpmg::default_tune(mg->nz, 8);
  if (v.pm != 0 && v.tune.smoother != tpmg::kSmScan) return hipErrorInvalidValue;   // nz beyond the scan form
  return tpmg::launch_smooth(v, 8, f, true, u_in, false, u_out, true, nullptr, sd, sc, omega, s);
}
