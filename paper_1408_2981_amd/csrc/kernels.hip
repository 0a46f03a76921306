// HIP kernels of the tensor-product multigrid solver, written for gfx950
// (CDNA4, wave64). Nothing here is a dense contraction, so there is no MFMA:
// every kernel is bound by HBM traffic, and the design goal is coalesced,
// once-only streaming of each field with the stencil rebuilt in registers
// from O(1) per-column scalars and O(nz) wave-uniform vertical vectors
// (paper Section 4.2: matrix-free reconstruction from factorised profiles).
//
// Operator (Appendix A, eq. ColumnEquation), flux form, for column T, level k:
//   (A u)_k = bh bv_k u_k + av_k sum_j ah_j (u_k - u_{T_j,k})
//           + arh (arv_{k+1} (u_k - u_{k+1}) + arv_k (u_k - u_{k-1}))
// with bh, ah_j, arh per column and bv, av, arv per level.
//
// Every kernel of the solve is written as a device body that takes its
// block's index and the block count of its problem's launch (GridPos). A
// single-problem kernel passes (blockIdx.x, gridDim.x); a batched kernel
// decodes its block from a table of segments, one per problem, and passes the
// problem-local values, so each problem of a batch is computed with exactly
// the block decomposition, and therefore the rounding, of its own solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "device.h"

namespace tpmg {
namespace {

__device__ __forceinline__ size_t tile_base(int col, int nz) {
  return static_cast<size_t>(col >> 6) * (static_cast<size_t>(kTile) * nz) + (col & 63);
}

template <typename T>
struct Lv {
  int n, npad, nz;
  const int32_t* __restrict__ nbr;
  const int32_t* __restrict__ code;
  const int32_t* __restrict__ halo;
  const T* __restrict__ bh;
  const T* __restrict__ arh;
  const T* __restrict__ ash;
  const T* __restrict__ pw;
  const T* __restrict__ bv;
  const T* __restrict__ av;
  const T* __restrict__ arv;
  const T* __restrict__ margin;
  // profiles that do not factorise (LevelView::pm > 0): per-(T, k)
  // coefficients, tiled like the vectors (fas: three planes, one per
  // neighbour; far: nz + 1 rows per tile, the radial faces)
  const T* __restrict__ fb;
  const T* __restrict__ far;
  const T* __restrict__ fas;
  // vertical advection (pm 3): omega^2 times the coefficients of a cell's
  // lower and upper face, tiled like the vectors
  const T* __restrict__ fxl;
  const T* __restrict__ fxu;
  // multicolour block-SOR: colour of every column and the colour this
  // smoother pass relaxes (pass < 0: every column, block-Jacobi)
  const int8_t* __restrict__ colour;
  int pass;
};

// whether a smoother pass relaxes column col (the other columns keep their
// values: u_out = u_in, or 0 for a pass from a zero guess)
template <typename T>
__device__ __forceinline__ bool relaxes(const Lv<T>& L, int col) {
  return L.pass < 0 || L.colour[col] == L.pass;
}

template <typename T>
__host__ __device__ Lv<T> view(const LevelView& L) {
  return Lv<T>{L.n,
               L.npad,
               L.nz,
               L.nbr,
               L.code,
               L.halo,
               static_cast<const T*>(L.beta_h),
               static_cast<const T*>(L.ar_h),
               static_cast<const T*>(L.as_h),
               static_cast<const T*>(L.pw),
               static_cast<const T*>(L.beta_v),
               static_cast<const T*>(L.as_v),
               static_cast<const T*>(L.ar_v),
               static_cast<const T*>(L.margin),
               static_cast<const T*>(L.fb),
               static_cast<const T*>(L.far),
               static_cast<const T*>(L.fas),
               static_cast<const T*>(L.fxl),
               static_cast<const T*>(L.fxu),
               L.colour,
               L.pass};
}

// The same view of a level descriptor held in the constant address space
// (the segment tables of batched launches, below).
template <typename T>
__device__ __forceinline__ Lv<T> view(const __attribute__((address_space(4))) LevelView& L) {
  return Lv<T>{L.n,
               L.npad,
               L.nz,
               L.nbr,
               L.code,
               L.halo,
               static_cast<const T*>(L.beta_h),
               static_cast<const T*>(L.ar_h),
               static_cast<const T*>(L.as_h),
               static_cast<const T*>(L.pw),
               static_cast<const T*>(L.beta_v),
               static_cast<const T*>(L.as_v),
               static_cast<const T*>(L.ar_v),
               static_cast<const T*>(L.margin),
               static_cast<const T*>(L.fb),
               static_cast<const T*>(L.far),
               static_cast<const T*>(L.fas),
               static_cast<const T*>(L.fxl),
               static_cast<const T*>(L.fxu),
               L.colour,
               L.pass};
}

// this block's index and the number of blocks of its problem's launch
struct GridPos {
  int b;
  int nb;
};

__device__ __forceinline__ GridPos whole_grid() { return GridPos{static_cast<int>(blockIdx.x), static_cast<int>(gridDim.x)}; }

// Blocks are dealt to the 8 XCDs round-robin; renumber them so that each
// XCD walks one contiguous range of tiles (or of tile chunks) and neighbour gathers across tile
// edges hit in that XCD's own L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
  return x * q + min(x, r) + i;
}

// per-column stencil data held in registers for a whole column sweep
template <typename T>
struct Column {
  T bh, arh, a0, a1, a2;
  size_t base, b0, b1, b2;   // tile offsets of the column and its neighbours
  size_t hb;                 // tile offset of the column's halo slot
  size_t abase;              // offset of the column in the (nz + 1)-row face arrays (full profiles)
  uint32_t code;             // where the wave finds each neighbour (see LevelView)
};

template <typename T>
__device__ __forceinline__ Column<T> load_column(const Lv<T>& L, int col) {
  Column<T> c;
  c.bh = L.bh[col];
  c.arh = L.arh[col];
  c.a0 = L.ash[col];
  c.a1 = L.ash[L.npad + col];
  c.a2 = L.ash[2 * L.npad + col];
  c.base = tile_base(col, L.nz);
  c.b0 = tile_base(L.nbr[col], L.nz);
  c.b1 = tile_base(L.nbr[L.npad + col], L.nz);
  c.b2 = tile_base(L.nbr[2 * L.npad + col], L.nz);
  c.hb = tile_base(L.halo[col], L.nz);
  c.abase = tile_base(col, L.nz + 1);
  c.code = static_cast<uint32_t>(L.code[col]);
  return c;
}

// Neighbour exchange inside a wave, one level at a time: the wave puts its
// 64 own values and the tile's 64 halo values of the level into its
// 128-entry LDS slice, and every lane takes its three neighbours at the slots
// its code names. LDS operations of one wave complete in order, so a slice is
// reused level after level without a barrier; the wave barriers only keep the
// compiler from moving the accesses across each other.
template <typename T>
struct Exchange {
  T* __restrict__ x;   // this wave's 128 entries
  __device__ __forceinline__ void put(int lane, T own, T halo) {
    x[lane] = own;
    x[kTile + lane] = halo;
    __builtin_amdgcn_wave_barrier();
  }
  __device__ __forceinline__ T get(const Column<T>& c, int j) const { return x[(c.code >> (8 * j)) & 0xffu]; }
  __device__ __forceinline__ void done() { __builtin_amdgcn_wave_barrier(); }
};

// (A u)_k in flux form from the own-column values um = u_{k-1}, uc = u_k,
// up = u_{k+1} and the neighbour-column values n0, n1, n2 at level k (every
// kernel evaluates a row through this one expression)
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// The fused multiply-adds are written out, so the rounding of a row does not
// depend on how a kernel's instance happens to be compiled.
//
// PM, the profile mode of the level (Section 4.2): 0 factorised (column
// scalars times vertical vectors, eq. TridiagonalFactorising); 1 the radial
// couplings per (T, k) and the rest factorised (the operator of
// TPMG^(partial)); 2 every coefficient per (T, k) (eq.
// TridiagonalNonFactorising); 3 as 2 with the vertical advection, whose
// couplings to the cell below (alphar^ - adv_lo) and above (alphar^ +
// adv_up) differ.
template <int PM, typename T>
__device__ __forceinline__ T coef_lower(const Lv<T>& L, const Column<T>& c, int k);
template <int PM, typename T>
__device__ __forceinline__ T coef_upper(const Lv<T>& L, const Column<T>& c, int k);

template <int PM = 0, typename T>
__device__ __forceinline__ T row_flux(const Lv<T>& L, const Column<T>& c, int k, T um, T uc, T up, T n0, T n1, T n2) {
  if constexpr (PM == 0) {
    const T h = fma_t(c.a2, uc - n2, fma_t(c.a1, uc - n1, c.a0 * (uc - n0)));
    const T v = fma_t(L.arv[k], uc - um, L.arv[k + 1] * (uc - up));
    return fma_t(c.arh, v, fma_t(L.av[k], h, (c.bh * L.bv[k]) * uc));
  } else {
    const size_t oa = c.abase + static_cast<size_t>(k) * kTile;
    const T v = PM == 3 ? fma_t(coef_lower<PM>(L, c, k), uc - um, coef_upper<PM>(L, c, k) * (uc - up))
                        : fma_t(L.far[oa], uc - um, L.far[oa + kTile] * (uc - up));
    if constexpr (PM == 1) {
      const T h = fma_t(c.a2, uc - n2, fma_t(c.a1, uc - n1, c.a0 * (uc - n0)));
      return v + fma_t(L.av[k], h, (c.bh * L.bv[k]) * uc);
    } else {
      const size_t o = c.base + static_cast<size_t>(k) * kTile;
      const size_t pl = static_cast<size_t>(L.npad) * L.nz;
      const T h = fma_t(L.fas[2 * pl + o], uc - n2, fma_t(L.fas[pl + o], uc - n1, L.fas[o] * (uc - n0)));
      return v + fma_t(L.fb[o], uc, h);
    }
  }
}

// Column excess e_k (mass plus horizontal couplings) and radial coupling
// through face k of a column, in the level's profile mode.
template <int PM, typename T>
__device__ __forceinline__ T coef_excess(const Lv<T>& L, const Column<T>& c, T esum, int k) {
  if constexpr (PM >= 2) {
    const size_t o = c.base + static_cast<size_t>(k) * kTile;
    const size_t pl = static_cast<size_t>(L.npad) * L.nz;
    return L.fb[o] + ((L.fas[o] + L.fas[pl + o]) + L.fas[2 * pl + o]);
  } else {
    return c.bh * L.bv[k] + esum * L.av[k];
  }
}
template <int PM, typename T>
__device__ __forceinline__ T coef_face(const Lv<T>& L, const Column<T>& c, int k) {
  if constexpr (PM >= 1)
    return L.far[c.abase + static_cast<size_t>(k) * kTile];
  else
    return c.arh * L.arv[k];
}
// coupling of row k to the cell below (l_k) and above (m_k); without
// advection both are the radial face's coupling
template <int PM, typename T>
__device__ __forceinline__ T coef_lower(const Lv<T>& L, const Column<T>& c, int k) {
  if constexpr (PM == 3)
    return coef_face<PM>(L, c, k) - L.fxl[c.base + static_cast<size_t>(k) * kTile];
  else
    return coef_face<PM>(L, c, k);
}
template <int PM, typename T>
__device__ __forceinline__ T coef_upper(const Lv<T>& L, const Column<T>& c, int k) {
  if constexpr (PM == 3)
    return coef_face<PM>(L, c, k + 1) + L.fxu[c.base + static_cast<size_t>(k) * kTile];
  else
    return coef_face<PM>(L, c, k + 1);
}

template <int PM = 0, typename T>
__device__ __forceinline__ T apply_row(const Lv<T>& L, const Column<T>& c, const T* __restrict__ u, int k, T um,
                                       T uc, T up) {
  const size_t o = static_cast<size_t>(k) * kTile;
  return row_flux<PM>(L, c, k, um, uc, up, u[c.b0 + o], u[c.b1 + o], u[c.b2 + o]);
}

// Values of a column at levels k0-1 .. k0+CH and of its neighbours at
// k0 .. k0+CH-1, all loaded before any is used (indices clamped into the
// column; the callers ignore the clamped entries)
template <typename T, int CH>
struct ChunkLoads {
  T xv[CH + 2], n0[CH], n1[CH], n2[CH];
  // own values of levels k0-1 .. k0+CH (clamped), neighbours of k0 .. k0+CH-1
  // through the wave's exchange slice (all 64 lanes active)
  __device__ __forceinline__ void load(const Column<T>& c, const T* __restrict__ u, int k0, int nz, Exchange<T> xc,
                                       int lane) {
    load_with(c, [&](size_t o) { return u[o]; }, k0, nz, xc, lane);
  }
  // the same with the value at offset o given by get(o)
  template <typename Get>
  __device__ __forceinline__ void load_with(const Column<T>& c, Get&& get, int k0, int nz, Exchange<T> xc,
                                            int lane) {
    T hv[CH];
#pragma unroll
    for (int i = 0; i < CH + 2; ++i) xv[i] = get(c.base + static_cast<size_t>(min(max(k0 - 1 + i, 0), nz - 1)) * kTile);
#pragma unroll
    for (int i = 0; i < CH; ++i) hv[i] = get(c.hb + static_cast<size_t>(min(k0 + i, nz - 1)) * kTile);
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      xc.put(lane, xv[i + 1], hv[i]);
      n0[i] = xc.get(c, 0);
      n1[i] = xc.get(c, 1);
      n2[i] = xc.get(c, 2);
      xc.done();
    }
  }
  // (A u)_{k0+i} for k0 + i < nz
  template <int PM = 0>
  __device__ __forceinline__ T row(const Lv<T>& L, const Column<T>& c, int k0, int i) const {
    const int k = k0 + i;
    const T um = k > 0 ? xv[i] : T(0);
    const T up = k + 1 < L.nz ? xv[i + 2] : T(0);
    return row_flux<PM>(L, c, k, um, xv[i + 1], up, n0[i], n1[i], n2[i]);
  }
};

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// deterministic block sum of two values (blockDim.x a multiple of 64, at
// most 16 waves); thread 0 writes out[2 * b + i]
__device__ __forceinline__ void block_sums(double (&v)[2], double* __restrict__ out, int b) {
  __shared__ double red[16][2];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  v[0] = wave_sum(v[0]);
  v[1] = wave_sum(v[1]);
  if (lane == 0) {
    red[w][0] = v[0];
    red[w][1] = v[1];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
    for (int i = 0; i < nw; ++i) {
      a += red[i][0];
      c += red[i][1];
    }
    out[2 * b] = a;
    out[2 * b + 1] = c;
  }
}

__device__ __forceinline__ bool finite(double v) { return v - v == 0.0; }

// Scalar updates of the flexible-CG recurrence from the deterministic sums
// (s0, s1) of all blocks' partials. done/iters serve batched solves, which
// test convergence on the device (||r|| <= rtol ||f||, as the host does for a
// single solve).
__device__ void fcg_scalars(int site, double s0, double s1, FcgScalars* __restrict__ sc, double rtol,
                            double div2) {
  switch (site) {
    case kFinInit:
      sc->rr = s0;
      sc->ff = s1;
      sc->rr0 = s0;
      sc->div2 = div2;
      sc->pq = 1.0;
      sc->rz = 0.0;
      sc->alpha = 0.0;
      sc->beta = 0.0;
      sc->rtol = rtol;
      sc->iters = 0;
      sc->seq = 0;
      sc->flushed = 0;
      sc->status = (finite(s0) && finite(s1)) ? 0 : 1;
      sc->done = (sc->status != 0 || sqrt(s0) <= rtol * sqrt(s1)) ? 1 : 0;
      break;
    case kFinAlpha:
      sc->pq = s0;
      if (!(s0 > 0.0) || !finite(s0) || !finite(sc->rz)) {
        sc->status = 1;
        sc->done = 1;
        sc->alpha = 0.0;
      } else {
        sc->alpha = sc->rz / s0;
      }
      sc->alpha_hist[sc->iters % kDirSlots] = sc->alpha;
      break;
    case kFinRR:
      sc->rr = s0;
      if (sc->status == 0) sc->iters += 1;
      if (!finite(s0)) {
        sc->status = 1;
        sc->done = 1;
      } else if (sqrt(s0) <= sc->rtol * sqrt(sc->ff)) {
        sc->done = 1;
      } else if (s0 > sc->div2 * sc->rr0) {
        sc->status = 2;   // diverged: the iterate is finite and kept
        sc->done = 1;
      }
      break;
    case kFinBeta:
      // (the first direction is z itself: no previous q enters)
      sc->beta = sc->iters == 0 ? 0.0 : -s0 / sc->pq;
      sc->rz = s1;
      break;
    case kKInit:
      sc->rz = sc->rr;
      sc->alpha = 1.0;
      sc->w = 1.0;
      sc->beta = 0.0;
      sc->iters = 0;
      break;
    case kKAlpha:
      if (!(s0 != 0.0) || !finite(s0) || !finite(sc->rz)) {
        sc->status = 1;
        sc->alpha = 0.0;
      } else {
        sc->alpha = sc->rz / s0;
      }
      break;
    case kKOmega:
      if (!(s1 > 0.0) || !finite(s0) || !finite(s1) || s0 == 0.0) {
        sc->status = 1;
        sc->w = 1.0;
      } else {
        sc->w = s0 / s1;
      }
      break;
    case kKRho:
      sc->rr = s1;
      sc->iters += 1;
      if (!(s0 != 0.0) || !finite(s0) || !finite(s1)) {
        sc->status = 1;
      } else {
        sc->beta = (s0 / sc->rz) * (sc->alpha / sc->w);
        sc->rz = s0;
      }
      break;
    default:
      break;
  }
}

// One block: sums the partials of nblocks blocks in a fixed order and
// applies them to the scalars. It runs as a kernel of its own: on this GPU
// each XCD has its own L2, and a kernel boundary is the cheap way to make
// all blocks' partials visible (a device-scope fence per block would write
// back the whole L2).
__device__ __forceinline__ void finalize_body(int site, const double* __restrict__ partials, int nblocks,
                                              FcgScalars* __restrict__ sc, double rtol, double div2 = kDefaultDiv2) {
  // thread t adds the partials t, t + blockDim.x, ... in that order, eight
  // pairs loaded ahead of their additions (the partials come from L2 or
  // memory: one dependent load per pair would serialise the latencies)
  double v[2] = {0.0, 0.0};
  const int nt = blockDim.x;
  for (int b0 = threadIdx.x; b0 < nblocks; b0 += 8 * nt) {
    double a0[8], a1[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int b = b0 + j * nt;
      a0[j] = b < nblocks ? partials[2 * b] : 0.0;
      a1[j] = b < nblocks ? partials[2 * b + 1] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      v[0] += a0[j];
      v[1] += a1[j];
    }
  }
  __shared__ double red[16][2];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = nt >> 6;
  v[0] = wave_sum(v[0]);
  v[1] = wave_sum(v[1]);
  if (lane == 0) {
    red[w][0] = v[0];
    red[w][1] = v[1];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, c = 0.0;
    for (int i = 0; i < nw; ++i) {
      a += red[i][0];
      c += red[i][1];
    }
    fcg_scalars(site, a, c, sc, rtol, div2);
  }
}

// ---------------------------------------------------------------------------
// stencil kernels: one wave per (tile, chunk of levels); the chunk length is
// chosen per grid so that small grids still launch enough waves
// ---------------------------------------------------------------------------

// MODE 0: y = A x, partials <x, y>. MODE 1: y = b - A x, partials <y, y>,
// <b, b>.
template <int MODE, int CH, int PM = 0>
__device__ __forceinline__ void spmv_body(const Lv<double>& L, int chunk_rt, const double* __restrict__ x,
                                          const double* __restrict__ b, double* __restrict__ y,
                                          double* __restrict__ partials, GridPos g, float* __restrict__ y32 = nullptr) {
  const int chunk = CH > 0 ? CH : chunk_rt;
  const int nchunks = (L.nz + chunk - 1) / chunk;
  const int lb = xcd_tile(g.b, g.nb);
  const int item = __builtin_amdgcn_readfirstlane(lb * 4 + (threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  double acc[2] = {0.0, 0.0};
  if (item < (L.npad >> 6) * nchunks) {
    const int tile = item / nchunks, chunk_i = item - tile * nchunks;
    const int k0 = chunk_i * chunk, k1 = min(L.nz, k0 + chunk);
    const Column<double> c = load_column(L, tile * kTile + lane);
    auto emit = [&](int k, double uc, double ax, double bk) {
      const size_t o = c.base + static_cast<size_t>(k) * kTile;
      if (MODE == 0) {
        y[o] = ax;
        acc[0] += uc * ax;
      } else {
        const double rk = bk - ax;
        y[o] = rk;
        if (y32) y32[o] = static_cast<float>(rk);
        acc[0] += rk * rk;
        acc[1] += bk * bk;
      }
    };
    if constexpr (CH > 0) {
      __shared__ double xbuf[kStencilWaves][2 * kTile];
      ChunkLoads<double, CH> ld;
      ld.load(c, x, k0, L.nz, Exchange<double>{xbuf[threadIdx.x >> 6]}, lane);
      double bb[MODE == 1 ? CH : 1];
      if (MODE == 1) {
#pragma unroll
        for (int i = 0; i < CH; ++i) bb[MODE == 1 ? i : 0] = b[c.base + static_cast<size_t>(min(k0 + i, L.nz - 1)) * kTile];
      }
#pragma unroll
      for (int i = 0; i < CH; ++i)
        if (k0 + i < k1)
          emit(k0 + i, ld.xv[i + 1], ld.template row<PM>(L, c, k0, i), MODE == 1 ? bb[MODE == 1 ? i : 0] : 0.0);
    } else {
      double um = k0 > 0 ? x[c.base + static_cast<size_t>(k0 - 1) * kTile] : 0.0;
      double uc = x[c.base + static_cast<size_t>(k0) * kTile];
      for (int k = k0; k < k1; ++k) {
        const size_t o = c.base + static_cast<size_t>(k) * kTile;
        const double up = k + 1 < L.nz ? x[o + kTile] : 0.0;
        emit(k, uc, apply_row<PM>(L, c, x, k, um, uc, up), MODE == 1 ? b[o] : 0.0);
        um = uc;
        uc = up;
      }
    }
  }
  block_sums(acc, partials, lb);
}

// Line smoother: damped block-Jacobi with a Thomas solve per column
// (eq. BlockJacobi). Forward sweep: residual r_k = f_k - (A u)_k and
// elimination in margin form s_k = e_k + l_k s_{k-1} / p_{k-1},
// p_k = s_k + m_k (e_k the column excess bh bv_k + av_k sum_j ah_j,
// l_k = arh arv_k, m_k = arh arv_{k+1}), d_k = (r_k + l_k d_{k-1}) / p_k;
// backward sweep x_k = d_k + (m_k / p_k) x_{k+1}, u_out = u_in + omega x.
template <typename T, typename TF, typename TO, bool ZERO, bool FCOPY>
__global__ __launch_bounds__(64) void k_smooth_fallback(Lv<T> L, const TF* __restrict__ f, const T* __restrict__ u_in,
                                               TO* __restrict__ u_out, T* __restrict__ fcopy,
                                               T* __restrict__ sd, T* __restrict__ sc, T omega) {
  const int lane = threadIdx.x;
  const int col = blockIdx.x * kTile + lane;
  const Column<T> c = load_column(L, col);
  const int nz = L.nz;
  const T esum = c.a0 + c.a1 + c.a2;
  T s_prev = T(0), ip_prev = T(1), d_prev = T(0);
  T um = T(0), uc = ZERO ? T(0) : u_in[c.base];
  for (int k = 0; k < nz; ++k) {
    const size_t o = c.base + static_cast<size_t>(k) * kTile;
    const T fk = static_cast<T>(f[o]);
    if (FCOPY) fcopy[o] = fk;
    T r = fk;
    T up = T(0);
    if (!ZERO) {
      up = k + 1 < nz ? u_in[o + kTile] : T(0);
      r = fk - apply_row(L, c, u_in, k, um, uc, up);
    }
    const T e = c.bh * L.bv[k] + esum * L.av[k];
    const T l = c.arh * L.arv[k];
    const T m = c.arh * L.arv[k + 1];
    const T s = e + l * (s_prev * ip_prev);
    const T ip = T(1) / (s + m);
    const T d = (r + l * d_prev) * ip;
    sd[o] = d;
    sc[o] = m * ip;
    s_prev = s;
    ip_prev = ip;
    d_prev = d;
    um = uc;
    uc = up;
  }
  T x = T(0);
  const bool upd = relaxes(L, col);
  for (int k = nz - 1; k >= 0; --k) {
    const size_t o = c.base + static_cast<size_t>(k) * kTile;
    x = sd[o] + sc[o] * x;
    const T uo = ZERO ? omega * x : u_in[o] + omega * x;
    u_out[o] = static_cast<TO>(upd ? uo : (ZERO ? T(0) : u_in[o]));
  }
}

__device__ __forceinline__ float fast_rcp(float p) { return __builtin_amdgcn_rcpf(p); }
__device__ __forceinline__ double fast_rcp(double p) {
  // hardware estimate refined by two Newton steps (a few ulp at most)
  double r = __builtin_amdgcn_rcp(p);
  double e = __builtin_fma(-p, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-p, r, 1.0);
  return __builtin_fma(r, e, r);
}

// Line smoother, LDS-staged form: one workgroup per tile of 64 columns.
//  1. every wave computes the residual r = f - A u_in for its own range of
//     levels (all loads independent, many in flight) into LDS;
//  2. wave 0 runs the margin-form Thomas recurrence of each column out of
//     LDS (forward: d_k and m_k / p_k; backward: x_k), in place, reading
//     LDS and the vertical coefficients kBatch levels ahead of the chain;
//  3. every wave writes u_out = u_in + omega x for its levels.
// LDS: two [nz][64] arrays of T and the three vertical vectors.
constexpr int kBatch = 8;

template <typename T, typename TF, typename TO, bool ZERO, bool FCOPY>
__global__ __launch_bounds__(1024) void k_smooth_lds(Lv<T> L, const TF* __restrict__ f, const T* __restrict__ u_in,
                                                     TO* __restrict__ u_out, T* __restrict__ fcopy, T omega) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nz = L.nz;
  T* __restrict__ rb = reinterpret_cast<T*>(smem);
  T* __restrict__ cb = rb + static_cast<size_t>(nz) * kTile;
  T* __restrict__ vb = cb + static_cast<size_t>(nz) * kTile;   // bv[nz], av[nz], arv[nz+1]
  T* __restrict__ va = vb + nz;
  T* __restrict__ vr = va + nz;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = blockDim.x >> 6;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int col = tile * kTile + lane;
  const int kw = (nz + nw - 1) / nw;
  const int k0 = min(nz, wave * kw), k1 = min(nz, k0 + kw);
  const Column<T> c = load_column(L, col);
  for (int i = threadIdx.x; i <= nz; i += blockDim.x) {
    if (i < nz) {
      vb[i] = L.bv[i];
      va[i] = L.av[i];
    }
    vr[i] = L.arv[i];
  }

  if (ZERO) {
#pragma unroll 8
    for (int k = k0; k < k1; ++k) {
      const size_t o = c.base + static_cast<size_t>(k) * kTile;
      const T fk = static_cast<T>(f[o]);
      if (FCOPY) fcopy[o] = fk;
      rb[k * kTile + lane] = fk;
    }
  } else {
#pragma unroll 8
    for (int k = k0; k < k1; ++k) {
      const size_t o = c.base + static_cast<size_t>(k) * kTile;
      const T um = k > 0 ? u_in[o - kTile] : T(0);
      const T uc = u_in[o];
      const T up = k + 1 < nz ? u_in[o + kTile] : T(0);
      const T fk = static_cast<T>(f[o]);
      if (FCOPY) fcopy[o] = fk;
      rb[k * kTile + lane] = fk - apply_row(L, c, u_in, k, um, uc, up);
    }
  }
  __syncthreads();
  if (wave == 0) {
    const T esum = c.a0 + c.a1 + c.a2;
    T s_prev = T(0), ip_prev = T(1), d_prev = T(0);
    for (int kb = 0; kb < nz; kb += kBatch) {
      T rr[kBatch], ee[kBatch], ll[kBatch], mm[kBatch];
#pragma unroll
      for (int i = 0; i < kBatch; ++i) {
        const int k = min(kb + i, nz - 1);
        rr[i] = rb[k * kTile + lane];
        ee[i] = c.bh * vb[k] + esum * va[k];
        ll[i] = c.arh * vr[k];
        mm[i] = c.arh * vr[k + 1];
      }
#pragma unroll
      for (int i = 0; i < kBatch; ++i) {
        if (kb + i < nz) {
          const int k = kb + i;
          const T s = ee[i] + ll[i] * (s_prev * ip_prev);
          const T ip = fast_rcp(s + mm[i]);
          const T d = (rr[i] + ll[i] * d_prev) * ip;
          rb[k * kTile + lane] = d;
          cb[k * kTile + lane] = mm[i] * ip;
          s_prev = s;
          ip_prev = ip;
          d_prev = d;
        }
      }
    }
    T x = T(0);
    for (int kt = nz; kt > 0; kt -= kBatch) {
      T dd[kBatch], cc[kBatch];
#pragma unroll
      for (int i = 0; i < kBatch; ++i) {
        const int k = max(kt - 1 - i, 0);
        dd[i] = rb[k * kTile + lane];
        cc[i] = cb[k * kTile + lane];
      }
#pragma unroll
      for (int i = 0; i < kBatch; ++i) {
        if (kt - 1 - i >= 0) {
          x = dd[i] + cc[i] * x;
          rb[(kt - 1 - i) * kTile + lane] = x;
        }
      }
    }
  }
  __syncthreads();
  const bool upd = relaxes(L, col);
#pragma unroll 8
  for (int k = k0; k < k1; ++k) {
    const size_t o = c.base + static_cast<size_t>(k) * kTile;
    const T x = rb[k * kTile + lane];
    const T uo = ZERO ? omega * x : u_in[o] + omega * x;
    u_out[o] = static_cast<TO>(upd ? uo : (ZERO ? T(0) : u_in[o]));
  }
}

// Margins of the margin-form Thomas factorisation, one thread per column:
// s_0 = e_0, s_k = e_k + l_k s_{k-1} / (s_{k-1} + l_k), with
// e_k = beta_h beta_v,k + (sum of the horizontal couplings) alpha_s,v,k and
// l_k = alpha_r,h alpha_r,v,k. FP64 throughout.
template <typename TO, int PM>
__global__ __launch_bounds__(256) void k_margins(Lv<double> L, TO* __restrict__ margin) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= L.npad) return;
  const Column<double> c = load_column(L, col);
  const double esum = c.a0 + c.a1 + c.a2;
  double sk = 0.0;
  for (int k = 0; k < L.nz; ++k) {
    const double e = coef_excess<PM>(L, c, esum, k);
    const double l = coef_lower<PM>(L, c, k);
    // (the pivot of row k-1 is s_{k-1} + m_{k-1}; without advection
    // m_{k-1} = l_k)
    const double mp = k > 0 ? coef_upper<PM>(L, c, k - 1) : 0.0;
    sk = k == 0 ? e : e + l * sk / (sk + mp);
    margin[c.base + static_cast<size_t>(k) * kTile] = static_cast<TO>(sk);
  }
}

// Line smoother, scan form (nz <= kScanWavesMax * KB): one workgroup per
// tile of 64 columns, wave w owns the levels [w*kb, (w+1)*kb) (kb <= KB) of
// every column and keeps them in registers. The column solve of the margin-form
// Thomas algorithm is evaluated in rounds of block scans over the waves:
//  1. pivots: the margins s_k = e_k + l_k s_{k-1} / (s_{k-1} + l_k) depend on
//     the operator only and are factorised once per level at setup
//     (k_margins); a wave loads the one entering its block, s_{k0-1}, and
//     forms its own pivots with one reciprocal per level;
//  2. elimination: d_k = (l_k d_{k-1} + r_k) / p_k, an affine map in d;
//  3. back substitution: x_k = (m_k / p_k) x_{k+1} + d_k, affine in x, its
//     block maps formed from the block's own d (composing the substitution
//     with the elimination instead, to save a round, loses the column's
//     near-null component in FP32 at extreme anisotropy).
// The chain is kb + 2 n_waves steps instead of 2 nz, only wave 0 runs the
// across-block chains, and the only workgroup-wide data in LDS are the
// per-wave summaries.

template <typename T>
__device__ __forceinline__ T rcp_of(T v) {
  return fast_rcp(v);
}

template <int KB, typename T, typename TF, typename TO, bool ZERO, bool FCOPY, bool DOTS, int PM = 0,
          bool PACK = false>
__device__ __forceinline__ void smooth_scan_body(const Lv<T>& L, const TF* __restrict__ f, const T* __restrict__ u_in,
                                                 TO* __restrict__ u_out, T* __restrict__ fcopy, T omega,
                                                 const double* __restrict__ q, double* __restrict__ partials,
                                                 GridPos g) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int nz = L.nz;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // waves that own levels of one tile. A batched launch sizes its blocks for
  // the deepest problem of the group (waves beyond a tile's own idle). With
  // PACK (batched sweeps without the dot products, whose partial sums are
  // one per tile as in the single launches) such a block holds several
  // tiles, one per nw waves (tpb of them; waves beyond those idle).
  const int nw = (nz + KB - 1) / KB;
  const int tpb = PACK ? max(1, static_cast<int>(blockDim.x >> 6) / nw) : 1;
  const int slot = PACK ? wave / nw : 0;   // the wave's tile in the block
  const int wt = wave - slot * nw;         // the wave's place in its tile
  // summaries: pivot map (4), elimination map (2), substitution map (2)
  T* __restrict__ sm = reinterpret_cast<T*>(smem);
  auto at = [&](int w, int q) -> T& { return sm[(static_cast<size_t>(w) * 8 + q) * kTile + lane]; };
  // after the summaries of all the block's waves: the exchange slices
  Exchange<T> xc{sm + static_cast<size_t>(blockDim.x >> 6) * 8 * kTile + static_cast<size_t>(wave) * 2 * kTile};
  const int ntiles = L.npad / kTile;
  const int tile_w = xcd_tile(g.b, g.nb) * tpb + slot;
  // a wave without a tile (beyond the block's tpb tiles, or past the last
  // tile) reads the last tile's column data, owns no level and stores nothing
  const bool live = !PACK || (slot < tpb && tile_w < ntiles);
  const int tile = live ? tile_w : ntiles - 1;
  const int col = tile * kTile + lane;
  const int kb = (nz + nw - 1) / nw;
  const int k0 = live ? min(nz, wt * kb) : nz;
  const int nb = min(nz, k0 + kb) - k0;
  const int w0 = slot * nw;           // the tile's first wave
  const Column<T> c = load_column(L, col);
  const T esum = c.a0 + c.a1 + c.a2;

  // column coefficients of level k0 + i, rebuilt from the per-column scalars
  // and the wave-uniform vertical vectors whenever needed (cheaper than
  // holding them: registers decide how many tiles a CU keeps in flight)
  auto e_of = [&](int i) -> T { return coef_excess<PM>(L, c, esum, k0 + i); };
  auto l_of = [&](int i) -> T { return coef_lower<PM>(L, c, k0 + i); };
  auto m_of = [&](int i) -> T { return coef_upper<PM>(L, c, k0 + i); };

  // ---- residual of the wave's levels, in registers. All loads are issued
  // before any is used: their level indices are clamped into the column (the
  // value of a clamped load is discarded), so no branch separates them and
  // the wave waits for memory once, not once per level.
  T r[KB], uu[KB];
  T s_in;   // margin s_{k0-1} entering the wave's block (factorised at setup)
  {
    TF fv[KB];
    T hv[ZERO ? 1 : KB];
    T below = T(0), above = T(0);
#pragma unroll
    for (int i = 0; i < KB; ++i) {
      const size_t ok = static_cast<size_t>(min(k0 + i, nz - 1)) * kTile;
      fv[i] = f[c.base + ok];
      if (!ZERO) {
        uu[i] = u_in[c.base + ok];
        hv[i] = u_in[c.hb + ok];
      }
    }
    s_in = L.margin[c.base + static_cast<size_t>(max(k0 - 1, 0)) * kTile];
    if (!ZERO) {
      const T b = u_in[c.base + static_cast<size_t>(max(k0 - 1, 0)) * kTile];
      const T a = u_in[c.base + static_cast<size_t>(min(k0 + nb, nz - 1)) * kTile];
      below = k0 > 0 ? b : T(0);
      above = k0 + nb < nz ? a : T(0);
    }
#pragma unroll
    for (int i = 0; i < KB; ++i) {
      if (i < nb) {
        const int k = k0 + i;
        const T fk = static_cast<T>(fv[i]);
        if (FCOPY) fcopy[c.base + static_cast<size_t>(k) * kTile] = fk;
        if (ZERO) {
          r[i] = fk;
          uu[i] = T(0);
        } else {
          const T uc = uu[i];
          const T um = i == 0 ? below : uu[i > 0 ? i - 1 : 0];
          const T next = i + 1 < KB ? uu[i + 1 < KB ? i + 1 : KB - 1] : above;
          const T up = i + 1 < nb ? next : above;
          xc.put(lane, uc, hv[i]);
          const T n0 = xc.get(c, 0), n1 = xc.get(c, 1), n2 = xc.get(c, 2);
          xc.done();
          r[i] = fk - row_flux<PM>(L, c, k, um, uc, up, n0, n1, n2);
        }
      }
    }
  }

  // local pivots p_k = s_k + m_k with s_k = e_k + l_k s_{k-1} / p_{k-1} (one
  // reciprocal per level; p_{k0-1} = s_in + m_{k0-1}, m_{k0-1} = l_{k0}); keep
  // the elimination factor l_k / p_k, the substitution factor m_k / p_k and
  // r_k / p_k
  T la[KB], mc[KB];
  {
    T s_prev = T(0), ip_prev = T(0);
    if (wt > 0) {
      s_prev = s_in;
      // the pivot of the level below the block, s_{k0-1} + m_{k0-1}
      ip_prev = rcp_of(s_prev + m_of(-1));
    }
#pragma unroll
    for (int i = 0; i < KB; ++i) {
      if (i < nb) {
        const T ei = e_of(i), li = l_of(i), mi = m_of(i);
        const T s = (k0 + i == 0) ? ei : ei + li * s_prev * ip_prev;
        const T ip = rcp_of(s + mi);
        la[i] = li * ip;
        mc[i] = mi * ip;
        r[i] *= ip;
        s_prev = s;
        ip_prev = ip;
      }
    }
  }

  // ---- round 2, elimination d_k = la_k d_{k-1} + r_k: the block's map
  // d_last = A d_in + B; the tile's first wave runs it up the column
  {
    T A = T(1), B = T(0);
#pragma unroll
    for (int i = 0; i < KB; ++i) {
      if (i < nb) {
        A = la[i] * A;
        B = la[i] * B + r[i];
      }
    }
    // (each wave overwrites only its own slots, which the tile's first wave
    // filled before the last barrier and this wave has read)
    at(wave, 0) = A;
    at(wave, 1) = B;
  }
  __syncthreads();
  if (wt == 0 && slot < tpb) {
    T d = T(0);
    for (int j = w0; j < w0 + nw; ++j) {
      const T aj = at(j, 0), bj = at(j, 1);
      at(j, 2) = d;
      d = aj * d + bj;
    }
  }
  __syncthreads();
  {
    T d = at(wave, 2);
#pragma unroll
    for (int i = 0; i < KB; ++i) {
      if (i < nb) {
        d = la[i] * d + r[i];
        r[i] = d;   // r now holds d
      }
    }
  }

  // ---- round 3, back substitution x_k = mc_k x_{k+1} + d_k: the block's map
  // x_first = C x_in + D from the block's own d; the tile's first wave runs it
  // down the column
  {
    T C = T(1), D = T(0);
#pragma unroll
    for (int i = KB - 1; i >= 0; --i) {
      if (i < nb) {
        C = mc[i] * C;
        D = mc[i] * D + r[i];
      }
    }
    at(wave, 3) = C;
    at(wave, 4) = D;
  }
  __syncthreads();
  if (wt == 0 && slot < tpb) {
    T x = T(0);
    for (int j = w0 + nw - 1; j >= w0; --j) {
      const T cj = at(j, 3), dj = at(j, 4);
      at(j, 5) = x;
      x = cj * x + dj;
    }
  }
  __syncthreads();
  T x = at(wave, 5);
  const bool upd = relaxes(L, col);
  double acc[2] = {0.0, 0.0};
#pragma unroll
  for (int i = KB - 1; i >= 0; --i) {
    if (i < nb) {
      x = mc[i] * x + r[i];
      const size_t o = c.base + static_cast<size_t>(k0 + i) * kTile;
      const T uo = upd ? (ZERO ? omega * x : uu[i] + omega * x) : (ZERO ? T(0) : uu[i]);
      const TO zo = static_cast<TO>(uo);
      u_out[o] = zo;
      if (DOTS) {
        acc[0] += static_cast<double>(zo) * q[o];
        // f read again rather than held since the start (registers bound
        // the tiles in flight; the line is still in cache)
        acc[1] += static_cast<double>(zo) * static_cast<double>(f[o]);
      }
    }
  }
  if (DOTS) block_sums(acc, partials, g.b);
}

// residual on the fine level, summed over the four children of each coarse
// cell (Algorithm 1 residual + restriction by summation, Section 5)
template <typename T, int CH, int PM = 0>
__device__ __forceinline__ void residual_restrict_body(const Lv<T>& L, int chunk_rt, int n_coarse,
                                                       const T* __restrict__ f, const T* __restrict__ u,
                                                       T* __restrict__ fc, GridPos g) {
  const int chunk = CH > 0 ? CH : chunk_rt;
  const int nchunks = (L.nz + chunk - 1) / chunk;
  const int item = __builtin_amdgcn_readfirstlane(xcd_tile(g.b, g.nb) * 4 + (threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  if (item >= (L.npad >> 6) * nchunks) return;
  const int tile = item / nchunks, chunk_i = item - tile * nchunks;
  const int k0 = chunk_i * chunk, k1 = min(L.nz, k0 + chunk);
  const int col = tile * kTile + lane;
  const int P = col >> 2;
  const Column<T> c = load_column(L, col);
  const size_t pb = tile_base(P, L.nz);
  auto emit = [&](int k, T r) {
    r += __shfl_xor(r, 1, 64);
    r += __shfl_xor(r, 2, 64);
    if ((lane & 3) == 0 && P < n_coarse) fc[pb + static_cast<size_t>(k) * kTile] = r;
  };
  if constexpr (CH > 0) {
    __shared__ T xbuf[kStencilWaves][2 * kTile];
    ChunkLoads<T, CH> ld;
    ld.load(c, u, k0, L.nz, Exchange<T>{xbuf[threadIdx.x >> 6]}, lane);
    T fv[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i) fv[i] = f[c.base + static_cast<size_t>(min(k0 + i, L.nz - 1)) * kTile];
#pragma unroll
    for (int i = 0; i < CH; ++i)
      if (k0 + i < k1) emit(k0 + i, fv[i] - ld.template row<PM>(L, c, k0, i));
  } else {
    T um = k0 > 0 ? u[c.base + static_cast<size_t>(k0 - 1) * kTile] : T(0);
    T uc = u[c.base + static_cast<size_t>(k0) * kTile];
    for (int k = k0; k < k1; ++k) {
      const size_t o = c.base + static_cast<size_t>(k) * kTile;
      const T up = k + 1 < L.nz ? u[o + kTile] : T(0);
      emit(k, f[o] - apply_row<PM>(L, c, u, k, um, uc, up));
      um = uc;
      uc = up;
    }
  }
}

// u_fine[c] += e_P + sum_j w_cj (e_{N_j(P)} - e_P), P = c / 4
template <typename T>
__device__ __forceinline__ void prolong_add_body(const Lv<T>& F, const Lv<T>& C, int chunk, const T* __restrict__ e,
                                                 T* __restrict__ u, GridPos g) {
  const int nchunks = (F.nz + chunk - 1) / chunk;
  const int item = __builtin_amdgcn_readfirstlane(xcd_tile(g.b, g.nb) * 4 + (threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  if (item >= (F.npad >> 6) * nchunks) return;
  const int tile = item / nchunks, chunk_i = item - tile * nchunks;
  const int k0 = chunk_i * chunk, k1 = min(F.nz, k0 + chunk);
  const int col = tile * kTile + lane;
  if (col >= F.n) return;
  const int P = col >> 2;
  const T w0 = F.pw[col], w1 = F.pw[F.npad + col], w2 = F.pw[2 * F.npad + col];
  const size_t bp = tile_base(P, F.nz);
  const size_t q0 = tile_base(C.nbr[P], F.nz), q1 = tile_base(C.nbr[C.npad + P], F.nz),
               q2 = tile_base(C.nbr[2 * C.npad + P], F.nz);
  const size_t base = tile_base(col, F.nz);
  for (int k = k0; k < k1; ++k) {
    const size_t ok = static_cast<size_t>(k) * kTile;
    const T ep = e[bp + ok];
    T v = ep + w0 * (e[q0 + ok] - ep);
    v = v + w1 * (e[q1 + ok] - ep);
    v = v + w2 * (e[q2 + ok] - ep);
    u[base + ok] = u[base + ok] + v;
  }
}

// ---------------------------------------------------------------------------
// flexible-CG BLAS-1: grid-stride loops over the padded vector with a fixed
// block count, deterministic reductions
// ---------------------------------------------------------------------------

__device__ __forceinline__ void fcg_update_body(double* __restrict__ x, double* __restrict__ r,
                                                const double* __restrict__ p, const double* __restrict__ q,
                                                const FcgScalars* __restrict__ sc, size_t len,
                                                double* __restrict__ partials, GridPos g) {
  const double alpha = sc->alpha;
  double acc[2] = {0.0, 0.0};
  for (size_t i = static_cast<size_t>(g.b) * blockDim.x + threadIdx.x; i < len;
       i += static_cast<size_t>(g.nb) * blockDim.x) {
    x[i] = __builtin_fma(alpha, p[i], x[i]);
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    acc[0] += ri * ri;
  }
  block_sums(acc, partials, g.b);
}

// <z, q>, <z, r> for the case where the smoother cannot fuse them
__device__ __forceinline__ void dots_body(const double* __restrict__ z, const double* __restrict__ q,
                                          const double* __restrict__ r, size_t len, double* __restrict__ partials,
                                          GridPos g) {
  double acc[2] = {0.0, 0.0};
  for (size_t i = static_cast<size_t>(g.b) * blockDim.x + threadIdx.x; i < len;
       i += static_cast<size_t>(g.nb) * blockDim.x) {
    const double zi = z[i];
    acc[0] += zi * q[i];
    acc[1] += zi * r[i];
  }
  block_sums(acc, partials, g.b);
}

template <typename TZ>
__device__ __forceinline__ void pupdate_body(const TZ* __restrict__ z, double* __restrict__ p,
                                             const FcgScalars* __restrict__ sc, size_t len, GridPos g) {
  const double beta = sc->beta;
  for (size_t i = static_cast<size_t>(g.b) * blockDim.x + threadIdx.x; i < len;
       i += static_cast<size_t>(g.nb) * blockDim.x)
    p[i] = static_cast<double>(z[i]) + beta * p[i];
}

// ---------------------------------------------------------------------------
// single-problem kernels
// ---------------------------------------------------------------------------

// Single solves: the sites of an iteration leave the scalars alone once
// they say done (an iteration queued ahead of the host's convergence test
// then changes nothing the solve returns); the kFinRR site publishes the
// iteration's record to the host ring when one is given.
__global__ __launch_bounds__(kFinThreads) void k_finalize(int site, const double* __restrict__ partials, int nblocks,
                                                  FcgScalars* __restrict__ sc, double rtol,
                                                  FcgRecord* __restrict__ ring, double div2) {
  const bool iter_site = site == kFinAlpha || site == kFinRR || site == kFinBeta;
  if (!(iter_site && sc->done)) finalize_body(site, partials, nblocks, sc, rtol, div2);
  if (site == kFinInit && ring != nullptr && threadIdx.x == 0) {
    // record 0: the initial residual, so that the host can decide while the
    // first iteration already runs
    FcgRecord* slot = ring;
    slot->rr = sc->rr;
    slot->ff = sc->ff;
    slot->status = sc->status;
    slot->done = sc->done;
    slot->iters = 0;
    __threadfence_system();
    slot->seq = 0;
  }
  if (site == kFinRR && ring != nullptr && threadIdx.x == 0) {
    const int seq = sc->seq + 1;
    sc->seq = seq;
    FcgRecord* slot = ring + (seq % kRecords);
    slot->rr = sc->rr;
    slot->status = sc->status;
    slot->done = sc->done;
    slot->iters = sc->iters;
    __threadfence_system();   // the payload is visible before the sequence number
    slot->seq = seq;
  }
}

template <int MODE, int CH, int PM>
__global__ __launch_bounds__(256) void k_spmv64(Lv<double> L, int chunk, const double* __restrict__ x,
                                                const double* __restrict__ b, double* __restrict__ y,
                                                double* __restrict__ partials, float* __restrict__ y32) {
  spmv_body<MODE, CH, PM>(L, chunk, x, b, y, partials, whole_grid(), y32);
}

// Occupancy: an FP32 sweep with up to 8 levels per wave fits two 16-wave
// workgroups per CU (at most 64 VGPRs, 8 waves per SIMD); with 16 levels per
// wave and an FP32 right-hand side, three 8-wave workgroups (at most 80
// VGPRs, 6 waves per SIMD); otherwise fewer. FP64 with 16 levels per wave
// needs more than 128 VGPRs and is limited to 8 waves (nz <= 128). wide: an
// FP64 right-hand side or the fused dots (16 levels per wave: 4 per SIMD).
template <int KB, typename T>
constexpr int scan_waves_per_simd(bool wide) {
  return (sizeof(T) == 4 && KB <= 8)     ? 8
         : (sizeof(T) == 4 && !wide)    ? 6
         : (sizeof(T) == 8 && KB == 16) ? 2
                                        : 4;
}
// profiles that do not factorise: the per-level coefficient loads need more
// registers, no FP32 bound beyond 4
template <int KB, typename T>
constexpr int scan_waves_per_simd_full() {
  return (sizeof(T) == 8 && KB == 16) ? 2 : 4;
}
template <int KB, typename T>
constexpr int scan_max_threads() {
  return 64 * ((sizeof(T) == 8 && KB == 16) ? 8 : kScanWavesMax);
}

template <int KB, typename T, typename TF, typename TO, bool ZERO, bool FCOPY, bool DOTS, int PM>
__global__ __launch_bounds__((scan_max_threads<KB, T>()),
                             (PM == 0 ? scan_waves_per_simd<KB, T>(DOTS || std::is_same<TF, double>::value)
                                      : scan_waves_per_simd_full<KB, T>())) void k_smooth_scan(
    Lv<T> L, const TF* __restrict__ f, const T* __restrict__ u_in, TO* __restrict__ u_out, T* __restrict__ fcopy,
    T omega, const double* __restrict__ q, double* __restrict__ partials) {
  smooth_scan_body<KB, T, TF, TO, ZERO, FCOPY, DOTS, PM>(L, f, u_in, u_out, fcopy, omega, q, partials, whole_grid());
}

template <typename T, int CH, int PM>
__global__ __launch_bounds__(256) void k_residual_restrict(Lv<T> L, int chunk, int n_coarse, const T* __restrict__ f,
                                                           const T* __restrict__ u, T* __restrict__ fc) {
  residual_restrict_body<T, CH, PM>(L, chunk, n_coarse, f, u, fc, whole_grid());
}

template <typename T>
__global__ __launch_bounds__(256) void k_prolong_add(Lv<T> F, Lv<T> C, int chunk, const T* __restrict__ e,
                                                     T* __restrict__ u) {
  prolong_add_body<T>(F, C, chunk, e, u, whole_grid());
}

__global__ __launch_bounds__(256) void k_fcg_update(double* __restrict__ x, double* __restrict__ r,
                                                    const double* __restrict__ p, const double* __restrict__ q,
                                                    const FcgScalars* __restrict__ sc, size_t len,
                                                    double* __restrict__ partials) {
  if (sc->done) return;
  fcg_update_body(x, r, p, q, sc, len, partials, whole_grid());
}

// p_k = z + beta p_{k-1} into slot k % kDirSlots. When the ring is full
// (k a positive multiple of kDirSlots) x first receives alpha p of the
// kDirSlots iterations before k, in order, element by element ahead of the
// slot's overwrite.
template <typename TZ>
__global__ __launch_bounds__(256) void k_pupdate_ring(const TZ* __restrict__ z, double* __restrict__ ring,
                                                      double* __restrict__ x, FcgScalars* __restrict__ sc,
                                                      size_t len) {
  if (sc->done) return;
  const int k = sc->iters;
  const double beta = sc->beta;
  const bool flush = k > 0 && k % kDirSlots == 0;
  const double* __restrict__ pp = ring + static_cast<size_t>((k + kDirSlots - 1) % kDirSlots) * len;
  double* __restrict__ pn = ring + static_cast<size_t>(k % kDirSlots) * len;
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < len;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    if (flush) {
      double xi = x[i];
#pragma unroll
      for (int j = 0; j < kDirSlots; ++j)
        xi = __builtin_fma(sc->alpha_hist[j], ring[static_cast<size_t>(j) * len + i], xi);
      x[i] = xi;
    }
    // (the first direction is z itself; the ring's previous slot is not read)
    pn[i] = k == 0 ? static_cast<double>(z[i]) : __builtin_fma(beta, pp[i], static_cast<double>(z[i]));
  }
  // (no block of this kernel reads flushed)
  if (flush && blockIdx.x == 0 && threadIdx.x == 0) sc->flushed = k;
}

template <int CH, int PM>
__global__ __launch_bounds__(256) void k_spmv_ring(Lv<double> L, int chunk, const double* __restrict__ ring,
                                                   size_t len, double* __restrict__ q, double* __restrict__ partials,
                                                   const FcgScalars* __restrict__ sc) {
  if (sc->done) return;
  const double* __restrict__ p = ring + static_cast<size_t>(sc->iters % kDirSlots) * len;
  spmv_body<0, CH, PM>(L, chunk, p, nullptr, q, partials, whole_grid());
}

// The direction update inside q = A p: p_k = z + beta p_{k-1} is formed on
// the fly at every point the operator reads (the expression of
// k_pupdate_ring, so the same bits), stored for the wave's own points, and
// the ring's flush, when due, runs on the same points first.
template <int CH, typename TZ, int PM = 0>
__device__ __forceinline__ void spmv_pring_body(const Lv<double>& L, const TZ* __restrict__ z,
                                                double* __restrict__ ring, size_t len, double* __restrict__ x,
                                                double* __restrict__ q, double* __restrict__ partials,
                                                FcgScalars* __restrict__ sc, GridPos g) {
  const int k = sc->iters;
  const double beta = sc->beta;
  const bool flush = k > 0 && k % kDirSlots == 0;
  const double* __restrict__ pp = ring + static_cast<size_t>((k + kDirSlots - 1) % kDirSlots) * len;
  double* __restrict__ pn = ring + static_cast<size_t>(k % kDirSlots) * len;
  const int nchunks = (L.nz + CH - 1) / CH;
  const int lb = xcd_tile(g.b, g.nb);
  const int item = __builtin_amdgcn_readfirstlane(lb * 4 + (threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  double acc[2] = {0.0, 0.0};
  if (item < (L.npad >> 6) * nchunks) {
    const int tile = item / nchunks, chunk_i = item - tile * nchunks;
    const int k0 = chunk_i * CH, k1 = min(L.nz, k0 + CH);
    const Column<double> c = load_column(L, tile * kTile + lane);
    __shared__ double xbuf[kStencilWaves][2 * kTile];
    ChunkLoads<double, CH> ld;
    // (the first direction is z itself; the ring's previous slot is not read)
    if (k == 0)
      ld.load_with(c, [&](size_t o) { return static_cast<double>(z[o]); }, k0, L.nz,
                   Exchange<double>{xbuf[threadIdx.x >> 6]}, lane);
    else
      ld.load_with(c, [&](size_t o) { return __builtin_fma(beta, pp[o], static_cast<double>(z[o])); }, k0, L.nz,
                   Exchange<double>{xbuf[threadIdx.x >> 6]}, lane);
#pragma unroll
    for (int i = 0; i < CH; ++i)
      if (k0 + i < k1) {
        const size_t o = c.base + static_cast<size_t>(k0 + i) * kTile;
        if (flush) {
          double xi = x[o];
#pragma unroll
          for (int j = 0; j < kDirSlots; ++j) xi = __builtin_fma(sc->alpha_hist[j], ring[static_cast<size_t>(j) * len + o], xi);
          x[o] = xi;
        }
        const double uc = ld.xv[i + 1];
        const double ax = ld.template row<PM>(L, c, k0, i);
        pn[o] = uc;
        q[o] = ax;
        acc[0] += uc * ax;
      }
  }
  block_sums(acc, partials, lb);
  // (no block of this kernel reads flushed)
  if (flush && g.b == 0 && threadIdx.x == 0) sc->flushed = k;
}

template <int CH, typename TZ, int PM>
__global__ __launch_bounds__(256) void k_spmv_pring(Lv<double> L, const TZ* __restrict__ z, double* __restrict__ ring,
                                                    size_t len, double* __restrict__ x, double* __restrict__ q,
                                                    double* __restrict__ partials, FcgScalars* __restrict__ sc) {
  if (sc->done) return;
  spmv_pring_body<CH, TZ, PM>(L, z, ring, len, x, q, partials, sc, whole_grid());
}

// r -= alpha q and <r, r>; with r32 also the FP32 rounding of the new r,
// which the next FP32 V-cycle reads as its finest right-hand side
__device__ __forceinline__ void rupdate_body(double* __restrict__ r, const double* __restrict__ q,
                                             const FcgScalars* __restrict__ sc, size_t len,
                                             double* __restrict__ partials, float* __restrict__ r32, GridPos g) {
  const double alpha = sc->alpha;
  double acc[2] = {0.0, 0.0};
  for (size_t i = static_cast<size_t>(g.b) * blockDim.x + threadIdx.x; i < len;
       i += static_cast<size_t>(g.nb) * blockDim.x) {
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    if (r32) r32[i] = static_cast<float>(ri);
    acc[0] += ri * ri;
  }
  block_sums(acc, partials, g.b);
}

__global__ __launch_bounds__(256) void k_rupdate(double* __restrict__ r, const double* __restrict__ q,
                                                 const FcgScalars* __restrict__ sc, size_t len,
                                                 double* __restrict__ partials, float* __restrict__ r32) {
  if (sc->done) return;
  rupdate_body(r, q, sc, len, partials, r32, whole_grid());
}


// x += alpha_j p_j of the iterations not yet added ([flushed, iters)), in
// order, each a fused multiply-add as in the per-iteration update.
__global__ __launch_bounds__(256) void k_flush(double* __restrict__ x, const double* __restrict__ ring,
                                               const FcgScalars* __restrict__ sc, size_t len) {
  const int first = sc->flushed, count = sc->iters - sc->flushed;
  if (count <= 0) return;
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < len;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    double xi = x[i];
    for (int j = 0; j < count; ++j) {
      const int it = first + j;
      xi = __builtin_fma(sc->alpha_hist[it % kDirSlots], ring[static_cast<size_t>(it % kDirSlots) * len + i], xi);
    }
    x[i] = xi;
  }
}

__global__ __launch_bounds__(256) void k_dots(const double* __restrict__ z, const double* __restrict__ q,
                                              const double* __restrict__ r, size_t len, double* __restrict__ partials) {
  dots_body(z, q, r, len, partials, whole_grid());
}

template <typename TZ>
__global__ __launch_bounds__(256) void k_pupdate(const TZ* __restrict__ z, double* __restrict__ p,
                                                 const FcgScalars* __restrict__ sc, size_t len) {
  pupdate_body(z, p, sc, len, whole_grid());
}

__global__ __launch_bounds__(256) void k_dots2(const double* __restrict__ a, const double* __restrict__ b,
                                               const double* __restrict__ c, const double* __restrict__ d,
                                               size_t len, double* __restrict__ partials) {
  double acc[2] = {0.0, 0.0};
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < len;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    acc[0] += a[i] * b[i];
    acc[1] += c[i] * d[i];
  }
  block_sums(acc, partials, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_bicg_p(const double* __restrict__ r, double* __restrict__ p,
                                                const double* __restrict__ v, const FcgScalars* __restrict__ sc,
                                                size_t len) {
  const double beta = sc->beta, w = sc->w;
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < len;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    p[i] = r[i] + beta * (p[i] - w * v[i]);
}

__global__ __launch_bounds__(256) void k_bicg_s(double* __restrict__ r, const double* __restrict__ v,
                                                const FcgScalars* __restrict__ sc, size_t len) {
  const double alpha = sc->alpha;
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < len;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    r[i] = r[i] - alpha * v[i];
}

__global__ __launch_bounds__(256) void k_bicg_x(double* __restrict__ x, double* __restrict__ r,
                                                const double* __restrict__ y, const double* __restrict__ z,
                                                const double* __restrict__ t, const double* __restrict__ rh,
                                                const FcgScalars* __restrict__ sc, size_t len,
                                                double* __restrict__ partials) {
  const double alpha = sc->alpha, w = sc->w;
  double acc[2] = {0.0, 0.0};
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < len;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    x[i] = x[i] + alpha * y[i] + w * z[i];
    const double ri = r[i] - w * t[i];
    r[i] = ri;
    acc[0] += rh[i] * ri;
    acc[1] += ri * ri;
  }
  block_sums(acc, partials, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_add(double* __restrict__ x, const double* __restrict__ y, size_t len) {
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < len;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    x[i] = x[i] + y[i];
}

__global__ __launch_bounds__(256) void k_fill(uint32_t* __restrict__ p, size_t words) {
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < words;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    p[i] = 0u;
}

__global__ __launch_bounds__(256) void k_pack(const double* __restrict__ cm, double* __restrict__ tiled, int n,
                                              int npad, int nz) {
  const size_t total = static_cast<size_t>(npad) * nz;
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int col = static_cast<int>(i / nz), k = static_cast<int>(i - static_cast<size_t>(col) * nz);
    tiled[tile_base(col, nz) + static_cast<size_t>(k) * kTile] = col < n ? cm[i] : 0.0;
  }
}

__global__ __launch_bounds__(256) void k_unpack(const double* __restrict__ tiled, double* __restrict__ cm, int n,
                                                int nz) {
  const size_t total = static_cast<size_t>(n) * nz;
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int col = static_cast<int>(i / nz), k = static_cast<int>(i - static_cast<size_t>(col) * nz);
    cm[i] = tiled[tile_base(col, nz) + static_cast<size_t>(k) * kTile];
  }
}

// ---------------------------------------------------------------------------
// batched kernels: one grouped launch covers several problems. segs[] is
// sorted by start; every segment starts at a multiple of 8 blocks, so the
// XCD of a block (blockIdx.x mod 8) equals that of its problem-local index.
// Problems whose scalars are marked done are skipped.
// ---------------------------------------------------------------------------

// The segment table is read through the constant address space: the table
// does not change during a launch, so its fields become scalar loads the
// compiler may repeat where they are used instead of holding every pointer
// of a level descriptor in registers (which took the grouped sweep from the
// 50 vector registers of the single one to 81, and its occupancy with it).
using CSeg = const __attribute__((address_space(4))) Seg;

__device__ __forceinline__ CSeg* find_segment(const Seg* __restrict__ segs_g, int nseg, GridPos& g) {
  CSeg* segs = (CSeg*)segs_g;
  const int b = blockIdx.x;
  int s = 0;
  for (int i = 1; i < nseg; ++i)
    if (segs[i].start <= b) s = i;
  CSeg* sg = &segs[__builtin_amdgcn_readfirstlane(s)];
  g.b = b - sg->start;
  g.nb = sg->nblocks;
  if (g.b >= g.nb) return nullptr;                      // alignment padding
  if (sg->sc != nullptr && sg->sc->done) return nullptr;  // converged problem
  return sg;
}

// (the occupancy bounds of the single sweep)
template <int KB, typename T, typename TF, typename TO, bool ZERO, bool FCOPY, bool DOTS, int PM>
__global__ __launch_bounds__((scan_max_threads<KB, T>()),
                             (PM == 0 ? scan_waves_per_simd<KB, T>(DOTS || std::is_same<TF, double>::value)
                                      : scan_waves_per_simd_full<KB, T>())) void kb_smooth_scan(
    const Seg* __restrict__ segs, int nseg, double omega) {
  GridPos g;
  CSeg* sg = find_segment(segs, nseg, g);
  if (!sg) return;
  smooth_scan_body<KB, T, TF, TO, ZERO, FCOPY, DOTS, PM, !DOTS>(
      view<T>(sg->L), static_cast<const TF*>(sg->in0), static_cast<const T*>(sg->in1), static_cast<TO*>(sg->out0),
      static_cast<T*>(sg->out1), static_cast<T>(omega), sg->q, sg->partials, g);
}

// (CH > 0: every segment's chunk is CH, the instance the single launches
// use for that chunk, so a batch forms the same bits)
template <typename T, int CH, int PM>
__global__ __launch_bounds__(256) void kb_residual_restrict(const Seg* __restrict__ segs, int nseg) {
  GridPos g;
  CSeg* sg = find_segment(segs, nseg, g);
  if (!sg) return;
  residual_restrict_body<T, CH, PM>(view<T>(sg->L), sg->chunk, sg->C.n, static_cast<const T*>(sg->in0),
                             static_cast<const T*>(sg->in1), static_cast<T*>(sg->out0), g);
}

template <typename T>
__global__ __launch_bounds__(256) void kb_prolong_add(const Seg* __restrict__ segs, int nseg) {
  GridPos g;
  CSeg* sg = find_segment(segs, nseg, g);
  if (!sg) return;
  prolong_add_body<T>(view<T>(sg->L), view<T>(sg->C), sg->chunk, static_cast<const T*>(sg->in0),
                      static_cast<T*>(sg->out0), g);
}

template <int CH, int PM>
__global__ __launch_bounds__(256) void kb_spmv64(const Seg* __restrict__ segs, int nseg) {
  GridPos g;
  CSeg* sg = find_segment(segs, nseg, g);
  if (!sg) return;
  spmv_body<0, CH, PM>(view<double>(sg->L), sg->chunk, static_cast<const double*>(sg->in0), nullptr,
                   static_cast<double*>(sg->out0), sg->partials, g);
}

template <typename TZ>
__global__ __launch_bounds__(256) void kb_pupdate(const Seg* __restrict__ segs, int nseg) {
  GridPos g;
  CSeg* sg = find_segment(segs, nseg, g);
  if (!sg) return;
  pupdate_body(static_cast<const TZ*>(sg->in0), static_cast<double*>(sg->out0), sg->sc, sg->len, g);
}

__global__ __launch_bounds__(256) void kb_fcg_update(const Seg* __restrict__ segs, int nseg) {
  GridPos g;
  CSeg* sg = find_segment(segs, nseg, g);
  if (!sg) return;
  fcg_update_body(static_cast<double*>(sg->out0), static_cast<double*>(sg->out1), static_cast<const double*>(sg->in0),
                  static_cast<const double*>(sg->in1), sg->sc, sg->len, sg->partials, g);
}

template <int CH, typename TZ, int PM>
__global__ __launch_bounds__(256) void kb_spmv_pring(const Seg* __restrict__ segs, int nseg) {
  GridPos g;
  CSeg* sg = find_segment(segs, nseg, g);
  if (!sg) return;
  spmv_pring_body<CH, TZ, PM>(view<double>(sg->L), static_cast<const TZ*>(sg->in0), sg->aux, sg->len,
                          static_cast<double*>(sg->out1), static_cast<double*>(sg->out0), sg->partials, sg->sc, g);
}

__global__ __launch_bounds__(256) void kb_rupdate(const Seg* __restrict__ segs, int nseg) {
  GridPos g;
  CSeg* sg = find_segment(segs, nseg, g);
  if (!sg) return;
  rupdate_body(static_cast<double*>(sg->out1), static_cast<const double*>(sg->in1), sg->sc, sg->len, sg->partials,
               static_cast<float*>(sg->out0), g);
}

// one block per problem
__global__ __launch_bounds__(kFinThreads) void kb_finalize(const Seg* __restrict__ segs, int nseg) {
  CSeg* sg = &((CSeg*)segs)[blockIdx.x];
  if (sg->sc->done) return;
  finalize_body(sg->site, sg->partials, sg->nblocks, sg->sc, 0.0);
}

unsigned grid_for(size_t work, unsigned cap) {
  size_t b = (work + 255) / 256;
  if (b < 1) b = 1;
  return static_cast<unsigned>(b < cap ? b : cap);
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

int stencil_chunk(int npad, int nz) {
  // largest levels-per-wave that still gives >= 4096 waves (latency hiding on
  // small grids), at most 16
  const size_t tiles = static_cast<size_t>(npad / kTile);
  for (int c = 16; c > 1; c >>= 1)
    if (tiles * static_cast<size_t>((nz + c - 1) / c) >= 4096) return c;
  return 1;
}

int effective_chunk(int tuned, int npad, int nz) { return tuned > 0 ? tuned : stencil_chunk(npad, nz); }

size_t stencil_blocks(int npad, int nz, int chunk) {
  const int c = effective_chunk(chunk, npad, nz);
  const size_t waves = static_cast<size_t>(npad / kTile) * ((nz + c - 1) / c);
  return (waves + 3) / 4;
}

int scan_waves(int nz, int scan_levels) { return (nz + scan_levels - 1) / scan_levels; }

// the scan kernel for nz <= 16 * KB; the LDS-staged kernel while its two
// [nz][64] arrays fit; the global-scratch kernel for any nz
size_t g_max_lds = 65536;

size_t lds_smoother_bytes(int nz, int prec) {
  return (2 * static_cast<size_t>(nz) * kTile + 3 * static_cast<size_t>(nz) + 1) * static_cast<size_t>(prec);
}

bool smoother_fits(int kind, int scan_levels, int nz, int prec) {
  switch (kind) {
    case kSmScan:
      return (scan_levels == 4 || scan_levels == 8 || scan_levels == 16) &&
             scan_waves(nz, scan_levels) <= ((prec == 8 && scan_levels == 16) ? 8 : kScanWavesMax);
    case kSmLds:
      return lds_smoother_bytes(nz, prec) <= g_max_lds;
    case kSmGlobal:
      return true;
    default:
      return false;
  }
}

LevelTune default_tune(int nz, int prec) {
  LevelTune t;
  if (smoother_fits(kSmScan, 8, nz, prec)) {
    t.smoother = kSmScan;
    t.scan_levels = 8;
  } else if (smoother_fits(kSmScan, 16, nz, prec)) {
    t.smoother = kSmScan;
    t.scan_levels = 16;
  } else if (smoother_fits(kSmLds, 0, nz, prec)) {
    t.smoother = kSmLds;
  } else {
    t.smoother = kSmGlobal;
  }
  return t;
}

unsigned pupdate_blocks(size_t len) { return grid_for(len, 2048); }

hipError_t launch_finalize(int site, const double* partials, int nblocks, FcgScalars* sc, double rtol, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinThreads), 0, s, site, partials, nblocks, sc, rtol, nullptr, kDefaultDiv2);
  return hipGetLastError();
}

// Calls fn(std::integral_constant<int, CH>): CH = chunk for the unrolled
// instances 1, 2, 4, 8, 16, else 0 (the loop over a runtime chunk).
template <typename Fn>
void chunk_variant(int chunk, Fn&& fn) {
  switch (chunk) {
    case 1: fn(std::integral_constant<int, 1>{}); break;
    case 2: fn(std::integral_constant<int, 2>{}); break;
    case 4: fn(std::integral_constant<int, 4>{}); break;
    case 8: fn(std::integral_constant<int, 8>{}); break;
    case 16: fn(std::integral_constant<int, 16>{}); break;
    default: fn(std::integral_constant<int, 0>{}); break;
  }
}

// Calls fn(std::integral_constant<int, PM>) for the profile mode of a level
// (0 factorised, 1 radial couplings per (T, k), 2 all coefficients per (T, k)).
template <typename Fn>
void profile_variant(int pm, Fn&& fn) {
  switch (pm) {
    case 1: fn(std::integral_constant<int, 1>{}); break;
    case 2: fn(std::integral_constant<int, 2>{}); break;
    case 3: fn(std::integral_constant<int, 3>{}); break;
    default: fn(std::integral_constant<int, 0>{}); break;
  }
}

hipError_t launch_spmv64(const LevelView& L, int mode, const double* x, const double* b, double* y,
                         double* partials, int site, FcgScalars* sc, hipStream_t s, double rtol, float* y32,
                         FcgRecord* ring, double div2) {
  const int chunk = effective_chunk(L.tune.chunk_spmv, L.npad, L.nz);
  const unsigned blocks = static_cast<unsigned>(stencil_blocks(L.npad, L.nz, chunk));
  const Lv<double> V = view<double>(L);
  profile_variant(L.pm, [&](auto pmc) {
    constexpr int PM = decltype(pmc)::value;
    chunk_variant(chunk, [&](auto chc) {
      constexpr int CH = decltype(chc)::value;
      if (mode == 0)
        hipLaunchKernelGGL((k_spmv64<0, CH, PM>), dim3(blocks), dim3(256), 0, s, V, chunk, x, b, y, partials,
                           static_cast<float*>(nullptr));
      else
        hipLaunchKernelGGL((k_spmv64<1, CH, PM>), dim3(blocks), dim3(256), 0, s, V, chunk, x, b, y, partials, y32);
    });
  });
  if (site != kFinNone)
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinThreads), 0, s, site, partials, static_cast<int>(blocks), sc, rtol, ring,
                       div2);
  return hipGetLastError();
}

template <typename X>
struct Type {
  using type = X;
};
template <bool B>
using Bool = std::integral_constant<bool, B>;

// Calls fn(Type<TF>, Type<TO>, Bool<ZERO>, Bool<FCOPY>, Bool<DOTS>) for the
// smoother variant of the flags; these are the combinations the V-cycle uses
// (T: precision of the level data).
template <typename T, typename Fn>
void smoother_variant(bool f_double, bool out_double, bool zero, bool fcopy, bool dots, Fn&& fn) {
  using D = Type<double>;
  using P = Type<T>;
  if (f_double && out_double) {
    if (dots && zero)
      fn(D{}, D{}, Bool<true>{}, Bool<false>{}, Bool<true>{});
    else if (dots)
      fn(D{}, D{}, Bool<false>{}, Bool<false>{}, Bool<true>{});
    else if (zero)
      fn(D{}, D{}, Bool<true>{}, Bool<false>{}, Bool<false>{});
    else
      fn(D{}, D{}, Bool<false>{}, Bool<false>{}, Bool<false>{});
  } else if (f_double) {
    if (dots && zero)
      fn(D{}, P{}, Bool<true>{}, Bool<false>{}, Bool<true>{});
    else if (dots)
      fn(D{}, P{}, Bool<false>{}, Bool<false>{}, Bool<true>{});
    else if (zero && fcopy)
      fn(D{}, P{}, Bool<true>{}, Bool<true>{}, Bool<false>{});
    else if (zero)
      fn(D{}, P{}, Bool<true>{}, Bool<false>{}, Bool<false>{});
    else
      fn(D{}, P{}, Bool<false>{}, Bool<false>{}, Bool<false>{});
  } else if (out_double) {
    if (zero)
      fn(P{}, D{}, Bool<true>{}, Bool<false>{}, Bool<false>{});
    else
      fn(P{}, D{}, Bool<false>{}, Bool<false>{}, Bool<false>{});
  } else {
    if (zero)
      fn(P{}, P{}, Bool<true>{}, Bool<false>{}, Bool<false>{});
    else
      fn(P{}, P{}, Bool<false>{}, Bool<false>{}, Bool<false>{});
  }
}

// Calls fn(std::integral_constant<int, KB>) for a valid levels-per-wave value.
template <typename Fn>
void scan_levels_variant(int kb, Fn&& fn) {
  if (kb == 4)
    fn(std::integral_constant<int, 4>{});
  else if (kb == 16)
    fn(std::integral_constant<int, 16>{});
  else
    fn(std::integral_constant<int, 8>{});
}

struct SmoothArgs {
  const void* f;
  const void* u_in;
  void* u_out;
  void* fcopy;
  void* sd;
  void* sc;
  double omega;
  const double* q;
  double* partials;
  FcgScalars* scal;
};

template <typename T>
static hipError_t smooth_t(const LevelView& Lg, bool f_double, bool zero, bool out_double, const SmoothArgs& a,
                           hipStream_t s) {
  const Lv<T> L = view<T>(Lg);
  const LevelTune& tn = Lg.tune;
  const bool dots = a.q != nullptr;
  const bool fcopy = a.fcopy != nullptr;
  const int prec = static_cast<int>(sizeof(T));
  const unsigned ntiles = static_cast<unsigned>(L.npad / kTile);
  const T* ui = static_cast<const T*>(a.u_in);
  T* fc = static_cast<T*>(a.fcopy);
  const T om = static_cast<T>(a.omega);
  if (!smoother_fits(tn.smoother, tn.scan_levels, L.nz, prec)) return hipErrorInvalidValue;
  if (tn.smoother == kSmScan) {
    if (Lg.margin == nullptr) return hipErrorInvalidValue;   // the scan form reads the stored margins
    const int waves = scan_waves(L.nz, tn.scan_levels);
    const size_t sl = scan_lds_bytes(waves, static_cast<int>(sizeof(T)));
    if (Lg.pm != 0 && tn.scan_levels == 4) return hipErrorInvalidValue;   // (no instance)
    scan_levels_variant(tn.scan_levels, [&](auto kbc) {
      constexpr int KB = decltype(kbc)::value;
      profile_variant(Lg.pm, [&](auto pmc) {
        constexpr int PM = decltype(pmc)::value;
        if constexpr (PM == 0 || KB != 4)
          smoother_variant<T>(f_double, out_double, zero, fcopy, dots, [&](auto tf, auto to, auto z, auto fcp, auto dt) {
            using TF = typename decltype(tf)::type;
            using TO = typename decltype(to)::type;
            hipLaunchKernelGGL((k_smooth_scan<KB, T, TF, TO, decltype(z)::value, decltype(fcp)::value,
                                              decltype(dt)::value, PM>),
                               dim3(ntiles), dim3(64 * waves), sl, s, L, static_cast<const TF*>(a.f), ui,
                               static_cast<TO*>(a.u_out), fc, om, a.q, a.partials);
          });
      });
    });
    if (dots)
      hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinThreads), 0, s, static_cast<int>(kFinBeta), a.partials,
                         static_cast<int>(ntiles), a.scal, 0.0, nullptr, kDefaultDiv2);
    return hipGetLastError();
  }
  if (dots) return hipErrorInvalidValue;   // only the scan kernel forms the dots
  if (Lg.pm != 0) return hipErrorInvalidValue;   // profiles that do not factorise: the scan kernel only
  if (tn.smoother == kSmLds) {
    const size_t lds = lds_smoother_bytes(L.nz, prec);
    const unsigned waves = static_cast<unsigned>(std::min(16, std::max(1, (L.nz + kBatch - 1) / kBatch)));
    smoother_variant<T>(f_double, out_double, zero, fcopy, false, [&](auto tf, auto to, auto z, auto fcp, auto) {
      using TF = typename decltype(tf)::type;
      using TO = typename decltype(to)::type;
      hipLaunchKernelGGL((k_smooth_lds<T, TF, TO, decltype(z)::value, decltype(fcp)::value>), dim3(ntiles),
                         dim3(64 * waves), lds, s, L, static_cast<const TF*>(a.f), ui, static_cast<TO*>(a.u_out), fc,
                         om);
    });
  } else {
    smoother_variant<T>(f_double, out_double, zero, fcopy, false, [&](auto tf, auto to, auto z, auto fcp, auto) {
      using TF = typename decltype(tf)::type;
      using TO = typename decltype(to)::type;
      hipLaunchKernelGGL((k_smooth_fallback<T, TF, TO, decltype(z)::value, decltype(fcp)::value>), dim3(ntiles),
                         dim3(kTile), 0, s, L, static_cast<const TF*>(a.f), ui, static_cast<TO*>(a.u_out), fc,
                         static_cast<T*>(a.sd), static_cast<T*>(a.sc), om);
    });
  }
  return hipGetLastError();
}

hipError_t launch_smooth(const LevelView& L, int prec, const void* f, bool f_double, const void* u_in,
                         bool zero_guess, void* u_out, bool out_double, void* fcopy, void* sd, void* sc,
                         double omega, hipStream_t s, const double* q, double* partials, FcgScalars* scal) {
  if (prec == 8) {
    const SmoothArgs a{f, u_in, u_out, nullptr, sd, sc, omega, q, partials, scal};
    return smooth_t<double>(L, true, zero_guess, true, a, s);
  }
  const SmoothArgs a{f, u_in, u_out, fcopy, sd, sc, omega, q, partials, scal};
  return smooth_t<float>(L, f_double, zero_guess, out_double, a, s);
}

hipError_t set_max_lds(size_t bytes) {
  g_max_lds = bytes;
  return hipSuccess;
}

hipError_t launch_residual_restrict(const LevelView& L, const LevelView& C, int prec, const void* f,
                                    const void* u, void* f_coarse, hipStream_t s) {
  const int chunk = effective_chunk(L.tune.chunk_rr, L.npad, L.nz);
  const unsigned blocks = static_cast<unsigned>(stencil_blocks(L.npad, L.nz, chunk));
  profile_variant(L.pm, [&](auto pmc) {
    constexpr int PM = decltype(pmc)::value;
    chunk_variant(chunk, [&](auto chc) {
      constexpr int CH = decltype(chc)::value;
      if (prec == 8)
        hipLaunchKernelGGL((k_residual_restrict<double, CH, PM>), dim3(blocks), dim3(256), 0, s, view<double>(L), chunk,
                           C.n, static_cast<const double*>(f), static_cast<const double*>(u),
                           static_cast<double*>(f_coarse));
      else
        hipLaunchKernelGGL((k_residual_restrict<float, CH, PM>), dim3(blocks), dim3(256), 0, s, view<float>(L), chunk,
                           C.n, static_cast<const float*>(f), static_cast<const float*>(u),
                           static_cast<float*>(f_coarse));
    });
  });
  return hipGetLastError();
}

hipError_t launch_prolong_add(const LevelView& F, const LevelView& C, int prec, const void* e_coarse,
                              void* u_fine, hipStream_t s) {
  const int chunk = effective_chunk(F.tune.chunk_pr, F.npad, F.nz);
  const unsigned blocks = static_cast<unsigned>(stencil_blocks(F.npad, F.nz, chunk));
  if (prec == 8)
    hipLaunchKernelGGL(k_prolong_add<double>, dim3(blocks), dim3(256), 0, s, view<double>(F), view<double>(C), chunk,
                       static_cast<const double*>(e_coarse), static_cast<double*>(u_fine));
  else
    hipLaunchKernelGGL(k_prolong_add<float>, dim3(blocks), dim3(256), 0, s, view<float>(F), view<float>(C), chunk,
                       static_cast<const float*>(e_coarse), static_cast<float*>(u_fine));
  return hipGetLastError();
}

hipError_t launch_margins(const LevelView& L64, int prec, void* margin, hipStream_t s) {
  const unsigned blocks = static_cast<unsigned>((L64.npad + 255) / 256);
  profile_variant(L64.pm, [&](auto pmc) {
    constexpr int PM = decltype(pmc)::value;
    if (prec == 8)
      hipLaunchKernelGGL((k_margins<double, PM>), dim3(blocks), dim3(256), 0, s, view<double>(L64),
                         static_cast<double*>(margin));
    else
      hipLaunchKernelGGL((k_margins<float, PM>), dim3(blocks), dim3(256), 0, s, view<double>(L64),
                         static_cast<float*>(margin));
  });
  return hipGetLastError();
}

hipError_t launch_fcg_update(double* x, double* r, const double* p, const double* q, FcgScalars* sc, size_t len,
                             double* partials, FcgRecord* ring, hipStream_t s) {
  hipLaunchKernelGGL(k_fcg_update, dim3(kRedBlocks), dim3(kRedThreads), 0, s, x, r, p, q, sc, len, partials);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinThreads), 0, s, static_cast<int>(kFinRR), partials, kRedBlocks, sc, 0.0,
                     ring, kDefaultDiv2);
  return hipGetLastError();
}

hipError_t launch_pupdate_ring(const void* z, bool z_double, double* ring, double* x, FcgScalars* sc, size_t len,
                               hipStream_t s) {
  if (z_double)
    hipLaunchKernelGGL(k_pupdate_ring<double>, dim3(pupdate_blocks(len)), dim3(256), 0, s,
                       static_cast<const double*>(z), ring, x, sc, len);
  else
    hipLaunchKernelGGL(k_pupdate_ring<float>, dim3(pupdate_blocks(len)), dim3(256), 0, s,
                       static_cast<const float*>(z), ring, x, sc, len);
  return hipGetLastError();
}

hipError_t launch_spmv_ring(const LevelView& L, const double* ring, size_t len, double* q, double* partials,
                            FcgScalars* sc, hipStream_t s) {
  const int chunk = effective_chunk(L.tune.chunk_spmv, L.npad, L.nz);
  const unsigned blocks = static_cast<unsigned>(stencil_blocks(L.npad, L.nz, chunk));
  const Lv<double> V = view<double>(L);
  profile_variant(L.pm, [&](auto pmc) {
    constexpr int PM = decltype(pmc)::value;
    chunk_variant(chunk, [&](auto chc) {
      constexpr int CH = decltype(chc)::value;
      hipLaunchKernelGGL((k_spmv_ring<CH, PM>), dim3(blocks), dim3(256), 0, s, V, chunk, ring, len, q, partials, sc);
    });
  });
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinThreads), 0, s, static_cast<int>(kFinAlpha), partials,
                     static_cast<int>(blocks), sc, 0.0, nullptr, kDefaultDiv2);
  return hipGetLastError();
}

bool spmv_pring_fits(const LevelView& L) {
  const int chunk = effective_chunk(L.tune.chunk_spmv, L.npad, L.nz);
  return chunk == 1 || chunk == 2 || chunk == 4 || chunk == 8 || chunk == 16;
}

hipError_t launch_spmv_pring(const LevelView& L, const void* z, bool z_double, double* ring, size_t len, double* x,
                             double* q, double* partials, FcgScalars* sc, hipStream_t s, int site) {
  if (!spmv_pring_fits(L)) return hipErrorInvalidValue;
  const int chunk = effective_chunk(L.tune.chunk_spmv, L.npad, L.nz);
  const unsigned blocks = static_cast<unsigned>(stencil_blocks(L.npad, L.nz, chunk));
  const Lv<double> V = view<double>(L);
  profile_variant(L.pm, [&](auto pmc) {
    constexpr int PM = decltype(pmc)::value;
    chunk_variant(chunk, [&](auto chc) {
      constexpr int CH = decltype(chc)::value;
      if constexpr (CH > 0) {
        if (z_double)
          hipLaunchKernelGGL((k_spmv_pring<CH, double, PM>), dim3(blocks), dim3(256), 0, s, V,
                             static_cast<const double*>(z), ring, len, x, q, partials, sc);
        else
          hipLaunchKernelGGL((k_spmv_pring<CH, float, PM>), dim3(blocks), dim3(256), 0, s, V,
                             static_cast<const float*>(z), ring, len, x, q, partials, sc);
      }
    });
  });
  if (site != kFinNone)
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinThreads), 0, s, site, partials, static_cast<int>(blocks), sc, 0.0, nullptr,
                       kDefaultDiv2);
  return hipGetLastError();
}

hipError_t launch_rupdate(double* r, const double* q, FcgScalars* sc, size_t len, double* partials, FcgRecord* ring,
                          hipStream_t s, float* r32) {
  hipLaunchKernelGGL(k_rupdate, dim3(kRedBlocks), dim3(kRedThreads), 0, s, r, q, sc, len, partials, r32);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinThreads), 0, s, static_cast<int>(kFinRR), partials, kRedBlocks, sc, 0.0,
                     ring, kDefaultDiv2);
  return hipGetLastError();
}

hipError_t launch_flush(double* x, const double* ring, const FcgScalars* sc, size_t len, hipStream_t s) {
  hipLaunchKernelGGL(k_flush, dim3(pupdate_blocks(len)), dim3(256), 0, s, x, ring, sc, len);
  return hipGetLastError();
}

hipError_t launch_dots(const double* z, const double* q, const double* r, size_t len, double* partials,
                       FcgScalars* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_dots, dim3(kRedBlocks), dim3(kRedThreads), 0, s, z, q, r, len, partials);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinThreads), 0, s, static_cast<int>(kFinBeta), partials, kRedBlocks, sc, 0.0, nullptr, kDefaultDiv2);
  return hipGetLastError();
}

hipError_t launch_pupdate(const void* z, bool z_double, double* p, const FcgScalars* sc, size_t len, hipStream_t s) {
  if (z_double)
    hipLaunchKernelGGL(k_pupdate<double>, dim3(pupdate_blocks(len)), dim3(256), 0, s, static_cast<const double*>(z), p,
                       sc, len);
  else
    hipLaunchKernelGGL(k_pupdate<float>, dim3(pupdate_blocks(len)), dim3(256), 0, s, static_cast<const float*>(z), p,
                       sc, len);
  return hipGetLastError();
}

hipError_t launch_dots2(const double* a, const double* b, const double* c, const double* d, size_t len,
                        double* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_dots2, dim3(kRedBlocks), dim3(kRedThreads), 0, s, a, b, c, d, len, partials);
  return hipGetLastError();
}

hipError_t launch_krylov_finalize(int stage, const double* partials, FcgScalars* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinThreads), 0, s, stage, partials, stage == kKInit ? 0 : kRedBlocks, sc,
                     0.0, nullptr, kDefaultDiv2);
  return hipGetLastError();
}

hipError_t launch_bicg_p(const double* r, double* p, const double* v, const FcgScalars* sc, size_t len,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_bicg_p, dim3(pupdate_blocks(len)), dim3(256), 0, s, r, p, v, sc, len);
  return hipGetLastError();
}

hipError_t launch_bicg_s(double* r, const double* v, const FcgScalars* sc, size_t len, hipStream_t s) {
  hipLaunchKernelGGL(k_bicg_s, dim3(pupdate_blocks(len)), dim3(256), 0, s, r, v, sc, len);
  return hipGetLastError();
}

hipError_t launch_bicg_x(double* x, double* r, const double* y, const double* z, const double* t, const double* rh,
                         const FcgScalars* sc, size_t len, double* partials, hipStream_t s) {
  hipLaunchKernelGGL(k_bicg_x, dim3(kRedBlocks), dim3(kRedThreads), 0, s, x, r, y, z, t, rh, sc, len, partials);
  return hipGetLastError();
}

hipError_t launch_add(double* x, const double* y, size_t len, hipStream_t s) {
  hipLaunchKernelGGL(k_add, dim3(grid_for(len, 2048)), dim3(256), 0, s, x, y, len);
  return hipGetLastError();
}

hipError_t launch_fill(void* p, size_t bytes, hipStream_t s) {
  const size_t words = bytes / 4;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(words, 2048)), dim3(256), 0, s, static_cast<uint32_t*>(p), words);
  return hipGetLastError();
}

hipError_t launch_pack(const double* cm, double* tiled, int n, int npad, int nz, hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3(grid_for(static_cast<size_t>(npad) * nz, 4096)), dim3(256), 0, s, cm, tiled, n,
                     npad, nz);
  return hipGetLastError();
}

hipError_t launch_unpack(const double* tiled, double* cm, int n, int npad, int nz, hipStream_t s) {
  hipLaunchKernelGGL(k_unpack, dim3(grid_for(static_cast<size_t>(n) * nz, 4096)), dim3(256), 0, s, tiled, cm, n,
                     nz);
  return hipGetLastError();
}

// ---- batched launches -----------------------------------------------------

// Calls fn(std::integral_constant<int, PM>) for the profile modes a batch can
// hold (0 factorised, 1 radial couplings per (T, k), 2 all coefficients per
// (T, k); the advective mode needs the non-symmetric solvers, not batched).
template <typename Fn>
void batch_profile_variant(int pm, Fn&& fn) {
  switch (pm) {
    case 1: fn(std::integral_constant<int, 1>{}); break;
    case 2: fn(std::integral_constant<int, 2>{}); break;
    default: fn(std::integral_constant<int, 0>{}); break;
  }
}

template <typename T>
static hipError_t batched_smooth_t(const BatchLaunch& b, hipStream_t s) {
  const dim3 grid(b.grid), block(b.block);
  if (!smoother_fits(kSmScan, b.scan_levels, 1, static_cast<int>(sizeof(T)))) return hipErrorInvalidValue;
  if (b.pm < 0 || b.pm > 2) return hipErrorInvalidValue;
  scan_levels_variant(b.scan_levels, [&](auto kbc) {
    constexpr int KB = decltype(kbc)::value;
    batch_profile_variant(b.pm, [&](auto pmc) {
      constexpr int PM = decltype(pmc)::value;
      smoother_variant<T>(b.f_double, b.out_double, b.zero, b.fcopy, b.dots,
                          [&](auto tf, auto to, auto z, auto fcp, auto dt) {
                            using TF = typename decltype(tf)::type;
                            using TO = typename decltype(to)::type;
                            hipLaunchKernelGGL((kb_smooth_scan<KB, T, TF, TO, decltype(z)::value, decltype(fcp)::value,
                                                               decltype(dt)::value, PM>),
                                               grid, block, b.lds, s, b.segs, b.nseg, b.omega);
                          });
    });
  });
  return hipGetLastError();
}

hipError_t launch_batched(const BatchLaunch& b, hipStream_t s) {
  if (b.pm < 0 || b.pm > 2) return hipErrorInvalidValue;
  switch (b.kind) {
    case kOpSmooth:
      if (b.prec == 8) return batched_smooth_t<double>(b, s);
      return batched_smooth_t<float>(b, s);
    case kOpRestrict:
      batch_profile_variant(b.pm, [&](auto pmc) {
        constexpr int PM = decltype(pmc)::value;
        chunk_variant(b.chunk, [&](auto chc) {
          constexpr int CH = decltype(chc)::value;
          if (b.prec == 8)
            hipLaunchKernelGGL((kb_residual_restrict<double, CH, PM>), dim3(b.grid), dim3(256), 0, s, b.segs, b.nseg);
          else
            hipLaunchKernelGGL((kb_residual_restrict<float, CH, PM>), dim3(b.grid), dim3(256), 0, s, b.segs, b.nseg);
        });
      });
      break;
    case kOpProlong:
      if (b.prec == 8)
        hipLaunchKernelGGL(kb_prolong_add<double>, dim3(b.grid), dim3(256), 0, s, b.segs, b.nseg);
      else
        hipLaunchKernelGGL(kb_prolong_add<float>, dim3(b.grid), dim3(256), 0, s, b.segs, b.nseg);
      break;
    case kOpSpmv:
      batch_profile_variant(b.pm, [&](auto pmc) {
        constexpr int PM = decltype(pmc)::value;
        chunk_variant(b.chunk, [&](auto chc) {
          constexpr int CH = decltype(chc)::value;
          hipLaunchKernelGGL((kb_spmv64<CH, PM>), dim3(b.grid), dim3(256), 0, s, b.segs, b.nseg);
        });
      });
      break;
    case kOpSpmvPRing:
      // (the plan only forms it for chunks with an instance)
      if (b.chunk == 0) return hipErrorInvalidValue;
      batch_profile_variant(b.pm, [&](auto pmc) {
        constexpr int PM = decltype(pmc)::value;
        chunk_variant(b.chunk, [&](auto chc) {
          constexpr int CH = decltype(chc)::value;
          if constexpr (CH > 0) {
            if (b.f_double)
              hipLaunchKernelGGL((kb_spmv_pring<CH, double, PM>), dim3(b.grid), dim3(256), 0, s, b.segs, b.nseg);
            else
              hipLaunchKernelGGL((kb_spmv_pring<CH, float, PM>), dim3(b.grid), dim3(256), 0, s, b.segs, b.nseg);
          }
        });
      });
      break;
    case kOpRupdate:
      hipLaunchKernelGGL(kb_rupdate, dim3(b.grid), dim3(256), 0, s, b.segs, b.nseg);
      break;
    case kOpPupdate:
      if (b.f_double)
        hipLaunchKernelGGL(kb_pupdate<double>, dim3(b.grid), dim3(256), 0, s, b.segs, b.nseg);
      else
        hipLaunchKernelGGL(kb_pupdate<float>, dim3(b.grid), dim3(256), 0, s, b.segs, b.nseg);
      break;
    case kOpUpdate:
      hipLaunchKernelGGL(kb_fcg_update, dim3(b.grid), dim3(256), 0, s, b.segs, b.nseg);
      break;
    case kOpFinalize:
      hipLaunchKernelGGL(kb_finalize, dim3(b.nseg), dim3(kFinThreads), 0, s, b.segs, b.nseg);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tpmg
