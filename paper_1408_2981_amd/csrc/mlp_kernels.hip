// gfx950 kernels of the per-column MLP (learned initial guess): a bf16
// matrix-core GEMM with fused epilogues, and the small elementwise and
// reduction kernels around it (features, standardisation, loss, bias
// gradients, Adam, weight copies, scaling moments).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "mlp_device.h"

namespace tpmg {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kTileCols = 64;

__device__ __forceinline__ size_t tiled_index(int col, int k, int nz) {
  return static_cast<size_t>(col >> 6) * 64 * nz + static_cast<size_t>(k) * 64 + (col & 63);
}

// ---------------------------------------------------------------------------
// GEMM: one workgroup of 4 waves computes a (64 WM) x (64 WN) tile of C; each
// wave a 64 x 64 block as 2 x 2 matrix-core products of 32 x 32 x 16 (bf16
// operands, FP32 accumulators). K advances through LDS in slices of BK
// (rows padded by 8 bf16 so the 16-byte operand reads spread over the
// banks); with K-contiguous operands the next slice's loads are in flight
// while the current one computes. Within a slice the 16-wide K chunks are
// taken in ascending order, so the accumulation order is that of K itself,
// whatever BK. Split-K partitions are multiples of kBK.
// Operand layout of the 32 x 32 x 16 product: lane l supplies row l % 32 of A
// (column l % 32 of B) at k = 8 (l / 32) .. 8 (l / 32) + 7; accumulator r of
// lane l holds row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.
// ---------------------------------------------------------------------------
constexpr int kBK = 32;
constexpr int kGemmBK = 64;   // K slice of the GEMM kernel

// LDS column of element (row, k) of a staged slice. A transposed operand is
// staged by scattering each lane's 8 consecutive rows (one k) into their
// rows, so the lanes of one store hit rows 8 apart, all in the same two of
// the 64 banks whatever the row padding; its 8-wide K groups are therefore
// placed at group XOR (row / 8) mod 8, which spreads those stores over the
// banks and keeps every group contiguous for the 16-byte operand reads.
template <bool T>
__device__ __forceinline__ int lds_col(int row, int k) {
  return T ? ((((k >> 3) ^ (row >> 3)) & 7) << 3 | (k & ~63) | (k & 7)) : k;
}

// Stages rows [r0, r0 + ROWS) x k [k0, k0 + BK) of a K-contiguous (T false)
// or R-contiguous (T true) operand into LDS as [row][lds_col(row, k)];
// entries outside r < R, k < kend are zero.
template <int ROWS, bool T, int BK>
__device__ __forceinline__ void stage(const bf16* __restrict__ src, int ld, int r0, int R, int k0, int kend,
                                      bf16 (*dst)[BK + 8]) {
  constexpr int kChunks = ROWS * BK / 8;   // 16-byte chunks of 8 bf16
  constexpr int kPerRow = BK / 8;
#pragma unroll
  for (int c = threadIdx.x; c < kChunks; c += 256) {
    if (!T) {
      const int row = c / kPerRow, kc = (c % kPerRow) * 8;
      const int r = r0 + row, k = k0 + kc;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (r < R && k < kend) v = *reinterpret_cast<const uint4*>(src + static_cast<size_t>(r) * ld + k);
      *reinterpret_cast<uint4*>(&dst[row][kc]) = v;
    } else {
      constexpr int kPerK = ROWS / 8;
      const int kk = c / kPerK, rc = (c - kk * kPerK) * 8;
      const int k = k0 + kk, r = r0 + rc;
      union {
        uint4 u;
        bf16 h[8];
      } v;
      v.u = make_uint4(0u, 0u, 0u, 0u);
      if (k < kend && r < R) v.u = *reinterpret_cast<const uint4*>(src + static_cast<size_t>(k) * ld + r);
#pragma unroll
      for (int i = 0; i < 8; ++i) dst[rc + i][lds_col<true>(rc + i, kk)] = v.h[i];
    }
  }
}

// The staging of a K-contiguous operand split in two, so that the next
// slice's loads are in flight while the current slice computes: fetch takes
// this thread's 16-byte chunks of rows [0, ROWS) x k [k0, k0 + BK) into
// registers (zero outside r < R, k < kend), put stores them as [row][k].
template <int ROWS, int BK>
struct StageRegs {
  static constexpr int kChunks = ROWS * BK / 8;
  static constexpr int kPerRow = BK / 8;
  static constexpr int kPer = (kChunks + 255) / 256;
  uint4 v[kPer];
  __device__ __forceinline__ void fetch(const bf16* __restrict__ src, int ld, int R, int k0, int kend) {
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int c = threadIdx.x + 256 * i;
      const int row = c / kPerRow, kc = (c % kPerRow) * 8;
      v[i] = make_uint4(0u, 0u, 0u, 0u);
      if (c < kChunks && row < R && k0 + kc < kend)
        v[i] = *reinterpret_cast<const uint4*>(src + static_cast<size_t>(row) * ld + k0 + kc);
    }
  }
  __device__ __forceinline__ void put(bf16 (*dst)[BK + 8]) const {
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int c = threadIdx.x + 256 * i;
      if (c < kChunks) *reinterpret_cast<uint4*>(&dst[c / kPerRow][(c % kPerRow) * 8]) = v[i];
    }
  }
};

template <int WM, int WN, bool TR, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  constexpr int BM = 64 * WM, BN = 64 * WN, BK = kGemmBK;
  __shared__ __align__(16) bf16 As[BM][BK + 8];
  __shared__ __align__(16) bf16 Bs[BN][BK + 8];
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  const int kbeg = blockIdx.z * g.ksplit;
  const int kend = min(g.K, kbeg + g.ksplit);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = (wave / WN) * 64, wn = (wave % WN) * 64;
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

  const int lr = lane & 31, lk = 8 * (lane >> 5);
  // output element (i, j, r) of this lane
  auto out_row = [&](int i, int r) { return m0 + wm + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); };
  auto out_col = [&](int j) { return n0 + wn + 32 * j + lr; };
  // this thread's word of ReLU mask bits (loaded before the products)
  const size_t mword = (static_cast<size_t>(blockIdx.y) * gridDim.x + blockIdx.x) * 256 + threadIdx.x;
  const uint64_t mk = EPI == kEpiMaskBf16 ? g.mask_bits[mword] : 0;
  uint64_t mb = 0;
  // this lane's bias (and de-standardisation) of its two output columns, in
  // registers before the products: read in the epilogue, each load would
  // wait behind the output stores the compiler cannot prove apart from it
  constexpr bool kBias = EPI == kEpiBiasReluBf16 || EPI == kEpiBiasF32 || EPI == kEpiInferTiled;
  float bj[2] = {0.0f, 0.0f}, sj[2] = {0.0f, 0.0f}, uj[2] = {0.0f, 0.0f};
  if (kBias)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = out_col(j);
      if (n < g.N) {
        bj[j] = g.bias[n];
        if (EPI == kEpiInferTiled) {
          sj[j] = g.sd[n];
          uj[j] = g.mu[n];
        }
      }
    }
  // row sums of A (bias gradient): the first column tile's threads, one row each
  const bool rsum = EPI == kEpiPartialF32 && g.row_sums && blockIdx.y == 0 && threadIdx.x < BM;
  float rs = 0.0f;
  StageRegs<BM, BK> ra;
  StageRegs<BN, BK> rb;
  const bf16* a0 = g.A + static_cast<size_t>(m0) * g.lda;
  const bf16* b0 = g.B + static_cast<size_t>(n0) * g.ldb;
  if (!TR && kbeg < kend) {
    ra.fetch(a0, g.lda, g.M - m0, kbeg, kend);
    rb.fetch(b0, g.ldb, g.N - n0, kbeg, kend);
  }
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    if (TR) {
      stage<BM, TR, BK>(g.A, g.lda, m0, g.M, k0, kend, As);
      stage<BN, TR, BK>(g.B, g.ldb, n0, g.N, k0, kend, Bs);
    } else {
      ra.put(As);
      rb.put(Bs);
    }
    __syncthreads();
    if (!TR && k0 + BK < kend) {
      ra.fetch(a0, g.lda, g.M - m0, k0 + BK, kend);
      rb.fetch(b0, g.ldb, g.N - n0, k0 + BK, kend);
    }
    if (rsum)
#pragma unroll
      for (int kk = 0; kk < BK; kk += 8) {
        const bf16x8 v = *reinterpret_cast<const bf16x8*>(&As[threadIdx.x][lds_col<TR>(threadIdx.x, kk)]);
#pragma unroll
        for (int q = 0; q < 8; ++q) rs += static_cast<float>(v[q]);
      }
#pragma unroll
    for (int ks = 0; ks < BK; ks += 16) {
      bf16x8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int row = wm + 32 * i + lr;
        a[i] = *reinterpret_cast<const bf16x8*>(&As[row][lds_col<TR>(row, ks + lk)]);
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int row = wn + 32 * j + lr;
        b[j] = *reinterpret_cast<const bf16x8*>(&Bs[row][lds_col<TR>(row, ks + lk)]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }

  const size_t pstride = g.pstride ? g.pstride : static_cast<size_t>(g.M) * g.N + (g.row_sums ? g.M : 0);
  if (rsum && m0 + static_cast<int>(threadIdx.x) < g.M)
    g.out_f32[static_cast<size_t>(blockIdx.z) * pstride + static_cast<size_t>(g.M) * g.N + m0 + threadIdx.x] = rs;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = out_row(i, r), n = out_col(j);
        if (m >= g.M || n >= g.N) continue;
        const float c = acc[i][j][r];
        const size_t o = static_cast<size_t>(m) * g.ldc + n;
        const int bit = 32 * i + 16 * j + r;
        if (EPI == kEpiBiasReluBf16) {
          const bf16 h = static_cast<bf16>(fmaxf(c + bj[j], 0.0f));
          g.out_bf16[o] = h;
          if (static_cast<float>(h) > 0.0f) mb |= uint64_t(1) << bit;
        } else if (EPI == kEpiBiasF32) {
          g.out_f32[o] = c + bj[j];
        } else if (EPI == kEpiMaskBf16) {
          g.out_bf16[o] = ((mk >> bit) & 1) ? static_cast<bf16>(c) : static_cast<bf16>(0.0f);
        } else if (EPI == kEpiPartialF32) {
          g.out_f32[static_cast<size_t>(blockIdx.z) * pstride + static_cast<size_t>(m) * g.N + n] = c;
        } else {
          g.out_f64[tiled_index(m, n, g.N)] = static_cast<double>((c + bj[j]) * sj[j] + uj[j]);
        }
      }
  if (EPI == kEpiBiasReluBf16 && g.mask_bits) g.mask_bits[mword] = mb;
}

// ---------------------------------------------------------------------------
// Inference, the whole network in one kernel: a block of 4 waves takes 64
// rows (one tile of columns of the solver's grid) from the tiled right-hand
// side through the features and the three layers, with the activations kept
// in LDS, so that only the right-hand side is read and only the guess is
// written. Each wave owns its output units, so it reads its weight
// fragments straight from memory (the 200 KB of weights stay in L2), a few
// 16-wide K slices ahead of the matrix cores, without staging or barriers
// inside a layer. Each layer is the GEMM above at the same operand rounding,
// K order and epilogue expression, so the result is the bits of the three
// separate products. Hidden width 256; nz a multiple of 32 up to 128, the
// padded feature width kp a multiple of 32 with nz + 3 <= kp <= nz + 32.
// ---------------------------------------------------------------------------
constexpr int kInferRows = 64;
constexpr int kInferHidden = 256;
constexpr int kInferAhead = 4;   // K slices of weight fragments in flight per wave
constexpr int kHLd = kInferHidden + 8;
template <int NZT>
constexpr int infer_xld() {
  return 32 * NZT + 40;
}
template <int NZT>
constexpr size_t infer_lds() {
  // features + hidden activations; the FP64 output staging reuses them
  const size_t act = static_cast<size_t>(kInferRows) * infer_xld<NZT>() * 2 + static_cast<size_t>(kInferRows) * kHLd * 2;
  const size_t out = static_cast<size_t>(32 * NZT) * kInferRows * 8;
  return act > out ? act : out;
}

// the B fragment of one 32 x 32 x 16 product: row n of a K-contiguous
// weight matrix, k .. k + 7 of this lane's half of the slice
__device__ __forceinline__ bf16x8 weight_fragment(const bf16* __restrict__ w, int ld, int n, int k) {
  return *reinterpret_cast<const bf16x8*>(w + static_cast<size_t>(n) * ld + k);
}

template <int NZT>
__global__ __launch_bounds__(256) void k_mlp_infer(InferArgs a) {
  constexpr int NZ = 32 * NZT;
  constexpr int XLd = infer_xld<NZT>();
  __shared__ __align__(16) unsigned char sm[infer_lds<NZT>()];
  bf16 (*Xs)[XLd] = reinterpret_cast<bf16 (*)[XLd]>(sm);
  bf16 (*Hs)[kHLd] = reinterpret_cast<bf16 (*)[kHLd]>(sm + static_cast<size_t>(kInferRows) * XLd * 2);
  const int m0 = blockIdx.x * kInferRows;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 31, lk = 8 * (lane >> 5);

  {
    // the features of the block's tile straight from the tiled right-hand
    // side (one coalesced row per level) and the neighbours' column means,
    // standardised and rounded as the features kernel does; zero beyond n.
    // Every load of the tile is issued before the first is used.
    const int cnt = min(kInferRows, a.n - m0);
    const size_t base = static_cast<size_t>(blockIdx.x) * kInferRows * NZ;
    constexpr int kPer = kInferRows * NZ / 256;
    double fv[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) fv[q] = a.f[base + threadIdx.x + 256 * q];
    double mean = 0.0;
    const int jm = threadIdx.x >> 6, cm = threadIdx.x & 63;
    if (jm < 3 && cm < cnt) mean = a.means[a.nbr[static_cast<size_t>(jm) * a.npad + m0 + cm]];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int i = threadIdx.x + 256 * q;
      const int k = i >> 6, c = i & 63;
      const float val = (static_cast<float>(fv[q]) - a.mu_x[k]) / a.sd_x[k];
      Xs[c][k] = c < cnt ? static_cast<bf16>(val) : static_cast<bf16>(0.0f);
    }
    if (jm < 3) {
      float val = 0.0f;
      if (cm < cnt) val = (static_cast<float>(mean) - a.mu_x[NZ + jm]) / a.sd_x[NZ + jm];
      Xs[cm][NZ + jm] = static_cast<bf16>(val);
    }
    // padding features
    const int pad = a.kp - NZ - 3;
    for (int i = threadIdx.x; i < kInferRows * pad; i += 256) {
      const int c = i / pad, j = 3 + (i - c * pad);
      Xs[c][NZ + j] = static_cast<bf16>(0.0f);
    }
  }
  __syncthreads();

  // layers 1 and 2: wave w owns hidden units [64 w, 64 w + 64) of all 64
  // rows; its fragments of slice s are rows 64 w + 32 j + lr, k 16 s + lk
  f32x16 acc[2][2];
  auto hidden_layer = [&](const bf16* __restrict__ w, int K, bool from_x) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;
    const int ns = K / 16;
    bf16x8 bq[kInferAhead][2];
#pragma unroll
    for (int d = 0; d < kInferAhead; ++d)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        if (d < ns) bq[d][j] = weight_fragment(w, K, 64 * wave + 32 * j + lr, 16 * d + lk);
    for (int s0 = 0; s0 < ns; s0 += kInferAhead) {
#pragma unroll
      for (int d = 0; d < kInferAhead; ++d) {
        const int sl = s0 + d;
        if (sl < ns) {
          const int k = 16 * sl + lk;
          bf16x8 av[2], bv[2];
#pragma unroll
          for (int i = 0; i < 2; ++i)
            av[i] = from_x ? *reinterpret_cast<const bf16x8*>(&Xs[32 * i + lr][k])
                           : *reinterpret_cast<const bf16x8*>(&Hs[32 * i + lr][k]);
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            bv[j] = bq[d][j];
            if (sl + kInferAhead < ns) bq[d][j] = weight_fragment(w, K, 64 * wave + 32 * j + lr, k + 16 * kInferAhead);
          }
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
      }
    }
  };
  auto hidden_out = [&](const float* __restrict__ bias) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int m = 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          const int nn = 64 * wave + 32 * j + lr;
          Hs[m][nn] = static_cast<bf16>(fmaxf(acc[i][j][r] + bias[nn], 0.0f));
        }
  };
  hidden_layer(a.w1, a.kp, true);
  hidden_out(a.b1);   // (layer 1 reads Xs only)
  __syncthreads();
  hidden_layer(a.w2, kInferHidden, false);
  __syncthreads();   // every wave is past its last read of Hs
  hidden_out(a.b2);
  __syncthreads();

  // layer 3: 2 x NZT products of 32 x 32, product t = wave + 4 q on rows
  // 32 (t % 2), levels 32 (t / 2); fragments rows 32 (t / 2) + lr of w3
  constexpr int kOwn = (2 * NZT + 3) / 4;
  constexpr int ns3 = kInferHidden / 16;
  f32x16 acc3[kOwn];
  bf16x8 bq3[kInferAhead][kOwn];
#pragma unroll
  for (int q = 0; q < kOwn; ++q) {
#pragma unroll
    for (int r = 0; r < 16; ++r) acc3[q][r] = 0.0f;
    const int t = wave + 4 * q;
#pragma unroll
    for (int d = 0; d < kInferAhead; ++d)
      if (t < 2 * NZT) bq3[d][q] = weight_fragment(a.w3, kInferHidden, 32 * (t >> 1) + lr, 16 * d + lk);
  }
  for (int s0 = 0; s0 < ns3; s0 += kInferAhead) {
#pragma unroll
    for (int d = 0; d < kInferAhead; ++d) {
      const int sl = s0 + d;
      const int k = 16 * sl + lk;
#pragma unroll
      for (int q = 0; q < kOwn; ++q) {
        const int t = wave + 4 * q;
        if (t < 2 * NZT) {
          const bf16x8 av = *reinterpret_cast<const bf16x8*>(&Hs[32 * (t & 1) + lr][k]);
          const bf16x8 bv = bq3[d][q];
          if (sl + kInferAhead < ns3)
            bq3[d][q] = weight_fragment(a.w3, kInferHidden, 32 * (t >> 1) + lr, k + 16 * kInferAhead);
          acc3[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc3[q], 0, 0, 0);
        }
      }
    }
  }
  __syncthreads();   // every wave is past its last read of Hs (the staging below overlays it)

  // de-standardise into [level][row] FP64 staging over the whole LDS, then
  // one coalesced 64-value row of the tiled guess per level
  double (*Os)[kInferRows] = reinterpret_cast<double (*)[kInferRows]>(sm);
#pragma unroll
  for (int q = 0; q < kOwn; ++q) {
    const int t = wave + 4 * q;
    if (t < 2 * NZT) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = 32 * (t & 1) + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int lev = 32 * (t >> 1) + lr;
        Os[lev][m] = static_cast<double>((acc3[q][r] + a.b3[lev]) * a.sd[lev] + a.mu[lev]);
      }
    }
  }
  __syncthreads();
  double* __restrict__ out = a.out + static_cast<size_t>(blockIdx.x) * kInferRows * NZ;
  for (int i = threadIdx.x; i < NZ * kInferRows; i += 256) {
    const int lev = i / kInferRows, m = i - lev * kInferRows;
    if (m0 + m < a.n) out[i] = Os[lev][m];
  }
}

// ---------------------------------------------------------------------------
// features, targets, standardisation
// ---------------------------------------------------------------------------

// mean over the levels of every real column of a tiled FP64 vector (FP64):
// one block per tile, four groups of levels per column summed apart (each
// load a coalesced 64-wide row) and combined in a fixed order
__global__ __launch_bounds__(256) void k_col_means(FineGrid g, const double* __restrict__ v, double* __restrict__ means) {
  __shared__ double part[4][kTileCols];
  const int c = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int t = blockIdx.x * kTileCols + c;
  const size_t base = static_cast<size_t>(blockIdx.x) * kTileCols * g.nz + c;
  double s = 0.0;
  for (int k = grp; k < g.nz; k += 4) s += v[base + static_cast<size_t>(k) * kTileCols];
  part[grp][c] = s;
  __syncthreads();
  if (grp == 0 && t < g.n) means[t] = ((part[0][c] + part[1][c]) + (part[2][c] + part[3][c])) / g.nz;
}

// out = a - b entry by entry over a tiled vector of len values
__global__ __launch_bounds__(256) void k_vec_sub(const double* __restrict__ a, const double* __restrict__ b,
                                                 double* __restrict__ out, size_t len) {
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < len;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    out[i] = a[i] - b[i];
}

// out = base + d on the real columns of a tiled vector, out = base on the
// tile padding (d is not read there)
__global__ __launch_bounds__(256) void k_add_guess(FineGrid g, const double* __restrict__ base,
                                                   const double* __restrict__ d, double* __restrict__ out) {
  const size_t len = static_cast<size_t>(g.npad) * g.nz;
  const size_t per_tile = static_cast<size_t>(kTileCols) * g.nz;
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < len;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const int col = static_cast<int>(i / per_tile) * kTileCols + static_cast<int>(i & (kTileCols - 1));
    out[i] = col < g.n ? base[i] + d[i] : base[i];
  }
}

// One tile of 64 columns per block: the tile's values (level-major, one
// coalesced row of 64 per level) are staged in LDS column-major with an odd
// stride, completed by the neighbour means, and written out as contiguous
// rows. MODE 0: raw features x[T][nz + 3]; MODE 1: standardised bf16 features
// xb[T][kp] (zeros beyond nz + 3); MODE 2: values y[T][nz].
template <int MODE>
__global__ __launch_bounds__(256) void k_columns_to_rows(FineGrid g, const double* __restrict__ v,
                                                         const double* __restrict__ means,
                                                         const float* __restrict__ mu, const float* __restrict__ sd,
                                                         int kp, void* __restrict__ out) {
  extern __shared__ float lds[];
  const int nz = g.nz;
  const int w = MODE == 2 ? nz : nz + 3;    // row length
  const int ws = MODE == 2 ? nz + 1 : nz + 3;   // LDS stride (odd: nz is a multiple of 8)
  const int tile = blockIdx.x;
  const size_t base = static_cast<size_t>(tile) * kTileCols * nz;
  for (int i = threadIdx.x; i < kTileCols * nz; i += blockDim.x) {
    const int k = i >> 6, c = i & 63;
    lds[c * ws + k] = static_cast<float>(v[base + i]);
  }
  const int cnt = min(kTileCols, g.n - tile * kTileCols);
  if (MODE != 2) {
    for (int i = threadIdx.x; i < kTileCols * 3; i += blockDim.x) {
      const int c = i / 3, j = i - 3 * c;
      const int t = tile * kTileCols + c;
      lds[c * ws + nz + j] = c < cnt ? static_cast<float>(means[g.nbr[static_cast<size_t>(j) * g.npad + t]]) : 0.0f;
    }
  }
  __syncthreads();
  if (MODE == 1) {
    bf16* xb = static_cast<bf16*>(out) + static_cast<size_t>(tile) * kTileCols * kp;
    for (int i = threadIdx.x; i < cnt * kp; i += blockDim.x) {
      const int c = i / kp, j = i - c * kp;
      const float val = j < w ? (lds[c * ws + j] - mu[j]) / sd[j] : 0.0f;
      xb[i] = static_cast<bf16>(val);
    }
  } else {
    float* o = static_cast<float*>(out) + static_cast<size_t>(tile) * kTileCols * w;
    for (int i = threadIdx.x; i < cnt * w; i += blockDim.x) {
      const int c = i / w, j = i - c * w;
      o[i] = lds[c * ws + j];
    }
  }
}

__global__ __launch_bounds__(256) void k_mlp_prep(const float* __restrict__ x, const float* __restrict__ y,
                                                  const int32_t* __restrict__ rows, size_t rows_total,
                                                  int* __restrict__ bad_row, int n, int nin, int kp, int nz,
                                                  const float* __restrict__ mu_x, const float* __restrict__ sd_x,
                                                  const float* __restrict__ mu_y, const float* __restrict__ sd_y,
                                                  bf16* __restrict__ xb, float* __restrict__ yt) {
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  const size_t first = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  // source row of batch row r, or -1 for an index outside [0, rows_total)
  auto source = [&](int r) -> long long {
    if (!rows) return r;
    const long long v = rows[r];
    if (v < 0 || static_cast<size_t>(v) >= rows_total) {
      *bad_row = 1;
      return -1;
    }
    return v;
  };
  const size_t tx = static_cast<size_t>(n) * kp;
  for (size_t i = first; i < tx; i += stride) {
    const int r = static_cast<int>(i / kp), j = static_cast<int>(i - static_cast<size_t>(r) * kp);
    const long long row = source(r);
    float v = 0.0f;
    if (j < nin && row >= 0) v = (x[static_cast<size_t>(row) * nin + j] - mu_x[j]) / sd_x[j];
    xb[i] = static_cast<bf16>(v);
  }
  if (!yt) return;
  const size_t ty = static_cast<size_t>(n) * nz;
  for (size_t i = first; i < ty; i += stride) {
    const int r = static_cast<int>(i / nz), k = static_cast<int>(i - static_cast<size_t>(r) * nz);
    const long long row = source(r);
    yt[i] = row >= 0 ? (y[static_cast<size_t>(row) * nz + k] - mu_y[k]) / sd_y[k] : 0.0f;
  }
}

// ---------------------------------------------------------------------------
// loss, bias gradients, partial sums
// ---------------------------------------------------------------------------

__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_mlp_mse(const float* __restrict__ y, const float* __restrict__ yt, size_t total,
                                                 float scale, bf16* __restrict__ dy, double* __restrict__ partials) {
  double s = 0.0;
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const float d = y[i] - yt[i];
    dy[i] = static_cast<bf16>(scale * d);
    s += static_cast<double>(d) * d;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_mlp_loss(const double* __restrict__ partials, int nblocks, double inv_total,
                                                  float* __restrict__ loss) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += partials[b];
  s = block_sum(s);
  if (threadIdx.x == 0) loss[0] = static_cast<float>(s * inv_total);
}

// out[i] = sum over p of part[p][i]: 64 elements x 4 groups of parts per
// block, the groups combined in a fixed order
__global__ __launch_bounds__(256) void k_sum_parts(const float* __restrict__ part, int nparts, size_t len,
                                                   float* __restrict__ out) {
  __shared__ float red[4][64];
  const int e = threadIdx.x & 63, grp = threadIdx.x >> 6;
  for (size_t i0 = static_cast<size_t>(blockIdx.x) * 64; i0 < len; i0 += static_cast<size_t>(gridDim.x) * 64) {
    const size_t i = i0 + e;
    float s = 0.0f;
    if (i < len)
      for (int p = grp; p < nparts; p += 4) s += part[static_cast<size_t>(p) * len + i];
    red[grp][e] = s;
    __syncthreads();
    if (grp == 0 && i < len) out[i] = (red[0][e] + red[1][e]) + (red[2][e] + red[3][e]);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// optimiser and weight copies
// ---------------------------------------------------------------------------

// Adam on every parameter, and for the weights the bf16 copies the products
// read (as k_refresh_weights writes them; the zero padding of the first
// layer's copy beyond nin is left as k_refresh_weights wrote it)
__global__ __launch_bounds__(256) void k_adam_copies(float* __restrict__ p, const float* __restrict__ g,
                                                     float* __restrict__ m, float* __restrict__ v, size_t n, float lr,
                                                     float bc1, float bc2, int nin, int h, int nz, int kp,
                                                     bf16* __restrict__ w1b, bf16* __restrict__ w2b,
                                                     bf16* __restrict__ w3b, bf16* __restrict__ w2t,
                                                     bf16* __restrict__ w3t) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const size_t oW2 = static_cast<size_t>(h) * nin + h, oW3 = oW2 + static_cast<size_t>(h) * h + h;
  const size_t eW1 = static_cast<size_t>(h) * nin, eW2 = oW2 + static_cast<size_t>(h) * h,
               eW3 = oW3 + static_cast<size_t>(nz) * h;
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi * bc1) / (sqrtf(vi * bc2) + eps);
    p[i] = pi;
    const bf16 w = static_cast<bf16>(pi);
    if (i < eW1) {
      const size_t o = i / nin;
      w1b[o * kp + (i - o * nin)] = w;
    } else if (i >= oW2 && i < eW2) {
      const size_t q = i - oW2, r = q / h, c = q - r * h;
      w2b[q] = w;
      w2t[c * h + r] = w;
    } else if (i >= oW3 && i < eW3) {
      const size_t q = i - oW3, r = q / h, c = q - r * h;
      w3b[q] = w;
      w3t[c * nz + r] = w;
    }
  }
}

__global__ __launch_bounds__(256) void k_refresh_weights(const float* __restrict__ params, int nin, int h, int nz,
                                                         int kp, bf16* __restrict__ w1b, bf16* __restrict__ w2b,
                                                         bf16* __restrict__ w3b, bf16* __restrict__ w2t,
                                                         bf16* __restrict__ w3t) {
  const float* W1 = params;
  const float* W2 = W1 + static_cast<size_t>(h) * nin + h;
  const float* W3 = W2 + static_cast<size_t>(h) * h + h;
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  const size_t first = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  for (size_t i = first; i < static_cast<size_t>(h) * kp; i += stride) {
    const int o = static_cast<int>(i / kp), k = static_cast<int>(i - static_cast<size_t>(o) * kp);
    w1b[i] = static_cast<bf16>(k < nin ? W1[static_cast<size_t>(o) * nin + k] : 0.0f);
  }
  for (size_t i = first; i < static_cast<size_t>(h) * h; i += stride) {
    const int r = static_cast<int>(i / h), c = static_cast<int>(i - static_cast<size_t>(r) * h);
    const bf16 w = static_cast<bf16>(W2[i]);
    w2b[i] = w;
    w2t[static_cast<size_t>(c) * h + r] = w;
  }
  for (size_t i = first; i < static_cast<size_t>(nz) * h; i += stride) {
    const int r = static_cast<int>(i / h), c = static_cast<int>(i - static_cast<size_t>(r) * h);
    const bf16 w = static_cast<bf16>(W3[i]);
    w3b[i] = w;
    w3t[static_cast<size_t>(c) * nz + r] = w;
  }
}

__global__ __launch_bounds__(256) void k_moment_partials(const float* __restrict__ a, size_t rows, int cols,
                                                         size_t chunk_rows, const double* __restrict__ mean,
                                                         double* __restrict__ part) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  const size_t r0 = static_cast<size_t>(blockIdx.y) * chunk_rows;
  const size_t r1 = std::min(rows, r0 + chunk_rows);
  double s = 0.0;
  if (mean) {
    const double mu = mean[j];
    for (size_t r = r0; r < r1; ++r) {
      const double d = static_cast<double>(a[r * cols + j]) - mu;
      s += d * d;
    }
  } else {
    for (size_t r = r0; r < r1; ++r) s += static_cast<double>(a[r * cols + j]);
  }
  part[static_cast<size_t>(blockIdx.y) * cols + j] = s;
}

unsigned grid_of(size_t work, unsigned cap = 4096) {
  const size_t b = (work + 255) / 256;
  return static_cast<unsigned>(std::max<size_t>(1, std::min<size_t>(b, cap)));
}

template <int WM, int WN, bool TR>
hipError_t gemm_tile(const GemmArgs& g, hipStream_t s) {
  const dim3 grid((g.M + 64 * WM - 1) / (64 * WM), (g.N + 64 * WN - 1) / (64 * WN), (g.K + g.ksplit - 1) / g.ksplit);
  switch (g.epi) {
    case kEpiBiasReluBf16:
      hipLaunchKernelGGL((k_gemm<WM, WN, TR, kEpiBiasReluBf16>), grid, dim3(256), 0, s, g);
      break;
    case kEpiBiasF32:
      hipLaunchKernelGGL((k_gemm<WM, WN, TR, kEpiBiasF32>), grid, dim3(256), 0, s, g);
      break;
    case kEpiMaskBf16:
      hipLaunchKernelGGL((k_gemm<WM, WN, TR, kEpiMaskBf16>), grid, dim3(256), 0, s, g);
      break;
    case kEpiPartialF32:
      hipLaunchKernelGGL((k_gemm<WM, WN, TR, kEpiPartialF32>), grid, dim3(256), 0, s, g);
      break;
    case kEpiInferTiled:
      hipLaunchKernelGGL((k_gemm<WM, WN, TR, kEpiInferTiled>), grid, dim3(256), 0, s, g);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

bool mlp_infer_fits(int hidden, int nz, int kp) {
  return hidden == kInferHidden && nz % 32 == 0 && nz >= 32 && nz <= 128 && kp % 32 == 0 && kp >= nz + 3 &&
         kp <= nz + 32;
}

hipError_t launch_mlp_col_means(const FineGrid& g, const double* f, double* means, hipStream_t s) {
  hipLaunchKernelGGL(k_col_means, dim3(g.npad / kTileCols), dim3(256), 0, s, g, f, means);
  return hipGetLastError();
}

hipError_t launch_mlp_infer(const InferArgs& a, hipStream_t s) {
  if (!mlp_infer_fits(kInferHidden, a.nz, a.kp) || a.n <= 0) return hipErrorInvalidValue;
  if (!a.f || !a.means || !a.nbr || !a.mu_x || !a.sd_x || a.npad < a.n || a.kp < a.nz + 3) return hipErrorInvalidValue;
  const unsigned blocks = static_cast<unsigned>((a.n + kInferRows - 1) / kInferRows);
  switch (a.nz / 32) {
    case 1: hipLaunchKernelGGL(k_mlp_infer<1>, dim3(blocks), dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_mlp_infer<2>, dim3(blocks), dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_mlp_infer<3>, dim3(blocks), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL(k_mlp_infer<4>, dim3(blocks), dim3(256), 0, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs& g0, hipStream_t s) {
  GemmArgs g = g0;
  if (g.M <= 0 || g.N <= 0 || g.K <= 0 || !g.A || !g.B) return hipErrorInvalidValue;
  if (g.ta != g.tb) return hipErrorInvalidValue;   // both operands K-contiguous, or both transposed
  if ((!g.ta && g.K % 8) || g.lda % 8 || g.ldb % 8) return hipErrorInvalidValue;
  if ((reinterpret_cast<uintptr_t>(g.A) | reinterpret_cast<uintptr_t>(g.B)) % 16) return hipErrorInvalidValue;
  auto up8 = [](int v) { return (v + 7) / 8 * 8; };
  if (!g.ta && (g.lda < g.K || g.ldb < g.K)) return hipErrorInvalidValue;
  if (g.ta && (g.lda < up8(g.M) || g.ldb < up8(g.N))) return hipErrorInvalidValue;
  if (g.row_sums && (g.epi != kEpiPartialF32 || !g.ta)) return hipErrorInvalidValue;
  if (g.epi == kEpiPartialF32) {
    if (g.ksplit <= 0 || g.ksplit % kBK) return hipErrorInvalidValue;
  } else {
    g.ksplit = (g.K + kBK - 1) / kBK * kBK;
  }
  switch (g.epi) {
    case kEpiBiasReluBf16:
    case kEpiMaskBf16:
      if (!g.out_bf16 || g.ldc < g.N) return hipErrorInvalidValue;
      if (g.epi == kEpiBiasReluBf16 && !g.bias) return hipErrorInvalidValue;
      if (g.epi == kEpiMaskBf16 && !g.mask_bits) return hipErrorInvalidValue;
      break;
    case kEpiBiasF32:
      if (!g.out_f32 || !g.bias || g.ldc < g.N) return hipErrorInvalidValue;
      break;
    case kEpiPartialF32:
      if (!g.out_f32) return hipErrorInvalidValue;
      break;
    case kEpiInferTiled:
      if (!g.out_f64 || !g.bias || !g.mu || !g.sd) return hipErrorInvalidValue;
      break;
    default:
      return hipErrorInvalidValue;
  }
  const bool tr = g.ta;
  if (g.N <= 64) return tr ? gemm_tile<4, 1, true>(g, s) : gemm_tile<4, 1, false>(g, s);
  if (g.M <= 64) return tr ? gemm_tile<1, 4, true>(g, s) : gemm_tile<1, 4, false>(g, s);
  return tr ? gemm_tile<2, 2, true>(g, s) : gemm_tile<2, 2, false>(g, s);
}

static hipError_t columns_to_rows(int mode, const FineGrid& g, const double* v, const double* means,
                                  const float* mu, const float* sd, int kp, void* out, hipStream_t s) {
  const int ws = mode == 2 ? g.nz + 1 : g.nz + 3;
  const size_t lds = static_cast<size_t>(kTileCols) * ws * sizeof(float);
  const dim3 grid(g.npad / kTileCols);
  if (mode == 0)
    hipLaunchKernelGGL(k_columns_to_rows<0>, grid, dim3(256), lds, s, g, v, means, mu, sd, kp, out);
  else if (mode == 1)
    hipLaunchKernelGGL(k_columns_to_rows<1>, grid, dim3(256), lds, s, g, v, means, mu, sd, kp, out);
  else
    hipLaunchKernelGGL(k_columns_to_rows<2>, grid, dim3(256), lds, s, g, v, means, mu, sd, kp, out);
  return hipGetLastError();
}

hipError_t launch_mlp_features(const FineGrid& g, const double* f, double* means, float* x, hipStream_t s) {
  hipLaunchKernelGGL(k_col_means, dim3(g.npad / kTileCols), dim3(256), 0, s, g, f, means);
  return columns_to_rows(0, g, f, means, nullptr, nullptr, 0, x, s);
}

hipError_t launch_mlp_features_bf16(const FineGrid& g, const double* f, double* means, const float* mu_x,
                                    const float* sd_x, int kp, bf16* xb, hipStream_t s) {
  hipLaunchKernelGGL(k_col_means, dim3(g.npad / kTileCols), dim3(256), 0, s, g, f, means);
  return columns_to_rows(1, g, f, means, mu_x, sd_x, kp, xb, s);
}

static unsigned vec_blocks(size_t len) {
  const size_t b = (len + 255) / 256;
  return static_cast<unsigned>(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}

hipError_t launch_vec_sub(const double* a, const double* b, double* out, size_t len, hipStream_t s) {
  hipLaunchKernelGGL(k_vec_sub, dim3(vec_blocks(len)), dim3(256), 0, s, a, b, out, len);
  return hipGetLastError();
}

hipError_t launch_add_guess(const FineGrid& g, const double* base, const double* d, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_add_guess, dim3(vec_blocks(static_cast<size_t>(g.npad) * g.nz)), dim3(256), 0, s, g, base, d,
                     out);
  return hipGetLastError();
}

hipError_t launch_mlp_targets(const FineGrid& g, const double* u, float* y, hipStream_t s) {
  return columns_to_rows(2, g, u, nullptr, nullptr, nullptr, 0, y, s);
}

hipError_t launch_mlp_prep(const float* x, const float* y, const int32_t* rows, size_t rows_total, int* bad_row,
                           int n, int n_in, int kp, int nz, const float* mu_x, const float* sd_x, const float* mu_y,
                           const float* sd_y, bf16* xb, float* yt, hipStream_t s) {
  if (rows && !bad_row) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mlp_prep, dim3(grid_of(static_cast<size_t>(n) * kp)), dim3(256), 0, s, x, y, rows, rows_total,
                     bad_row, n, n_in, kp, nz, mu_x, sd_x, mu_y, sd_y, xb, yt);
  return hipGetLastError();
}

int mlp_mse_blocks(int n, int nz) { return static_cast<int>(grid_of(static_cast<size_t>(n) * nz, 1024)); }

hipError_t launch_mlp_mse(const float* y, const float* yt, int n, int nz, bf16* dy, double* partials, float* loss,
                          hipStream_t s) {
  const size_t total = static_cast<size_t>(n) * nz;
  const int nb = mlp_mse_blocks(n, nz);
  hipLaunchKernelGGL(k_mlp_mse, dim3(nb), dim3(256), 0, s, y, yt, total, 2.0f / static_cast<float>(total), dy,
                     partials);
  if (loss)
    hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, s, partials, nb, 1.0 / static_cast<double>(total), loss);
  return hipGetLastError();
}

hipError_t launch_sum_parts(const float* part, int nparts, size_t len, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_parts, dim3(static_cast<unsigned>(std::min<size_t>((len + 63) / 64, 4096))), dim3(256), 0, s,
                     part, nparts, len, out);
  return hipGetLastError();
}

hipError_t launch_adam_copies(float* p, const float* g, float* m, float* v, size_t n, float lr, int t, int n_in,
                              int hidden, int nz, int kp, bf16* w1b, bf16* w2b, bf16* w3b, bf16* w2t, bf16* w3t,
                              hipStream_t s) {
  const double bc1 = 1.0 / (1.0 - std::pow(0.9, t)), bc2 = 1.0 / (1.0 - std::pow(0.999, t));
  hipLaunchKernelGGL(k_adam_copies, dim3(grid_of(n)), dim3(256), 0, s, p, g, m, v, n, lr, static_cast<float>(bc1),
                     static_cast<float>(bc2), n_in, hidden, nz, kp, w1b, w2b, w3b, w2t, w3t);
  return hipGetLastError();
}

hipError_t launch_refresh_weights(const float* params, int n_in, int hidden, int nz, int kp, bf16* w1b, bf16* w2b,
                                  bf16* w3b, bf16* w2t, bf16* w3t, hipStream_t s) {
  const size_t work = std::max({static_cast<size_t>(hidden) * kp, static_cast<size_t>(hidden) * hidden,
                                static_cast<size_t>(nz) * hidden});
  hipLaunchKernelGGL(k_refresh_weights, dim3(grid_of(work)), dim3(256), 0, s, params, n_in, hidden, nz, kp, w1b, w2b,
                     w3b, w2t, w3t);
  return hipGetLastError();
}

size_t moment_chunk_rows(size_t rows) {
  const size_t chunks = std::min<size_t>(kMomentChunksMax, std::max<size_t>(1, (rows + 255) / 256));
  return (rows + chunks - 1) / chunks;
}

hipError_t launch_moment_partials(const float* a, size_t rows, int cols, const double* mean, double* part,
                                  hipStream_t s) {
  const size_t cr = moment_chunk_rows(rows);
  const unsigned chunks = static_cast<unsigned>((rows + cr - 1) / cr);
  hipLaunchKernelGGL(k_moment_partials, dim3((cols + 255) / 256, chunks), dim3(256), 0, s, a, rows, cols, cr, mean,
                     part);
  return hipGetLastError();
}

}  // namespace tpmg
