// Device side of the per-column MLP (learned initial guess): launchers of
// the gfx950 kernels. Matrices are row-major; bf16 is the 16-bit brain
// float; every launcher enqueues on `s` and returns hipGetLastError() or
// hipErrorInvalidValue for a shape it does not support.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "device.h"

namespace tpmg {

using bf16 = __bf16;

// C[m][n] = sum_k A(m, k) B(n, k) for m < M, n < N, k < K, with
// A(m, k) = ta ? A[k * lda + m] : A[m * lda + k] and likewise B. Products of
// bf16 on the matrix cores, FP32 sums. Requirements (checked): lda, ldb
// multiples of 8, 16-byte aligned A and B; not transposed: K a multiple of
// 8, lda >= K (ldb >= K); transposed: lda >= M rounded up to 8 (ldb >= N),
// the entries between M and that bound are read but reach only discarded
// outputs.
enum GemmEpilogue {
  kEpiBiasReluBf16 = 0,  // out_bf16[m ldc + n] = bf16(max(C + bias[n], 0))
  kEpiBiasF32 = 1,       // out_f32[m ldc + n] = C + bias[n]
  kEpiMaskBf16 = 2,      // out_bf16[m ldc + n] = (ReLU mask bit of (m, n), mask_bits) ? bf16(C) : 0
  kEpiPartialF32 = 3,    // out_f32[z S + m N + n] = C over the z-th slice of ksplit values of k (S: pstride)
  kEpiInferTiled = 4,    // out_f64 tiled (column m, level n) = (C + bias[n]) sd[n] + mu[n]
};

struct GemmArgs {
  const bf16* A = nullptr;
  const bf16* B = nullptr;
  int lda = 0, ldb = 0;
  int M = 0, N = 0, K = 0;
  int ksplit = 0;            // kEpiPartialF32: k values per slice (multiple of 32); else K
  // kEpiPartialF32 with transposed operands: also the sums over k of each row
  // of A (a layer's bias gradient beside its weight gradient); the partials
  // of slice z are then out_f32[z S + m N + n] and, for the row sums,
  // out_f32[z S + M N + m], S the partial stride
  bool row_sums = false;
  // kEpiPartialF32: the distance between the partials of consecutive K slices
  // (0: M N, + M with row_sums)
  size_t pstride = 0;
  bool ta = false, tb = false;
  int epi = kEpiBiasF32;
  const float* bias = nullptr;
  // ReLU masks as bits: kEpiBiasReluBf16 (optional) writes, for every thread
  // of every workgroup, one 64-bit word whose bit 32 i + 16 j + r is set when
  // its output (i, j, r) is > 0 after the bf16 rounding; kEpiMaskBf16 reads the
  // words a kEpiBiasReluBf16 product of the same M and N wrote (same tiles,
  // so the same output positions per thread) as its mask
  uint64_t* mask_bits = nullptr;
  bf16* out_bf16 = nullptr;
  float* out_f32 = nullptr;
  int ldc = 0;
  double* out_f64 = nullptr;  // kEpiInferTiled: tiled FP64 vector with nz = N levels
  const float* mu = nullptr;
  const float* sd = nullptr;
};
hipError_t launch_gemm(const GemmArgs& g, hipStream_t s);

// Inference in one kernel: the features of launch_mlp_features_bf16 formed
// from the tiled right-hand side f, the column means (launch_mlp_col_means)
// and the neighbour table [3][npad], then the three products of the
// kEpiBiasReluBf16, kEpiBiasReluBf16, kEpiInferTiled GEMMs (same bits):
// w1 [256][kp], w2 [256][256], w3 [nz][256] bf16, biases and scalings FP32,
// out the tiled FP64 guess (nz levels; n columns, the tile padding left
// untouched). Supported: hidden 256, nz a multiple of 32 up to 128, kp a
// multiple of 8 up to 160 (mlp_infer_fits).
struct InferArgs {
  int kp = 0, n = 0, nz = 0;
  const double* f = nullptr;
  const double* means = nullptr;
  const int32_t* nbr = nullptr;
  int npad = 0;
  const float *mu_x = nullptr, *sd_x = nullptr;
  const bf16 *w1 = nullptr, *w2 = nullptr, *w3 = nullptr;
  const float *b1 = nullptr, *b2 = nullptr, *b3 = nullptr, *mu = nullptr, *sd = nullptr;
  double* out = nullptr;
};
bool mlp_infer_fits(int hidden, int nz, int kp);
// means[T] = mean over the levels of column T of the tiled vector f (FP64).
hipError_t launch_mlp_col_means(const FineGrid& g, const double* f, double* means, hipStream_t s);
hipError_t launch_mlp_infer(const InferArgs& a, hipStream_t s);

// x[T][j]: the column's right-hand side (j < nz) and the vertical means of
// neighbours 0..2 (j = nz + i), from a tiled FP64 vector; means: scratch of
// n doubles (the column means). The _bf16 form writes the standardised,
// bf16-rounded rows xb[T][kp] instead (zeros beyond nz + 3).
hipError_t launch_mlp_features(const FineGrid& g, const double* f, double* means, float* x, hipStream_t s);
hipError_t launch_mlp_features_bf16(const FineGrid& g, const double* f, double* means, const float* mu_x,
                                    const float* sd_x, int kp, bf16* xb, hipStream_t s);
// out = a - b over a tiled vector of len values (the increment of a right-hand
// side or a solution between two steps of a sequence).
hipError_t launch_vec_sub(const double* a, const double* b, double* out, size_t len, hipStream_t s);
// out = base + d on the real columns of the tiled vector, base on the padding.
hipError_t launch_add_guess(const FineGrid& g, const double* base, const double* d, double* out, hipStream_t s);
// y[T][k] = u(T, k), FP32.
hipError_t launch_mlp_targets(const FineGrid& g, const double* u, float* y, hipStream_t s);

// Gathers rows (rows == nullptr: rows 0..n-1), standardises and rounds:
// xb[r][j] = bf16((x[row][j] - mu_x[j]) / sd_x[j]) for j < n_in, 0 up to kp;
// yt (optional) [r][k] = (y[row][k] - mu_y[k]) / sd_y[k]. An index outside
// [0, rows_total) is not read: its row becomes zeros and *bad_row is set.
hipError_t launch_mlp_prep(const float* x, const float* y, const int32_t* rows, size_t rows_total, int* bad_row,
                           int n, int n_in, int kp, int nz, const float* mu_x, const float* sd_x, const float* mu_y,
                           const float* sd_y, bf16* xb, float* yt, hipStream_t s);

// d = y - yt; dy = bf16(scale d); loss_partials[b] = sum of d^2 per block
// (FP64), then (loss not NULL) loss[0] = sum over blocks / (n nz), FP32.
hipError_t launch_mlp_mse(const float* y, const float* yt, int n, int nz, bf16* dy, double* partials,
                          float* loss, hipStream_t s);
int mlp_mse_blocks(int n, int nz);

// out[i] = sum_p part[p * len + i] (fixed order), FP32.
hipError_t launch_sum_parts(const float* part, int nparts, size_t len, float* out, hipStream_t s);

// Adam (t: the step count from 1) on the n packed parameters, also writing
// the bf16 copies of the weights the products read (as
// launch_refresh_weights, whose zero padding of w1b it keeps)
hipError_t launch_adam_copies(float* p, const float* g, float* m, float* v, size_t n, float lr, int t, int n_in,
                              int hidden, int nz, int kp, bf16* w1b, bf16* w2b, bf16* w3b, bf16* w2t, bf16* w3t,
                              hipStream_t s);

// bf16 copies of the weights: w1b [hidden][kp] (zero beyond n_in), w2b, w3b,
// and the transposes w2t [hidden][hidden], w3t [hidden][nz].
hipError_t launch_refresh_weights(const float* params, int n_in, int hidden, int nz, int kp, bf16* w1b, bf16* w2b,
                                  bf16* w3b, bf16* w2t, bf16* w3t, hipStream_t s);

// Per-column sums over rows of a [rows][cols] FP32 matrix, in FP64:
// partials [chunks][cols] of a (mean == nullptr) or of (a - mean)^2, chunk c
// covering rows [c chunk_rows, (c + 1) chunk_rows).
constexpr int kMomentChunksMax = 2048;
size_t moment_chunk_rows(size_t rows);
hipError_t launch_moment_partials(const float* a, size_t rows, int cols, const double* mean, double* part,
                                  hipStream_t s);

}  // namespace tpmg
