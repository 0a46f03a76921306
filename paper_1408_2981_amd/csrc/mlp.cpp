// C ABI of the per-column MLP (learned initial guess): workspace carving,
// argument checks, and the sequences of kernel launches for features,
// forward pass, gradients, Adam steps and inference.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <string>
#include <vector>

#include "../../include/tpmg_mlp.h"
#include "mlp_device.h"

namespace {

tpmg_status fail(tpmg_status s, const std::string& m) {
  tpmg_set_last_error(m.c_str());
  return s;
}

#define MLP_HIP(call)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return fail(TPMG_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* b) : base(static_cast<char*>(b)) {}
  template <typename T>
  T* take(size_t n) {
    off = (off + 255) / 256 * 256;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
};

constexpr int kSplitMax = 64;   // K slices of the weight-gradient products
constexpr uint32_t kFileMagic = 0x504c4d54u;   // file tag of saved networks

size_t param_count(int nz, int h) {
  const size_t nin = static_cast<size_t>(nz) + 3;
  return h * nin + h + static_cast<size_t>(h) * h + h + static_cast<size_t>(nz) * h + nz;
}

bool shape_ok(int nz, int h, int rows) {
  return nz >= 8 && nz <= 256 && nz % 8 == 0 && (h == 64 || h == 128 || h == 256 || h == 512) && rows >= 1 &&
         rows <= (1 << 22);
}

}  // namespace

using tpmg::bf16;

struct tpmg_mlp {
  int nz = 0, h = 0, nin = 0, kp = 0, max_rows = 0;
  hipStream_t stream = nullptr;
  int adam_t = 0;
  size_t np = 0;
  // FP32 master parameters (packed), gradients, Adam moments
  float *params = nullptr, *grads = nullptr, *am = nullptr, *av = nullptr;
  // bf16 weights and transposes
  bf16 *w1b = nullptr, *w2b = nullptr, *w3b = nullptr, *w2t = nullptr, *w3t = nullptr;
  // scaling (device FP32, host FP64)
  float *mu_x = nullptr, *sd_x = nullptr, *mu_y = nullptr, *sd_y = nullptr;
  std::vector<double> h_mu_x, h_sd_x, h_mu_y, h_sd_y;
  // activations of up to max_rows rows
  bf16 *xb = nullptr, *h1 = nullptr, *h2 = nullptr, *dy = nullptr, *dh2 = nullptr, *dh1 = nullptr;
  // ReLU masks of h1 and h2 as bits, written by the training forward pass
  uint64_t *bits1 = nullptr, *bits2 = nullptr;
  float *y = nullptr, *yt = nullptr;
  // reductions
  float* gpart = nullptr;     // kSplitMax x np: partial gradients of the K slices
  double* lpart = nullptr;    // loss partials
  float* loss = nullptr;
  double* mpart = nullptr;    // moment partials
  double* mvec = nullptr;     // column means for the second moment pass
  int* bad_row = nullptr;     // set by a batch that names a row outside [0, rows_total)
  // inference before line relaxation, and the relaxation's scratch (tiled FP64)
  double *guess = nullptr, *rsd = nullptr, *rsc = nullptr;
  double* dvec = nullptr;   // the increment of a right-hand side or a solution (tiled)
  double* colmean = nullptr;  // column means of a right-hand side (features)

  // parameter offsets in the packed array
  size_t oW1() const { return 0; }
  size_t ob1() const { return static_cast<size_t>(h) * nin; }
  size_t oW2() const { return ob1() + h; }
  size_t ob2() const { return oW2() + static_cast<size_t>(h) * h; }
  size_t oW3() const { return ob2() + h; }
  size_t ob3() const { return oW3() + static_cast<size_t>(nz) * h; }
};

namespace {

void carve(tpmg_mlp& m, Carve& c) {
  const size_t R = m.max_rows;
  m.np = param_count(m.nz, m.h);
  m.params = c.take<float>(m.np);
  m.grads = c.take<float>(m.np);
  m.am = c.take<float>(m.np);
  m.av = c.take<float>(m.np);
  m.w1b = c.take<bf16>(static_cast<size_t>(m.h) * m.kp);
  m.w2b = c.take<bf16>(static_cast<size_t>(m.h) * m.h);
  m.w3b = c.take<bf16>(static_cast<size_t>(m.nz) * m.h);
  m.w2t = c.take<bf16>(static_cast<size_t>(m.h) * m.h);
  m.w3t = c.take<bf16>(static_cast<size_t>(m.h) * m.nz);
  m.mu_x = c.take<float>(m.nin);
  m.sd_x = c.take<float>(m.nin);
  m.mu_y = c.take<float>(m.nz);
  m.sd_y = c.take<float>(m.nz);
  m.xb = c.take<bf16>(R * m.kp);
  m.h1 = c.take<bf16>(R * m.h);
  m.h2 = c.take<bf16>(R * m.h);
  m.dy = c.take<bf16>(R * m.nz);
  m.dh2 = c.take<bf16>(R * m.h);
  m.dh1 = c.take<bf16>(R * m.h);
  // (at most one word per thread of 4 waves per 64 x 64 outputs, whatever the tile)
  const size_t words = (R + 63) / 64 * ((static_cast<size_t>(m.h) + 63) / 64) * 256;
  m.bits1 = c.take<uint64_t>(words);
  m.bits2 = c.take<uint64_t>(words);
  m.y = c.take<float>(R * m.nz);
  m.yt = c.take<float>(R * m.nz);
  m.gpart = c.take<float>(kSplitMax * m.np);
  m.lpart = c.take<double>(1024);
  m.loss = c.take<float>(1);
  m.mpart = c.take<double>(static_cast<size_t>(tpmg::kMomentChunksMax) * m.nin);
  m.mvec = c.take<double>(m.nin);
  m.bad_row = c.take<int>(1);
  const size_t tiled = static_cast<size_t>((m.max_rows + 63) / 64 * 64) * m.nz;
  m.guess = c.take<double>(tiled);
  m.rsd = c.take<double>(tiled);
  m.rsc = c.take<double>(tiled);
  m.dvec = c.take<double>(tiled);
  m.colmean = c.take<double>(m.max_rows);
}

tpmg_status check(const tpmg_mlp* m) {
  if (!m) return fail(TPMG_ERR_ARG, "mlp handle is NULL");
  return TPMG_OK;
}

hipError_t upload_scaling(tpmg_mlp& m) {
  std::vector<float> v(2 * static_cast<size_t>(m.nin) + 2 * static_cast<size_t>(m.nz));
  for (int j = 0; j < m.nin; ++j) {
    v[j] = static_cast<float>(m.h_mu_x[j]);
    v[m.nin + j] = static_cast<float>(m.h_sd_x[j]);
  }
  for (int k = 0; k < m.nz; ++k) {
    v[2 * m.nin + k] = static_cast<float>(m.h_mu_y[k]);
    v[2 * m.nin + m.nz + k] = static_cast<float>(m.h_sd_y[k]);
  }
  hipError_t e = hipMemcpyAsync(m.mu_x, v.data(), m.nin * sizeof(float), hipMemcpyHostToDevice, m.stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(m.sd_x, v.data() + m.nin, m.nin * sizeof(float), hipMemcpyHostToDevice, m.stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(m.mu_y, v.data() + 2 * m.nin, m.nz * sizeof(float), hipMemcpyHostToDevice, m.stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(m.sd_y, v.data() + 2 * m.nin + m.nz, m.nz * sizeof(float), hipMemcpyHostToDevice, m.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m.stream);
  return e;
}

hipError_t refresh(tpmg_mlp& m) {
  return tpmg::launch_refresh_weights(m.params, m.nin, m.h, m.nz, m.kp, m.w1b, m.w2b, m.w3b, m.w2t, m.w3t, m.stream);
}

// one Adam step on m.grads, with the bf16 weight copies refreshed in it
hipError_t adam_step(tpmg_mlp& m, float lr) {
  return tpmg::launch_adam_copies(m.params, m.grads, m.am, m.av, m.np, lr, m.adam_t, m.nin, m.h, m.nz, m.kp, m.w1b,
                                  m.w2b, m.w3b, m.w2t, m.w3t, m.stream);
}

// forward pass over n prepared rows (m.xb): h1, h2, then the third product
// with the given epilogue
hipError_t forward(tpmg_mlp& m, int n, int epi3, float* y_out, double* u_out, bool mask_bits = false) {
  const float* P = m.params;
  tpmg::GemmArgs g;
  g.A = m.xb;
  g.lda = m.kp;
  g.B = m.w1b;
  g.ldb = m.kp;
  g.M = n;
  g.N = m.h;
  g.K = m.kp;
  g.epi = tpmg::kEpiBiasReluBf16;
  g.bias = P + m.ob1();
  g.out_bf16 = m.h1;
  g.ldc = m.h;
  g.mask_bits = mask_bits ? m.bits1 : nullptr;
  hipError_t e = tpmg::launch_gemm(g, m.stream);
  if (e != hipSuccess) return e;
  g.A = m.h1;
  g.lda = m.h;
  g.B = m.w2b;
  g.ldb = m.h;
  g.K = m.h;
  g.bias = P + m.ob2();
  g.out_bf16 = m.h2;
  g.mask_bits = mask_bits ? m.bits2 : nullptr;
  e = tpmg::launch_gemm(g, m.stream);
  if (e != hipSuccess) return e;
  tpmg::GemmArgs g3;
  g3.A = m.h2;
  g3.lda = m.h;
  g3.B = m.w3b;
  g3.ldb = m.h;
  g3.M = n;
  g3.N = m.nz;
  g3.K = m.h;
  g3.epi = epi3;
  g3.bias = P + m.ob3();
  g3.out_f32 = y_out;
  g3.ldc = m.nz;
  g3.out_f64 = u_out;
  g3.mu = m.mu_y;
  g3.sd = m.sd_y;
  return tpmg::launch_gemm(g3, m.stream);
}

// weight gradient dW [M][N] = sum over the batch of a(b, m) c(b, n), a and c
// row-major [batch][lda] and [batch][ldc], written to grads + off
// K slices of the weight-gradient products: about 256 workgroups for the
// largest layer, at least 32 rows each; the same for every layer, so that
// one sum over the slices forms all the gradients
int grad_ksplit(int batch) {
  int ksplit = (batch + kSplitMax - 1) / kSplitMax;
  return std::max(32, (ksplit + 31) / 32 * 32);
}

// partial gradients of a layer's weights W [M][N] and bias b [M], which
// follows W in the packed parameters: the product a^T c over each K slice of
// the batch (a: the layer's output gradients [batch][M], c: its inputs
// [batch][N]) with the row sums of a (the bias gradient) beside it, at
// offset off of that slice's row of m.gpart (rows of np entries)
hipError_t weight_grad(tpmg_mlp& m, const bf16* a, int lda, int M, const bf16* c, int ldc, int N, int batch,
                       size_t off) {
  tpmg::GemmArgs g;
  g.A = a;
  g.lda = lda;
  g.B = c;
  g.ldb = ldc;
  g.ta = g.tb = true;
  g.M = M;
  g.N = N;
  g.K = batch;
  g.ksplit = grad_ksplit(batch);
  g.epi = tpmg::kEpiPartialF32;
  g.row_sums = true;
  g.pstride = m.np;
  g.out_f32 = m.gpart + off;
  return tpmg::launch_gemm(g, m.stream);
}

// loss and gradients of the batch into m.grads and m.loss
hipError_t backprop(tpmg_mlp& m, const float* x, const float* yv, size_t rows_total, const int32_t* rows, int batch,
                    bool want_loss = true) {
  hipError_t e = tpmg::launch_mlp_prep(x, yv, rows, rows_total, m.bad_row, batch, m.nin, m.kp, m.nz, m.mu_x, m.sd_x,
                                       m.mu_y, m.sd_y, m.xb, m.yt, m.stream);
  if (e == hipSuccess) e = forward(m, batch, tpmg::kEpiBiasF32, m.y, nullptr, true);
  // (the batch loss, into m.loss, only when it is read)
  if (e == hipSuccess)
    e = tpmg::launch_mlp_mse(m.y, m.yt, batch, m.nz, m.dy, m.lpart, want_loss ? m.loss : nullptr, m.stream);
  if (e != hipSuccess) return e;
  // output layer
  e = weight_grad(m, m.dy, m.nz, m.nz, m.h2, m.h, m.h, batch, m.oW3());
  // dh2 = (dy W3) * [h2 > 0]
  tpmg::GemmArgs g;
  g.A = m.dy;
  g.lda = m.nz;
  g.B = m.w3t;
  g.ldb = m.nz;
  g.M = batch;
  g.N = m.h;
  g.K = m.nz;
  g.epi = tpmg::kEpiMaskBf16;
  g.mask_bits = m.bits2;   // (this product's M and N are those of layer 2's)
  g.out_bf16 = m.dh2;
  g.ldc = m.h;
  if (e == hipSuccess) e = tpmg::launch_gemm(g, m.stream);
  if (e == hipSuccess) e = weight_grad(m, m.dh2, m.h, m.h, m.h1, m.h, m.h, batch, m.oW2());
  // dh1 = (dh2 W2) * [h1 > 0]
  g.A = m.dh2;
  g.lda = m.h;
  g.B = m.w2t;
  g.ldb = m.h;
  g.K = m.h;
  g.mask_bits = m.bits1;
  g.out_bf16 = m.dh1;
  if (e == hipSuccess) e = tpmg::launch_gemm(g, m.stream);
  if (e == hipSuccess) e = weight_grad(m, m.dh1, m.h, m.h, m.xb, m.kp, m.nin, batch, m.oW1());
  // every parameter's gradient: the sum over the K slices
  const int ksplit = grad_ksplit(batch);
  if (e == hipSuccess) e = tpmg::launch_sum_parts(m.gpart, (batch + ksplit - 1) / ksplit, m.np, m.grads, m.stream);
  return e;
}

tpmg_status check_batch_args(const tpmg_mlp* m, const float* x, const float* y, size_t rows_total,
                             const int32_t* rows, int batch) {
  if (!x || !y || !rows) return fail(TPMG_ERR_ARG, "NULL device buffer");
  if (batch < 1 || batch > m->max_rows) return fail(TPMG_ERR_ARG, "batch must be in 1..max_rows");
  if (rows_total < 1) return fail(TPMG_ERR_ARG, "rows_total must be >= 1");
  return TPMG_OK;
}

// after a synchronisation: reports (and clears) a batch index that was out of range
tpmg_status check_bad_row(tpmg_mlp& m) {
  int bad = 0;
  MLP_HIP(hipMemcpyAsync(&bad, m.bad_row, sizeof(int), hipMemcpyDeviceToHost, m.stream));
  MLP_HIP(hipStreamSynchronize(m.stream));
  if (!bad) return TPMG_OK;
  MLP_HIP(hipMemsetAsync(m.bad_row, 0, sizeof(int), m.stream));
  MLP_HIP(hipStreamSynchronize(m.stream));
  return fail(TPMG_ERR_ARG, "a batch named a row outside [0, rows_total): those rows were replaced by zeros");
}

tpmg_status check_grid(const tpmg_mlp* m, const tpmg_mg* mg, tpmg::FineGrid* g) {
  if (!mg || !tpmg_fine_grid(mg, g)) return fail(TPMG_ERR_ARG, "mg handle is NULL");
  if (g->nz != m->nz) return fail(TPMG_ERR_ARG, "the grid's nz differs from the network's");
  return TPMG_OK;
}

}  // namespace

extern "C" {

tpmg_status tpmg_mlp_param_count(int nz, int hidden, size_t* n) {
  if (!n) return fail(TPMG_ERR_ARG, "n is NULL");
  if (!shape_ok(nz, hidden, 1)) return fail(TPMG_ERR_ARG, "unsupported nz or hidden width");
  *n = param_count(nz, hidden);
  return TPMG_OK;
}

tpmg_status tpmg_mlp_workspace_size(int nz, int hidden, int max_rows, size_t* bytes) {
  if (!bytes) return fail(TPMG_ERR_ARG, "bytes is NULL");
  if (!shape_ok(nz, hidden, max_rows)) return fail(TPMG_ERR_ARG, "unsupported nz, hidden width or max_rows");
  tpmg_mlp m;
  m.nz = nz;
  m.h = hidden;
  m.nin = nz + 3;
  m.kp = (m.nin + 31) / 32 * 32;
  m.max_rows = max_rows;
  Carve c(nullptr);
  carve(m, c);
  *bytes = c.off + 256;
  return TPMG_OK;
}

tpmg_status tpmg_mlp_create(int nz, int hidden, int max_rows, void* d_workspace, size_t bytes, void* hip_stream,
                            tpmg_mlp** out) {
  if (!out) return fail(TPMG_ERR_ARG, "out is NULL");
  *out = nullptr;
  size_t need = 0;
  tpmg_status st = tpmg_mlp_workspace_size(nz, hidden, max_rows, &need);
  if (st != TPMG_OK) return st;
  if (!d_workspace || reinterpret_cast<uintptr_t>(d_workspace) % 256)
    return fail(TPMG_ERR_ARG, "workspace must be a non-NULL 256-byte aligned device pointer");
  if (bytes < need) return fail(TPMG_ERR_NOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  auto* m = new tpmg_mlp();
  m->nz = nz;
  m->h = hidden;
  m->nin = nz + 3;
  m->kp = (m->nin + 31) / 32 * 32;
  m->max_rows = max_rows;
  m->stream = static_cast<hipStream_t>(hip_stream);
  Carve c(d_workspace);
  carve(*m, c);
  m->h_mu_x.assign(m->nin, 0.0);
  m->h_sd_x.assign(m->nin, 1.0);
  m->h_mu_y.assign(m->nz, 0.0);
  m->h_sd_y.assign(m->nz, 1.0);
  hipError_t e = hipMemsetAsync(d_workspace, 0, c.off, m->stream);
  if (e == hipSuccess) e = refresh(*m);
  if (e == hipSuccess) e = upload_scaling(*m);
  if (e != hipSuccess) {
    delete m;
    return fail(TPMG_ERR_DEVICE, std::string("mlp setup: ") + hipGetErrorString(e));
  }
  *out = m;
  return TPMG_OK;
}

tpmg_status tpmg_mlp_set_params(tpmg_mlp* m, const float* params) {
  tpmg_status st = check(m);
  if (st != TPMG_OK) return st;
  if (!params) return fail(TPMG_ERR_ARG, "params is NULL");
  for (size_t i = 0; i < m->np; ++i)
    if (!std::isfinite(params[i])) return fail(TPMG_ERR_ARG, "parameters must be finite");
  MLP_HIP(hipMemcpyAsync(m->params, params, m->np * sizeof(float), hipMemcpyHostToDevice, m->stream));
  MLP_HIP(hipMemsetAsync(m->am, 0, m->np * sizeof(float), m->stream));
  MLP_HIP(hipMemsetAsync(m->av, 0, m->np * sizeof(float), m->stream));
  MLP_HIP(refresh(*m));
  MLP_HIP(hipStreamSynchronize(m->stream));
  m->adam_t = 0;
  return TPMG_OK;
}

tpmg_status tpmg_mlp_get_params(tpmg_mlp* m, float* params) {
  tpmg_status st = check(m);
  if (st != TPMG_OK) return st;
  if (!params) return fail(TPMG_ERR_ARG, "params is NULL");
  MLP_HIP(hipMemcpyAsync(params, m->params, m->np * sizeof(float), hipMemcpyDeviceToHost, m->stream));
  MLP_HIP(hipStreamSynchronize(m->stream));
  return check_bad_row(*m);
}

tpmg_status tpmg_mlp_set_scaling(tpmg_mlp* m, const double* mu_x, const double* sd_x, const double* mu_y,
                                 const double* sd_y) {
  tpmg_status st = check(m);
  if (st != TPMG_OK) return st;
  if (!mu_x || !sd_x || !mu_y || !sd_y) return fail(TPMG_ERR_ARG, "NULL scaling array");
  for (int j = 0; j < m->nin; ++j)
    if (!(sd_x[j] > 0.0) || !std::isfinite(sd_x[j]) || !std::isfinite(mu_x[j]))
      return fail(TPMG_ERR_ARG, "feature scaling must be finite with sd > 0");
  for (int k = 0; k < m->nz; ++k)
    if (!(sd_y[k] > 0.0) || !std::isfinite(sd_y[k]) || !std::isfinite(mu_y[k]))
      return fail(TPMG_ERR_ARG, "target scaling must be finite with sd > 0");
  m->h_mu_x.assign(mu_x, mu_x + m->nin);
  m->h_sd_x.assign(sd_x, sd_x + m->nin);
  m->h_mu_y.assign(mu_y, mu_y + m->nz);
  m->h_sd_y.assign(sd_y, sd_y + m->nz);
  MLP_HIP(upload_scaling(*m));
  return TPMG_OK;
}

tpmg_status tpmg_mlp_get_scaling(const tpmg_mlp* m, double* mu_x, double* sd_x, double* mu_y, double* sd_y) {
  tpmg_status st = check(m);
  if (st != TPMG_OK) return st;
  if (mu_x) std::copy(m->h_mu_x.begin(), m->h_mu_x.end(), mu_x);
  if (sd_x) std::copy(m->h_sd_x.begin(), m->h_sd_x.end(), sd_x);
  if (mu_y) std::copy(m->h_mu_y.begin(), m->h_mu_y.end(), mu_y);
  if (sd_y) std::copy(m->h_sd_y.begin(), m->h_sd_y.end(), sd_y);
  return TPMG_OK;
}

tpmg_status tpmg_mlp_fit_scaling(tpmg_mlp* m, const float* d_x, const float* d_y, size_t rows) {
  tpmg_status st = check(m);
  if (st != TPMG_OK) return st;
  if (!d_x || !d_y) return fail(TPMG_ERR_ARG, "NULL device buffer");
  if (rows < 1) return fail(TPMG_ERR_ARG, "rows must be >= 1");
  const size_t cr = tpmg::moment_chunk_rows(rows);
  const size_t chunks = (rows + cr - 1) / cr;
  auto moments = [&](const float* a, int cols, std::vector<double>& mu, std::vector<double>& sd) -> hipError_t {
    std::vector<double> part(chunks * cols);
    hipError_t e = tpmg::launch_moment_partials(a, rows, cols, nullptr, m->mpart, m->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(part.data(), m->mpart, part.size() * sizeof(double), hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) return e;
    mu.assign(cols, 0.0);
    for (size_t c = 0; c < chunks; ++c)
      for (int j = 0; j < cols; ++j) mu[j] += part[c * cols + j];
    for (int j = 0; j < cols; ++j) mu[j] /= static_cast<double>(rows);
    e = hipMemcpyAsync(m->mvec, mu.data(), cols * sizeof(double), hipMemcpyHostToDevice, m->stream);
    if (e == hipSuccess) e = tpmg::launch_moment_partials(a, rows, cols, m->mvec, m->mpart, m->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(part.data(), m->mpart, part.size() * sizeof(double), hipMemcpyDeviceToHost, m->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
    if (e != hipSuccess) return e;
    sd.assign(cols, 0.0);
    for (size_t c = 0; c < chunks; ++c)
      for (int j = 0; j < cols; ++j) sd[j] += part[c * cols + j];
    for (int j = 0; j < cols; ++j) {
      sd[j] = std::sqrt(sd[j] / static_cast<double>(rows));
      if (!(sd[j] > 0.0)) sd[j] = 1.0;
    }
    return hipSuccess;
  };
  std::vector<double> mx, sx, my, sy;
  MLP_HIP(moments(d_x, m->nin, mx, sx));
  MLP_HIP(moments(d_y, m->nz, my, sy));
  m->h_mu_x = mx;
  m->h_sd_x = sx;
  m->h_mu_y = my;
  m->h_sd_y = sy;
  MLP_HIP(upload_scaling(*m));
  return TPMG_OK;
}

tpmg_status tpmg_mlp_features(tpmg_mlp* m, const tpmg_mg* mg, const double* d_f, float* d_x) {
  tpmg_status st = check(m);
  if (st != TPMG_OK) return st;
  tpmg::FineGrid g;
  if ((st = check_grid(m, mg, &g)) != TPMG_OK) return st;
  if (!d_f || !d_x) return fail(TPMG_ERR_ARG, "NULL device buffer");
  if (g.n > m->max_rows) return fail(TPMG_ERR_ARG, "the grid has more columns than max_rows");
  MLP_HIP(tpmg::launch_mlp_features(g, d_f, m->colmean, d_x, m->stream));
  return TPMG_OK;
}

tpmg_status tpmg_mlp_targets(tpmg_mlp* m, const tpmg_mg* mg, const double* d_u, float* d_y) {
  tpmg_status st = check(m);
  if (st != TPMG_OK) return st;
  tpmg::FineGrid g;
  if ((st = check_grid(m, mg, &g)) != TPMG_OK) return st;
  if (!d_u || !d_y) return fail(TPMG_ERR_ARG, "NULL device buffer");
  MLP_HIP(tpmg::launch_mlp_targets(g, d_u, d_y, m->stream));
  return TPMG_OK;
}

tpmg_status tpmg_mlp_forward(tpmg_mlp* m, const float* d_x, int rows, float* d_y) {
  tpmg_status st = check(m);
  if (st != TPMG_OK) return st;
  if (!d_x || !d_y) return fail(TPMG_ERR_ARG, "NULL device buffer");
  if (rows < 1 || rows > m->max_rows) return fail(TPMG_ERR_ARG, "rows must be in 1..max_rows");
  MLP_HIP(tpmg::launch_mlp_prep(d_x, nullptr, nullptr, 0, nullptr, rows, m->nin, m->kp, m->nz, m->mu_x, m->sd_x,
                                m->mu_y, m->sd_y, m->xb, nullptr, m->stream));
  MLP_HIP(forward(*m, rows, tpmg::kEpiBiasF32, d_y, nullptr));
  return TPMG_OK;
}

tpmg_status tpmg_mlp_gradients(tpmg_mlp* m, const float* d_x, const float* d_y, size_t rows_total,
                               const int32_t* d_rows, int batch, float* loss, float* grads) {
  tpmg_status st = check(m);
  if (st != TPMG_OK) return st;
  if ((st = check_batch_args(m, d_x, d_y, rows_total, d_rows, batch)) != TPMG_OK) return st;
  MLP_HIP(backprop(*m, d_x, d_y, rows_total, d_rows, batch));
  if (loss) MLP_HIP(hipMemcpyAsync(loss, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->stream));
  if (grads) MLP_HIP(hipMemcpyAsync(grads, m->grads, m->np * sizeof(float), hipMemcpyDeviceToHost, m->stream));
  MLP_HIP(hipStreamSynchronize(m->stream));
  return check_bad_row(*m);
}

tpmg_status tpmg_mlp_train_step(tpmg_mlp* m, const float* d_x, const float* d_y, size_t rows_total,
                                const int32_t* d_rows, int batch, float lr, float* loss) {
  tpmg_status st = check(m);
  if (st != TPMG_OK) return st;
  if ((st = check_batch_args(m, d_x, d_y, rows_total, d_rows, batch)) != TPMG_OK) return st;
  if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(TPMG_ERR_ARG, "lr must be finite and > 0");
  MLP_HIP(backprop(*m, d_x, d_y, rows_total, d_rows, batch, loss != nullptr));
  m->adam_t += 1;
  MLP_HIP(adam_step(*m, lr));
  if (loss) {
    MLP_HIP(hipMemcpyAsync(loss, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->stream));
    MLP_HIP(hipStreamSynchronize(m->stream));
    return check_bad_row(*m);
  }
  return TPMG_OK;
}

tpmg_status tpmg_mlp_train_epoch(tpmg_mlp* m, const float* d_x, const float* d_y, size_t rows_total,
                                 const int32_t* d_perm, int steps, int batch, float lr, int loss_every, float* losses) {
  tpmg_status st = check(m);
  if (st != TPMG_OK) return st;
  if (steps < 1) return fail(TPMG_ERR_ARG, "steps must be >= 1");
  if ((st = check_batch_args(m, d_x, d_y, rows_total, d_perm, batch)) != TPMG_OK) return st;
  if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(TPMG_ERR_ARG, "lr must be finite and > 0");
  if (loss_every < 0 || (loss_every > 0 && !losses)) return fail(TPMG_ERR_ARG, "loss_every > 0 needs losses");
  int sampled = 0;
  for (int k = 0; k < steps; ++k) {
    const bool sample = loss_every > 0 && (k % loss_every == 0 || k == steps - 1);
    MLP_HIP(backprop(*m, d_x, d_y, rows_total, d_perm + static_cast<size_t>(k) * batch, batch, sample));
    if (sample)
      MLP_HIP(hipMemcpyAsync(losses + sampled++, m->loss, sizeof(float), hipMemcpyDeviceToHost, m->stream));
    m->adam_t += 1;
    MLP_HIP(adam_step(*m, lr));
  }
  MLP_HIP(hipStreamSynchronize(m->stream));
  return check_bad_row(*m);
}

tpmg_status tpmg_mlp_infer(tpmg_mlp* m, const tpmg_mg* mg, const double* d_f, int relax, double* d_u0) {
  tpmg_status st = check(m);
  if (st != TPMG_OK) return st;
  tpmg::FineGrid g;
  if ((st = check_grid(m, mg, &g)) != TPMG_OK) return st;
  if (!d_f || !d_u0) return fail(TPMG_ERR_ARG, "NULL device buffer");
  if (d_f == d_u0) return fail(TPMG_ERR_ARG, "f and u0 must not alias");
  if (g.n > m->max_rows) return fail(TPMG_ERR_ARG, "the grid has more columns than max_rows");
  if (relax != 0 && relax != 1) return fail(TPMG_ERR_ARG, "relax must be 0 or 1");
  if (g.stream != m->stream) return fail(TPMG_ERR_ARG, "the network and mg must share one stream");
  double* out = relax ? m->guess : d_u0;
  if (tpmg::mlp_infer_fits(m->h, m->nz, m->kp)) {
    // one kernel from the right-hand side to the guess (features formed in it)
    MLP_HIP(tpmg::launch_mlp_col_means(g, d_f, m->colmean, m->stream));
    tpmg::InferArgs a;
    a.kp = m->kp;
    a.n = g.n;
    a.nz = m->nz;
    a.f = d_f;
    a.means = m->colmean;
    a.nbr = g.nbr;
    a.npad = g.npad;
    a.mu_x = m->mu_x;
    a.sd_x = m->sd_x;
    a.w1 = m->w1b;
    a.w2 = m->w2b;
    a.w3 = m->w3b;
    a.b1 = m->params + m->ob1();
    a.b2 = m->params + m->ob2();
    a.b3 = m->params + m->ob3();
    a.mu = m->mu_y;
    a.sd = m->sd_y;
    a.out = out;
    MLP_HIP(tpmg::launch_mlp_infer(a, m->stream));
  } else {
    MLP_HIP(tpmg::launch_mlp_features_bf16(g, d_f, m->colmean, m->mu_x, m->sd_x, m->kp, m->xb, m->stream));
    MLP_HIP(forward(*m, g.n, tpmg::kEpiInferTiled, nullptr, out));
  }
  if (!relax) return TPMG_OK;
  MLP_HIP(tpmg_relax_finest(mg, d_f, m->guess, d_u0, m->rsd, m->rsc, 1.0, m->stream));
  return TPMG_OK;
}

tpmg_status tpmg_mlp_features_increment(tpmg_mlp* m, const tpmg_mg* mg, const double* d_f, const double* d_f_prev,
                                        float* d_x) {
  tpmg_status st = check(m);
  if (st != TPMG_OK) return st;
  tpmg::FineGrid g;
  if ((st = check_grid(m, mg, &g)) != TPMG_OK) return st;
  if (!d_f || !d_f_prev || !d_x) return fail(TPMG_ERR_ARG, "NULL device buffer");
  if (g.n > m->max_rows) return fail(TPMG_ERR_ARG, "the grid has more columns than max_rows");
  MLP_HIP(tpmg::launch_vec_sub(d_f, d_f_prev, m->dvec, static_cast<size_t>(g.npad) * g.nz, m->stream));
  MLP_HIP(tpmg::launch_mlp_features(g, m->dvec, m->colmean, d_x, m->stream));
  return TPMG_OK;
}

tpmg_status tpmg_mlp_targets_increment(tpmg_mlp* m, const tpmg_mg* mg, const double* d_u, const double* d_u_prev,
                                       float* d_y) {
  tpmg_status st = check(m);
  if (st != TPMG_OK) return st;
  tpmg::FineGrid g;
  if ((st = check_grid(m, mg, &g)) != TPMG_OK) return st;
  if (!d_u || !d_u_prev || !d_y) return fail(TPMG_ERR_ARG, "NULL device buffer");
  if (g.n > m->max_rows) return fail(TPMG_ERR_ARG, "the grid has more columns than max_rows");
  MLP_HIP(tpmg::launch_vec_sub(d_u, d_u_prev, m->dvec, static_cast<size_t>(g.npad) * g.nz, m->stream));
  MLP_HIP(tpmg::launch_mlp_targets(g, m->dvec, d_y, m->stream));
  return TPMG_OK;
}

tpmg_status tpmg_mlp_infer_increment(tpmg_mlp* m, const tpmg_mg* mg, const double* d_f, const double* d_f_prev,
                                     const double* d_u_prev, int relax, double* d_u0) {
  tpmg_status st = check(m);
  if (st != TPMG_OK) return st;
  tpmg::FineGrid g;
  if ((st = check_grid(m, mg, &g)) != TPMG_OK) return st;
  if (!d_f || !d_f_prev || !d_u_prev || !d_u0) return fail(TPMG_ERR_ARG, "NULL device buffer");
  if (d_u0 == d_f || d_u0 == d_f_prev || d_u0 == d_u_prev)
    return fail(TPMG_ERR_ARG, "u0 must not alias f, f_prev or u_prev");
  if (g.n > m->max_rows) return fail(TPMG_ERR_ARG, "the grid has more columns than max_rows");
  if (relax != 0 && relax != 1) return fail(TPMG_ERR_ARG, "relax must be 0 or 1");
  if (g.stream != m->stream) return fail(TPMG_ERR_ARG, "the network and mg must share one stream");
  MLP_HIP(tpmg::launch_vec_sub(d_f, d_f_prev, m->dvec, static_cast<size_t>(g.npad) * g.nz, m->stream));
  // the network's increment into guess (real columns), then u_prev + increment
  if ((st = tpmg_mlp_infer(m, mg, m->dvec, 0, m->guess)) != TPMG_OK) return st;
  if (!relax) {
    MLP_HIP(tpmg::launch_add_guess(g, d_u_prev, m->guess, d_u0, m->stream));
    return TPMG_OK;
  }
  MLP_HIP(tpmg::launch_add_guess(g, d_u_prev, m->guess, m->guess, m->stream));
  MLP_HIP(tpmg_relax_finest(mg, d_f, m->guess, d_u0, m->rsd, m->rsc, 1.0, m->stream));
  return TPMG_OK;
}

tpmg_status tpmg_mlp_save(tpmg_mlp* m, const char* path) {
  tpmg_status st = check(m);
  if (st != TPMG_OK) return st;
  if (!path) return fail(TPMG_ERR_ARG, "path is NULL");
  std::vector<float> p(m->np);
  if ((st = tpmg_mlp_get_params(m, p.data())) != TPMG_OK) return st;
  std::ofstream out(path, std::ios::binary | std::ios::trunc);
  if (!out) return fail(TPMG_ERR_ARG, std::string("cannot write ") + path);
  const int32_t hdr[4] = {static_cast<int32_t>(kFileMagic), m->nz, m->h, 1};
  out.write(reinterpret_cast<const char*>(hdr), sizeof(hdr));
  out.write(reinterpret_cast<const char*>(p.data()), p.size() * sizeof(float));
  for (const auto* v : {&m->h_mu_x, &m->h_sd_x, &m->h_mu_y, &m->h_sd_y})
    out.write(reinterpret_cast<const char*>(v->data()), v->size() * sizeof(double));
  out.close();
  if (!out) return fail(TPMG_ERR_ARG, std::string("write failed: ") + path);
  return TPMG_OK;
}

tpmg_status tpmg_mlp_load(tpmg_mlp* m, const char* path) {
  tpmg_status st = check(m);
  if (st != TPMG_OK) return st;
  if (!path) return fail(TPMG_ERR_ARG, "path is NULL");
  std::ifstream in(path, std::ios::binary);
  if (!in) return fail(TPMG_ERR_ARG, std::string("cannot read ") + path);
  int32_t hdr[4] = {0, 0, 0, 0};
  in.read(reinterpret_cast<char*>(hdr), sizeof(hdr));
  if (!in || hdr[0] != static_cast<int32_t>(kFileMagic) || hdr[3] != 1)
    return fail(TPMG_ERR_ARG, std::string("not a saved network: ") + path);
  if (hdr[1] != m->nz || hdr[2] != m->h) return fail(TPMG_ERR_ARG, "saved network has a different shape");
  std::vector<float> p(m->np);
  in.read(reinterpret_cast<char*>(p.data()), p.size() * sizeof(float));
  std::vector<double> mx(m->nin), sx(m->nin), my(m->nz), sy(m->nz);
  for (auto* v : {&mx, &sx, &my, &sy}) in.read(reinterpret_cast<char*>(v->data()), v->size() * sizeof(double));
  if (!in) return fail(TPMG_ERR_ARG, std::string("truncated file: ") + path);
  if ((st = tpmg_mlp_set_scaling(m, mx.data(), sx.data(), my.data(), sy.data())) != TPMG_OK) return st;
  return tpmg_mlp_set_params(m, p.data());
}

void tpmg_mlp_destroy(tpmg_mlp* m) { delete m; }

}  // extern "C"
