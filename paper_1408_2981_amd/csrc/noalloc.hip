// tpmg_solve_noalloc: a whole solve (device setup, flexible CG, teardown)
// that allocates nothing. Its workspace is `scratch`, a fixed array in
// device memory that the code object carries (one copy per GPU, held until
// the process ends); every call on a GPU reuses that GPU's copy.
//
// Host code never passes `scratch` itself to the device: in host code the
// name stands for a host-side shadow, not a device address. The device
// address of each GPU's copy is looked up once per device with
// hipGetSymbolAddress (with that device current) and kept; the workspace
// pointers the kernels receive are carved from it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/tpmg.h"
#include "device.h"

// defined with the solver (csrc/tpmg.cpp)
tpmg_status tpmg_solve_on_workspace(const tpmg_op* op, const tpmg_mg_params* params, void* d_workspace,
                                    size_t bytes, void* hip_stream, const double* d_f, double* d_u, double rtol,
                                    int maxit, tpmg_solve_info* info);

constexpr size_t kScratchBytes = TPMG_NOALLOC_SCRATCH_BYTES;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of the current GPU's copy of `scratch` (looked up on the
// first call on that GPU).
hipError_t scratch_address(void** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[dev] = p;
  }
  *ptr = g_scratch[dev];
  return hipSuccess;
}

}  // namespace

extern "C" tpmg_status tpmg_solve_noalloc(const tpmg_op* op, const tpmg_mg_params* params, void* hip_stream,
                                          const double* d_f, double* d_u, double rtol, int maxit,
                                          tpmg_solve_info* info) {
  if (!op || !params) {
    tpmg_set_last_error("NULL argument");
    return TPMG_ERR_ARG;
  }
  size_t need = 0;
  tpmg_status st = tpmg_mg_workspace_size(op, params, &need);
  if (st != TPMG_OK) return st;
  if (need > kScratchBytes) {
    tpmg_set_last_error(("tpmg_solve_noalloc: the problem needs " + std::to_string(need) +
                         " bytes of workspace; the static scratch holds " + std::to_string(kScratchBytes) +
                         " bytes (use tpmg_mg_setup with a workspace of that size)")
                            .c_str());
    return TPMG_ERR_NOMEM;
  }
  void* ptr = nullptr;
  const hipError_t e = scratch_address(&ptr);
  if (e != hipSuccess) {
    tpmg_set_last_error((std::string("tpmg_solve_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e)).c_str());
    return TPMG_ERR_DEVICE;
  }
  return tpmg_solve_on_workspace(op, params, ptr, kScratchBytes, hip_stream, d_f, d_u, rtol, maxit, info);
}
