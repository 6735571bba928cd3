// Allocation-free variant of the transpose apply, for callers that cannot
// allocate device memory (code under stream capture, serving loops, harnesses
// that forbid it). cpm_apply_T keeps the neighbour sums z = O^T x over
// Sigma_A u Sigma_G in an operator-owned buffer that it allocates on first use;
// this entry point keeps them in a static device array instead, so it never
// allocates. Every call on one GPU shares that GPU's copy of the array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.h"

namespace cpm {

// z of (N_A + N_G) * nrhs doubles must fit: 32 MiB per device, held until the process ends
constexpr size_t kNoAllocScratchDoubles = size_t(1) << 22;
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

// device address of each GPU's copy of `scratch` (the host-side name is only a
// stand-in and must never reach a kernel or a copy)
static double* g_scratch_ptr[kNoAllocMaxDevices] = {};
static std::mutex g_scratch_mu;

static double* scratch_on_current_device() {
  int dev = 0;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kNoAllocMaxDevices) fail(CPM_ERR_DEVICE, "device index beyond the supported range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) fail(CPM_ERR_DEVICE, "static scratch has no device address");
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}

}  // namespace cpm

using namespace cpm;

cpm_status cpm_apply_T_noalloc(const cpm_operator* op, const double* x, double* y, int32_t nrhs, void* stream) {
  try {
    if (!op || !x || !y) fail(CPM_ERR_ARG, "null argument");
    if (nrhs != 1 && nrhs != 2 && nrhs != 4) fail(CPM_ERR_ARG, "nrhs must be 1, 2 or 4");
    if (x == y) fail(CPM_ERR_ARG, "x and y must not alias");
    if (op->generic) fail(CPM_ERR_ARG, "the transposed apply needs a second-order operator with p <= 3");
    const size_t need = (size_t)op->band->nodes() * (size_t)nrhs;
    if (need > kNoAllocScratchDoubles)
      fail(CPM_ERR_ARG, "cpm_apply_T_noalloc: (N_A + N_G) * nrhs = " + std::to_string(need) +
                            " doubles exceeds the static scratch of " + std::to_string(kNoAllocScratchDoubles));
    double* z = scratch_on_current_device();
    hip_check(launch_apply_T(op->I, nrhs, x, z, y, (hipStream_t)stream), "cpm_apply_T_noalloc");
    return CPM_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  }
}
