// Gradient of a loss with respect to the shift c of A(c) = c I + K (Sec. 2.1,
// eq. lapBel: c enters A only through the identity). For u = A^-1 f and the
// adjoint solution lambda of A^T lambda = dL/du, differentiating A u = f gives
// dL/dc = -lambda . u. The inner product is reduced in a fixed order that does
// not depend on timing: each block sums one chunk of kGradChunk consecutive
// elements (thread t takes elements t, t + 256, ... of the chunk, then a
// butterfly over the wavefront, then the four wavefront sums in order), and
// one wavefront adds the chunk sums (lane l takes chunks l, l + 64, ...).
#include <hip/hip_runtime.h>

#include "common.h"

#pragma clang fp contract(off)

namespace cpm {

constexpr int kGradThreads = 256;
constexpr int kGradPerThread = 16;
constexpr int64_t kGradChunk = (int64_t)kGradThreads * kGradPerThread;

__device__ __forceinline__ double grad_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ void __launch_bounds__(kGradThreads) k_grad_part(int64_t n, const double* __restrict__ x,
                                                            const double* __restrict__ y, double* __restrict__ part) {
  __shared__ double red[kGradThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kGradChunk;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kGradPerThread; ++k) {
    const int64_t i = base + (int64_t)k * kGradThreads + threadIdx.x;
    if (i < n) s += x[i] * y[i];
  }
  s = grad_wave_sum(s);
  if (__lane_id() == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kGradThreads / 64; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(64) k_grad_final(int64_t nchunks, const double* __restrict__ part, double scale,
                                                   double* __restrict__ out) {
  double s = 0.0;
  for (int64_t c = threadIdx.x; c < nchunks; c += 64) s += part[c];
  s = grad_wave_sum(s);
  if (threadIdx.x == 0) out[0] = scale * s;
}

int64_t grad_chunks(int64_t n) { return (n + kGradChunk - 1) / kGradChunk; }

hipError_t launch_scaled_dot(int64_t n, const double* x, const double* y, double scale, double* part, double* out,
                             hipStream_t s) {
  const int64_t nc = grad_chunks(n);
  if (nc > 0) hipLaunchKernelGGL(k_grad_part, dim3((unsigned)nc), dim3(kGradThreads), 0, s, n, x, y, part);
  hipLaunchKernelGGL(k_grad_final, dim3(1), dim3(64), 0, s, nc, part, scale, out);
  return hipGetLastError();
}

}  // namespace cpm

using namespace cpm;

cpm_status cpm_shift_gradient(const cpm_operator* op, const double* lambda, const double* u, int32_t nrhs,
                              double* grad, void* stream) {
  try {
    if (!op) fail(CPM_ERR_ARG, "cpm_shift_gradient: null operator");
    if (nrhs != 1 && nrhs != 2 && nrhs != 4) fail(CPM_ERR_ARG, "cpm_shift_gradient: nrhs must be 1, 2 or 4");
    const int64_t n = op->band->nA * nrhs;
    if (!grad || (n > 0 && (!lambda || !u))) fail(CPM_ERR_ARG, "cpm_shift_gradient: null argument");
    const int64_t nc = grad_chunks(n);
    op->d_part.alloc((size_t)(nc > 0 ? nc : 1));
    hip_check(launch_scaled_dot(n, lambda, u, -1.0, op->d_part.p, grad, (hipStream_t)stream), "cpm_shift_gradient");
    return CPM_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  }
}
