// Two-level Schwarz: a coarse-grid correction added to the one-level (O)RAS
// preconditioner. The one-level method's iteration count grows with the number
// of subdomains (Sec. 5, Table 3, weak scaling); a coarse space is the standard
// remedy. Coarse space (Nicolaides, SIAM J. Numer. Anal. 24, 1987): one basis
// vector per subdomain, equal to 1 on the nodes the subdomain owns, R0 (N_S x N_A).
// Galerkin coarse matrix A0 = R0 A R0^T, built on the device with the operator
// (A applied to the indicator vectors of the subdomains, four at a time) and
// inverted on the host (partial pivoting). Combinations with the one-level M1:
//   additive:     z = M1^-1 r + R0^T A0^-1 R0 r
//   coarse first: z_c = R0^T A0^-1 R0 r,  z = z_c + M1^-1 (r - A z_c)
// All reductions run in a fixed order (deterministic results).
#include <hip/hip_runtime.h>

#include "coarse.h"

#pragma clang fp contract(off)

namespace cpm {

constexpr int kCoarseThreads = 256;

__device__ __forceinline__ double coarse_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// c[(coff + j) R + q] = sum over the nodes i owned by subdomain j of r[(vec_off + i) R + q]
template <int R>
__global__ void __launch_bounds__(kCoarseThreads) k_coarse_restrict(DevCoarse C, const double* __restrict__ r,
                                                                    double* __restrict__ c) {
  __shared__ double red[kCoarseThreads / 64][R];
  const int j = blockIdx.x;
  if (j >= C.n) return;
  const int b = C.own_ptr[j], e = C.own_ptr[j + 1];
  double acc[R];
#pragma unroll
  for (int q = 0; q < R; ++q) acc[q] = 0.0;
  for (int k = b + (int)threadIdx.x; k < e; k += kCoarseThreads) {
    const int64_t i = C.vec_off + C.own_idx[k];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] += r[i * R + q];
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const double s = coarse_wave_sum(acc[q]);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = s;
  }
  __syncthreads();
  if (threadIdx.x < R) {
    double s = 0.0;
    for (int w = 0; w < kCoarseThreads / 64; ++w) s += red[w][threadIdx.x];
    c[(C.coff + j) * R + threadIdx.x] = s;
  }
}

// e[(coff + j) R + q] = sum_k A0^-1[j, k] c[(coff + k) R + q], one wavefront per row j
template <int R>
__global__ void __launch_bounds__(kCoarseThreads) k_coarse_solve(DevCoarse C, const double* __restrict__ c,
                                                                 double* __restrict__ e) {
  const int j = blockIdx.x * (kCoarseThreads / 64) + (threadIdx.x >> 6);
  if (j >= C.n) return;
  const int lane = threadIdx.x & 63;
  double acc[R];
#pragma unroll
  for (int q = 0; q < R; ++q) acc[q] = 0.0;
  const double* row = C.ainv + (int64_t)j * C.n;
  for (int k = lane; k < C.n; k += 64) {
    const double a = row[k];
#pragma unroll
    for (int q = 0; q < R; ++q) acc[q] += a * c[(C.coff + k) * R + q];
  }
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const double s = coarse_wave_sum(acc[q]);
    if (lane == 0) e[(C.coff + j) * R + q] = s;
  }
}

// z[(vec_off + i) R + q] = (add ? z : 0) + e[(coff + owner[i]) R + q]
template <int R>
__global__ void __launch_bounds__(kCoarseThreads) k_coarse_prolong(DevCoarse C, const double* __restrict__ e,
                                                                   double* __restrict__ z, int add) {
  const int64_t i = (int64_t)blockIdx.x * kCoarseThreads + threadIdx.x;
  if (i >= C.nA) return;
  const int j = C.owner[i];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int64_t k = (C.vec_off + i) * R + q;
    const double v = e[(C.coff + j) * R + q];
    z[k] = add ? z[k] + v : v;
  }
}

// x[i R + q] = 1 when node i is owned by subdomain j0 + q (< n), else 0: four coarse basis vectors
__global__ void __launch_bounds__(kCoarseThreads) k_coarse_indicators(DevCoarse C, int j0, double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * kCoarseThreads + threadIdx.x;
  if (i >= C.nA) return;
  const int j = C.owner[i];
#pragma unroll
  for (int q = 0; q < 4; ++q) x[i * 4 + q] = (j == j0 + q) ? 1.0 : 0.0;
}

// y = a - b over n entries (y may alias a or b)
__global__ void __launch_bounds__(kCoarseThreads) k_coarse_sub(int64_t n, const double* a, const double* b,
                                                               double* y) {
  const int64_t i = (int64_t)blockIdx.x * kCoarseThreads + threadIdx.x;
  if (i < n) y[i] = a[i] - b[i];
}

static dim3 cgrid(int64_t n) { return dim3((unsigned)((n + kCoarseThreads - 1) / kCoarseThreads)); }

hipError_t coarse_restrict(const DevCoarse& C, int R, const double* r, double* c, hipStream_t s) {
  if (C.n <= 0) return hipSuccess;
  if (R == 1) hipLaunchKernelGGL(k_coarse_restrict<1>, dim3(C.n), dim3(kCoarseThreads), 0, s, C, r, c);
  else if (R == 2) hipLaunchKernelGGL(k_coarse_restrict<2>, dim3(C.n), dim3(kCoarseThreads), 0, s, C, r, c);
  else if (R == 4) hipLaunchKernelGGL(k_coarse_restrict<4>, dim3(C.n), dim3(kCoarseThreads), 0, s, C, r, c);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t coarse_solve(const DevCoarse& C, int R, const double* c, double* e, hipStream_t s) {
  if (C.n <= 0) return hipSuccess;
  const dim3 g((unsigned)((C.n + kCoarseThreads / 64 - 1) / (kCoarseThreads / 64)));
  if (R == 1) hipLaunchKernelGGL(k_coarse_solve<1>, g, dim3(kCoarseThreads), 0, s, C, c, e);
  else if (R == 2) hipLaunchKernelGGL(k_coarse_solve<2>, g, dim3(kCoarseThreads), 0, s, C, c, e);
  else if (R == 4) hipLaunchKernelGGL(k_coarse_solve<4>, g, dim3(kCoarseThreads), 0, s, C, c, e);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t coarse_prolong(const DevCoarse& C, int R, const double* e, double* z, bool add, hipStream_t s) {
  if (C.n <= 0 || C.nA <= 0) return hipSuccess;
  if (R == 1) hipLaunchKernelGGL(k_coarse_prolong<1>, cgrid(C.nA), dim3(kCoarseThreads), 0, s, C, e, z, add ? 1 : 0);
  else if (R == 2) hipLaunchKernelGGL(k_coarse_prolong<2>, cgrid(C.nA), dim3(kCoarseThreads), 0, s, C, e, z, add ? 1 : 0);
  else if (R == 4) hipLaunchKernelGGL(k_coarse_prolong<4>, cgrid(C.nA), dim3(kCoarseThreads), 0, s, C, e, z, add ? 1 : 0);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t coarse_indicators(const DevCoarse& C, int j0, double* x, hipStream_t s) {
  if (C.nA <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_coarse_indicators, cgrid(C.nA), dim3(kCoarseThreads), 0, s, C, j0, x);
  return hipGetLastError();
}

hipError_t coarse_sub(int64_t n, const double* a, const double* b, double* y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_coarse_sub, cgrid(n), dim3(kCoarseThreads), 0, s, n, a, b, y);
  return hipGetLastError();
}

}  // namespace cpm
