// IMEX-Euler right-hand sides of the Gray-Scott system on a surface (paper
// Sec. 1, eq. rdsys; Sec. 4.1.5, eq. grayscott): the reaction is explicit and
// the diffusion implicit, so each species w solves
//   (1/(mu_w dt) - Lap_S^h) w^{n+1} = (w^n/dt + R_w(u^n, v^n)) / mu_w
// with R_u = -u v^2 + F (1 - u), R_v = u v^2 - (F + k) v.
#include <hip/hip_runtime.h>

#include "common.h"

namespace cpm {

__global__ void k_gray_scott_rhs(int64_t n, const double* __restrict__ u, const double* __restrict__ v, double F,
                                 double k, double inv_dt, double inv_mu_u, double inv_mu_v, double* __restrict__ fu,
                                 double* __restrict__ fv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = u[i], b = v[i];
  const double abb = a * b * b;
  fu[i] = (a * inv_dt + (-abb + F * (1.0 - a))) * inv_mu_u;
  fv[i] = (b * inv_dt + (abb - (F + k) * b)) * inv_mu_v;
}

}  // namespace cpm

using namespace cpm;

cpm_status cpm_gray_scott_rhs(int64_t n, const double* u, const double* v, double F, double k, double dt,
                              double mu_u, double mu_v, double* fu, double* fv, void* stream) {
  if (n < 0 || (n > 0 && (!u || !v || !fu || !fv)) || !(dt > 0) || !(mu_u > 0) || !(mu_v > 0)) {
    set_error("cpm_gray_scott_rhs: bad argument");
    return CPM_ERR_ARG;
  }
  if (n == 0) return CPM_OK;
  hipLaunchKernelGGL(k_gray_scott_rhs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream, n, u, v,
                     F, k, 1.0 / dt, 1.0 / mu_u, 1.0 / mu_v, fu, fv);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("cpm_gray_scott_rhs: ") + hipGetErrorString(e));
    return CPM_ERR_DEVICE;
  }
  return CPM_OK;
}
