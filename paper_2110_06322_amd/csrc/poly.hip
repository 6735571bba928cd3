// Operator algebra (Sec. 3.1.2 grid functions: the identity and the
// Laplace-Beltrami operator added and composed; Sec. 4.1.2: the shifted
// biharmonic c + Lap_S^2). Sums and compositions of these are polynomials
// P(L) = sum_k a_k L^k in L = Lap_S^h, applied matrix-free by repeated
// operator applies: with the stabilized operator A(c) = c I - L of the band,
// L v = c v - A(c) v, so every power costs one fused apply and one
// elementwise pass:
//   y = a_0 x;  v_0 = x;  v_k = c v_{k-1} - A v_{k-1};  y += a_k v_k.
#include <hip/hip_runtime.h>

#include "common.h"
#include "krylov.h"

#pragma clang fp contract(off)

namespace cpm {

constexpr int kPolyThreads = 256;

__global__ void __launch_bounds__(kPolyThreads) k_poly_scale(int64_t n, double a, const double* __restrict__ x,
                                                            double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * kPolyThreads + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

// vn = c v - av (vn may alias av); y += a vn
__global__ void __launch_bounds__(kPolyThreads) k_poly_step(int64_t n, double c, double a, const double* v,
                                                           const double* av, double* vn, double* y) {
  const int64_t i = (int64_t)blockIdx.x * kPolyThreads + threadIdx.x;
  if (i >= n) return;
  const double w = c * v[i] - av[i];
  vn[i] = w;
  y[i] = y[i] + a * w;
}

// the same step over the packed vectors of a batch (R interleaved right-hand sides per
// node), with each chunk's instance shift
__global__ void __launch_bounds__(kPolyThreads) k_poly_step_chunks(int R, const Chunk* __restrict__ chunks,
                                                                  const double* __restrict__ shift, double a,
                                                                  const double* v, const double* av, double* vn,
                                                                  double* y) {
  const Chunk ch = chunks[blockIdx.x];
  const double c = shift[ch.inst];
  const int64_t e0 = ch.node0 * R, ne = ch.nodes * R;
  for (int64_t k = threadIdx.x; k < ne; k += kPolyThreads) {
    const int64_t i = e0 + k;
    const double w = c * v[i] - av[i];
    vn[i] = w;
    y[i] = y[i] + a * w;
  }
}

static dim3 pgrid(int64_t n) { return dim3((unsigned)((n + kPolyThreads - 1) / kPolyThreads)); }

hipError_t poly_scale(int64_t n, double a, const double* x, double* y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_poly_scale, pgrid(n), dim3(kPolyThreads), 0, s, n, a, x, y);
  return hipGetLastError();
}

hipError_t poly_step(int64_t n, double c, double a, const double* v, const double* av, double* vn, double* y,
                     hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_poly_step, pgrid(n), dim3(kPolyThreads), 0, s, n, c, a, v, av, vn, y);
  return hipGetLastError();
}

hipError_t poly_step_chunks(int R, const Chunk* chunks, int nchunks, const double* shift, double a, const double* v,
                            const double* av, double* vn, double* y, hipStream_t s) {
  if (nchunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_poly_step_chunks, dim3(nchunks), dim3(kPolyThreads), 0, s, R, chunks, shift, a, v, av, vn, y);
  return hipGetLastError();
}

}  // namespace cpm

using namespace cpm;

cpm_status cpm_poly_apply(const cpm_operator* op, int32_t ncoef, const double* coef, const double* x, double* y,
                          int32_t nrhs, void* stream) {
  try {
    if (!op || !coef || !x || !y) fail(CPM_ERR_ARG, "null argument");
    if (ncoef < 1 || ncoef > kMaxPoly) fail(CPM_ERR_ARG, "ncoef must be in 1..5");
    if (nrhs != 1 && nrhs != 2 && nrhs != 4) fail(CPM_ERR_ARG, "nrhs must be 1, 2 or 4");
    if (x == y) fail(CPM_ERR_ARG, "x and y must not alias");
    for (int k = 0; k < ncoef; ++k)
      if (!std::isfinite(coef[k])) fail(CPM_ERR_ARG, "non-finite coefficient");
    const hipStream_t s = (hipStream_t)stream;
    const int64_t n = op->band->nA * nrhs;
    hip_check(poly_scale(n, coef[0], x, y, s), "cpm_poly_apply");
    if (ncoef == 1) return CPM_OK;
    op->d_poly.alloc((size_t)n * 2);
    const int variant = (nrhs == 1 && op->apply_variant == kApplyTwoPass && !op->twopass) ? kApplyPipelined
                                                                                         : op->apply_variant;
    // v_k lives in buffer (k - 1) mod 2: the apply of v_{k-1} writes A v_{k-1} there and the
    // step overwrites it in place with v_k
    const double* v = x;
    for (int k = 1; k < ncoef; ++k) {
      double* buf = op->d_poly.p + (size_t)((k - 1) & 1) * n;
      hip_check(launch_apply(op->apply_args(), nrhs, variant, v, buf, s), "cpm_poly_apply");
      hip_check(poly_step(n, op->c, coef[k], v, buf, buf, y, s), "cpm_poly_apply");
      v = buf;
    }
    return CPM_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  }
}
