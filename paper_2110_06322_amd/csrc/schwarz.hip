// (O)RAS preconditioner apply, z = sum_j Rt_j^T U_j^-1 L_j^-1 R_j r (paper Sec. 2.2,
// restricted recombination on the disjoint pieces): one workgroup per
// subdomain (and instance). The local vector lives in LDS; both triangular
// solves run without barriers: wavefront w takes positions w, w+16, ... of a
// level schedule (a topological order of the sweep), one lane per stored
// entry, waits on per-row completion flags (LDS acquire/release), and
// publishes its row after a fixed-order wavefront reduction. The earliest
// unfinished schedule position always has all its inputs, so the sweep always
// advances; a bounded wait sets an error flag instead of spinning forever. Only rows the
// subdomain owns are written back: no two workgroups write the same entry.
#include <hip/hip_runtime.h>

#include "schwarz.h"

namespace cpm {

constexpr int kSchwarzThreads = 1024;
constexpr int kSpinLimit = 1 << 22;

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ bool wait_flag(int* f, int level, int32_t* err) {
  int spins = 0;
  while (__hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < level) {
    __builtin_amdgcn_s_sleep(1);
    if (++spins > kSpinLimit) {
      __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
  }
  return true;
}

// One triangular sweep. The rows follow a level schedule (a topological order
// of the sweep's dependencies); wavefront `wave` takes schedule positions
// wave, wave+nw, ...; the pointers and first 64 entries of its next row are
// loaded while the current row waits for its inputs.
template <class T, int NRHS, bool BACKWARD>
__device__ __forceinline__ void sweep(int n, int wave, int nw, int lane, const uint16_t* __restrict__ sched,
                                      const int64_t* __restrict__ ptr,
                                      const uint16_t* __restrict__ col, const T* __restrict__ val,
                                      const T* __restrict__ dinv, T* xv, int* done, int32_t* err) {
  constexpr int LEVEL = BACKWARD ? 2 : 1;
  int i = 0;
  auto row_of = [&](int it) { const int pos = wave + it * nw; return pos < n ? (int)sched[pos] : 0; };
  int q = row_of(0);
  bool valid = wave < n;
  int64_t b = 0, e = 0;
  int k = -1;
  T v = (T)0, dq = (T)0;
  if (valid) {
    b = ptr[q];
    e = ptr[q + 1];
    if (b + lane < e) { k = col[b + lane]; v = val[b + lane]; }
    if (BACKWARD) dq = dinv[q];
  }
  while (valid) {
    // prefetch the next row of this wavefront
    const int qn = row_of(i + 1);
    const bool nvalid = wave + (i + 1) * nw < n;
    int64_t bn = 0, en = 0;
    T dn = (T)0;
    if (nvalid) {
      bn = ptr[qn];
      en = ptr[qn + 1];
      if (BACKWARD) dn = dinv[qn];
    }
    T acc[NRHS];
#pragma unroll
    for (int r = 0; r < NRHS; ++r) acc[r] = (T)0;
    if (k >= 0) {
      wait_flag(&done[k], LEVEL, err);
#pragma unroll
      for (int r = 0; r < NRHS; ++r) acc[r] += v * xv[k * NRHS + r];
    }
    for (int64_t t = b + 64 + lane; t < e; t += 64) {   // rows longer than a wavefront
      const int kk = col[t];
      const T vv = val[t];
      wait_flag(&done[kk], LEVEL, err);
#pragma unroll
      for (int r = 0; r < NRHS; ++r) acc[r] += vv * xv[kk * NRHS + r];
    }
    int kn = -1;
    T vn = (T)0;
    if (nvalid && bn + lane < en) { kn = col[bn + lane]; vn = val[bn + lane]; }
#pragma unroll
    for (int r = 0; r < NRHS; ++r) acc[r] = wave_sum(acc[r]);
    if (lane == 0) {
      if (BACKWARD) {
#pragma unroll
        for (int r = 0; r < NRHS; ++r) xv[q * NRHS + r] = (xv[q * NRHS + r] - acc[r]) * dq;
      } else {
#pragma unroll
        for (int r = 0; r < NRHS; ++r) xv[q * NRHS + r] -= acc[r];
      }
      __hip_atomic_store(&done[q], LEVEL, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    q = qn;
    valid = nvalid;
    b = bn;
    e = en;
    k = kn;
    v = vn;
    dq = dn;
    ++i;
  }
}

template <class T, int NRHS>
__global__ void __launch_bounds__(kSchwarzThreads) k_schwarz(const DevPC* __restrict__ pcs,
                                                            const WorkItem* __restrict__ work, int nwork,
                                                            const double* __restrict__ rin, double* __restrict__ zout) {
  extern __shared__ double smem_d[];
  if ((int)blockIdx.x >= nwork) return;
  const WorkItem wi = work[blockIdx.x];
  const DevPC& P = pcs[wi.inst];
  const DevSub sub = P.subs[wi.idx];
  const int n = sub.n;
  T* xv = reinterpret_cast<T*>(smem_d);
  int* done = reinterpret_cast<int*>(xv + (size_t)n * NRHS);
  const int tid = threadIdx.x, wave = tid >> 6, lane = __lane_id(), nw = blockDim.x >> 6;
  const int32_t* in_idx = P.in_idx + sub.row_off;
  const int32_t* out_idx = P.out_idx + sub.row_off;
  const int64_t* lp = P.lptr + sub.ptr_off;
  const int64_t* up = P.uptr + sub.ptr_off;
  const T* lv = reinterpret_cast<const T*>(P.lval);
  const T* uv = reinterpret_cast<const T*>(P.uval);
  const T* di = reinterpret_cast<const T*>(P.dinv) + sub.row_off;
  const double* rb = rin + P.vec_off * NRHS;
  double* zb = zout + P.vec_off * NRHS;

  for (int q = tid; q < n; q += blockDim.x) {
    const int64_t g = in_idx[q];
#pragma unroll
    for (int r = 0; r < NRHS; ++r) xv[q * NRHS + r] = (T)rb[g * NRHS + r];
    done[q] = 0;
  }
  __syncthreads();

  // forward: y_q = r_q - sum_{k<q} l_qk y_k (unit lower triangle)
  sweep<T, NRHS, false>(n, wave, nw, lane, P.schedL + sub.row_off, lp, P.lcol, lv, nullptr, xv, done,
                        P.error_flag);
  __syncthreads();
  // backward: z_q = (y_q - sum_{k>q} u_qk z_k) / u_qq
  sweep<T, NRHS, true>(n, wave, nw, lane, P.schedU + sub.row_off, up, P.ucol, uv, di, xv, done,
                       P.error_flag);
  __syncthreads();

  for (int q = tid; q < n; q += blockDim.x) {
    const int32_t o = out_idx[q];
    if (o < 0) {
      const int64_t g = o & 0x7fffffff;
#pragma unroll
      for (int r = 0; r < NRHS; ++r) zb[g * NRHS + r] = (double)xv[q * NRHS + r];
    }
  }
}

template <class T, int NRHS>
static hipError_t launch_t(const DevPC* pcs, const WorkItem* work, int nwork, int max_rows, const double* r,
                           double* z, hipStream_t s) {
  const size_t shm = (size_t)max_rows * (NRHS * sizeof(T) + sizeof(int));
  int dev = 0, lim = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (shm > (size_t)lim) return hipErrorInvalidConfiguration;
  if (shm > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k_schwarz<T, NRHS>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)shm);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_schwarz<T, NRHS>), dim3(nwork), dim3(kSchwarzThreads), shm, s, pcs, work, nwork, r, z);
  return hipGetLastError();
}

hipError_t launch_schwarz(const DevPC* pcs, const WorkItem* work, int nwork, int max_rows, int fp32, int nrhs,
                          const double* r, double* z, hipStream_t s) {
  if (nwork == 0) return hipSuccess;
  if (fp32) {
    if (nrhs == 1) return launch_t<float, 1>(pcs, work, nwork, max_rows, r, z, s);
    if (nrhs == 2) return launch_t<float, 2>(pcs, work, nwork, max_rows, r, z, s);
    if (nrhs == 4) return launch_t<float, 4>(pcs, work, nwork, max_rows, r, z, s);
  } else {
    if (nrhs == 1) return launch_t<double, 1>(pcs, work, nwork, max_rows, r, z, s);
    if (nrhs == 2) return launch_t<double, 2>(pcs, work, nwork, max_rows, r, z, s);
    if (nrhs == 4) return launch_t<double, 4>(pcs, work, nwork, max_rows, r, z, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace cpm
