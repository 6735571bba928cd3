// Batched FGMRES building blocks (Sec. 4.1.1: GMRES is the default Krylov
// method). Vectors of several systems are packed: instance i owns nodes
// [off_i, off_i + nA_i) of every packed vector, each node holding R
// interleaved right-hand sides; system s = i*R + r. Reductions are
// deterministic: each chunk (a contiguous slice of one instance) writes its
// partial sums, and a second kernel adds a system's chunks in a fixed order.
#include <hip/hip_runtime.h>

#include "krylov.h"

// Vector kernels are bandwidth-bound: keep multiply and add separate so that
// every right-hand-side count rounds identically (a batch of R systems
// reproduces each solo solve bit for bit).
#pragma clang fp contract(off)

namespace cpm {

constexpr int kVecThreads = 256;
// chunk count (of kChunkNodes nodes) from which the dot kernel groups basis vectors
constexpr int kDotsGroupChunks = 4096;

template <int R>
__device__ __forceinline__ bool inst_active(const int32_t* act, int inst) {
  bool a = false;
#pragma unroll
  for (int r = 0; r < R; ++r) a = a || act[inst * R + r];
  return a;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// block-wide sum of R accumulators (fixed order); result valid in thread 0
template <int R>
__device__ __forceinline__ void block_sum(double* acc, double* red) {
  const int lane = __lane_id(), wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    double v = wave_sum(acc[r]);
    if (lane == 0) red[wave * R + r] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      double s = 0;
      for (int q = 0; q < nw; ++q) s += red[q * R + r];
      acc[r] = s;
    }
  }
}

// part[(i*nchunks + c)*R + r] = <V_i, w> over chunk c, for the MB basis
// vectors i = blockIdx.y*MB + b < m of this block. Every (i, c) sum is formed
// in the same order whatever MB is (thread t adds nodes t, t + blockDim, ...,
// then the fixed block reduction), so MB only trades blocks for reuse of w.
template <int R, int MB>
__global__ void __launch_bounds__(kVecThreads) k_dots(const double* __restrict__ V0, int64_t vstride,
                                                      const double* __restrict__ w, const Chunk* __restrict__ chunks,
                                                      int nchunks, int m, const int32_t* __restrict__ act,
                                                      double* __restrict__ part) {
  __shared__ double red[16 * R * MB];
  const int c = blockIdx.x, i0 = blockIdx.y * MB;
  const Chunk ch = chunks[c];
  if (!inst_active<R>(act, ch.inst)) {   // uniform over the block: a stopped instance's sums are 0
    if (threadIdx.x == 0) {
#pragma unroll
      for (int b = 0; b < MB; ++b)
        if (i0 + b < m) {
#pragma unroll
          for (int r = 0; r < R; ++r) part[((int64_t)(i0 + b) * nchunks + c) * R + r] = 0.0;
        }
    }
    return;
  }
  double acc[MB * R];
#pragma unroll
  for (int k = 0; k < MB * R; ++k) acc[k] = 0.0;
  {
    for (int64_t n = threadIdx.x; n < ch.nodes; n += blockDim.x) {
      const int64_t e = (ch.node0 + n) * R;
      double wv[R];
#pragma unroll
      for (int r = 0; r < R; ++r) wv[r] = w[e + r];
#pragma unroll
      for (int b = 0; b < MB; ++b) {
        if (i0 + b < m) {
          const double* v = V0 + (int64_t)(i0 + b) * vstride;
#pragma unroll
          for (int r = 0; r < R; ++r) acc[b * R + r] += v[e + r] * wv[r];
        }
      }
    }
  }
  block_sum<MB * R>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int b = 0; b < MB; ++b)
      if (i0 + b < m) {
#pragma unroll
        for (int r = 0; r < R; ++r) part[((int64_t)(i0 + b) * nchunks + c) * R + r] = acc[b * R + r];
      }
  }
}

// out[s*ld + i] (= or +=) sum over the chunks of inst(s) of part[(i*nchunks + c)*R + r].
// One wavefront per (s, i): lane l adds chunks l, l+64, ... in order, then a
// fixed butterfly over the lanes; the order depends only on the instance's
// chunk count, so a batch reproduces each solo solve.
template <int R>
__global__ void __launch_bounds__(256) k_reduce(const double* __restrict__ part, int m, int nchunks,
                                                const int32_t* __restrict__ cbeg, int ns, double* __restrict__ out,
                                                int ld, double* __restrict__ accum, int accum_ld) {
  const int t = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (t >= ns * m) return;   // uniform over the wavefront
  const int lane = __lane_id();
  const int s = t / m, i = t % m;
  const int inst = s / R, r = s % R;
  const double* pp = part + (int64_t)i * nchunks * R + r;
  const int c0 = cbeg[inst], c1 = cbeg[inst + 1];
  double sum = 0.0;
  for (int c = c0 + lane; c < c1; c += 64) sum += pp[(int64_t)c * R];
  sum = wave_sum(sum);
  if (lane == 0) {
    out[(int64_t)s * ld + i] = sum;
    if (accum) accum[(int64_t)s * accum_ld + i] += sum;
  }
}

// w -= sum_{i<m} hv[s][i] V_i; optionally norm partials of the new w
template <int R>
__global__ void __launch_bounds__(kVecThreads) k_update(const double* __restrict__ V0, int64_t vstride, int m,
                                                        double* __restrict__ w, const Chunk* __restrict__ chunks,
                                                        const int32_t* __restrict__ act, const double* __restrict__ hv,
                                                        int ld, double* __restrict__ part_norm) {
  __shared__ double red[16 * R];
  __shared__ double hs[kMaxRestart * R];
  const int c = blockIdx.x;
  const Chunk ch = chunks[c];
  if (!inst_active<R>(act, ch.inst)) {   // uniform over the block: nothing to update, norms 0
    if (part_norm && threadIdx.x == 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) part_norm[(int64_t)c * R + r] = 0.0;
    }
    return;
  }
  bool on[R];
#pragma unroll
  for (int r = 0; r < R; ++r) on[r] = act[ch.inst * R + r] != 0;
  for (int t = threadIdx.x; t < m * R; t += blockDim.x) {
    const int i = t / R, r = t % R;
    hs[t] = hv[(int64_t)(ch.inst * R + r) * ld + i];
  }
  __syncthreads();
  double acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
  if (inst_active<R>(act, ch.inst)) {
    for (int64_t n = threadIdx.x; n < ch.nodes; n += blockDim.x) {
      const int64_t e = (ch.node0 + n) * R;
      double v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = w[e + r];
      for (int i = 0; i < m; ++i) {
        const double* vi = V0 + (int64_t)i * vstride + e;
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] -= hs[i * R + r] * vi[r];
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (on[r]) w[e + r] = v[r];
        acc[r] += on[r] ? v[r] * v[r] : 0.0;
      }
    }
  }
  if (part_norm) {
    block_sum<R>(acc, red);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) part_norm[(int64_t)c * R + r] = acc[r];
    }
  }
}

// out = a * x (per system scale a[s]) for active systems
template <int R>
__global__ void __launch_bounds__(kVecThreads) k_scale(const double* __restrict__ x, double* __restrict__ out,
                                                       const Chunk* __restrict__ chunks, const int32_t* __restrict__ act,
                                                       const double* __restrict__ a) {
  const Chunk ch = chunks[blockIdx.x];
  if (!inst_active<R>(act, ch.inst)) return;
  double sc[R];
  bool on[R];
#pragma unroll
  for (int r = 0; r < R; ++r) { sc[r] = a[ch.inst * R + r]; on[r] = act[ch.inst * R + r] != 0; }
  for (int64_t n = threadIdx.x; n < ch.nodes; n += blockDim.x) {
    const int64_t e = (ch.node0 + n) * R;
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (on[r]) out[e + r] = sc[r] * x[e + r];
  }
}

// out = x for instances flagged in copy_inst (instances without a preconditioner)
template <int R>
__global__ void __launch_bounds__(kVecThreads) k_copy(const double* __restrict__ x, double* __restrict__ out,
                                                      const Chunk* __restrict__ chunks,
                                                      const int32_t* __restrict__ copy_inst) {
  const Chunk ch = chunks[blockIdx.x];
  if (!copy_inst[ch.inst]) return;
  for (int64_t n = threadIdx.x; n < ch.nodes; n += blockDim.x) {
    const int64_t e = (ch.node0 + n) * R;
#pragma unroll
    for (int r = 0; r < R; ++r) out[e + r] = x[e + r];
  }
}

// r = f - t and norm partials of r (all systems); or norm partials of f when t == nullptr
template <int R>
__global__ void __launch_bounds__(kVecThreads) k_residual(const double* __restrict__ f, const double* __restrict__ t,
                                                          double* __restrict__ r, const Chunk* __restrict__ chunks,
                                                          double* __restrict__ part) {
  __shared__ double red[16 * R];
  const int c = blockIdx.x;
  const Chunk ch = chunks[c];
  double acc[R];
#pragma unroll
  for (int q = 0; q < R; ++q) acc[q] = 0.0;
  for (int64_t n = threadIdx.x; n < ch.nodes; n += blockDim.x) {
    const int64_t e = (ch.node0 + n) * R;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      double v = t ? f[e + q] - t[e + q] : f[e + q];
      if (r) r[e + q] = v;
      acc[q] += v * v;
    }
  }
  block_sum<R>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < R; ++q) part[(int64_t)c * R + q] = acc[q];
  }
}

// x += sum_{i < steps[s]} y[s][i] Z_i
template <int R>
__global__ void __launch_bounds__(kVecThreads) k_xupdate(double* __restrict__ x, const double* __restrict__ Z0,
                                                         int64_t zstride, const Chunk* __restrict__ chunks,
                                                         const int32_t* __restrict__ steps, const double* __restrict__ y,
                                                         int ld) {
  __shared__ double ys[kMaxRestart * R];
  __shared__ int ks[R];
  const Chunk ch = chunks[blockIdx.x];
  int kmax = 0;
  for (int t = threadIdx.x; t < kMaxRestart * R; t += blockDim.x) {
    const int i = t / R, r = t % R;
    const int s = ch.inst * R + r;
    ys[t] = i < steps[s] ? y[(int64_t)s * ld + i] : 0.0;
  }
  if (threadIdx.x < R) ks[threadIdx.x] = steps[ch.inst * R + threadIdx.x];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < R; ++r) kmax = max(kmax, ks[r]);
  if (kmax == 0) return;
  for (int64_t n = threadIdx.x; n < ch.nodes; n += blockDim.x) {
    const int64_t e = (ch.node0 + n) * R;
    double v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = x[e + r];
    for (int i = 0; i < kmax; ++i) {
      const double* zi = Z0 + (int64_t)i * zstride + e;
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] += ys[i * R + r] * zi[r];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) x[e + r] = v[r];
  }
}

// Arnoldi column j of every active system: Givens rotations and the residual
// estimate. The column accumulated by the two Gram-Schmidt passes is consumed
// and cleared here (and at each cycle start), ready for the next step.
__global__ void k_givens(GmresState S, int j, int ns) {
  __shared__ int cnt[1024 / 64];
  const int s = threadIdx.x;
  int alive = 0;
  if (s < ns && S.act[s]) {
    const int m = S.m, ldh = m + 1;
    double* __restrict__ Hj = S.H + (int64_t)s * ldh * m + (int64_t)j * ldh;
    double* g = S.g + (int64_t)s * (m + 1);
    double* __restrict__ cs = S.cs + (int64_t)s * m;
    double* __restrict__ sn = S.sn + (int64_t)s * m;
    double* __restrict__ col = S.hcol + (int64_t)s * (m + 1);
    const double hn = sqrt(S.nrm2[s]);
    // earlier rotations applied to the new column; only the running entry is
    // carried, the other operands are independent loads
    double carry = col[0];
    for (int i = 0; i < j; ++i) {
      const double b = col[i + 1], c = cs[i], sv = sn[i];
      Hj[i] = c * carry + sv * b;
      carry = -sv * carry + c * b;
    }
    for (int i = 0; i <= j; ++i) col[i] = 0.0;
    const double a = carry, b = hn;
    const double den = hypot(a, b);
    const double c = den > 0 ? a / den : 1.0, sv = den > 0 ? b / den : 0.0;
    cs[j] = c;
    sn[j] = sv;
    Hj[j] = den;
    Hj[j + 1] = 0.0;
    g[j + 1] = -sv * g[j];
    g[j] = c * g[j];
    S.steps[s] = j + 1;
    S.scale[s] = hn > 0 ? 1.0 / hn : 0.0;
    const double est = fabs(g[j + 1]);
    S.est[s] = est;
    bool finite = isfinite(hn) && isfinite(est) && isfinite(den);
    if (!finite) S.bad[s] = 1;
    if (!finite || est <= S.tol_in[s] || hn == 0.0 || den == 0.0 || j + 1 >= m || j + 1 >= S.budget[s])
      S.act[s] = 0;
    else alive = 1;
  }
  // count active systems (fixed order)
  const int lane = __lane_id(), wave = threadIdx.x >> 6;
  unsigned long long b = __ballot(alive);
  if (lane == 0) cnt[wave] = __popcll(b);
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) tot += cnt[q];
    *S.n_active = tot;
  }
}

// back substitution H y = g for each system with steps > 0
__global__ void k_hsolve(GmresState S, int ns) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  const int k = S.steps[s], m = S.m, ldh = m + 1;
  const double* H = S.H + (int64_t)s * ldh * m;
  const double* g = S.g + (int64_t)s * (m + 1);
  double* y = S.y + (int64_t)s * m;
  for (int i = k - 1; i >= 0; --i) {
    double v = g[i];
    for (int q = i + 1; q < k; ++q) v -= H[i + q * ldh] * y[q];
    y[i] = H[i + i * ldh] != 0.0 ? v / H[i + i * ldh] : 0.0;
  }
}

// start of a cycle: g = (beta, 0, ...), hcol = 0, steps = 0, scale = 1/beta
__global__ void k_cycle_init(GmresState S, int ns) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  const int m = S.m;
  double* g = S.g + (int64_t)s * (m + 1);
  double* col = S.hcol + (int64_t)s * (m + 1);
  for (int i = 0; i <= m; ++i) g[i] = 0.0;
  for (int i = 0; i <= m; ++i) col[i] = 0.0;
  g[0] = S.beta[s];
  S.steps[s] = 0;
  S.scale[s] = S.beta[s] > 0 ? 1.0 / S.beta[s] : 0.0;
}

// ---------------------------------------------------------------- launchers
#define CPM_R_DISPATCH(R, ...) \
  switch (R) { \
    case 1: { constexpr int RR = 1; __VA_ARGS__; break; } \
    case 2: { constexpr int RR = 2; __VA_ARGS__; break; } \
    case 4: { constexpr int RR = 4; __VA_ARGS__; break; } \
    default: return hipErrorInvalidValue; \
  }

hipError_t vec_dots(int R, const double* V0, int64_t vstride, int m, const double* w, const Chunk* chunks,
                    int nchunks, const int32_t* act, double* part, hipStream_t s) {
  if (nchunks == 0 || m == 0) return hipSuccess;
  // Large packed vectors: one block per chunk and group of 8 basis vectors, so
  // that w is read once per group and the launch holds 8x fewer blocks; small
  // ones keep a block per (chunk, vector) to fill the chip.
  if (nchunks >= kDotsGroupChunks) {
    CPM_R_DISPATCH(R, hipLaunchKernelGGL((k_dots<RR, 8>), dim3(nchunks, (m + 7) / 8), dim3(kVecThreads), 0, s, V0,
                                         vstride, w, chunks, nchunks, m, act, part));
  } else {
    CPM_R_DISPATCH(R, hipLaunchKernelGGL((k_dots<RR, 1>), dim3(nchunks, m), dim3(kVecThreads), 0, s, V0, vstride,
                                         w, chunks, nchunks, m, act, part));
  }
  return hipGetLastError();
}

hipError_t vec_reduce(int R, const double* part, int m, int nchunks, const int32_t* cbeg, int ns, double* out,
                      int ld, double* accum, int accum_ld, hipStream_t s) {
  const int n = ns * m;
  if (n == 0) return hipSuccess;
  CPM_R_DISPATCH(R, hipLaunchKernelGGL((k_reduce<RR>), dim3((n + 3) / 4), dim3(256), 0, s, part, m, nchunks,
                                       cbeg, ns, out, ld, accum, accum_ld));
  return hipGetLastError();
}

hipError_t vec_update(int R, const double* V0, int64_t vstride, int m, double* w, const Chunk* chunks, int nchunks,
                      const int32_t* act, const double* hv, int ld, double* part_norm, hipStream_t s) {
  if (nchunks == 0) return hipSuccess;
  CPM_R_DISPATCH(R, hipLaunchKernelGGL((k_update<RR>), dim3(nchunks), dim3(kVecThreads), 0, s, V0, vstride, m, w,
                                       chunks, act, hv, ld, part_norm));
  return hipGetLastError();
}

hipError_t vec_scale(int R, const double* x, double* out, const Chunk* chunks, int nchunks, const int32_t* act,
                     const double* a, hipStream_t s) {
  if (nchunks == 0) return hipSuccess;
  CPM_R_DISPATCH(R, hipLaunchKernelGGL((k_scale<RR>), dim3(nchunks), dim3(kVecThreads), 0, s, x, out, chunks, act, a));
  return hipGetLastError();
}

hipError_t vec_copy(int R, const double* x, double* out, const Chunk* chunks, int nchunks, const int32_t* copy_inst,
                    hipStream_t s) {
  if (nchunks == 0) return hipSuccess;
  CPM_R_DISPATCH(R, hipLaunchKernelGGL((k_copy<RR>), dim3(nchunks), dim3(kVecThreads), 0, s, x, out, chunks, copy_inst));
  return hipGetLastError();
}

hipError_t vec_residual(int R, const double* f, const double* t, double* r, const Chunk* chunks, int nchunks,
                        double* part, hipStream_t s) {
  if (nchunks == 0) return hipSuccess;
  CPM_R_DISPATCH(R, hipLaunchKernelGGL((k_residual<RR>), dim3(nchunks), dim3(kVecThreads), 0, s, f, t, r, chunks, part));
  return hipGetLastError();
}

hipError_t vec_xupdate(int R, double* x, const double* Z0, int64_t zstride, const Chunk* chunks, int nchunks,
                       const int32_t* steps, const double* y, int ld, hipStream_t s) {
  if (nchunks == 0) return hipSuccess;
  CPM_R_DISPATCH(R, hipLaunchKernelGGL((k_xupdate<RR>), dim3(nchunks), dim3(kVecThreads), 0, s, x, Z0, zstride,
                                       chunks, steps, y, ld));
  return hipGetLastError();
}

hipError_t gmres_givens(const GmresState& S, int j, int ns, hipStream_t s) {
  hipLaunchKernelGGL(k_givens, dim3(1), dim3(((ns + 63) / 64) * 64), 0, s, S, j, ns);
  return hipGetLastError();
}

hipError_t gmres_hsolve(const GmresState& S, int ns, hipStream_t s) {
  hipLaunchKernelGGL(k_hsolve, dim3((ns + 63) / 64), dim3(64), 0, s, S, ns);
  return hipGetLastError();
}

hipError_t gmres_cycle_init(const GmresState& S, int ns, hipStream_t s) {
  hipLaunchKernelGGL(k_cycle_init, dim3((ns + 63) / 64), dim3(64), 0, s, S, ns);
  return hipGetLastError();
}

}  // namespace cpm
