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

#include <type_traits>

#include "schwarz.h"

namespace cpm {

constexpr int kSchwarzThreads = 1024;

// true when the gate says instance `inst` has nothing to do
__device__ __forceinline__ bool gate_skip(const Gate& g, int inst) {
  if (g.count && *g.count == 0) return true;
  if (g.act) {
    int any = 0;
    for (int r = 0; r < g.nrhs; ++r) any |= g.act[inst * g.nrhs + r];
    return any == 0;
  }
  return false;
}

constexpr int kSpinLimit = 1 << 22;

// a bounded wait that expired: the error flag is set with a global store (a flat
// store would stay pending in both memory counters and make every later wait of
// the sweep drain all loads in flight)
__device__ __forceinline__ void set_error(int32_t* err) {
  __hip_atomic_store((__attribute__((address_space(1))) int32_t*)err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

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
      set_error(err);
      return false;
    }
  }
  return true;
}

// Wavefront sum into lane 63 with DPP: inclusive scan inside each 16-lane row
// (row_shr 1, 2, 4, 8), then the row totals are carried by row_bcast15 and
// row_bcast31. Fixed order, no LDS traffic.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int l2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWMASK, 0xf, true);
  const int h2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWMASK, 0xf, true);
  return __hiloint2double(h2, l2);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xf, true));
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_any(double v) { return dpp_d<CTRL, ROWMASK>(v); }
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_any(float v) { return dpp_f<CTRL, ROWMASK>(v); }

template <class T>
__device__ __forceinline__ T wave_sum_to_63(T v) {
  v += dpp_any<0x111, 0xf>(v);   // row_shr:1
  v += dpp_any<0x112, 0xf>(v);   // row_shr:2
  v += dpp_any<0x114, 0xf>(v);   // row_shr:4
  v += dpp_any<0x118, 0xf>(v);   // row_shr:8
  v += dpp_any<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_any<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  return v;                      // lane 63 holds the wavefront total
}

// One triangular sweep. Rows follow a level schedule (a topological order of
// the sweep's dependencies); wavefront `wave` takes schedule positions wave,
// wave+nw, .... Each position has a 64-bit record (row, length, entry offset)
// and its entries are stored in schedule order; the record two positions
// ahead and the entries one position ahead are loaded while the current row
// waits for its inputs.
template <class T, int NRHS, bool BACKWARD>
__device__ __forceinline__ void sweep(int n, int wave, int nw, int lane, const uint64_t* __restrict__ rec,
                                      const uint16_t* __restrict__ col, const T* __restrict__ val,
                                      const T* __restrict__ dinv, T* xv, int* done, int32_t* err) {
  constexpr int LEVEL = BACKWARD ? 2 : 1;
  int pos = wave;
  if (pos >= n) return;
  uint64_t r0 = rec[pos];
  uint64_t r1 = pos + nw < n ? rec[pos + nw] : 0ull;
  int k = -1;
  T v = (T)0, dq = (T)0;
  {
    const int len = (int)((r0 >> 32) & 0xffff);
    const int64_t off = (int64_t)(r0 & 0xffffffffull);
    if (lane < len) { k = col[off + lane]; v = val[off + lane]; }
    if (BACKWARD) dq = dinv[(int)(r0 >> 48)];
  }
  for (;;) {
    const int q = (int)(r0 >> 48);
    const int len = (int)((r0 >> 32) & 0xffff);
    const int64_t off = (int64_t)(r0 & 0xffffffffull);
    const bool has1 = pos + nw < n;
    // prefetch: record two ahead, entries of the next row
    const uint64_t r2 = pos + 2 * nw < n ? rec[pos + 2 * nw] : 0ull;
    int kn = -1;
    T vn = (T)0, dn = (T)0;
    if (has1) {
      const int len1 = (int)((r1 >> 32) & 0xffff);
      const int64_t off1 = (int64_t)(r1 & 0xffffffffull);
      if (lane < len1) { kn = col[off1 + lane]; vn = val[off1 + lane]; }
      if (BACKWARD) dn = dinv[(int)(r1 >> 48)];
    }
    T acc[NRHS];
#pragma unroll
    for (int r = 0; r < NRHS; ++r) acc[r] = (T)0;
    if (k >= 0) {
      wait_flag(&done[k], LEVEL, err);
#pragma unroll
      for (int r = 0; r < NRHS; ++r) acc[r] += v * xv[k * NRHS + r];
    }
    for (int t = 64 + lane; t < len; t += 64) {   // rows longer than a wavefront
      const int kk = col[off + t];
      const T vv = val[off + t];
      wait_flag(&done[kk], LEVEL, err);
#pragma unroll
      for (int r = 0; r < NRHS; ++r) acc[r] += vv * xv[kk * NRHS + r];
    }
#pragma unroll
    for (int r = 0; r < NRHS; ++r) acc[r] = wave_sum_to_63(acc[r]);
    if (lane == 63) {
      if (BACKWARD) {
#pragma unroll
        for (int r = 0; r < NRHS; ++r) xv[q * NRHS + r] = (xv[q * NRHS + r] - acc[r]) * dq;
      } else {
#pragma unroll
        for (int r = 0; r < NRHS; ++r) xv[q * NRHS + r] -= acc[r];
      }
      __hip_atomic_store(&done[q], LEVEL, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    if (!has1) break;
    pos += nw;
    r0 = r1;
    r1 = r2;
    k = kn;
    v = vn;
    dq = dn;
  }
}

template <class T, int NRHS>
__global__ void __launch_bounds__(kSchwarzThreads) k_schwarz(const DevPC* __restrict__ pcs,
                                                            const WorkItem* __restrict__ work, int nwork,
                                                            const double* __restrict__ rin, double* __restrict__ zout,
                                                            Gate gate) {
  extern __shared__ double smem_d[];
  if ((int)blockIdx.x >= nwork) return;
  const WorkItem wi = work[blockIdx.x];
  if (gate_skip(gate, wi.inst)) return;
  const DevPC& P = pcs[wi.inst];
  const DevSub sub = P.subs[wi.idx];
  const int n = sub.n;
  T* xv = reinterpret_cast<T*>(smem_d);
  int* done = reinterpret_cast<int*>(xv + (size_t)n * NRHS);
  const int tid = threadIdx.x, wave = tid >> 6, lane = __lane_id(), nw = blockDim.x >> 6;
  const int32_t* in_idx = P.in_idx + sub.row_off;
  const int32_t* out_idx = P.out_idx + sub.row_off;
  const T* lv = reinterpret_cast<const T*>(P.lval) + sub.lbase;
  const T* uv = reinterpret_cast<const T*>(P.uval) + sub.ubase;
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
  sweep<T, NRHS, false>(n, wave, nw, lane, P.recL + sub.row_off, P.lcol + sub.lbase, lv, nullptr, xv, done,
                        P.error_flag);
  __syncthreads();
  // backward: z_q = (y_q - sum_{k>q} u_qk z_k) / u_qq
  sweep<T, NRHS, true>(n, wave, nw, lane, P.recU + sub.row_off, P.ucol + sub.ubase, uv, di, xv, done,
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

// ---- value-as-flag variant
//
// The solution arrays start filled with a signalling-NaN bit pattern that no
// arithmetic produces; a row's first right-hand-side component is published
// with a release store after the others, so a waiting wavefront polls the
// value it needs and gets it in the same load. Input values are read from HBM
// by the wavefront that owns the row (no gather phase), forward results go to
// one array and backward results to another, saving one LDS round trip per
// dependency and per row against the flag-array variant.
template <class T>
struct Sentinel;
template <>
struct Sentinel<double> {
  using Bits = unsigned long long;
  static constexpr Bits kBits = 0x7ff40000deadbeefull;
};
template <>
struct Sentinel<float> {
  using Bits = unsigned int;
  static constexpr Bits kBits = 0x7fa0beefu;
};

template <class T>
__device__ __forceinline__ T bits_to(typename Sentinel<T>::Bits b) {
  T v;
  __builtin_memcpy(&v, &b, sizeof(T));
  return v;
}
template <class T>
__device__ __forceinline__ typename Sentinel<T>::Bits to_bits(T v) {
  typename Sentinel<T>::Bits b;
  __builtin_memcpy(&b, &v, sizeof(T));
  return b;
}

// wait until slot p (component 0 of a row) holds a value, return it
template <class T, bool SLEEP>
__device__ __forceinline__ T wait_value(T* p, int32_t* err) {
  using Bits = typename Sentinel<T>::Bits;
  Bits* bp = reinterpret_cast<Bits*>(p);
  int spins = 0;
  for (;;) {
    const Bits b = __hip_atomic_load(bp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (b != Sentinel<T>::kBits) {
      // acquire limited to LDS: global loads in flight (the next rows' prefetch)
      // need not complete first
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
      return bits_to<T>(b);
    }
    if (SLEEP) __builtin_amdgcn_s_sleep(1);
    if (++spins > kSpinLimit) {
      set_error(err);
      return (T)0;
    }
  }
}

template <class T, int NRHS, bool SLEEP>
__device__ __forceinline__ void dep_accumulate(const T* src, int k, T v, T* acc, int32_t* err) {
  const T x0 = wait_value<T, SLEEP>(const_cast<T*>(src) + (size_t)k * NRHS, err);
  acc[0] += v * x0;
#pragma unroll
  for (int r = 1; r < NRHS; ++r) acc[r] += v * src[(size_t)k * NRHS + r];
}

// global-memory view of a pointer: loads through it are global (vector memory
// counter only), not flat loads that also hold the LDS counter the sweeps wait on
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gmem(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}

// what one wavefront holds for one row: record, entries (two per lane) and its
// own value (forward: r_q; backward: 1/u_qq)
template <class T, int NRHS>
struct SweepRow {
  uint64_t rec;
  int k0, k1;
  T v0, v1;
  T own[NRHS];
  T dq;
};

// One sweep of the value-as-flag variant. Forward (BACKWARD = false): dst_q =
// r_q - sum_k l_qk dst_k, r_q read from HBM through the schedule-ordered input
// index. Backward: dst_q = (y_q - sum_k u_qk dst_k) * dinv_q with y from the
// forward array. Every load of the loop is unconditional (indices clamped into
// the padded arrays) and two row buffers are used in turn, so the next row's
// entries and right-hand side stay in flight while the current row waits for
// its dependencies. Rows have at most 128 entries (two per lane).
template <class T, int NRHS, bool BACKWARD, bool SLEEP>
__device__ __forceinline__ void sweep_v(int n, int wave, int nw, int lane, const uint64_t* __restrict__ rec_,
                                        const uint16_t* __restrict__ col_, const T* __restrict__ val_,
                                        const T* __restrict__ dinv_, const int32_t* __restrict__ gsched_,
                                        const double* __restrict__ rb_, const T* yv, T* dst, int32_t* err) {
  const auto rec = gmem(rec_);
  const auto col = gmem(col_);
  const auto val = gmem(val_);
  const auto dinv = gmem(dinv_);
  const auto gsched = gmem(gsched_);
  const auto rb = gmem(rb_);
  int pos = wave;
  if (pos >= n) return;
  const int last = n - 1;
  auto slot = [&](uint64_t r, int l) {
    const int len = (int)((r >> 32) & 0xffff);
    return (int64_t)(r & 0xffffffffull) + min(l, max(len - 1, 0));
  };
  auto fetch = [&](SweepRow<T, NRHS>& D, uint64_t r, int g) {
    D.rec = r;
    D.k0 = col[slot(r, lane)];
    D.k1 = col[slot(r, lane + 64)];
    D.v0 = val[slot(r, lane)];
    D.v1 = val[slot(r, lane + 64)];
    if (BACKWARD) {
      D.dq = dinv[(int)(r >> 48)];
    } else {
      D.dq = (T)0;
#pragma unroll
      for (int q = 0; q < NRHS; ++q) D.own[q] = (T)rb[(int64_t)g * NRHS + q];
    }
  };
  auto solve_row = [&](SweepRow<T, NRHS>& D) {
    const int q = (int)(D.rec >> 48);
    const int len = (int)((D.rec >> 32) & 0xffff);
    if (BACKWARD) {
#pragma unroll
      for (int r = 0; r < NRHS; ++r) D.own[r] = yv[(size_t)q * NRHS + r];   // y_q, complete before this sweep
    }
    T acc[NRHS];
#pragma unroll
    for (int r = 0; r < NRHS; ++r) acc[r] = (T)0;
    if (lane < len) dep_accumulate<T, NRHS, SLEEP>(dst, D.k0, D.v0, acc, err);
    if (lane + 64 < len) dep_accumulate<T, NRHS, SLEEP>(dst, D.k1, D.v1, acc, err);
#pragma unroll
    for (int r = 0; r < NRHS; ++r) acc[r] = wave_sum_to_63(acc[r]);
    if (lane == 63) {
      T out[NRHS];
#pragma unroll
      for (int r = 0; r < NRHS; ++r) out[r] = BACKWARD ? (D.own[r] - acc[r]) * D.dq : D.own[r] - acc[r];
#pragma unroll
      for (int r = 1; r < NRHS; ++r) dst[(size_t)q * NRHS + r] = out[r];
      // release limited to LDS: global loads in flight need not complete first;
      // readers pair it with an LDS-only acquire
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
      __hip_atomic_store(reinterpret_cast<typename Sentinel<T>::Bits*>(dst + (size_t)q * NRHS), to_bits<T>(out[0]),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  };
  // records and input indices two rows ahead, entries and own values one row ahead
  SweepRow<T, NRHS> A, B;
  uint64_t rn = rec[min(pos + nw, last)];
  int gn = BACKWARD ? 0 : gsched[min(pos + nw, last)];
  fetch(A, rec[pos], BACKWARD ? 0 : gsched[pos]);
  for (;;) {
    const uint64_t rnn = rec[min(pos + 2 * nw, last)];
    const int gnn = BACKWARD ? 0 : gsched[min(pos + 2 * nw, last)];
    fetch(B, rn, gn);
    solve_row(A);
    if (pos + nw >= n) break;
    pos += nw;
    rn = rec[min(pos + 2 * nw, last)];
    gn = BACKWARD ? 0 : gsched[min(pos + 2 * nw, last)];
    fetch(A, rnn, gnn);
    solve_row(B);
    if (pos + nw >= n) break;
    pos += nw;
  }
}

template <class T, int NRHS, bool SLEEP>
__global__ void __launch_bounds__(kSchwarzThreads) k_schwarz_v(const DevPC* __restrict__ pcs,
                                                              const WorkItem* __restrict__ work, int nwork,
                                                              const double* __restrict__ rin,
                                                              double* __restrict__ zout,
                                                              Gate gate) {
  extern __shared__ double smem_d[];
  if ((int)blockIdx.x >= nwork) return;
  const WorkItem wi = work[blockIdx.x];
  if (gate_skip(gate, wi.inst)) return;
  const DevPC& P = pcs[wi.inst];
  const DevSub sub = P.subs[wi.idx];
  const int n = sub.n;
  T* yv = reinterpret_cast<T*>(smem_d);
  T* zv = yv + (size_t)n * NRHS;
  const int tid = threadIdx.x, wave = tid >> 6, lane = __lane_id(), nw = blockDim.x >> 6;
  const int32_t* in_idx = P.in_idx + sub.row_off;
  const int32_t* out_idx = P.out_idx + sub.row_off;
  const T* lv = reinterpret_cast<const T*>(P.lval) + sub.lbase;
  const T* uv = reinterpret_cast<const T*>(P.uval) + sub.ubase;
  const T* di = reinterpret_cast<const T*>(P.dinv) + sub.row_off;
  const double* rb = rin + P.vec_off * NRHS;
  double* zb = zout + P.vec_off * NRHS;
  const T sent = bits_to<T>(Sentinel<T>::kBits);
  for (int q = tid; q < 2 * n * NRHS; q += blockDim.x) yv[q] = sent;
  __syncthreads();
  sweep_v<T, NRHS, false, SLEEP>(n, wave, nw, lane, P.recL + sub.row_off, P.lcol + sub.lbase, lv, nullptr,
                                 P.gL + sub.row_off, rb, nullptr, yv, P.error_flag);
  __syncthreads();
  sweep_v<T, NRHS, true, SLEEP>(n, wave, nw, lane, P.recU + sub.row_off, P.ucol + sub.ubase, uv, di, nullptr,
                                nullptr, yv, zv, P.error_flag);
  __syncthreads();
  for (int q = tid; q < n; q += blockDim.x) {
    const int32_t o = out_idx[q];
    if (o < 0) {
      const int64_t g = o & 0x7fffffff;
#pragma unroll
      for (int r = 0; r < NRHS; ++r) zb[g * NRHS + r] = (double)zv[(size_t)q * NRHS + r];
    }
  }
}

// ---- packet variant
//
// For orderings whose levels hold many rows (the distance order), a wavefront
// takes a packet of up to four rows of one level at once: lane group g (16
// lanes) solves the packet's row g, lane t of the group taking entries t,
// t+16, ... up to the packet's length class (4, 8 or 12 entries per lane, rows
// of up to 64, 128 or 192 entries; the host packs rows of one class together,
// and each class has its own unrolled poll and sum code, while entries are
// always fetched as 12 slots, which keeps the two row buffers in registers).
// The dependencies of a row are all issued before the first wait and re-polled
// together until none reads the sentinel, and the group's sum is formed in a
// fixed order (entries of a lane in increasing order, then a DPP prefix sum
// over the 16 lanes). Rows of one packet never depend on each other, and
// packets follow the level order, so the earliest unfinished packet always has
// its inputs: the sweep always advances.
template <class T, int NRHS>
struct PacketRow {
  uint64_t rec;
  int len;                     // stored entries of the group's row (0 for an empty slot)
  bool live;                   // the group has a row in this packet
  int cls;                     // length class of the packet (wave-uniform)
  int start;                   // first schedule position of the packet's level (level waits)
  int nrows;                   // rows in the packet
  int k[kPacketEntries];
  T v[kPacketEntries];
  T own[NRHS];
  T dq;
};

template <class T>
__device__ __forceinline__ T row16_sum_to_15(T v) {
  v += dpp_any<0x111, 0xf>(v);   // row_shr:1
  v += dpp_any<0x112, 0xf>(v);   // row_shr:2
  v += dpp_any<0x114, 0xf>(v);   // row_shr:4
  v += dpp_any<0x118, 0xf>(v);   // row_shr:8
  return v;                      // lane 15 of each 16-lane row holds the row total
}

// FLAGS = false: values double as flags (dst starts filled with the sentinel,
// yv holds the forward result in the backward sweep). FLAGS = true: one value
// array (dst = yv, solved in place) and per-row completion flags `done`
// (forward publishes level 1, backward level 2); less local memory, one more
// LDS round trip per dependency, the same arithmetic in the same order.
// LVL = true (value form, one right-hand side): no per-dependency polls; a
// packet waits until the sweep's count of completed rows `cnt` reaches the first
// position of its level (from the packet word), then reads its dependencies, and
// its publication adds its rows to the count. A level therefore starts only once
// every row of the previous level is complete, so a count above the first
// position of a level certifies every lower level; one uniform LDS read per poll
// instead of one per dependency. (In a level wider than 4095 rows a packet waits
// for a count 4095 below its own first position, which some rows of its own level
// help reach: slower, still every lower level.) The same arithmetic in the same
// order.
template <class T, int NRHS, bool BACKWARD, bool SLEEP, bool FLAGS, bool LVL = false>
__device__ __forceinline__ void sweep_p(int n, int npk, int wave, int nw, int lane, const uint32_t* __restrict__ pk_,
                                        const uint64_t* __restrict__ rec_, const uint16_t* __restrict__ col_,
                                        const T* __restrict__ val_, const T* __restrict__ dinv_,
                                        const int32_t* __restrict__ gsched_, const double* __restrict__ rb_,
                                        const T* yv, T* dst, int* done, int32_t* err, int* cnt = nullptr) {
  static_assert(!LVL || (!FLAGS && NRHS == 1), "level waits take the value form with one right-hand side");
  constexpr int LEVEL = BACKWARD ? 2 : 1;
  // one right-hand side keeps three packets' entries in registers where the register
  // budget of the form's thread count allows it (all but the FP64 flag form)
  constexpr bool DEEP = NRHS == 1 && (!FLAGS || sizeof(T) == 4);
  using Bits = typename Sentinel<T>::Bits;
  const auto pk = gmem(pk_);
  const auto rec = gmem(rec_);
  const auto col = gmem(col_);
  const auto val = gmem(val_);
  const auto dinv = gmem(dinv_);
  const auto gsched = gmem(gsched_);
  const auto rb = gmem(rb_);
  // A bounded wait that expires sets the error flag with a global store (a flat
  // store would leave both memory counters pending). The level-wait form records
  // it and stores once the sweep ends: a vector store inside its poll loop leaves
  // the compiler unable to count the entry loads in flight.
  const auto errg = (__attribute__((address_space(1))) int32_t*)err;
  bool timed_out = false;
  auto expired = [&]() {
    if constexpr (LVL) timed_out = true;
    else __hip_atomic_store(errg, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  auto report = [&]() {
    if (LVL && timed_out) __hip_atomic_store(errg, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  int p = wave;
  if (p >= npk) return;
  const int last = npk - 1;
  const int g = lane >> 4, t = lane & 15;
  // schedule position of this lane group's row in a packet (clamped into the packet)
  auto posof = [&](uint32_t w) { return (int)((w >> 4) & 0xffffu) + min(g, (int)(w & 3u)); };
  auto class_of = [&](uint32_t w) { return __builtin_amdgcn_readfirstlane((int)((w >> 2) & 3u)); };
  // Entries t, t+16, ... of the row, loaded unconditionally at immediate offsets
  // from one address: slots past the row's end read the entries that follow it
  // (the factor arrays are padded), and solve_row masks them out.
  // (NJc: entry slots per lane, a std::integral_constant)
  auto fetch_n = [&](auto NJc, PacketRow<T, NRHS>& D, uint32_t w, uint64_t r, int gi) __attribute__((always_inline)) {
    constexpr int NJ = decltype(NJc)::value;
    D.rec = r;
    D.live = g <= (int)(w & 3u);
    D.len = D.live ? (int)((r >> 32) & 0xffff) : 0;
    const int64_t e0 = (int64_t)(r & 0xffffffffull) + t;
    const auto cp = col + e0;
    const auto vp = val + e0;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      // uniform: only the slots of the packet's class, or all of them in the deep
      // pipeline (a fixed number of loads per fetch keeps its waits exact)
      if (DEEP || j < packet_slots(D.cls)) {
        D.k[j] = cp[kPacketLanes * j];
        D.v[j] = vp[kPacketLanes * j];
      }
    }
    if (BACKWARD) {
      D.dq = dinv[(int)(r >> 48)];
    } else {
      D.dq = (T)0;
#pragma unroll
      for (int q = 0; q < NRHS; ++q) D.own[q] = (T)rb[(int64_t)gi * NRHS + q];
    }
  };
  auto solve_n = [&](auto NJc, PacketRow<T, NRHS>& D) __attribute__((always_inline)) {
    constexpr int NJ = decltype(NJc)::value;
    const int q = (int)(D.rec >> 48);
    if (BACKWARD) {
#pragma unroll
      for (int r = 0; r < NRHS; ++r) D.own[r] = yv[(size_t)q * NRHS + r];   // y_q, complete before this sweep
    }
    // dependency slots; masked entries read slot n, which always holds 0 and is
    // always complete, so every poll is unconditional
    int kk[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) kk[j] = t + kPacketLanes * j < D.len ? (int)D.k[j] : n;
    // wait for every dependency: all polls issued together, pending ones re-polled
    Bits b[NJ];
    int spins = 0;
    if constexpr (LVL) {
      // every row of the lower levels complete (the count is uniform over the wavefront)
      const int start = __builtin_amdgcn_readfirstlane(D.start);
      if (start > 0) {
        while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) < start) {
          if (SLEEP) __builtin_amdgcn_s_sleep(1);
          if (++spins > kSpinLimit) {
            expired();
            break;
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
#pragma unroll
      for (int j = 0; j < NJ; ++j) b[j] = to_bits<T>(dst[(size_t)kk[j] * NRHS]);
    } else if constexpr (FLAGS) {
      int f[NJ];
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        f[j] = __hip_atomic_load(done + kk[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      for (;;) {
        bool pending = false;
#pragma unroll
        for (int j = 0; j < NJ; ++j) pending |= f[j] < LEVEL;
        if (!pending) break;
        if (SLEEP) __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) {
          expired();
          break;
        }
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          if (f[j] < LEVEL) f[j] = __hip_atomic_load(done + kk[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
#pragma unroll
      for (int j = 0; j < NJ; ++j) b[j] = to_bits<T>(dst[(size_t)kk[j] * NRHS]);
    } else {
      const Bits sent = Sentinel<T>::kBits;
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        b[j] = __hip_atomic_load(reinterpret_cast<Bits*>(dst + (size_t)kk[j] * NRHS), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
      for (;;) {
        bool pending = false;
#pragma unroll
        for (int j = 0; j < NJ; ++j) pending |= b[j] == sent;
        if (!pending) break;
        if (SLEEP) __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) {
          expired();
#pragma unroll
          for (int j = 0; j < NJ; ++j) b[j] = 0;
          break;
        }
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          if (b[j] == sent)
            b[j] = __hip_atomic_load(reinterpret_cast<Bits*>(dst + (size_t)kk[j] * NRHS), __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    }
    T acc[NRHS];
#pragma unroll
    for (int r = 0; r < NRHS; ++r) acc[r] = (T)0;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const T vj = t + kPacketLanes * j < D.len ? D.v[j] : (T)0;
      acc[0] += vj * bits_to<T>(b[j]);
#pragma unroll
      for (int r = 1; r < NRHS; ++r) acc[r] += vj * dst[(size_t)kk[j] * NRHS + r];
    }
#pragma unroll
    for (int r = 0; r < NRHS; ++r) acc[r] = row16_sum_to_15(acc[r]);
    if (t == kPacketLanes - 1 && D.live) {
      T out[NRHS];
#pragma unroll
      for (int r = 0; r < NRHS; ++r) out[r] = BACKWARD ? (D.own[r] - acc[r]) * D.dq : D.own[r] - acc[r];
      if constexpr (FLAGS) {
#pragma unroll
        for (int r = 0; r < NRHS; ++r) dst[(size_t)q * NRHS + r] = out[r];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __hip_atomic_store(done + q, LEVEL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      } else {
#pragma unroll
        for (int r = 1; r < NRHS; ++r) dst[(size_t)q * NRHS + r] = out[r];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __hip_atomic_store(reinterpret_cast<Bits*>(dst + (size_t)q * NRHS), to_bits<T>(out[0]), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
    if constexpr (LVL) {
      // the packet's values are written (the wavefront's LDS stores complete) before its
      // rows are counted
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
      if (lane == 0) __hip_atomic_fetch_add(cnt, D.nrows, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  };
  auto fetch = [&](PacketRow<T, NRHS>& D, uint32_t w, uint64_t r, int gi) __attribute__((always_inline)) {
    D.cls = class_of(w);
    D.start = (int)((w >> 4) & 0xffffu) - (int)(w >> 20);   // level waits: rows to count first
    D.nrows = (int)(w & 3u) + 1;
    fetch_n(std::integral_constant<int, kPacketEntries>{}, D, w, r, gi);
  };
  auto solve_row = [&](PacketRow<T, NRHS>& D) __attribute__((always_inline)) {
    if (D.cls == 0) solve_n(std::integral_constant<int, packet_slots(0)>{}, D);
    else if (D.cls == 1) solve_n(std::integral_constant<int, packet_slots(1)>{}, D);
    else solve_n(std::integral_constant<int, packet_slots(2)>{}, D);
  };
  if constexpr (DEEP) {
    // Entries two packets ahead: each step issues the packet word four packets
    // ahead and the record three ahead first, then the entries two ahead, then
    // solves. Vector loads complete in issue order, so a step waits only for
    // loads issued at least one step earlier (the current packet's entries and
    // the lookahead words and records), and the entries fetched by the previous
    // step stay in flight across this packet's polls and sums.
    PacketRow<T, NRHS> A, B, C;
    auto word = [&](int q) { return pk[min(q, last)]; };
    auto gpos = [&](uint32_t w) { return BACKWARD ? 0 : gsched[posof(w)]; };
    uint32_t w0 = word(p), w1 = word(p + nw);
    const uint64_t r0 = rec[posof(w0)], r1 = rec[posof(w1)];
    const int g0 = gpos(w0), g1 = gpos(w1);
    uint32_t w2 = word(p + 2 * nw), w3 = word(p + 3 * nw);
    uint64_t r2 = rec[posof(w2)];
    int g2 = gpos(w2);
    fetch(A, w0, r0, g0);
    fetch(B, w1, r1, g1);
    auto step = [&](PacketRow<T, NRHS>& cur, PacketRow<T, NRHS>& ahead) {
      const uint32_t w4 = word(p + 4 * nw);
      const uint64_t r3 = rec[posof(w3)];
      const int g3 = gpos(w3);
      fetch(ahead, w2, r2, g2);   // packet p + 2nw (clamped to the last packet near the end)
      solve_row(cur);
      if (p + nw > last) return false;
      p += nw;
      w2 = w3;
      r2 = r3;
      g2 = g3;
      w3 = w4;
      return true;
    };
    while (step(A, C) && step(B, A) && step(C, B)) {
    }
    report();
    return;
  }
  // packet words three packets ahead, records two ahead, entries one ahead
  // (fetched right after the previous packet is published)
  PacketRow<T, NRHS> A, B;
  uint32_t w1 = pk[min(p + nw, last)], w2 = pk[min(p + 2 * nw, last)];
  uint64_t r1 = rec[posof(w1)];
  int g1 = BACKWARD ? 0 : gsched[posof(w1)];
  {
    const uint32_t w0 = pk[p];
    fetch(A, w0, rec[posof(w0)], BACKWARD ? 0 : gsched[posof(w0)]);
  }
  auto step = [&](PacketRow<T, NRHS>& cur, PacketRow<T, NRHS>& nxt) {
    const uint64_t r2 = rec[posof(w2)];
    const int g2 = BACKWARD ? 0 : gsched[posof(w2)];
    const uint32_t w3 = pk[min(p + 3 * nw, last)];
    // the next packet's entries are issued after this packet is published: they
    // are not needed before its dependencies (a level later) are complete
    solve_row(cur);
    if (p + nw > last) return false;
    fetch(nxt, w1, r1, g1);
    p += nw;
    w1 = w2;
    r1 = r2;
    g1 = g2;
    w2 = w3;
    return true;
  };
  while (step(A, B) && step(B, A)) {
  }
  report();
}

template <class T, int NRHS, bool SLEEP, bool FLAGS, bool LVL = false>
__global__ void __launch_bounds__(packet_max_threads(sizeof(T) == 4, NRHS, FLAGS)) k_schwarz_p(const DevPC* __restrict__ pcs,
                                                              const WorkItem* __restrict__ work, int nwork,
                                                              const double* __restrict__ rin,
                                                              double* __restrict__ zout, Gate gate) {
  extern __shared__ double smem_d[];
  if ((int)blockIdx.x >= nwork) return;
  const WorkItem wi = work[blockIdx.x];
  if (gate_skip(gate, wi.inst)) return;
  const DevPC& P = pcs[wi.inst];
  const DevSub sub = P.subs[wi.idx];
  const int n = sub.n;
  // slot n of each array is the always-complete zero the masked entries read
  const int n1 = n + 1;
  T* yv = reinterpret_cast<T*>(smem_d);
  T* zv = FLAGS ? yv : yv + (size_t)n1 * NRHS;                // FLAGS: solved in place
  int* done = reinterpret_cast<int*>(yv + (size_t)n1 * NRHS); // FLAGS only
  // LVL: completed-row counts of the forward and backward sweeps, after the two value arrays
  int* cnt = reinterpret_cast<int*>(yv + 2 * (size_t)n1 * NRHS);
  const int tid = threadIdx.x, wave = tid >> 6, lane = __lane_id(), nw = blockDim.x >> 6;
  const int32_t* out_idx = P.out_idx + sub.row_off;
  const T* lv = reinterpret_cast<const T*>(P.lval) + sub.lbase;
  const T* uv = reinterpret_cast<const T*>(P.uval) + sub.ubase;
  const T* di = reinterpret_cast<const T*>(P.dinv) + sub.row_off;
  const double* rb = rin + P.vec_off * NRHS;
  double* zb = zout + P.vec_off * NRHS;
  if (FLAGS) {
    for (int q = tid; q < n1; q += blockDim.x) done[q] = q < n ? 0 : 2;
    for (int r = tid; r < NRHS; r += blockDim.x) yv[(size_t)n * NRHS + r] = (T)0;
  } else {
    const T sent = bits_to<T>(Sentinel<T>::kBits);
    for (int q = tid; q < 2 * n1 * NRHS; q += blockDim.x)
      yv[q] = (q % (n1 * NRHS)) < n * NRHS ? sent : (T)0;
    if (LVL && tid < 2) cnt[tid] = 0;
  }
  __syncthreads();
  sweep_p<T, NRHS, false, SLEEP, FLAGS, LVL>(n, sub.npkL, wave, nw, lane, P.pk + sub.pk_off, P.recL + sub.row_off,
                                             P.lcol + sub.lbase, lv, nullptr, P.gL + sub.row_off, rb, nullptr, yv,
                                             done, P.error_flag, cnt);
  __syncthreads();
  sweep_p<T, NRHS, true, SLEEP, FLAGS, LVL>(n, sub.npkU, wave, nw, lane, P.pk + sub.pk_off + sub.npkL,
                                            P.recU + sub.row_off, P.ucol + sub.ubase, uv, di, nullptr, nullptr, yv,
                                            zv, done, P.error_flag, cnt + 1);
  __syncthreads();
  for (int q = tid; q < n; q += blockDim.x) {
    const int32_t o = out_idx[q];
    if (o < 0) {
      const int64_t g = o & 0x7fffffff;
#pragma unroll
      for (int r = 0; r < NRHS; ++r) zb[g * NRHS + r] = (double)zv[(size_t)q * NRHS + r];
    }
  }
}

static hipError_t lds_ok(const void* kern, size_t shm) {
  int dev = 0, lim = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return hipErrorInvalidDevice;
  if (shm > (size_t)lim) return hipErrorInvalidConfiguration;
  if (shm > 65536) return hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  return hipSuccess;
}

template <class T, int NRHS>
static hipError_t launch_t(const SchwarzCfg& cfg, const DevPC* pcs, const WorkItem* work, int nwork, int max_rows,
                           int max_len, const double* r, double* z, hipStream_t s, const Gate& gate) {
  const int threads = cfg.threads > 0 ? cfg.threads : kSchwarzThreads;
  if (cfg.variant == kSchwarzPacketLevel) {
    // level waits: value form, one right-hand side, two sweep counters after the arrays
    if constexpr (NRHS == 1) {
      if (max_len > kPacketLanes * kPacketEntries) return hipErrorInvalidValue;
      const size_t shm = schwarz_value_lds(max_rows + 1, 1, sizeof(T)) + 2 * sizeof(int);
      if (shm > kSchwarzMaxLds) return hipErrorInvalidConfiguration;
      const int pthreads = min(threads, packet_max_threads(sizeof(T) == 4, 1, false));
      const void* kern = cfg.sleep ? (const void*)k_schwarz_p<T, 1, true, false, true>
                                   : (const void*)k_schwarz_p<T, 1, false, false, true>;
      hipError_t e = lds_ok(kern, shm);
      if (e != hipSuccess) return e;
      if (cfg.sleep)
        hipLaunchKernelGGL((k_schwarz_p<T, 1, true, false, true>), dim3(nwork), dim3(pthreads), shm, s, pcs, work,
                           nwork, r, z, gate);
      else
        hipLaunchKernelGGL((k_schwarz_p<T, 1, false, false, true>), dim3(nwork), dim3(pthreads), shm, s, pcs, work,
                           nwork, r, z, gate);
      return hipGetLastError();
    } else {
      return hipErrorInvalidConfiguration;
    }
  }
  if (cfg.variant == kSchwarzPacket || cfg.variant == kSchwarzPacketFlags) {
    // packet factors: the value form when its two arrays fit, else the flag form
    // (the same arithmetic); rows longer than a packet's lanes take are not packed
    // one extra slot per array: the always-complete zero of masked entries
    const bool flags = cfg.variant == kSchwarzPacketFlags ||
                       schwarz_value_lds(max_rows + 1, NRHS, sizeof(T)) > kSchwarzMaxLds;
    if (max_len > kPacketLanes * kPacketEntries) return hipErrorInvalidValue;
    // the flag form may stand in for the value form: keep within its register
    // budget (the thread count does not change results)
    const int pthreads = min(threads, packet_max_threads(sizeof(T) == 4, NRHS, flags));
    const size_t shm = flags ? (size_t)(max_rows + 1) * (NRHS * sizeof(T) + sizeof(int))
                             : schwarz_value_lds(max_rows + 1, NRHS, sizeof(T));
    const void* kern = flags ? (cfg.sleep ? (const void*)k_schwarz_p<T, NRHS, true, true>
                                          : (const void*)k_schwarz_p<T, NRHS, false, true>)
                             : (cfg.sleep ? (const void*)k_schwarz_p<T, NRHS, true, false>
                                          : (const void*)k_schwarz_p<T, NRHS, false, false>);
    hipError_t e = lds_ok(kern, shm);
    if (e != hipSuccess) return e;
    if (flags && cfg.sleep)
      hipLaunchKernelGGL((k_schwarz_p<T, NRHS, true, true>), dim3(nwork), dim3(pthreads), shm, s, pcs, work, nwork, r,
                         z, gate);
    else if (flags)
      hipLaunchKernelGGL((k_schwarz_p<T, NRHS, false, true>), dim3(nwork), dim3(pthreads), shm, s, pcs, work, nwork, r,
                         z, gate);
    else if (cfg.sleep)
      hipLaunchKernelGGL((k_schwarz_p<T, NRHS, true, false>), dim3(nwork), dim3(pthreads), shm, s, pcs, work, nwork, r,
                         z, gate);
    else
      hipLaunchKernelGGL((k_schwarz_p<T, NRHS, false, false>), dim3(nwork), dim3(pthreads), shm, s, pcs, work, nwork,
                         r, z, gate);
    return hipGetLastError();
  }
  if (cfg.variant == kSchwarzValueFlags && max_len <= kSchwarzValueMaxLen &&
      schwarz_value_lds(max_rows, NRHS, sizeof(T)) <= kSchwarzMaxLds) {
    const size_t shm = schwarz_value_lds(max_rows, NRHS, sizeof(T));
    if (cfg.sleep) {
      hipError_t e = lds_ok((const void*)k_schwarz_v<T, NRHS, true>, shm);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_schwarz_v<T, NRHS, true>), dim3(nwork), dim3(threads), shm, s, pcs, work, nwork, r, z, gate);
    } else {
      hipError_t e = lds_ok((const void*)k_schwarz_v<T, NRHS, false>, shm);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL((k_schwarz_v<T, NRHS, false>), dim3(nwork), dim3(threads), shm, s, pcs, work, nwork, r, z, gate);
    }
    return hipGetLastError();
  }
  const size_t shm = (size_t)max_rows * (NRHS * sizeof(T) + sizeof(int));
  hipError_t e = lds_ok((const void*)k_schwarz<T, NRHS>, shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_schwarz<T, NRHS>), dim3(nwork), dim3(threads), shm, s, pcs, work, nwork, r, z, gate);
  return hipGetLastError();
}

hipError_t launch_schwarz(const SchwarzCfg& cfg, const DevPC* pcs, const WorkItem* work, int nwork, int max_rows,
                          int max_len, int fp32, int nrhs, const double* r, double* z, hipStream_t s,
                          const Gate& gate) {
  if (nwork == 0) return hipSuccess;
  if (fp32) {
    if (nrhs == 1) return launch_t<float, 1>(cfg, pcs, work, nwork, max_rows, max_len, r, z, s, gate);
    if (nrhs == 2) return launch_t<float, 2>(cfg, pcs, work, nwork, max_rows, max_len, r, z, s, gate);
    if (nrhs == 4) return launch_t<float, 4>(cfg, pcs, work, nwork, max_rows, max_len, r, z, s, gate);
  } else {
    if (nrhs == 1) return launch_t<double, 1>(cfg, pcs, work, nwork, max_rows, max_len, r, z, s, gate);
    if (nrhs == 2) return launch_t<double, 2>(cfg, pcs, work, nwork, max_rows, max_len, r, z, s, gate);
    if (nrhs == 4) return launch_t<double, 4>(cfg, pcs, work, nwork, max_rows, max_len, r, z, s, gate);
  }
  return hipErrorInvalidValue;
}

}  // namespace cpm
