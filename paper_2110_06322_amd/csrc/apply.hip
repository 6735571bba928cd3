// Matrix-free CPM operator kernels for CDNA4 (gfx950).
//
//   (E u)_j   = sum_{a in {0..p}^d} prod_k l_{a_k}(s_jk) u[b_j + a]          (Sec. 2.1)
//   (A u)_i   = (c + 2d/h^2) u_i - h^-2 sum_{nbr n of i} (E u)_n               (eq. lapBel)
//   (A^T y)_k = (c + 2d/h^2) y_k - h^-2 sum_{j : k in cube(j)} W_jk (O^T y)_j
// with b_j = floor((cp_j - lo)/h - (p-1)/2), s_j = (cp_j - lo)/h - b_j and the
// Lagrange basis on nodes 0..p in product form (equal to the barycentric form
// of the paper's reference in exact arithmetic).
//
// Forward apply: one workgroup per 8^3-node tile (16^2 in 2-D). It stages the
// tile's interpolation footprint of u into LDS (one wavefront per 64-node
// brick, lane = node, compacted loads addressed with mbcnt over the brick's
// occupancy mask), evaluates every extension row the tile's stencils need
// (tile nodes plus the face halo) into an LDS box, then applies the
// (2d+1)-point stencil from LDS. Every extension row is read from HBM once
// per tile that needs it and no intermediate vector goes back to HBM. The
// per-tile lists (jobs, footprint bricks) are built once on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <map>
#include <mutex>
#include <utility>

#include "device.h"

namespace cpm {

// ------------------------------------------------------------- helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

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


// number of set bits of m strictly below this lane
__device__ __forceinline__ int mbcnt64(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

__device__ __forceinline__ int popc_below(uint64_t m, int bit) {
  uint64_t below = bit == 0 ? 0ull : ((~0ull) >> (64 - bit));
  return __popcll(m & below);
}

template <int D>
__device__ __forceinline__ void local_of(int bit, int* l) {
  if (D == 3) { l[0] = bit >> 4; l[1] = (bit >> 2) & 3; l[2] = bit & 3; }
  else { l[0] = bit >> 3; l[1] = bit & 7; l[2] = 0; }
}
template <int D>
__device__ __forceinline__ int bit_of(int l0, int l1, int l2) {
  return D == 3 ? l0 * 16 + l1 * 4 + l2 : l0 * 8 + l1;
}
template <int D> constexpr int kEdge = D == 3 ? 4 : 8;
template <int D> constexpr int kShift = D == 3 ? 2 : 3;
template <int D> constexpr int kTile = 2 * kEdge<D>;   // tile edge in nodes

// brick id holding grid node g, or -1
template <int D>
__device__ __forceinline__ int brick_at(const DevInst& I, const int* g) {
  int r = 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    int b = (g[k] >> kShift<D>) - I.bm_lo[k];
    if (b < 0 || b >= I.bm_dim[k] || g[k] < 0) return -1;
    r = r * I.bm_dim[k] + b;
  }
  return I.bmap[r];
}

// node index (Sigma_A then Sigma_G) of grid node g, -1 if not in the band
template <int D>
__device__ __forceinline__ int node_at(const DevInst& I, const int* g) {
  int id = brick_at<D>(I, g);
  if (id < 0) return -1;
  int bit = bit_of<D>(g[0] & (kEdge<D> - 1), g[1] & (kEdge<D> - 1), D == 3 ? (g[2] & 3) : 0);
  uint64_t mA = I.maskA[id];
  if ((mA >> bit) & 1ull) return I.offA[id] + popc_below(mA, bit);
  uint64_t mG = I.maskG[id];
  if ((mG >> bit) & 1ull) return I.nA + I.offG[id] + popc_below(mG, bit);
  return -1;
}

// Pointers of the instance read through the global address space: loads through
// a pointer taken from a struct would otherwise be flat loads, which also count in
// the counter the LDS reads of the extension rows wait on and so force those waits
// to drain every outstanding load.
template <class T>
using gptr = const __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> as_global(const T* p) {
  return (gptr<T>)p;
}
// list records read field by field through global pointers
__device__ __forceinline__ Job load_job(gptr<Job> p) {
  Job j;
  j.node = p->node;
  j.slot = p->slot;
  return j;
}
__device__ __forceinline__ FootBrick load_footbrick(gptr<FootBrick> p) {
  FootBrick f;
  f.mask = p->mask;
  f.off = p->off;
  f.lds = p->lds;
  return f;
}

// Lagrange basis on nodes 0..P at s, product form
template <int P>
__device__ __forceinline__ void lagrange(double s, double* w) {
  if (P == 1) { w[0] = 1.0 - s; w[1] = s; }
  else if (P == 2) {
    double a = s, b = s - 1.0, c = s - 2.0;
    w[0] = 0.5 * b * c; w[1] = -a * c; w[2] = 0.5 * a * b;
  } else if (P == 3) {
    double a = s, b = s - 1.0, c = s - 2.0, e = s - 3.0;
    const double i6 = 1.0 / 6.0;
    w[0] = -i6 * (b * c) * e; w[1] = 0.5 * (a * c) * e;
    w[2] = -0.5 * (a * b) * e; w[3] = i6 * (a * b) * c;
  } else if (P == 4) {
    const double a = s, b = s - 1.0, c = s - 2.0, d = s - 3.0, e = s - 4.0;
    const double i24 = 1.0 / 24.0, i6 = 1.0 / 6.0;
    w[0] = i24 * ((b * c) * (d * e)); w[1] = -i6 * ((a * c) * (d * e));
    w[2] = 0.25 * ((a * b) * (d * e)); w[3] = -i6 * ((a * b) * (c * e));
    w[4] = i24 * ((a * b) * (c * d));
  } else {
    const double a = s, b = s - 1.0, c = s - 2.0, d = s - 3.0, e = s - 4.0, f = s - 5.0;
    const double i120 = 1.0 / 120.0, i24 = 1.0 / 24.0, i12 = 1.0 / 12.0;
    w[0] = -i120 * (((b * c) * (d * e)) * f); w[1] = i24 * (((a * c) * (d * e)) * f);
    w[2] = -i12 * (((a * b) * (d * e)) * f); w[3] = i12 * (((a * b) * (c * e)) * f);
    w[4] = -i24 * (((a * b) * (c * d)) * f); w[5] = i120 * (((a * b) * (c * d)) * e);
  }
}

// cube corner b and per-axis weights of the extension row whose closest point
// in grid units is t = (cp - lo)/h
template <int D, int P>
__device__ __forceinline__ void erow_weights(const double* t, int* b, double (*w)[P + 1]) {
#pragma unroll
  for (int k = 0; k < D; ++k) {
    double bf = floor(t[k] - (P - 1) * 0.5);
    b[k] = (int)bf;
    lagrange<P>(t[k] - bf, w[k]);
  }
}

// closest point of node j in grid units (precomputed on the host with an IEEE division)
template <int D>
__device__ __forceinline__ void load_tcp(const DevInst& I, int j, double* t) {
  const int n = I.nA + I.nG;
  const gptr<double> tcp = as_global(I.tcp);
#pragma unroll
  for (int k = 0; k < D; ++k) t[k] = tcp[(int64_t)k * n + j];
}

// Extension row (closest point cp given in grid units) evaluated with per-node
// index lookups into a global vector
// (slow path: test hook and tiles whose footprint does not fit in LDS).
template <int D, int P, int NRHS>
__device__ void erow_global(const DevInst& I, const double* cp, const double* __restrict__ x, double* out) {
  int b[3] = {0, 0, 0};
  double w[D][P + 1];
  erow_weights<D, P>(cp, b, w);
#pragma unroll
  for (int r = 0; r < NRHS; ++r) out[r] = 0.0;
  if (D == 3) {
    for (int a0 = 0; a0 <= P; ++a0) {
      double acc1[NRHS];
#pragma unroll
      for (int r = 0; r < NRHS; ++r) acc1[r] = 0.0;
      for (int a1 = 0; a1 <= P; ++a1) {
        double acc2[NRHS];
#pragma unroll
        for (int r = 0; r < NRHS; ++r) acc2[r] = 0.0;
        for (int a2 = 0; a2 <= P; ++a2) {
          int g[3] = {b[0] + a0, b[1] + a1, b[2] + a2};
          int j = node_at<3>(I, g);
          if (j < 0 || j >= I.nA) continue;  // cannot happen on a closed band
          const double* xp = x + (I.vec_off + j) * NRHS;
#pragma unroll
          for (int r = 0; r < NRHS; ++r) acc2[r] += w[2][a2] * xp[r];
        }
#pragma unroll
        for (int r = 0; r < NRHS; ++r) acc1[r] += w[1][a1] * acc2[r];
      }
#pragma unroll
      for (int r = 0; r < NRHS; ++r) out[r] += w[0][a0] * acc1[r];
    }
  } else {
    for (int a0 = 0; a0 <= P; ++a0) {
      double acc1[NRHS];
#pragma unroll
      for (int r = 0; r < NRHS; ++r) acc1[r] = 0.0;
      for (int a1 = 0; a1 <= P; ++a1) {
        int g[3] = {b[0] + a0, b[1] + a1, 0};
        int j = node_at<2>(I, g);
        if (j < 0 || j >= I.nA) continue;  // cannot happen on a closed band
        const double* xp = x + (I.vec_off + j) * NRHS;
#pragma unroll
        for (int r = 0; r < NRHS; ++r) acc1[r] += w[1][a1] * xp[r];
      }
#pragma unroll
      for (int r = 0; r < NRHS; ++r) out[r] += w[0][a0] * acc1[r];
    }
  }
}

// Sum over one run of the last axis of a cube: acc[r] = sum_a w[a] x[node(g + a e_last)][r].
// All cube nodes are active, so inside one brick the run's indices are consecutive: the
// run costs one brick lookup plus one per brick boundary it crosses. Returns false when a
// node is missing (impossible on a closed band; the run then contributes nothing).
template <int D, int P, int NRHS>
__device__ __forceinline__ bool run_sum(const DevInst& I, int* g, const double* w, const double* __restrict__ x,
                                        double* acc) {
  constexpr int E = kEdge<D>;
  const int g0 = g[D - 1];
  int zl = g0 & (E - 1);
  int j = node_at<D>(I, g);
  bool ok = j >= 0 && j < I.nA;
#pragma unroll
  for (int r = 0; r < NRHS; ++r) acc[r] = 0.0;
#pragma unroll
  for (int a = 0; a <= P; ++a) {
    if (a > 0) {
      if (++zl == E) {
        zl = 0;
        g[D - 1] = g0 + a;
        j = node_at<D>(I, g);
        ok = ok && j >= 0 && j < I.nA;
      } else {
        ++j;
      }
    }
    if (ok) {
      const double* xp = x + (I.vec_off + j) * NRHS;
#pragma unroll
      for (int r = 0; r < NRHS; ++r) acc[r] += w[a] * xp[r];
    }
  }
  return ok;
}

// Extension row through global memory for the two-kernel apply: erow_global's weights and
// summation order, with the cube's nodes located run by run (run_sum).
template <int D, int P, int NRHS>
__device__ void erow_runs(const DevInst& I, const double* cp, const double* __restrict__ x, double* out) {
  int b[3] = {0, 0, 0};
  double w[D][P + 1];
  erow_weights<D, P>(cp, b, w);
#pragma unroll
  for (int r = 0; r < NRHS; ++r) out[r] = 0.0;
  if (D == 3) {
    for (int a0 = 0; a0 <= P; ++a0) {
      double acc1[NRHS];
#pragma unroll
      for (int r = 0; r < NRHS; ++r) acc1[r] = 0.0;
      for (int a1 = 0; a1 <= P; ++a1) {
        int g[3] = {b[0] + a0, b[1] + a1, b[2]};
        double acc2[NRHS];
        if (!run_sum<3, P, NRHS>(I, g, w[2], x, acc2)) continue;
#pragma unroll
        for (int r = 0; r < NRHS; ++r) acc1[r] += w[1][a1] * acc2[r];
      }
#pragma unroll
      for (int r = 0; r < NRHS; ++r) out[r] += w[0][a0] * acc1[r];
    }
  } else {
    for (int a0 = 0; a0 <= P; ++a0) {
      int g[3] = {b[0] + a0, b[1], 0};
      double acc1[NRHS];
      if (!run_sum<2, P, NRHS>(I, g, w[1], x, acc1)) continue;
#pragma unroll
      for (int r = 0; r < NRHS; ++r) out[r] += w[0][a0] * acc1[r];
    }
  }
}

// Extension row evaluated from the LDS footprint box U (node (x, y, z) of the
// grid at U[x*s0 + y*s1 + z - fbase]; 2-D: U[x*s0 + y - fbase]).
template <int D, int P>
__device__ __forceinline__ double erow_lds(const double* t, const double* U, int s0, int s1, int fbase) {
  int b[3] = {0, 0, 0};
  double w[D][P + 1];
  erow_weights<D, P>(t, b, w);
  double out = 0.0;
  if constexpr (D == 3) {
    const int base = b[0] * s0 + b[1] * s1 + b[2] - fbase;
#pragma unroll
    for (int a0 = 0; a0 <= P; ++a0) {
      // up to cubic interpolation the plane's (P+1)^2 values are read before they are
      // combined, so that its LDS reads are in flight together rather than one column at
      // a time (higher degrees read column by column: their planes exceed the registers)
      constexpr int PB = P <= 3 ? P + 1 : 1;
      double c[PB][P + 1];
      double acc1 = 0.0;
#pragma unroll
      for (int a1b = 0; a1b <= P; a1b += PB) {
#pragma unroll
        for (int q = 0; q < PB; ++q) {
          const double* col = U + base + a0 * s0 + (a1b + q) * s1;
#pragma unroll
          for (int a2 = 0; a2 <= P; ++a2) c[q][a2] = col[a2];
        }
#pragma unroll
        for (int q = 0; q < PB; ++q) {
          double acc2 = 0.0;
#pragma unroll
          for (int a2 = 0; a2 <= P; ++a2) acc2 += w[2][a2] * c[q][a2];
          acc1 += w[1][a1b + q] * acc2;
        }
      }
      out += w[0][a0] * acc1;
    }
  } else {
    const int base = b[0] * s0 + b[1] - fbase;
#pragma unroll
    for (int a0 = 0; a0 <= P; ++a0) {
      const double* col = U + base + a0 * s0;
      double acc1 = 0.0;
#pragma unroll
      for (int a1 = 0; a1 <= P; ++a1) acc1 += w[1][a1] * col[a1];
      out += w[0][a0] * acc1;
    }
  }
  return out;
}

// (2d+1)-point stencil row from the LDS box of extension values (slot vi)
template <int D>
__device__ __forceinline__ double stencil_row(const double* V, int vi, double diag, double inv_h2, double xi) {
  constexpr int W = (D == 3 ? 8 : 16) + 2;
  constexpr int S0 = D == 3 ? W * W : W, S1 = D == 3 ? W : 1, S2 = 1;
  double s = V[vi - S0] + V[vi + S0];
  s += V[vi - S1] + V[vi + S1];
  if (D == 3) s += V[vi - S2] + V[vi + S2];
  return diag * xi - inv_h2 * s;
}

// LDS offset of lane (node l of a brick) inside a footprint box with strides s0, s1
template <int D>
__device__ __forceinline__ int lane_box_offset(const int* l, int s0, int s1) {
  return D == 3 ? l[0] * s0 + l[1] * s1 + l[2] : l[0] * s0 + l[1];
}

// Work item w of n for block i so that consecutive work items run on the same
// XCD (the dispatcher deals workgroups to the 8 XCDs round-robin).
__device__ __forceinline__ int xcd_remap(int i, int n) {
  const int X = 8;
  int q = n / X, r = n % X;
  int xcd = i % X, k = i / X;
  return xcd * q + min(xcd, r) + k;
}

// ------------------------------------------------------------- kernels
// v = E u over all nodes of Sigma_A u Sigma_G (one right-hand side)
template <int D, int P>
__global__ void __launch_bounds__(256) k_extend(DevInst I, const double* __restrict__ u, double* __restrict__ v) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= I.nA + I.nG) return;
  double cp[3], out[1];
  load_tcp<D>(I, j, cp);
  erow_global<D, P, 1>(I, cp, u, out);
  if (I.esgn) out[0] *= I.esgn[j];
  v[j] = out[0];
}

template <int D, int NRHS>
__device__ __forceinline__ int vbox_index(const int* l) {
  // tile-local coordinates in [-1, T] -> box of edge T+2
  constexpr int W = kTile<D> + 2;
  return D == 3 ? (((l[0] + 1) * W + (l[1] + 1)) * W + (l[2] + 1)) * NRHS
                : ((l[0] + 1) * W + (l[1] + 1)) * NRHS;
}

template <int D, int NRHS>
constexpr int vbox_doubles() {
  constexpr int W = kTile<D> + 2;
  return (D == 3 ? W * W * W : W * W) * NRHS;
}

// LDS bytes of the fused apply besides the footprint U: the box of extension values
template <int D>
constexpr size_t tile_lds_extra() {
  return (size_t)vbox_doubles<D, 1>() * 8;
}

// Fused y = A x over the tiles of one or more instances, one workgroup per
// tile (used for several right-hand sides). The host lists, per tile, its
// extension-row jobs (node, slot in the LDS box V), the Sigma_A bricks inside
// its brick-aligned interpolation footprint box and its own bricks, so a tile
// costs two dependent HBM levels (records, then data). The closest points of
// a thread's jobs and the x values of its stencil rows are fetched before the
// footprint is staged. Per right-hand side:
//  C. stage the footprint of x into LDS (one wavefront per brick, lane = node);
//  D. evaluate the jobs' extension rows into V;
//  E. (2d+1)-point stencil from V for the tile's active nodes.
template <int D, int P, int NRHS>
__global__ void __launch_bounds__(512) k_apply_tile(const DevInst* __restrict__ insts,
                                                    const WorkItem* __restrict__ work, int nwork, int ucap,
                                                    const double* __restrict__ x, double* __restrict__ y,
                                                    Gate gate) {
  extern __shared__ double smem[];
  constexpr int NT = 512, NW = NT / 64;
  constexpr int E = kEdge<D>;
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  if (w >= nwork) return;
  const WorkItem wi = work[w];
  if (gate_skip(gate, wi.inst)) return;
  const DevInst& I = insts[wi.inst];
  const DevTile& tile = I.tiles[wi.idx];
  const int s0 = tile.fstr[0], s1 = tile.fstr[1], fbase = tile.fbase;
  const int fcnt = tile.fb_cnt, nj = tile.job_cnt;
  const gptr<FootBrick> fb = as_global(I.fbrec) + tile.fb_off;
  const gptr<Job> jl = as_global(I.jobs) + tile.job_off;
  const gptr<double> esgn = as_global(I.esgn);
  double* U = smem;
  double* V = U + ucap;
  const int tid = threadIdx.x, lane = lane_id();
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const double* xb = x + I.vec_off * NRHS;
  double* yb = y + I.vec_off * NRHS;
  int l[3];
  local_of<D>(lane, l);
  const int loff = lane_box_offset<D>(l, s0, s1);

  // jobs of this thread (at most two: a tile has at most 2^d*64 band nodes plus its face halo)
  int slot0 = -1, slot1 = -1;
  double cp0[3] = {0, 0, 0}, cp1[3] = {0, 0, 0}, sg0 = 1.0, sg1 = 1.0;
  if (tid < nj) {
    const Job j = load_job(jl + tid);
    slot0 = j.slot;
    load_tcp<D>(I, j.node, cp0);
    if (esgn) sg0 = esgn[j.node];
  }
  if (tid + NT < nj) {
    const Job j = load_job(jl + tid + NT);
    slot1 = j.slot;
    load_tcp<D>(I, j.node, cp1);
    if (esgn) sg1 = esgn[j.node];
  }
  // stencil row of this thread: wavefront = tile brick, lane = node
  uint64_t mS = 0;
  int row = 0, vi = 0;
  double xi[NRHS];
  if (wave < (1 << D)) {
    mS = tile.mA[wave];
    row = tile.oA[wave] + mbcnt64(mS);
    const int sub[3] = {D == 3 ? (wave >> 2) : (wave >> 1), D == 3 ? ((wave >> 1) & 1) : (wave & 1),
                        D == 3 ? (wave & 1) : 0};
    int ll[3] = {l[0] + sub[0] * E, l[1] + sub[1] * E, l[2] + sub[2] * E};
    vi = vbox_index<D, 1>(ll);
  }
  const bool has_row = (mS >> lane) & 1ull;
  if (has_row) {
#pragma unroll
    for (int r = 0; r < NRHS; ++r) xi[r] = xb[(int64_t)row * NRHS + r];
  }

#pragma unroll 1
  for (int r = 0; r < NRHS; ++r) {
    // ---- C. stage the footprint of x (8 bricks per wavefront in flight)
#pragma unroll 1
    for (int q0 = wave; q0 < fcnt; q0 += 8 * NW) {
      double val[8];
      int slot[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = q0 + u * NW;
        slot[u] = -1;
        if (q < fcnt) {
          const FootBrick rec = load_footbrick(fb + q);
          if ((rec.mask >> lane) & 1ull) {
            slot[u] = rec.lds + loff;
            val[u] = xb[(int64_t)(rec.off + mbcnt64(rec.mask)) * NRHS + r];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (slot[u] >= 0) U[slot[u]] = val[u];
    }
    __syncthreads();
    // ---- D. extension rows
    if (slot0 >= 0) {
      double e = erow_lds<D, P>(cp0, U, s0, s1, fbase);
      if (I.esgn) e *= sg0;
      V[slot0] = e;
    }
    if (slot1 >= 0) {
      double e = erow_lds<D, P>(cp1, U, s0, s1, fbase);
      if (I.esgn) e *= sg1;
      V[slot1] = e;
    }
    __syncthreads();
    // ---- E. stencil
    if (has_row) yb[(int64_t)row * NRHS + r] = stencil_row<D>(V, vi, I.diag, I.inv_h2, xi[r]);
    if (r + 1 < NRHS) __syncthreads();
  }
}

// ---- pipelined single-right-hand-side apply
//
// A persistent workgroup walks the tiles of one contiguous range (the work
// list is split into 8 ranges, one per XCD, so tiles that share footprint
// data run on the same L2). Three tiles are in flight per workgroup: while
// the extension rows of tile k are evaluated, the gathered data of tile k+1
// (closest points of its jobs, its footprint of x, its stencil x values) and
// the lists of tile k+2 (jobs, footprint brick records) are in transit.

// uniform per-tile values (the footprint record dwords are spread over lanes)
struct PipeRec {
  int inst, s0, s1, fbase, fb_off, fb_cnt, job_off, job_cnt, oA;
  uint64_t mA;
};

// A tile record travels as one vector load, lane j holding dword j of the
// record, and is unpacked with readlane one iteration later: vector loads
// complete in order, so unlike scalar loads they never hold up the LDS waits
// of the extension rows.
constexpr int kTileDwords = (int)(sizeof(DevTile) / 4);
static_assert(sizeof(DevTile) % 4 == 0 && kTileDwords <= 64, "tile record must fit one dword per lane");

__device__ __forceinline__ uint32_t pipe_rec_raw(const DevTile* __restrict__ wtiles, int w, int lane) {
  return lane < kTileDwords ? reinterpret_cast<const uint32_t*>(wtiles + w)[lane] : 0u;
}

template <int D>
__device__ __forceinline__ PipeRec pipe_unpack(uint32_t rw, int wave, const Gate& gate) {
  auto f = [&](size_t byte_off) { return (int)__builtin_amdgcn_readlane(rw, (int)(byte_off / 4)); };
  PipeRec R;
  R.inst = f(offsetof(DevTile, inst));
  if (gate.act && gate_skip(gate, R.inst)) {   // an instance whose systems have stopped: an empty tile
    R.s0 = R.s1 = R.fbase = R.fb_off = R.fb_cnt = R.job_off = R.job_cnt = R.oA = 0;
    R.mA = 0ull;
    return R;
  }
  R.s0 = f(offsetof(DevTile, fstr));
  R.s1 = f(offsetof(DevTile, fstr) + 4);
  R.fbase = f(offsetof(DevTile, fbase));
  R.fb_off = f(offsetof(DevTile, fb_off));
  R.fb_cnt = f(offsetof(DevTile, fb_cnt));
  R.job_off = f(offsetof(DevTile, job_off));
  R.job_cnt = f(offsetof(DevTile, job_cnt));
  R.oA = 0;
  R.mA = 0ull;
  if (wave < (1 << D)) {
    R.oA = (int)__builtin_amdgcn_readlane(rw, (int)(offsetof(DevTile, oA) / 4) + wave);
    const uint32_t lo = __builtin_amdgcn_readlane(rw, (int)(offsetof(DevTile, mA) / 4) + 2 * wave);
    const uint32_t hi = __builtin_amdgcn_readlane(rw, (int)(offsetof(DevTile, mA) / 4) + 2 * wave + 1);
    R.mA = ((uint64_t)hi << 32) | lo;
  }
  return R;
}

// lists of one tile held by one thread: up to two jobs and one dword of the
// wavefront's footprint brick records (lane 4u+f holds dword f of record wave+8u)
struct PipeList {
  int node0, slot0, node1, slot1;
  uint32_t fbw;
};

// instance values a pipeline stage needs, kept in scalar registers and
// reloaded only when the stage's tile belongs to another instance (tiles of
// one instance are contiguous in the work list), so the steady state issues
// no scalar loads
struct InstView {
  gptr<double> tcp;
  gptr<double> esgn;        // extension-row signs, or null
  gptr<Job> jobs;
  gptr<FootBrick> fbrec;
  int64_t vec_off;          // offset of the output (y, or extension values in the two-pass kernel)
  int64_t xoff;             // offset of x
  double diag, inv_h2;
  int ntot, inst;
};

template <bool TWO = false>
__device__ __forceinline__ void inst_refresh(InstView& v, const DevInst* __restrict__ insts, int i) {
  if (i == v.inst) return;
  const DevInst& I = insts[i];
  v.tcp = as_global(I.tcp);
  v.esgn = as_global(I.esgn);
  v.jobs = as_global(TWO ? I.jobsE : I.jobs);
  v.fbrec = as_global(TWO ? I.fbrecE : I.fbrec);
  v.vec_off = TWO ? I.vnode_off : I.vec_off;
  v.xoff = I.vec_off;
  v.diag = I.diag;
  v.inv_h2 = I.inv_h2;
  v.ntot = I.nA + I.nG;
  v.inst = i;
}

template <int D>
__device__ __forceinline__ void view_tcp(const InstView& V, int j, double* t) {
#pragma unroll
  for (int k = 0; k < D; ++k) t[k] = V.tcp[(int64_t)k * V.ntot + j];
}

template <int D>
__device__ __forceinline__ PipeList pipe_list(const InstView& I, const PipeRec& R, int tid, int wave, int lane) {
  PipeList L;
  L.node0 = 0; L.slot0 = -1; L.node1 = 0; L.slot1 = -1; L.fbw = 0;
  if (tid < R.job_cnt) {
    const Job j = load_job(I.jobs + R.job_off + tid);
    L.node0 = j.node;
    L.slot0 = j.slot;
  }
  if (tid + 512 < R.job_cnt) {
    const Job j = load_job(I.jobs + R.job_off + tid + 512);
    L.node1 = j.node;
    L.slot1 = j.slot;
  }
  const int q = wave + 8 * (lane >> 2);
  if (lane < 32 && q < R.fb_cnt) L.fbw = reinterpret_cast<gptr<uint32_t>>(I.fbrec + R.fb_off + q)[lane & 3];
  return L;
}

// gathered data of one tile held by one thread
template <int D>
struct PipeData {
  double t0[3];          // closest point (grid units) of the first job (a second job, needed
                         // only by tiles with more than 512 jobs, is fetched when evaluated)
  double sval[8];        // footprint values this lane stages
  int sidx[8];           // their LDS slots, -1 = none
  double xi;             // x at the stencil row
};

template <int D>
__device__ __forceinline__ void pipe_data(const InstView& I, const PipeRec& R, const PipeList& L,
                                          const double* __restrict__ x, const int* l, int wave, int lane,
                                          PipeData<D>& Dt) {
  const double* xb = x + I.xoff;
#pragma unroll
  for (int k = 0; k < 3; ++k) Dt.t0[k] = 0.0;
  if (L.slot0 >= 0) view_tcp<D>(I, L.node0, Dt.t0);
  const int loff = lane_box_offset<D>(l, R.s0, R.s1);
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    Dt.sidx[u] = -1;
    Dt.sval[u] = 0.0;
    if (wave + 8 * u < R.fb_cnt) {
      const uint32_t mlo = __builtin_amdgcn_readlane(L.fbw, 4 * u);
      const uint32_t mhi = __builtin_amdgcn_readlane(L.fbw, 4 * u + 1);
      const int off = (int)__builtin_amdgcn_readlane(L.fbw, 4 * u + 2);
      const int lds = (int)__builtin_amdgcn_readlane(L.fbw, 4 * u + 3);
      const uint64_t m = ((uint64_t)mhi << 32) | mlo;
      if ((m >> lane) & 1ull) {
        Dt.sidx[u] = lds + loff;
        Dt.sval[u] = xb[off + mbcnt64(m)];
      }
    }
  }
  Dt.xi = 0.0;
  if ((R.mA >> lane) & 1ull) Dt.xi = xb[R.oA + mbcnt64(R.mA)];
}

// TWO = true: the extension pass of the two-pass apply. The jobs are the tile's
// own band nodes (no face halo), each extension row goes to y[vnode_off + node]
// (the scratch vector of extension values) and the work-ordered tile copies
// carry no Sigma_A masks, so the stencil stage is empty.
template <int D, int P, bool TWO>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) k_apply_pipe(const DevInst* __restrict__ insts,
                                                    const DevTile* __restrict__ wtiles,
                                                    const PipeSpan* __restrict__ plan, int ucap,
                                                    const double* __restrict__ x, double* __restrict__ y,
                                                    Gate gate) {
  extern __shared__ double smem[];
  if (gate.count && *gate.count == 0) return;
  constexpr int E = kEdge<D>;
  double* U = smem;
  double* V = U + ucap;
  const int tid = threadIdx.x, lane = lane_id();
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  int l[3];
  local_of<D>(lane, l);
  const PipeSpan span = plan[blockIdx.x];
  const int per = span.step, w_end = span.end;
  int w = span.first;
  if (w >= w_end) return;  // uniform over the workgroup, before any barrier

  // slot in V of this thread's stencil row (fixed: wavefront = tile brick, lane = node)
  int vi = 0;
  if (wave < (1 << D)) {
    const int sub[3] = {D == 3 ? (wave >> 2) : (wave >> 1), D == 3 ? ((wave >> 1) & 1) : (wave & 1),
                        D == 3 ? (wave & 1) : 0};
    int ll[3] = {l[0] + sub[0] * E, l[1] + sub[1] * E, l[2] + sub[2] * E};
    vi = vbox_index<D, 1>(ll);
  }

  // prologue: data of tile w, lists of w+per, raw record of w+2per
  InstView V0, V1, V2;   // instance views of the stencil, data and list stages
  V0.inst = V1.inst = V2.inst = -1;
  PipeRec R0 = pipe_unpack<D>(pipe_rec_raw(wtiles, w, lane), wave, gate);
  inst_refresh<TWO>(V1, insts, R0.inst);
  PipeList L0 = pipe_list<D>(V1, R0, tid, wave, lane);
  PipeData<D> D0;
  pipe_data<D>(V1, R0, L0, x, l, wave, lane, D0);
  const bool v1 = w + per < w_end, v2 = w + 2 * per < w_end;
  PipeRec R1 = v1 ? pipe_unpack<D>(pipe_rec_raw(wtiles, w + per, lane), wave, gate) : R0;
  inst_refresh<TWO>(V2, insts, R1.inst);
  PipeList L1 = v1 ? pipe_list<D>(V2, R1, tid, wave, lane) : L0;
  uint32_t W2 = v2 ? pipe_rec_raw(wtiles, w + 2 * per, lane) : 0u;

#pragma unroll 1
  for (; w < w_end; w += per) {
    inst_refresh<TWO>(V0, insts, R0.inst);
    const InstView& I = V0;
    // ---- stage this tile's footprint of x
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (D0.sidx[u] >= 0) U[D0.sidx[u]] = D0.sval[u];
    const bool has_row = (R0.mA >> lane) & 1ull;
    const int row = R0.oA + mbcnt64(R0.mA);
    const double xi = D0.xi;
    const double diag = I.diag, inv_h2 = I.inv_h2;
    double* yb = y + I.vec_off;
    const int s0 = R0.s0, s1 = R0.s1, fbase = R0.fbase;
    const int slot0 = L0.slot0, slot1 = L0.slot1, node0 = L0.node0, node1 = L0.node1;
    double t0[3] = {D0.t0[0], D0.t0[1], D0.t0[2]};
    __syncthreads();
    // closest point of a second job (tiles of more than 512 jobs), issued before the next
    // tiles' loads: vector loads complete in order, so waiting for it later does not
    // wait for those
    double t1[3] = {0.0, 0.0, 0.0};
    if (slot1 >= 0) view_tcp<D>(I, node1, t1);
    // ---- next tiles' loads: data of w+per, lists of w+2per, record of w+3per
    const bool n1 = w + per < w_end, n2 = w + 2 * per < w_end, n3 = w + 3 * per < w_end;
    if (n1) {
      inst_refresh<TWO>(V1, insts, R1.inst);
      pipe_data<D>(V1, R1, L1, x, l, wave, lane, D0);
    }
    PipeRec R2 = R1;
    PipeList L2 = L1;
    if (n2) {
      R2 = pipe_unpack<D>(W2, wave, gate);
      inst_refresh<TWO>(V2, insts, R2.inst);
      L2 = pipe_list<D>(V2, R2, tid, wave, lane);
    }
    const uint32_t W3 = n3 ? pipe_rec_raw(wtiles, w + 3 * per, lane) : 0u;
    // ---- extension rows of this tile
    if (slot0 >= 0) {
      double e = erow_lds<D, P>(t0, U, s0, s1, fbase);
      if (I.esgn) e *= I.esgn[node0];
      if constexpr (TWO) yb[node0] = e;
      else V[slot0] = e;
    }
    if (slot1 >= 0) {
      double e = erow_lds<D, P>(t1, U, s0, s1, fbase);
      if (I.esgn) e *= I.esgn[node1];
      if constexpr (TWO) yb[node1] = e;
      else V[slot1] = e;
    }
    __syncthreads();
    // ---- stencil
    if (has_row) yb[row] = stencil_row<D>(V, vi, diag, inv_h2, xi);
    R0 = R1; L0 = L1;
    R1 = R2; L1 = L2;
    W2 = W3;
  }
}

// Slow path for tiles whose footprint exceeds the LDS budget: each active
// node evaluates its 2d neighbours' extension rows with index lookups.
template <int D, int P, int NRHS>
__global__ void __launch_bounds__(256) k_apply_fallback(const DevInst* __restrict__ insts,
                                                        const WorkItem* __restrict__ work, int nwork,
                                                        const double* __restrict__ x, double* __restrict__ y,
                                                        Gate gate) {
  constexpr int NB = D == 3 ? 8 : 4, E = kEdge<D>;
  const int w = blockIdx.x;
  if (w >= nwork) return;
  const WorkItem wi = work[w];
  if (gate_skip(gate, wi.inst)) return;
  const DevInst& I = insts[wi.inst];
  const DevTile& tile = I.tiles[wi.idx];
  const int wave = threadIdx.x >> 6, lane = lane_id();
  for (int q = wave; q < NB; q += (blockDim.x >> 6)) {
    const uint64_t mA = tile.mA[q];
    if (!((mA >> lane) & 1ull)) continue;
    const int i = tile.oA[q] + mbcnt64(mA);
    const int sub[3] = {D == 3 ? (q >> 2) : (q >> 1), D == 3 ? ((q >> 1) & 1) : (q & 1), D == 3 ? (q & 1) : 0};
    int l[3];
    local_of<D>(lane, l);
    int g[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < D; ++k) g[k] = tile.origin[k] + sub[k] * E + l[k];
    // neighbour sum in the fused kernel's order: (x- + x+), then + (y- + y+), then + (z- + z+)
    double s[NRHS];
#pragma unroll
    for (int r = 0; r < NRHS; ++r) s[r] = 0.0;
    for (int k = 0; k < D; ++k) {
      double pr[NRHS];
#pragma unroll
      for (int r = 0; r < NRHS; ++r) pr[r] = 0.0;
      for (int sd = -1; sd <= 1; sd += 2) {
        int gn[3] = {g[0], g[1], g[2]};
        gn[k] += sd;
        int j = node_at<D>(I, gn);
        double out[NRHS];
#pragma unroll
        for (int r = 0; r < NRHS; ++r) out[r] = 0.0;
        if (j >= 0) {  // always on a closed band
          double cp[3];
          load_tcp<D>(I, j, cp);
          erow_global<D, P, NRHS>(I, cp, x, out);
          if (I.esgn) {
            const double sgn = I.esgn[j];
#pragma unroll
            for (int r = 0; r < NRHS; ++r) out[r] *= sgn;
          }
        }
#pragma unroll
        for (int r = 0; r < NRHS; ++r) pr[r] = sd < 0 ? out[r] : pr[r] + out[r];
      }
#pragma unroll
      for (int r = 0; r < NRHS; ++r) s[r] = k == 0 ? pr[r] : s[r] + pr[r];
    }
#pragma unroll
    for (int r = 0; r < NRHS; ++r) {
      const int64_t e = (I.vec_off + i) * NRHS + r;
      y[e] = I.diag * x[e] - I.inv_h2 * s[r];
    }
  }
}

// Extension pass, slow path: the bricks of the extension-pass tiles whose footprint
// exceeds the LDS budget (one wavefront per brick, lane = node, rows evaluated from
// global memory); each item names its instance and brick.
template <int D, int P>
__global__ void __launch_bounds__(256) k_extend_bricks(const DevInst* __restrict__ insts,
                                                       const WorkItem* __restrict__ items, int nitems,
                                                       const double* __restrict__ x, double* __restrict__ v,
                                                       Gate gate) {
  const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= nitems) return;
  const WorkItem wi = items[w];
  if (gate_skip(gate, wi.inst)) return;
  const DevInst& I = insts[wi.inst];
  const int lane = lane_id();
  const int id = wi.idx;
  if (id < 0 || id >= I.nbricks) return;
  const uint64_t mA = I.maskA[id], mG = I.maskG[id];
  int node = -1;
  if ((mA >> lane) & 1ull) node = I.offA[id] + mbcnt64(mA);
  else if ((mG >> lane) & 1ull) node = I.nA + I.offG[id] + mbcnt64(mG);
  if (node < 0) return;
  double cp[3], out[1];
  load_tcp<D>(I, node, cp);
  erow_runs<D, P, 1>(I, cp, x, out);
  if (I.esgn) out[0] *= I.esgn[node];
  v[I.vnode_off + node] = out[0];
}

// Stencil pass of the two-pass apply: y_i = (c + 2d/h^2) x_i - h^-2 sum_n v_n
// with v the extension values of Sigma_A u Sigma_G written by the extension
// pass. One workgroup per tile with active nodes, one wavefront per brick,
// lane = node. A node's grid neighbours lie in its own brick or in the brick
// across one face; the masks and offsets of those 2d + 1 bricks are uniform
// over the wavefront (scalar loads), so a neighbour's index is a popcount.
// The sum is formed in the fused kernel's order (x pair, y pair, z pair).
template <int D>
__global__ void __launch_bounds__(512) k_stencil(const DevInst* __restrict__ insts, const WorkItem* __restrict__ work,
                                                 int nwork, const double* __restrict__ v, const double* __restrict__ x,
                                                 double* __restrict__ y, Gate gate) {
  constexpr int E = kEdge<D>;
  const int w = xcd_remap(blockIdx.x, gridDim.x);
  if (w >= nwork) return;
  const WorkItem wi = work[w];
  if (gate_skip(gate, wi.inst)) return;
  const DevInst& I = insts[wi.inst];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = lane_id();
  if (wave >= (1 << D)) return;
  const DevTile& tile = I.tiles[wi.idx];
  const uint64_t mA = tile.mA[wave];
  if (!((mA >> lane) & 1ull)) return;
  const int id = tile.bid[wave];
  const int row = tile.oA[wave] + mbcnt64(mA);
  int l[3];
  local_of<D>(lane, l);
  const double* vb = v + I.vnode_off;
  double nb[2 * D];
#pragma unroll
  for (int k = 0; k < D; ++k)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      int ln[3] = {l[0], l[1], l[2]};
      ln[k] += s ? 1 : -1;
      int b = id;
      if (ln[k] < 0 || ln[k] >= E) {
        b = as_global(I.bnbr)[id * 2 * D + 2 * k + s];
        ln[k] = (ln[k] + E) & (E - 1);
      }
      const int bit = bit_of<D>(ln[0], ln[1], ln[2]);
      const uint64_t ma = as_global(I.maskA)[b];
      int j;
      if ((ma >> bit) & 1ull) j = as_global(I.offA)[b] + popc_below(ma, bit);
      else j = I.nA + as_global(I.offG)[b] + popc_below(as_global(I.maskG)[b], bit);
      nb[2 * k + s] = vb[j];
    }
  double sum = nb[0] + nb[1];
  sum += nb[2] + nb[3];
  if (D == 3) sum += nb[4] + nb[5];
  const int64_t e = I.vec_off + row;
  y[e] = I.diag * x[e] - I.inv_h2 * sum;
}

// ---- transpose: z = O^T y over Sigma_A u Sigma_G (z_j = sum of y over the active grid
// neighbours of node j, in the order -x, +x, -y, +y, -z, +z). One wavefront per brick; a
// neighbour lies in the node's brick or in the brick across one face.
template <int D, int NRHS>
__global__ void __launch_bounds__(256) k_OT(DevInst I, const double* __restrict__ y, double* __restrict__ z,
                                            Gate gate, int inst) {
  constexpr int E = kEdge<D>;
  if (gate_skip(gate, inst)) return;
  const int id = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (id >= I.nbricks) return;
  const int lane = lane_id();
  const uint64_t mA = I.maskA[id], mG = I.maskG[id];
  if (!(((mA | mG) >> lane) & 1ull)) return;
  const int j = ((mA >> lane) & 1ull) ? I.offA[id] + mbcnt64(mA) : I.nA + I.offG[id] + mbcnt64(mG);
  int l[3];
  local_of<D>(lane, l);
  double s[NRHS];
#pragma unroll
  for (int r = 0; r < NRHS; ++r) s[r] = 0.0;
#pragma unroll
  for (int k = 0; k < D; ++k)
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      int ln[3] = {l[0], l[1], l[2]};
      ln[k] += sd ? 1 : -1;
      int b = id;
      if (ln[k] < 0 || ln[k] >= E) {
        b = I.bnbr[id * 2 * D + 2 * k + sd];
        ln[k] = (ln[k] + E) & (E - 1);
      }
      if (b < 0) continue;
      const int bit = bit_of<D>(ln[0], ln[1], ln[2]);
      const uint64_t ma = I.maskA[b];
      if (!((ma >> bit) & 1ull)) continue;
      const int64_t n = I.vec_off + I.offA[b] + popc_below(ma, bit);
#pragma unroll
      for (int r = 0; r < NRHS; ++r) s[r] += y[n * NRHS + r];
    }
#pragma unroll
  for (int r = 0; r < NRHS; ++r) z[(int64_t)j * NRHS + r] = s[r];
}

// ---- transpose: y_out = diag y - h^-2 E^T z. One wavefront per brick with active nodes,
// a lane per node of the brick. The extension rows whose interpolation cube overlaps the
// brick (a list in ascending row order) are staged 64 at a time in LDS: cube corner
// relative to the brick, per-axis weights, and sign times z. Every lane then adds the
// contributions of the staged rows whose cube holds its node, in list order; a row's
// weights are computed once per overlapped brick instead of once per cube node.
template <int D, int P, int NRHS>
__global__ void __launch_bounds__(64) k_ET(DevInst I, const double* __restrict__ yin, const double* __restrict__ z,
                                           double* __restrict__ yout, Gate gate, int inst) {
  constexpr int E = kEdge<D>, NW = D * (P + 1);
  __shared__ int32_t s_rel[64];
  __shared__ double s_w[64][NW];
  __shared__ double s_z[64][NRHS];
  if (gate_skip(gate, inst)) return;
  if ((int)blockIdx.x >= I.ntbricks) return;
  const int id = I.tbricks[xcd_remap(blockIdx.x, gridDim.x)];   // neighbouring bricks share an XCD's L2
  const int lane = threadIdx.x;
  int l[3] = {0, 0, 0}, org[3] = {0, 0, 0};
  local_of<D>(lane, l);
#pragma unroll
  for (int k = 0; k < D; ++k) org[k] = I.bcoord[id * 3 + k] * E;
  const uint64_t mA = I.maskA[id];
  double acc[NRHS];
#pragma unroll
  for (int r = 0; r < NRHS; ++r) acc[r] = 0.0;
  const int rb = I.trow_ptr[id], re = I.trow_ptr[id + 1];
  for (int c0 = rb; c0 < re; c0 += 64) {
    const int nr = min(64, re - c0);
    if (lane < nr) {
      const int j = I.trows[c0 + lane];
      double t[3];
      load_tcp<D>(I, j, t);
      int rel = 0;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const double bf = floor(t[k] - (P - 1) * 0.5);
        double w[P + 1];
        lagrange<P>(t[k] - bf, w);
#pragma unroll
        for (int a = 0; a <= P; ++a) s_w[lane][k * (P + 1) + a] = w[a];
        rel |= (((int)bf - org[k] + 16) & 0xff) << (8 * k);   // corner - origin in [-P, E-1], biased
      }
      s_rel[lane] = rel;
      const double sg = I.esgn ? I.esgn[j] : 1.0;
#pragma unroll
      for (int r = 0; r < NRHS; ++r) s_z[lane][r] = sg * z[(int64_t)j * NRHS + r];
    }
    __syncthreads();
    for (int q = 0; q < nr; ++q) {
      const int rel = s_rel[q];
      int a[3] = {0, 0, 0};
      bool in = true;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        a[k] = l[k] - (((rel >> (8 * k)) & 0xff) - 16);
        in = in && a[k] >= 0 && a[k] <= P;
      }
      if (in) {
        double w = s_w[q][a[0]];
#pragma unroll
        for (int k = 1; k < D; ++k) w *= s_w[q][k * (P + 1) + a[k]];
#pragma unroll
        for (int r = 0; r < NRHS; ++r) acc[r] += w * s_z[q][r];
      }
    }
    __syncthreads();
  }
  if (!((mA >> lane) & 1ull)) return;
  const int64_t row = I.vec_off + I.offA[id] + mbcnt64(mA);
#pragma unroll
  for (int r = 0; r < NRHS; ++r) {
    const int64_t e = row * NRHS + r;
    yout[e] = I.diag * yin[e] - I.inv_h2 * acc[r];
  }
}

// ---- two-kernel apply (fourth-order stencil, or interpolation degree 4 or 5).
// Pass 1: v = E x at every node of Sigma_A u Sigma_G, R right-hand sides (signed rows of
// open surfaces included); v is the instance's own scratch, indexed by node.
template <int D, int P, int R>
__global__ void __launch_bounds__(256) k_gen_extend(DevInst I, const double* __restrict__ x, double* __restrict__ v,
                                                    Gate gate, int inst) {
  if (gate_skip(gate, inst)) return;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= I.nA + I.nG) return;
  double t[3], out[R];
  load_tcp<D>(I, j, t);
  erow_runs<D, P, R>(I, t, x, out);
  const double sg = I.esgn ? I.esgn[j] : 1.0;
#pragma unroll
  for (int r = 0; r < R; ++r) v[(int64_t)j * R + r] = sg * out[r];
}

// Pass 2: y = diag x - w (sum of the stencil's extension values), one wavefront per brick
// with active nodes. Order 2: w = 1/h^2, the six (four) nearest neighbours, summed in
// pairs per axis. Order 4: w = 1/(12h^2), 16 times the nearest pairs' sum minus the sum of
// the pairs two steps away. A neighbour lies in the node's brick or the one across a face
// (bricks are at least 4 nodes wide).
template <int D, int R, int ORDER>
__global__ void __launch_bounds__(256) k_gen_stencil(DevInst I, const double* __restrict__ v,
                                                     const double* __restrict__ x, double* __restrict__ y,
                                                     Gate gate, int inst) {
  constexpr int E = kEdge<D>;
  if (gate_skip(gate, inst)) return;
  const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= I.ntbricks) return;
  const int id = I.tbricks[w];
  const int lane = lane_id();
  const uint64_t mA = I.maskA[id];
  if (!((mA >> lane) & 1ull)) return;
  int l[3];
  local_of<D>(lane, l);
  double s1[R], s2[R];
#pragma unroll
  for (int r = 0; r < R; ++r) { s1[r] = 0.0; s2[r] = 0.0; }
#pragma unroll
  for (int step = 1; step <= ORDER / 2; ++step)
#pragma unroll
    for (int k = 0; k < D; ++k) {
      double pr[2][R];
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        int ln[3] = {l[0], l[1], l[2]};
        ln[k] += sd ? step : -step;
        int b = id;
        if (ln[k] < 0 || ln[k] >= E) {
          b = I.bnbr[id * 2 * D + 2 * k + sd];
          ln[k] = (ln[k] + E) & (E - 1);
        }
        int j = -1;
        if (b >= 0) {
          const int bit = bit_of<D>(ln[0], ln[1], ln[2]);
          const uint64_t ma = I.maskA[b], mg = I.maskG[b];
          if ((ma >> bit) & 1ull) j = I.offA[b] + popc_below(ma, bit);
          else if ((mg >> bit) & 1ull) j = I.nA + I.offG[b] + popc_below(mg, bit);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) pr[sd][r] = j >= 0 ? v[(int64_t)j * R + r] : 0.0;
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double q = pr[0][r] + pr[1][r];
        if (step == 1) s1[r] += q;
        else s2[r] += q;
      }
    }
  const int64_t row = I.vec_off + I.offA[id] + mbcnt64(mA);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const double sum = ORDER == 2 ? s1[r] : 16.0 * s1[r] - s2[r];
    const int64_t e = row * R + r;
    y[e] = I.diag * x[e] - I.inv_h2 * sum;
  }
}

template <int D, int P, int R>
static hipError_t launch_generic_t(const GenericPlan& G, const double* x, double* y, hipStream_t s,
                                   const Gate& gate) {
  for (int i = 0; i < G.ninst; ++i) {
    const DevInst& I = G.inst[i];
    const int n = I.nA + I.nG;
    if (n == 0 || I.ntbricks == 0) continue;
    double* v = G.vscr + G.voff[i] * R;
    bool done = false;
    if constexpr (R == 1) {
      const GenericEPass* e = G.epass ? &G.epass[i] : nullptr;
      if (e && e->dinst && (e->pipe.nplan > 0 || e->nfb > 0)) {
        // the extension pass's tiles name instance 0: gate them by this instance only in a
        // batch of one (a batch's other instances keep their own activity flags)
        const Gate eg = G.ninst == 1 ? gate : Gate{};
        if (e->pipe.nplan > 0)
          hipLaunchKernelGGL((k_apply_pipe<D, P, true>), dim3(e->pipe.nplan), dim3(512),
                             (size_t)e->ucap * sizeof(double), s, e->dinst, e->pipe.wtiles, e->pipe.plan, e->ucap,
                             x, G.vscr, eg);
        if (e->nfb > 0)
          hipLaunchKernelGGL((k_extend_bricks<D, P>), dim3((e->nfb + 3) / 4), dim3(256), 0, s, e->dinst, e->fb,
                             e->nfb, x, G.vscr, eg);
        done = true;
      }
    }
    if (!done)
      hipLaunchKernelGGL((k_gen_extend<D, P, R>), dim3((n + 255) / 256), dim3(256), 0, s, I, x, v, gate, i);
    if (I.order == 4)
      hipLaunchKernelGGL((k_gen_stencil<D, R, 4>), dim3((I.ntbricks + 3) / 4), dim3(256), 0, s, I, v, x, y, gate, i);
    else
      hipLaunchKernelGGL((k_gen_stencil<D, R, 2>), dim3((I.ntbricks + 3) / 4), dim3(256), 0, s, I, v, x, y, gate, i);
  }
  return hipGetLastError();
}

static hipError_t launch_generic(const GenericPlan& G, int d, int p, int nrhs, const double* x, double* y,
                                 hipStream_t s, const Gate& gate) {
  if (!G.vscr || !G.inst || !G.voff) return hipErrorInvalidValue;
#define CPM_CASE(D, P, R) \
  if (d == D && p == P && nrhs == R) return launch_generic_t<D, P, R>(G, x, y, s, gate);
#define CPM_CASES(D, P) CPM_CASE(D, P, 1) CPM_CASE(D, P, 2) CPM_CASE(D, P, 4)
  CPM_CASES(3, 1) CPM_CASES(3, 2) CPM_CASES(3, 3) CPM_CASES(3, 4) CPM_CASES(3, 5)
  CPM_CASES(2, 1) CPM_CASES(2, 2) CPM_CASES(2, 3) CPM_CASES(2, 4) CPM_CASES(2, 5)
#undef CPM_CASES
#undef CPM_CASE
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------- launchers
// Persistent grid of the pipelined apply: resident workgroups per CU (from the
// occupancy calculator, cached per kernel and LDS size) times the CU count,
// no more than the tiles, rounded up to a multiple of 8 (one share per XCD).
static int pipe_grid(int nwork, size_t shm, const void* kern) {
  static std::mutex mu;
  static std::map<std::pair<const void*, size_t>, int> cache;
  static int ncu = 0;
  int per_cu = 0;
  {
    std::lock_guard<std::mutex> lock(mu);
    if (ncu == 0) {
      int dev = 0;
      if (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
        ncu = 256;
    }
    auto it = cache.find({kern, shm});
    if (it != cache.end()) {
      per_cu = it->second;
    } else {
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 512, shm) != hipSuccess || per_cu <= 0)
        per_cu = 1;
      cache[{kern, shm}] = per_cu;
    }
  }
  int g = std::min(ncu * per_cu, nwork);
  return ((g + 7) / 8) * 8;
}

template <int D, int P, int NRHS>
static hipError_t launch_apply_t(const ApplyArgs& A, int variant, const double* x, double* y, hipStream_t s,
                                 const Gate& gate) {
  if (NRHS == 1 && variant == kApplyTwoPass) {
    // extension rows of every band node into the scratch vector, then the stencil
    if (!A.twopass || !A.vscr || (A.pipeE.nplan > 0 && (!A.pipeE.wtiles || !A.pipeE.plan))) return hipErrorInvalidValue;
    const size_t shmE = (size_t)A.ucapE * sizeof(double);
    if (A.pipeE.nplan > 0)
      hipLaunchKernelGGL((k_apply_pipe<D, P, true>), dim3(A.pipeE.nplan), dim3(512), shmE, s, A.insts, A.pipeE.wtiles,
                         A.pipeE.plan, A.ucapE, x, A.vscr, gate);
    if (A.nfbE > 0)
      hipLaunchKernelGGL((k_extend_bricks<D, P>), dim3((A.nfbE + 3) / 4), dim3(256), 0, s, A.insts, A.fbE, A.nfbE, x,
                         A.vscr, gate);
    if (A.nswork > 0)
      hipLaunchKernelGGL((k_stencil<D>), dim3(A.nswork), dim3(512), 0, s, A.insts, A.swork, A.nswork, A.vscr, x, y,
                         gate);
    return hipGetLastError();
  }
  if (A.nwork > 0) {
    const size_t shm = (size_t)A.ucap * sizeof(double) + tile_lds_extra<D>();
    if (NRHS == 1 && variant == kApplyPipelined) {
      if (!A.pipe.wtiles || !A.pipe.plan || A.pipe.nplan <= 0) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_apply_pipe<D, P, false>), dim3(A.pipe.nplan), dim3(512), shm, s, A.insts, A.pipe.wtiles,
                         A.pipe.plan, A.ucap, x, y, gate);
    } else {
      hipLaunchKernelGGL((k_apply_tile<D, P, NRHS>), dim3(A.nwork), dim3(512), shm, s, A.insts, A.work, A.nwork,
                         A.ucap, x, y, gate);
    }
  }
  if (A.nfb > 0)
    hipLaunchKernelGGL((k_apply_fallback<D, P, NRHS>), dim3(A.nfb), dim3(256), 0, s, A.insts, A.fb, A.nfb, x, y,
                       gate);
  return hipGetLastError();
}

hipError_t launch_apply(const ApplyArgs& A, int nrhs, int variant, const double* x, double* y, hipStream_t s,
                        const Gate& gate) {
  const int d = A.d, p = A.p;
  if (A.gen) return launch_generic(*A.gen, d, p, nrhs, x, y, s, gate);
#define CPM_CASE(D, P, R) \
  if (d == D && p == P && nrhs == R)                                                              \
    return launch_apply_t<D, P, R>(A, variant, x, y, s, gate);
  CPM_CASE(3, 3, 1) CPM_CASE(3, 3, 2) CPM_CASE(3, 3, 4)
  CPM_CASE(3, 2, 1) CPM_CASE(3, 2, 2) CPM_CASE(3, 2, 4)
  CPM_CASE(3, 1, 1) CPM_CASE(3, 1, 2) CPM_CASE(3, 1, 4)
  CPM_CASE(2, 3, 1) CPM_CASE(2, 3, 2) CPM_CASE(2, 3, 4)
  CPM_CASE(2, 2, 1) CPM_CASE(2, 2, 2) CPM_CASE(2, 2, 4)
  CPM_CASE(2, 1, 1) CPM_CASE(2, 1, 2) CPM_CASE(2, 1, 4)
#undef CPM_CASE
  return hipErrorInvalidValue;
}

int apply_pipe_grid(int d, int p, int nwork, int ucap, bool extension_pass) {
#define CPM_CASE(D, P)                                                                             \
  if (d == D && p == P)                                                                            \
    return extension_pass ? pipe_grid(nwork, (size_t)ucap * sizeof(double), (const void*)k_apply_pipe<D, P, true>) \
                          : pipe_grid(nwork, (size_t)ucap * sizeof(double) + tile_lds_extra<D>(),          \
                                      (const void*)k_apply_pipe<D, P, false>);
  CPM_CASE(3, 3) CPM_CASE(3, 2) CPM_CASE(3, 1) CPM_CASE(2, 3) CPM_CASE(2, 2) CPM_CASE(2, 1)
#undef CPM_CASE
  // degrees 4 and 5 have only the extension pass (the two-kernel apply)
#define CPM_CASE(D, P)                                                                             \
  if (d == D && p == P)                                                                            \
    return extension_pass ? pipe_grid(nwork, (size_t)ucap * sizeof(double), (const void*)k_apply_pipe<D, P, true>) : 0;
  CPM_CASE(3, 5) CPM_CASE(3, 4) CPM_CASE(2, 5) CPM_CASE(2, 4)
#undef CPM_CASE
  return 0;
}

hipError_t launch_extend(const DevInst& I, const double* u, double* v, hipStream_t s) {
  const int n = I.nA + I.nG;
  if (n == 0) return hipSuccess;
  dim3 g((n + 255) / 256), b(256);
#define CPM_CASE(D, P) \
  if (I.d == D && I.p == P) { hipLaunchKernelGGL((k_extend<D, P>), g, b, 0, s, I, u, v); return hipGetLastError(); }
  CPM_CASE(3, 5) CPM_CASE(3, 4) CPM_CASE(3, 3) CPM_CASE(3, 2) CPM_CASE(3, 1)
  CPM_CASE(2, 5) CPM_CASE(2, 4) CPM_CASE(2, 3) CPM_CASE(2, 2) CPM_CASE(2, 1)
#undef CPM_CASE
  return hipErrorInvalidValue;
}

template <int D, int P, int NRHS>
static hipError_t launch_apply_T_t(const DevInst& I, const double* x, double* z, double* y, hipStream_t s,
                                   const Gate& gate, int inst) {
  if (!I.bnbr || !I.trow_ptr || !I.trows || !I.tbricks) return hipErrorInvalidValue;
  dim3 g((I.nbricks + 3) / 4), b(256);
  hipLaunchKernelGGL((k_OT<D, NRHS>), g, b, 0, s, I, x, z, gate, inst);
  if (I.ntbricks > 0)
    hipLaunchKernelGGL((k_ET<D, P, NRHS>), dim3(I.ntbricks), dim3(64), 0, s, I, x, z, y, gate, inst);
  return hipGetLastError();
}

hipError_t launch_apply_T(const DevInst& I, int nrhs, const double* x, double* zscratch, double* y, hipStream_t s,
                          const Gate& gate, int inst) {
  if (I.nbricks == 0) return hipSuccess;
#define CPM_CASE(D, P, R) \
  if (I.d == D && I.p == P && nrhs == R) return launch_apply_T_t<D, P, R>(I, x, zscratch, y, s, gate, inst);
  CPM_CASE(3, 3, 1) CPM_CASE(3, 3, 2) CPM_CASE(3, 3, 4)
  CPM_CASE(3, 2, 1) CPM_CASE(3, 2, 2) CPM_CASE(3, 2, 4)
  CPM_CASE(3, 1, 1) CPM_CASE(3, 1, 2) CPM_CASE(3, 1, 4)
  CPM_CASE(2, 3, 1) CPM_CASE(2, 3, 2) CPM_CASE(2, 3, 4)
  CPM_CASE(2, 2, 1) CPM_CASE(2, 2, 2) CPM_CASE(2, 2, 4)
  CPM_CASE(2, 1, 1) CPM_CASE(2, 1, 2) CPM_CASE(2, 1, 4)
#undef CPM_CASE
  return hipErrorInvalidValue;
}

}  // namespace cpm
