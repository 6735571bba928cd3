// Host-side helpers: HIP error checks, device buffers, the operator object.
#pragma once

#include <hip/hip_runtime_api.h>

#include <memory>
#include <string>
#include <vector>

#include "device.h"
#include "internal.h"

namespace cpm {

inline void hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    fail(CPM_ERR_OOM, std::string(what) + ": device allocation failed");
  fail(CPM_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Owning device allocation.
template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t count) {
    if (count <= n && p) return;
    release();
    if (count == 0) return;
    hip_check(hipMalloc((void**)&p, count * sizeof(T)), "hipMalloc");
    n = count;
  }
  void upload(const T* src, size_t count) {
    alloc(count);
    if (count) hip_check(hipMemcpy(p, src, count * sizeof(T), hipMemcpyHostToDevice), "upload");
  }
  void upload(const std::vector<T>& v) { upload(v.data(), v.size()); }
};

// kernel launchers (apply.hip)
// gate: lets Krylov cycles skip instances whose systems have stopped (see Gate)
hipError_t launch_apply(const ApplyArgs& A, int nrhs, int variant, const double* x, double* y, hipStream_t s,
                        const Gate& gate = Gate{});
// workgroups of the persistent apply for a work list (a multiple of 8: as many
// as are resident at once, at most one per work item, rounded up)
int apply_pipe_grid(int d, int p, int nwork, int ucap, bool extension_pass = false);
// Orders a work list for the persistent apply and gives each of `grid`
// workgroups its span (workgroup b runs on XCD b mod 8 and takes tiles of that
// XCD's eighth of the list). Lists of at most kCostOrderMaxTiles items are
// balanced by cost (heaviest first, each to the least loaded workgroup of its
// XCD, whose tiles then lie contiguous); longer lists keep their order and the
// workgroups of an XCD walk its eighth with a stride, so that tiles processed
// at the same time are neighbours in L2.
void plan_pipe(std::vector<WorkItem>& work, const std::vector<int32_t>& cost, int grid,
               std::vector<PipeSpan>& plan);
hipError_t launch_extend(const DevInst& I, const double* u, double* v, hipStream_t s);
hipError_t launch_apply_T(const DevInst& I, int nrhs, const double* x, double* zscratch, double* y,
                          hipStream_t s, const Gate& gate = Gate{}, int inst = 0);

// operator algebra (poly.hip): y = a x; vn = c v - av, y += a vn (vn may alias av)
hipError_t poly_scale(int64_t n, double a, const double* x, double* y, hipStream_t s);
hipError_t poly_step(int64_t n, double c, double a, const double* v, const double* av, double* vn, double* y,
                     hipStream_t s);
struct Chunk;
hipError_t poly_step_chunks(int R, const Chunk* chunks, int nchunks, const double* shift, double a, const double* v,
                            const double* av, double* vn, double* y, hipStream_t s);

inline int vbox_nodes(int d) { return d == 3 ? 10 * 10 * 10 : 18 * 18; }
// footprint bricks a tile may stage in the pipelined apply (8 per wavefront)
constexpr int kMaxFootBricks = 64;
// work lists of at most this many tiles are balanced by cost (up to 16 tiles
// per workgroup of a 512-workgroup persistent apply; beyond that the balance
// gained is small and brick order's L2 locality is worth more)
constexpr int kCostOrderMaxTiles = 8192;
// fixed cost of a tile in the balance, in extension rows
constexpr int kTileCostBase = 128;

// LDS of the fused apply besides the footprint: the tile's box of extension values
inline size_t tile_lds_extra_bytes(int d) { return (size_t)vbox_nodes(d) * 8; }
constexpr size_t kApplyLdsBytes = 64 * 1024;
// highest polynomial degree + 1 of the operator algebra (cpm_poly_apply, polynomial solves)
constexpr int kMaxPoly = 5;

}  // namespace cpm

struct cpm_batch_s;
struct cpm_operator_s {
  std::shared_ptr<const cpm_band_s> band;   // host copy (preconditioner setup reads it)
  double c = 1.0;
  cpm::DevInst I{};                         // device pointers, vec_off = 0
  cpm::DevBuf<cpm::DevInst> d_inst;
  cpm::DevBuf<double> d_tcp;   // interpolation points in grid units, SoA
  cpm::DevBuf<double> d_sgn;   // extension-row signs (open surfaces with Dirichlet boundaries only)
  cpm::DevBuf<uint64_t> d_maskA, d_maskG;
  cpm::DevBuf<int32_t> d_offA, d_offG, d_bcoord, d_bmap, d_bptr, d_brows, d_tlist;
  cpm::DevBuf<cpm::DevTile> d_tiles;
  cpm::DevBuf<cpm::FootBrick> d_fbrec;
  cpm::DevBuf<cpm::Job> d_jobs;
  std::vector<cpm::DevTile> tiles;          // host copy
  std::vector<int32_t> tile_fvol;           // footprint nodes per tile
  cpm::DevBuf<cpm::WorkItem> d_work, d_fb;      // (instance 0, tile) lists: LDS path / fallback
  cpm::DevBuf<cpm::DevTile> d_wtiles;           // tiles of d_work in work order
  cpm::DevBuf<cpm::PipeSpan> d_plan;            // spans of the persistent apply's workgroups
  int nplan = 0;
  cpm::PipeWork pipe() const { return cpm::PipeWork{d_wtiles.p, d_plan.p, nplan}; }
  std::vector<cpm::WorkItem> h_work, h_fb;
  int nwork = 0, nfb = 0, ucap = 0;
  int apply_variant = cpm::kApplyPipelined;   // one-RHS apply kernel (tunable)
  // two-pass apply: extension-pass tile lists (own band nodes only) and work plan, the
  // stencil pass's tile list, face-neighbour bricks, the scratch of extension values
  bool twopass = false;
  cpm::DevBuf<cpm::FootBrick> d_fbrecE;
  cpm::DevBuf<cpm::Job> d_jobsE;
  cpm::DevBuf<int32_t> d_bnbr;
  std::vector<cpm::DevTile> tilesE;
  std::vector<cpm::WorkItem> h_workE, h_swork, h_fbE;
  cpm::DevBuf<cpm::WorkItem> d_fbE;
  cpm::DevBuf<cpm::DevTile> d_wtilesE;
  cpm::DevBuf<cpm::PipeSpan> d_planE;
  cpm::DevBuf<cpm::WorkItem> d_swork;
  int nplanE = 0, ucapE = 0;
  mutable cpm::DevBuf<double> d_v;
  // stencil order; generic: the two-kernel apply (order 4, or p > 3) through gen
  int order = 2;
  int lds_bytes = (int)cpm::kApplyLdsBytes;   // LDS budget of the fused apply's tiles
  bool generic = false;
  int64_t gvoff = 0;
  cpm::GenericEPass gep;
  cpm::GenericPlan gen;
  cpm::ApplyArgs apply_args() const {
    cpm::ApplyArgs A;
    A.gen = generic ? &gen : nullptr;
    A.d = I.d; A.p = I.p; A.insts = d_inst.p;
    A.work = d_work.p; A.nwork = nwork; A.pipe = pipe(); A.ucap = ucap;
    A.fb = d_fb.p; A.nfb = nfb;
    A.twopass = twopass;
    A.pipeE = cpm::PipeWork{d_wtilesE.p, d_planE.p, nplanE};
    A.ucapE = ucapE;
    A.swork = d_swork.p; A.nswork = (int)h_swork.size();
    A.fbE = d_fbE.p; A.nfbE = (int)h_fbE.size();
    A.vscr = d_v.p;
    return A;
  }
  // workspace of single solves (one solve at a time per operator)
  mutable std::shared_ptr<cpm_batch_s> solve_cache;
  mutable int64_t solve_cache_key = -1;
  mutable cpm::DevBuf<double> d_z;          // transpose scratch [(nA+nG) * 4]
  mutable cpm::DevBuf<double> d_part;       // chunk sums of cpm_shift_gradient
  mutable cpm::DevBuf<double> d_poly;       // two vectors of cpm_poly_apply
  int64_t nA() const { return band->nA; }
};
