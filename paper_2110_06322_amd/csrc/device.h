// Plain-old-data layouts shared by the host setup code and the HIP kernels.
#pragma once

#include <cstdint>

namespace cpm {

// One operator instance as the kernels see it. Node arrays are indexed
// Sigma_A first (0..nA-1) then Sigma_G (nA..nA+nG-1).
struct DevTile {
  int32_t origin[3];   // node coordinates of the tile's lower corner
  int32_t fstr[2];     // LDS strides of the footprint box along x and y (z stride 1)
  int32_t fbase;       // dot(flo, (fstr[0], fstr[1], 1)), flo the box's lower corner
  int32_t fb_off;      // footprint brick records fbrec[fb_off .. fb_off+fb_cnt)
  int32_t fb_cnt;
  int32_t job_off;     // extension-row jobs jobs[job_off .. job_off+job_cnt)
  int32_t job_cnt;
  int32_t fvol;        // doubles of LDS the footprint box occupies (with padding)
  int32_t inst;        // instance of the tile in work-ordered copies (0 in an operator's own list)
  int32_t oA[8];       // the tile's bricks (3-D index bx*4+by*2+bz, 2-D bx*2+by):
  uint64_t mA[8];      //   first Sigma_A index and Sigma_A occupancy (0 when absent)
  int32_t bid[8];      //   and brick id (-1 when absent)
};

// a Sigma_A brick overlapping a tile's footprint box (the box is brick aligned,
// so all 64 nodes of the brick lie inside it)
struct FootBrick {
  uint64_t mask;       // Sigma_A occupancy
  int32_t off;         // first Sigma_A index of the brick
  int32_t lds;         // LDS index of the brick's lower corner node
};

// an extension row a tile evaluates: node index (Sigma_A then Sigma_G) and its slot in
// the tile's LDS box of edge T+2 (tile nodes and the face halo)
struct Job {
  int32_t node;
  int32_t slot;
};

struct DevInst {
  int32_t d, p, nA, nG;
  double h, inv_h2, diag;   // order 2: diag = c + 2d/h^2, inv_h2 = 1/h^2; order 4: c + 30d/(12h^2), 1/(12h^2)
  int32_t order;            // stencil order of the operator (2 or 4)
  double lo[3];
  const double* tcp;        // interpolation points in grid units (ip - lo)/h, SoA [d][nA+nG] (ip = cp
                            // except for mirrored Dirichlet rows of open surfaces)
  const double* esgn;       // sign of each extension row [nA+nG], or null when all are +1
  const uint64_t* maskA;
  const uint64_t* maskG;
  const int32_t* offA;
  const int32_t* offG;
  const int32_t* bcoord;    // [nbricks][3]
  const int32_t* bmap;      // dense brick map over [bm_lo, bm_lo+bm_dim), -1 = none
  int32_t bm_lo[3], bm_dim[3];
  const DevTile* tiles;
  const FootBrick* fbrec;   // per-tile footprint brick records
  const Job* jobs;          // per-tile extension-row jobs
  int32_t ntiles;
  int32_t nbricks;
  // transpose: for each brick with active nodes, the extension rows whose interpolation
  // cube overlaps it (ascending row ids)
  const int32_t* trow_ptr;     // [nbricks+1]
  const int32_t* trows;
  const int32_t* tbricks;      // bricks with active nodes
  int32_t ntbricks;
  int64_t vec_off;          // offset of this instance's vectors inside a packed batch (doubles / nrhs)
  // two-pass apply: per-tile lists of the extension pass (jobs = the tile's own band
  // nodes, no face halo), the face-neighbour bricks of every brick, and the offset of
  // this instance's extension values inside a packed batch (nodes of Sigma_A u Sigma_G)
  const FootBrick* fbrecE;
  const Job* jobsE;
  const int32_t* bnbr;      // [nbricks][2d]: brick across face (axis k, side s) at 2k+s, -1 = none
  int64_t vnode_off;
};

// apply kernels for one right-hand side: persistent pipelined (default), one workgroup per
// tile, or two passes (extension rows of every band node once, written to a scratch vector,
// then the (2d+1)-point stencil from it)
constexpr int kApplyPipelined = 0;
constexpr int kApplyPerTile = 1;
constexpr int kApplyTwoPass = 2;

// Work gate of the operator and preconditioner kernels inside Krylov cycles.
// count (device int, may be null): every system has stopped when it reads 0;
// act (device [instances * nrhs], may be null): instance i is skipped when none
// of act[i*nrhs .. i*nrhs + nrhs) is set.
struct Gate {
  const int32_t* count = nullptr;
  const int32_t* act = nullptr;
  int32_t nrhs = 1;
};

// (instance, item) pair of a work list: a tile, a subdomain or a vector chunk
struct WorkItem {
  int32_t inst, idx;
};

// work items one workgroup of the persistent apply takes: positions first,
// first + step, ... below end of the work list
struct PipeSpan {
  int32_t first, end, step, pad;
};

// persistent apply's view of a work list: wtiles[w] is a copy of the tile of
// work item w (with its instance), read in one load instead of a work item ->
// instance -> tile chain; plan[b] the span of workgroup b (nplan workgroups)
struct PipeWork {
  const DevTile* wtiles = nullptr;
  const PipeSpan* plan = nullptr;
  int nplan = 0;
};

// What an apply launch needs of an operator or a batch: the fused kernel's tile
// list (and its persistent work plan), the slow-path list, and for the two-pass
// variant the extension pass's plan, the stencil pass's list and a scratch
// vector of N_A + N_G extension values per instance.
// Two-kernel apply of operators the fused kernels do not cover (fourth-order stencil, or
// interpolation degree above 3): host copies of the instances, the node offset of each
// instance's extension values in the scratch vector (times nrhs), and that vector.
struct GenericEPass {
  // one right-hand side, p <= 3: the extension pass of the two-pass apply (LDS tiles) instead
  // of the per-row global gathers; its tiles name instance 0, so dinst points at this
  // instance's record in device memory and v is written at vnode_off + node
  const DevInst* dinst = nullptr;   // device
  PipeWork pipe;
  int ucap = 0;
  const WorkItem* fb = nullptr;     // bricks of the extension-pass tiles whose footprint exceeds the LDS budget
  int nfb = 0;
};

struct GenericPlan {
  const DevInst* inst = nullptr;    // host array of ninst
  const int64_t* voff = nullptr;    // host array of ninst (equal to each instance's vnode_off)
  int ninst = 0;
  double* vscr = nullptr;           // device, sum of (nA + nG) over the instances, times nrhs
  const GenericEPass* epass = nullptr;   // host array of ninst, or null
};

struct ApplyArgs {
  const GenericPlan* gen = nullptr;   // set: every apply takes the two-kernel path
  int d = 3, p = 3;
  const DevInst* insts = nullptr;
  const WorkItem* work = nullptr;
  int nwork = 0;
  PipeWork pipe;
  int ucap = 0;
  const WorkItem* fb = nullptr;
  int nfb = 0;
  bool twopass = false;
  PipeWork pipeE;
  int ucapE = 0;
  const WorkItem* swork = nullptr;
  int nswork = 0;
  const WorkItem* fbE = nullptr;   // bricks of the extension-pass tiles whose footprint exceeds the LDS budget
  int nfbE = 0;
  double* vscr = nullptr;
};

}  // namespace cpm
