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
  double h, inv_h2, diag;   // diag = c + 2d/h^2
  double lo[3];
  const double* tcp;        // closest points in grid units (cp - lo)/h, SoA [d][nA+nG]
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
  // transpose: extension rows bucketed by their cube's lower-corner node (an active node)
  const int32_t* bucket_ptr;   // [nA+1]
  const int32_t* bucket_rows;  // [nA+nG], extension-row ids sorted by corner
  int64_t vec_off;          // offset of this instance's vectors inside a packed batch (doubles / nrhs)
};

// apply kernels for one right-hand side: persistent pipelined (default) or one workgroup per tile
constexpr int kApplyPipelined = 0;
constexpr int kApplyPerTile = 1;

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

}  // namespace cpm
