// Plain-old-data layouts shared by the host setup code and the HIP kernels.
#pragma once

#include <cstdint>

namespace cpm {

// One operator instance as the kernels see it. Node arrays are indexed
// Sigma_A first (0..nA-1) then Sigma_G (nA..nA+nG-1).
struct DevTile {
  int32_t origin[3];   // node coordinates of the tile's lower corner
  int32_t brick[8];    // brick ids (-1 when absent); 3-D index bx*4+by*2+bz, 2-D bx*2+by
  int32_t flo[3];      // LDS footprint of the tile's interpolation cubes: lower corner
  int32_t fdim[3];     //   and extent (node units)
  int32_t fb_off;      // non-empty bricks overlapping the footprint: fbricks[fb_off .. fb_off+fb_cnt)
  int32_t fb_cnt;
};

constexpr int kMaxFootprintBricks = 256;

struct DevInst {
  int32_t d, p, nA, nG;
  double h, inv_h2, diag;   // diag = c + 2d/h^2
  double lo[3];
  const double* cp;         // SoA [d][nA+nG]
  const uint64_t* maskA;
  const uint64_t* maskG;
  const int32_t* offA;
  const int32_t* offG;
  const int32_t* bcoord;    // [nbricks][3]
  const int32_t* bmap;      // dense brick map over [bm_lo, bm_lo+bm_dim), -1 = none
  int32_t bm_lo[3], bm_dim[3];
  const DevTile* tiles;
  const int32_t* fbricks;   // per-tile footprint brick lists
  int32_t ntiles;
  int32_t nbricks;
  // transpose: extension rows bucketed by their cube's lower-corner node (an active node)
  const int32_t* bucket_ptr;   // [nA+1]
  const int32_t* bucket_rows;  // [nA+nG], extension-row ids sorted by corner
  int64_t vec_off;          // offset of this instance's vectors inside a packed batch (doubles / nrhs)
};

// (instance, item) pair of a work list: a tile, a subdomain or a vector chunk
struct WorkItem {
  int32_t inst, idx;
};

}  // namespace cpm
