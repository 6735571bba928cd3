// Internal declarations shared by the host setup code and the HIP kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cpm.h"

namespace cpm {

// ------------------------------------------------------------------ errors
struct Error {
  cpm_status code;
  std::string msg;
};
void set_error(const std::string& msg);
[[noreturn]] void fail(cpm_status code, const std::string& msg);

// ------------------------------------------------------------------ geometry
// Bricks are 4x4x4 nodes in 3-D and 8x8 in 2-D: 64 nodes, one bit each in a
// 64-bit occupancy mask, one wavefront lane each. Local index, last axis
// fastest: 3-D l = 16 lx + 4 ly + lz, 2-D l = 8 lx + ly.
constexpr int kBrickNodes = 64;
inline int brick_edge(int d) { return d == 3 ? 4 : 8; }
inline int brick_shift(int d) { return d == 3 ? 2 : 3; }

struct Surface {
  int kind;
  double params[3];
  double center[3];
};
void closest_point(const Surface& s, int d, const double* x, double* cp);

}  // namespace cpm

// The band as built on the host (node order: Sigma_A bricks, then Sigma_G bricks).
struct cpm_band_s {
  int d = 3, p = 3;
  int reach = 1;                 // the ghost set holds the nodes within `reach` steps along an axis of Sigma_A
  double h = 0, gamma = 0;
  double lo[3] = {0, 0, 0};
  int32_t shape[3] = {1, 1, 1};
  int64_t nA = 0, nG = 0, nBand = 0;
  int closure_iterations = 0;
  // bricks holding at least one node of Sigma_A u Sigma_G, in storage order
  std::vector<int32_t> bcoord;   // [nb][3] brick coordinates
  std::vector<uint64_t> maskA, maskG;
  std::vector<int32_t> offA, offG;  // first node index of the brick in Sigma_A / Sigma_G
  // dense brick map over the bricks' bounding box [bm_lo, bm_lo + bm_dim)
  int32_t bm_lo[3] = {0, 0, 0}, bm_dim[3] = {1, 1, 1};
  std::vector<int32_t> bmap;     // brick id or -1
  // per node (Sigma_A then Sigma_G): grid index and closest point, [node][axis]
  std::vector<int32_t> gidx;
  std::vector<double> cp;
  // extension rows interpolate at ip with sign sgn: ip = cp and sign +1, except on open
  // surfaces for nodes whose closest point lies on a Dirichlet boundary (ip = cp of the
  // mirror image 2 cp - x, sign -1); sgn is empty when every sign is +1
  std::vector<double> ip;
  std::vector<double> sgn;
  int64_t nodes() const { return nA + nG; }
  int64_t nbricks() const { return (int64_t)maskA.size(); }
  // node index of grid point g (global index: Sigma_A then Sigma_G), -1 if absent
  int64_t lookup(const int32_t* g) const;
};

namespace cpm {
// Tiles of the fused apply: 2x2x2 bricks (8^3 nodes) in 3-D, 2x2 (16^2) in 2-D.
struct TileHost {
  int32_t origin[3];     // node coordinates of the tile's lower corner
  int32_t brick[8];      // brick ids (-1 absent), index = bx*4 + by*2 + bz (3-D), bx*2+by (2-D)
  int32_t flo[3];        // u-footprint lower corner (node coordinates)
  int32_t fdim[3];       // u-footprint extent
};
}  // namespace cpm
