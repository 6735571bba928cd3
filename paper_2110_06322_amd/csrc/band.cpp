// Host construction of the CPM computational band (paper Sec. 2.1).
//
// Sets built (the paper states their properties; these are the definitions):
//   B_gamma = grid nodes x with |x - cp(x)| <= gamma (1 + 1e-10);
//   Sigma_A = union over x in B_gamma of the interpolation cube of cp(x),
//             b + {0..p}^d with b = floor((cp - lo)/h - (p-1)/2);
//   Sigma_G = grid neighbours (+-e_k) of Sigma_A that are not in Sigma_A;
//   closure : the cube of every node of Sigma_A u Sigma_G lies in Sigma_A
//             (checked; a missing node is added at most once, else an error).
// Storage: 64-node bricks (4^3 in 3-D, 8^2 in 2-D) with one occupancy bit per
// node, ordered along a Morton curve over 2^d-brick tiles; Sigma_A nodes come
// first (brick order, then local index), then Sigma_G nodes. Closest points
// use the same IEEE operation order as the textbook formulas (no FMA
// contraction), so independent implementations agree bit for bit.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <climits>
#include <cstring>
#include <limits>
#include <memory>
#include <numeric>

#include "internal.h"

namespace cpm {

static inline double sq(double v) { return v * v; }

void closest_point(const Surface& s, int d, const double* x, double* cp) {
  switch (s.kind) {
    case CPM_SURF_CIRCLE:
    case CPM_SURF_SPHERE: {
      double q[3];
      for (int k = 0; k < d; ++k) q[k] = x[k] - s.center[k];
      double n = d == 2 ? std::sqrt(q[0] * q[0] + q[1] * q[1])
                        : std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
      double f = s.params[0] / n;
      for (int k = 0; k < d; ++k) cp[k] = s.center[k] + f * q[k];
      return;
    }
    case CPM_SURF_TORUS: {
      // nearest point of the centre circle, then radially inside the tube
      const double R = s.params[0], r = s.params[1];
      double rho = std::sqrt(x[0] * x[0] + x[1] * x[1]);
      double sr = R / rho;
      double qx = sr * x[0], qy = sr * x[1];
      double ex = x[0] - qx, ey = x[1] - qy;
      double m = std::sqrt(ex * ex + ey * ey + x[2] * x[2]);
      double f = r / m;
      cp[0] = qx + f * ex;
      cp[1] = qy + f * ey;
      cp[2] = f * x[2];
      return;
    }
    case CPM_SURF_ELLIPSOID: {
      // y_k = a_k^2 x_k / (a_k^2 + t), t the root of
      // F(t) = sum_k (a_k x_k/(a_k^2 + t))^2 - 1 (decreasing for t > -amin^2),
      // bracketed by [-amin^2 + amin |x_kmin|, -amin^2 + |a x|] (Eberly 2013),
      // bisected until the midpoint stops moving.
      const double* a = s.params;
      double a2[3] = {a[0] * a[0], a[1] * a[1], a[2] * a[2]};
      int kmin = 0;
      for (int k = 1; k < 3; ++k)
        if (a[k] < a[kmin]) kmin = k;
      double ax[3] = {x[0] * a[0], x[1] * a[1], x[2] * a[2]};
      // Zero coordinates along every smallest axis and sum over the other axes of
      // (a_k x_k / (a_k^2 - amin^2))^2 below 1: F has no root above -amin^2 and the
      // point lies on the medial set, where two mirror closest points exist. NaN.
      {
        bool on_min_axis = false;
        double frest = 0.0;
        for (int k = 0; k < 3; ++k) {
          if (x[k] == 0.0) continue;
          if (a[k] == a[kmin]) on_min_axis = true;
          else {
            double r = ax[k] / (a2[k] - a2[kmin]);
            frest += r * r;
          }
        }
        if (!on_min_axis && frest < 1.0) {
          cp[0] = cp[1] = cp[2] = std::numeric_limits<double>::quiet_NaN();
          return;
        }
      }
      double nrm = std::sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
      double lo = -a2[kmin] + a[kmin] * std::fabs(x[kmin]);
      double hi = -a2[kmin] + nrm;
      for (int it = 0; it < 2000; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        double r0 = ax[0] / (a2[0] + mid), r1 = ax[1] / (a2[1] + mid), r2 = ax[2] / (a2[2] + mid);
        double F = r0 * r0 + r1 * r1 + r2 * r2 - 1.0;
        if (F > 0.0) lo = mid;
        else if (F < 0.0) hi = mid;
        else { lo = mid; hi = mid; }
      }
      double t = 0.5 * (lo + hi);
      for (int k = 0; k < 3; ++k) cp[k] = a2[k] * x[k] / (a2[k] + t);
      return;
    }
    default:
      fail(CPM_ERR_ARG, "unknown surface kind");
  }
}

}  // namespace cpm

using namespace cpm;

int64_t cpm_band_s::lookup(const int32_t* g) const {
  const int sh = brick_shift(d), E = brick_edge(d);
  int32_t b[3] = {0, 0, 0}, l[3] = {0, 0, 0};
  for (int k = 0; k < d; ++k) {
    if (g[k] < 0 || g[k] >= shape[k]) return -1;
    b[k] = (g[k] >> sh) - bm_lo[k];
    if (b[k] < 0 || b[k] >= bm_dim[k]) return -1;
    l[k] = g[k] & (E - 1);
  }
  int64_t bi = d == 3 ? ((int64_t)b[0] * bm_dim[1] + b[1]) * bm_dim[2] + b[2]
                      : (int64_t)b[0] * bm_dim[1] + b[1];
  int32_t id = bmap[bi];
  if (id < 0) return -1;
  int bit = d == 3 ? l[0] * 16 + l[1] * 4 + l[2] : l[0] * 8 + l[1];
  uint64_t below = (bit == 0) ? 0ull : ((~0ull) >> (64 - bit));
  if ((maskA[id] >> bit) & 1ull) return offA[id] + __builtin_popcountll(maskA[id] & below);
  if ((maskG[id] >> bit) & 1ull) return nA + offG[id] + __builtin_popcountll(maskG[id] & below);
  return -1;
}

namespace {

struct Grid {
  int d, p;
  double h, lo[3];
  int32_t shape[3];
  int E, sh;
  int32_t bshape[3];
};

inline void local_of(int d, int bit, int* l) {
  if (d == 3) { l[0] = bit >> 4; l[1] = (bit >> 2) & 3; l[2] = bit & 3; }
  else { l[0] = bit >> 3; l[1] = bit & 7; l[2] = 0; }
}
inline int bit_of(int d, const int* l) { return d == 3 ? l[0] * 16 + l[1] * 4 + l[2] : l[0] * 8 + l[1]; }

// Dense brick-mask field over a brick bounding box.
struct MaskField {
  int d;
  int32_t lo[3], dim[3];
  std::vector<uint64_t> A, G;
  int64_t index(const int32_t* b) const {
    int64_t i = 0;
    for (int k = 0; k < d; ++k) {
      int32_t v = b[k] - lo[k];
      if (v < 0 || v >= dim[k]) return -1;
      i = i * dim[k] + v;
    }
    return i;
  }
  void coords(int64_t i, int32_t* b) const {
    for (int k = d - 1; k >= 0; --k) { b[k] = (int32_t)(i % dim[k]) + lo[k]; i /= dim[k]; }
  }
};

inline uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  uint64_t m = 0;
  for (int i = 0; i < 21; ++i) {
    m |= (uint64_t)((x >> i) & 1) << (3 * i + 2);
    m |= (uint64_t)((y >> i) & 1) << (3 * i + 1);
    m |= (uint64_t)((z >> i) & 1) << (3 * i);
  }
  return m;
}

void cube_base(const Grid& G, const double* cp, int32_t* b) {
  for (int k = 0; k < G.d; ++k) {
    double t = (cp[k] - G.lo[k]) / G.h;
    b[k] = (int32_t)std::floor(t - (G.p - 1) / 2.0);
  }
}

}  // namespace

namespace {

// Closest points of the surface, from an analytic kind or a caller's callback,
// evaluated for many points at once; flag = 1 marks a closest point on a
// boundary part with homogeneous Dirichlet conditions (open surfaces).
struct CpSource {
  const Surface* S = nullptr;
  cpm_cp_callback cb = nullptr;
  void* ctx = nullptr;
  int d = 3;
  void eval(int64_t n, const double* x, double* cp, int32_t* flag) const {
    if (n <= 0) return;
    if (S) {
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < n; ++i) closest_point(*S, d, x + i * d, cp + i * d);
      std::fill(flag, flag + n, 0);
      return;
    }
    const int64_t chunk = int64_t(1) << 20;
    for (int64_t s0 = 0; s0 < n; s0 += chunk) {
      const int64_t m = std::min(chunk, n - s0);
      if (cb(m, x + s0 * d, cp + s0 * d, flag + s0, ctx) != 0) fail(CPM_ERR_ARG, "closest point callback failed");
    }
  }
  // cp, the interpolation point ip (cp, or for a Dirichlet-flagged point the closest
  // point of its mirror image 2 cp - x) and the sign of the extension row (+1 / -1)
  void interp(int64_t n, const double* x, double* cp, double* ip, double* sg) const {
    std::vector<int32_t> flag(n > 0 ? n : 1);
    eval(n, x, cp, flag.data());
    std::vector<int64_t> mir;
    for (int64_t i = 0; i < n; ++i) {
      for (int k = 0; k < d; ++k) ip[i * d + k] = cp[i * d + k];
      sg[i] = 1.0;
      if (flag[i]) mir.push_back(i);
    }
    if (mir.empty()) return;
    std::vector<double> xb(mir.size() * d), cpb(mir.size() * d);
    std::vector<int32_t> fb(mir.size());
    for (size_t q = 0; q < mir.size(); ++q)
      for (int k = 0; k < d; ++k) xb[q * d + k] = 2.0 * cp[mir[q] * d + k] - x[mir[q] * d + k];
    eval((int64_t)mir.size(), xb.data(), cpb.data(), fb.data());
    for (size_t q = 0; q < mir.size(); ++q) {
      for (int k = 0; k < d; ++k) ip[mir[q] * d + k] = cpb[q * d + k];
      sg[mir[q]] = -1.0;
    }
  }
};

cpm_band_s* build_band_impl(const CpSource& src, int32_t d, double h, int32_t p, const double* lo, const double* hi,
                            double gamma, int32_t reach) {
  if (gamma <= 0) {
    double a = (p + 1) / 2.0;
    gamma = h * std::sqrt((d - 1) * a * a + (reach + a) * (reach + a));
  }
  Grid G;
  G.d = d; G.p = p; G.h = h;
  G.E = brick_edge(d); G.sh = brick_shift(d);
  for (int k = 0; k < 3; ++k) { G.lo[k] = 0; G.shape[k] = 1; G.bshape[k] = 1; }
  for (int k = 0; k < d; ++k) {
    if (!(hi[k] > lo[k])) fail(CPM_ERR_ARG, "hi must exceed lo");
    G.lo[k] = lo[k];
    double n = std::floor((hi[k] - lo[k]) / h + 0.5) + 1;
    if (n > 1.0e6) fail(CPM_ERR_ARG, "grid too large");
    G.shape[k] = (int32_t)n;
    G.bshape[k] = (G.shape[k] + G.E - 1) / G.E;
  }
  const double thr = gamma * (1.0 + 1e-10);
  const double halfdiag = std::sqrt((double)d) * 0.5 * (G.E - 1) * h;
  const int64_t kChunk = int64_t(1) << 20;
  auto brick_of = [&](int64_t bi, int32_t* b) {
    int64_t r = bi;
    for (int k = d - 1; k >= 0; --k) { b[k] = (int32_t)(r % G.bshape[k]); r /= G.bshape[k]; }
  };

  // ---- pass 1: candidate bricks by the 1-Lipschitz distance bound at brick centres
  int64_t nbr_all = (int64_t)G.bshape[0] * G.bshape[1] * (d == 3 ? G.bshape[2] : 1);
  std::vector<uint8_t> cand(nbr_all, 0);
  {
    std::vector<double> x, cp;
    std::vector<int32_t> fl;
    for (int64_t s0 = 0; s0 < nbr_all; s0 += kChunk) {
      const int64_t m = std::min(kChunk, nbr_all - s0);
      x.resize(m * d);
      cp.resize(m * d);
      fl.resize(m);
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < m; ++i) {
        int32_t b[3] = {0, 0, 0};
        brick_of(s0 + i, b);
        for (int k = 0; k < d; ++k) x[i * d + k] = G.lo[k] + (b[k] * G.E + 0.5 * (G.E - 1)) * h;
      }
      src.eval(m, x.data(), cp.data(), fl.data());
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < m; ++i) {
        double sd = 0;
        for (int k = 0; k < d; ++k) sd += sq(x[i * d + k] - cp[i * d + k]);
        if (!(std::sqrt(sd) > thr + halfdiag + 1e-9)) cand[s0 + i] = 1;  // NaN keeps the brick
      }
    }
  }
  // bounding box of candidates, grown by 2 bricks for cubes and neighbours (mirrored
  // interpolation points stay within the band's reach of the surface)
  MaskField F;
  F.d = d;
  int32_t bl[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, bh[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
  std::vector<int64_t> cand_list;
  for (int64_t bi = 0; bi < nbr_all; ++bi) {
    if (!cand[bi]) continue;
    cand_list.push_back(bi);
    int32_t b[3];
    brick_of(bi, b);
    for (int k = 0; k < d; ++k) { bl[k] = std::min(bl[k], b[k]); bh[k] = std::max(bh[k], b[k]); }
  }
  if (cand_list.empty()) fail(CPM_ERR_BAND, "the surface does not meet the grid");
  std::vector<uint8_t>().swap(cand);
  int64_t fsize = 1;
  for (int k = 0; k < 3; ++k) { F.lo[k] = 0; F.dim[k] = 1; }
  for (int k = 0; k < d; ++k) {
    F.lo[k] = bl[k] - 2;
    F.dim[k] = bh[k] - bl[k] + 5;
    fsize *= F.dim[k];
  }
  F.A.assign(fsize, 0);
  F.G.assign(fsize, 0);

  const int P1 = p + 1;
  const int ncube = d == 3 ? P1 * P1 * P1 : P1 * P1;
  auto mark_cube = [&](const double* ipv, std::vector<uint64_t>& M) -> bool {
    int32_t b[3] = {0, 0, 0};
    cube_base(G, ipv, b);
    for (int q = 0; q < ncube; ++q) {
      int32_t g[3] = {0, 0, 0};
      int r = q;
      for (int k = d - 1; k >= 0; --k) { g[k] = b[k] + r % P1; r /= P1; }
      int32_t bb[3] = {0, 0, 0};
      int l[3] = {0, 0, 0};
      for (int k = 0; k < d; ++k) {
        if (g[k] < 0 || g[k] >= G.shape[k]) return false;
        bb[k] = g[k] >> G.sh;
        l[k] = g[k] & (G.E - 1);
      }
      int64_t fi = F.index(bb);
      if (fi < 0) return false;
      __atomic_fetch_or(&M[fi], 1ull << bit_of(d, l), __ATOMIC_RELAXED);
    }
    return true;
  };

  // ---- pass 2: band nodes; mark the cubes of their interpolation points into Sigma_A
  int64_t nband = 0;
  bool outside = false;
  double bad_x[3] = {0, 0, 0}, bad_cp[3] = {0, 0, 0};
  {
    const int64_t per = kChunk / kBrickNodes;
    std::vector<double> x, cp, ip, sg, xs;
    std::vector<int32_t> fl;
    for (size_t c0 = 0; c0 < cand_list.size(); c0 += per) {
      const size_t c1 = std::min(cand_list.size(), c0 + per);
      x.clear();
      for (size_t ci = c0; ci < c1; ++ci) {
        int32_t b[3] = {0, 0, 0};
        brick_of(cand_list[ci], b);
        for (int bit = 0; bit < kBrickNodes; ++bit) {
          int l[3];
          local_of(d, bit, l);
          int32_t g[3] = {0, 0, 0};
          bool in = true;
          for (int k = 0; k < d; ++k) {
            g[k] = b[k] * G.E + l[k];
            if (g[k] >= G.shape[k]) in = false;
          }
          if (!in) continue;
          for (int k = 0; k < d; ++k) x.push_back(G.lo[k] + g[k] * h);
        }
      }
      const int64_t m = (int64_t)x.size() / d;
      cp.resize(m * d);
      fl.resize(m);
      src.eval(m, x.data(), cp.data(), fl.data());
      // keep the band nodes, then their interpolation points
      xs.clear();
      for (int64_t i = 0; i < m; ++i) {
        double sd = 0;
        for (int k = 0; k < d; ++k) sd += (x[i * d + k] - cp[i * d + k]) * (x[i * d + k] - cp[i * d + k]);
        if (!(std::sqrt(sd) <= thr)) continue;
        for (int k = 0; k < d; ++k) xs.push_back(x[i * d + k]);
      }
      const int64_t nb = (int64_t)xs.size() / d;
      nband += nb;
      cp.resize(nb * d);
      ip.resize(nb * d);
      sg.resize(nb);
      src.interp(nb, xs.data(), cp.data(), ip.data(), sg.data());
#pragma omp parallel for schedule(dynamic, 1024)
      for (int64_t i = 0; i < nb; ++i) {
        if (!mark_cube(&ip[i * d], F.A)) {
#pragma omp critical(cpm_band_outside)
          if (!outside) {
            outside = true;
            for (int k = 0; k < 3; ++k) { bad_x[k] = k < d ? xs[i * d + k] : 0.0; bad_cp[k] = k < d ? ip[i * d + k] : 0.0; }
          }
        }
      }
    }
  }
  if (outside) {
    char msg[256];
    std::snprintf(msg, sizeof msg,
                  "an interpolation cube leaves the grid box (node x = (%g, %g, %g), interpolation point (%g, %g, %g))",
                  bad_x[0], bad_x[1], bad_x[2], bad_cp[0], bad_cp[1], bad_cp[2]);
    fail(CPM_ERR_BAND, msg);
  }

  // nodes of a mask field as coordinates (brick order of the field)
  auto node_coords = [&](const std::vector<uint64_t>& M1, const std::vector<uint64_t>* M2, std::vector<double>& x) {
    x.clear();
    for (int64_t fi = 0; fi < fsize; ++fi) {
      uint64_t m = M1[fi] | (M2 ? (*M2)[fi] : 0ull);
      if (!m) continue;
      int32_t b[3] = {0, 0, 0};
      F.coords(fi, b);
      while (m) {
        int bit = __builtin_ctzll(m);
        m &= m - 1;
        int l[3];
        local_of(d, bit, l);
        for (int k = 0; k < d; ++k) x.push_back(G.lo[k] + (b[k] * G.E + l[k]) * h);
      }
    }
  };

  // ---- Sigma_G and the closure check
  int iters = 0;
  for (;;) {
    std::fill(F.G.begin(), F.G.end(), 0ull);
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t fi = 0; fi < fsize; ++fi) {
      uint64_t m = F.A[fi];
      if (!m) continue;
      int32_t b[3] = {0, 0, 0};
      F.coords(fi, b);
      while (m) {
        int bit = __builtin_ctzll(m);
        m &= m - 1;
        int l[3];
        local_of(d, bit, l);
        for (int k = 0; k < d; ++k)
          for (int s = -reach; s <= reach; ++s) {
            if (s == 0) continue;
            int32_t g[3] = {0, 0, 0};
            for (int q = 0; q < d; ++q) g[q] = b[q] * G.E + l[q];
            g[k] += s;
            if (g[k] < 0 || g[k] >= G.shape[k]) {
#pragma omp atomic write
              outside = true;
              continue;
            }
            int32_t bb[3] = {0, 0, 0};
            int ll[3] = {0, 0, 0};
            for (int q = 0; q < d; ++q) { bb[q] = g[q] >> G.sh; ll[q] = g[q] & (G.E - 1); }
            int64_t fj = F.index(bb);
            if (fj < 0) {
#pragma omp atomic write
              outside = true;
              continue;
            }
            uint64_t bitm = 1ull << bit_of(d, ll);
            if (!(F.A[fj] & bitm)) __atomic_fetch_or(&F.G[fj], bitm, __ATOMIC_RELAXED);
          }
      }
    }
    if (outside) fail(CPM_ERR_BAND, "a ghost node leaves the grid box");
    // closure: the cube of every node of Sigma_A u Sigma_G must lie in Sigma_A
    std::vector<uint64_t> add(fsize, 0ull);
    std::vector<double> x, cp, ip, sg;
    node_coords(F.A, &F.G, x);
    const int64_t n = (int64_t)x.size() / d;
    cp.resize(n * d);
    ip.resize(n * d);
    sg.resize(n);
    src.interp(n, x.data(), cp.data(), ip.data(), sg.data());
    bool bad = false;
    int64_t degenerate = -1;
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
      bool finite = true;
      for (int k = 0; k < d; ++k) finite = finite && std::isfinite(ip[i * d + k]);
      if (!finite) {
#pragma omp critical(cpm_band_degenerate)
        if (degenerate < 0) degenerate = i;
      } else if (!mark_cube(&ip[i * d], add)) {
#pragma omp atomic write
        bad = true;
      }
    }
    if (degenerate >= 0) {
      char msg[256];
      std::snprintf(msg, sizeof msg,
                    "the band node x = (%g, %g, %g) has no unique closest point (the band reaches the medial "
                    "axis; refine h)", x[degenerate * d], x[degenerate * d + 1], d == 3 ? x[degenerate * d + 2] : 0.0);
      fail(CPM_ERR_BAND, msg);
    }
    if (bad) fail(CPM_ERR_BAND, "an interpolation cube leaves the grid box");
    bool grew = false;
    for (int64_t fi = 0; fi < fsize; ++fi)
      if (add[fi] & ~F.A[fi]) { grew = true; F.A[fi] |= add[fi]; }
    if (!grew) break;
    if (++iters > 1) fail(CPM_ERR_BAND, "band closure did not converge");
  }

  // ---- storage order: Morton over 2^d-brick tiles, then brick within tile
  auto* B = new cpm_band_s();
  std::unique_ptr<cpm_band_s> guard(B);
  B->d = d; B->p = p; B->h = h; B->gamma = gamma; B->reach = reach;
  for (int k = 0; k < 3; ++k) { B->lo[k] = G.lo[k]; B->shape[k] = G.shape[k]; }
  B->nBand = nband;
  B->closure_iterations = iters;
  std::vector<std::pair<uint64_t, int64_t>> order;
  for (int64_t fi = 0; fi < fsize; ++fi) {
    if (!(F.A[fi] | F.G[fi])) continue;
    int32_t b[3] = {0, 0, 0};
    F.coords(fi, b);
    uint64_t key = morton3((uint32_t)(b[0] >> 1), (uint32_t)(b[1] >> 1), (uint32_t)(b[2] >> 1));
    int sub = d == 3 ? (b[0] & 1) * 4 + (b[1] & 1) * 2 + (b[2] & 1) : (b[0] & 1) * 2 + (b[1] & 1);
    order.push_back({(key << 3) | (uint64_t)sub, fi});
  }
  std::sort(order.begin(), order.end());
  const int64_t nb = (int64_t)order.size();
  B->bcoord.resize(nb * 3);
  B->maskA.resize(nb);
  B->maskG.resize(nb);
  B->offA.resize(nb);
  B->offG.resize(nb);
  int64_t na = 0, ng = 0;
  int32_t lo_b[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi_b[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
  for (int64_t i = 0; i < nb; ++i) {
    int64_t fi = order[i].second;
    int32_t b[3] = {0, 0, 0};
    F.coords(fi, b);
    for (int k = 0; k < 3; ++k) B->bcoord[i * 3 + k] = b[k];
    for (int k = 0; k < d; ++k) { lo_b[k] = std::min(lo_b[k], b[k]); hi_b[k] = std::max(hi_b[k], b[k]); }
    B->maskA[i] = F.A[fi];
    B->maskG[i] = F.G[fi];
    B->offA[i] = (int32_t)na;
    B->offG[i] = (int32_t)ng;
    na += __builtin_popcountll(F.A[fi]);
    ng += __builtin_popcountll(F.G[fi]);
  }
  if (na + ng > INT32_MAX) fail(CPM_ERR_ARG, "band too large for 32-bit node indices");
  B->nA = na;
  B->nG = ng;
  int64_t bmsize = 1;
  for (int k = 0; k < 3; ++k) { B->bm_lo[k] = 0; B->bm_dim[k] = 1; }
  for (int k = 0; k < d; ++k) {
    B->bm_lo[k] = lo_b[k];
    B->bm_dim[k] = hi_b[k] - lo_b[k] + 1;
    bmsize *= B->bm_dim[k];
  }
  B->bmap.assign(bmsize, -1);
  for (int64_t i = 0; i < nb; ++i) {
    int64_t r = 0;
    for (int k = 0; k < d; ++k) r = r * B->bm_dim[k] + (B->bcoord[i * 3 + k] - B->bm_lo[k]);
    B->bmap[r] = (int32_t)i;
  }
  // per-node grid index, closest point, interpolation point and sign, in storage order
  const int64_t nn = na + ng;
  B->gidx.assign(nn * d, 0);
  std::vector<double> x(nn * d);
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < nb; ++i) {
    for (int set = 0; set < 2; ++set) {
      uint64_t m = set == 0 ? B->maskA[i] : B->maskG[i];
      int64_t base = set == 0 ? B->offA[i] : na + B->offG[i];
      int64_t j = 0;
      while (m) {
        int bit = __builtin_ctzll(m);
        m &= m - 1;
        int l[3];
        local_of(d, bit, l);
        int64_t node = base + j++;
        for (int k = 0; k < d; ++k) {
          int32_t g = B->bcoord[i * 3 + k] * G.E + l[k];
          B->gidx[node * d + k] = g;
          x[node * d + k] = G.lo[k] + g * h;
        }
      }
    }
  }
  B->cp.assign(nn * d, 0.0);
  B->ip.assign(nn * d, 0.0);
  std::vector<double> sg(nn);
  src.interp(nn, x.data(), B->cp.data(), B->ip.data(), sg.data());
  bool mirrored = false;
  for (int64_t i = 0; i < nn; ++i) mirrored = mirrored || sg[i] != 1.0;
  if (mirrored) B->sgn.swap(sg);
  return guard.release();
}

}  // namespace

namespace {

cpm_status band_build_any(const char* who, const cpm_surface* surface, cpm_cp_callback cb, void* ctx, int32_t d,
                          double h, int32_t p, const double* lo, const double* hi, double gamma, int32_t reach,
                          cpm_band** out) {
  try {
    if (!lo || !hi || !out || (!surface && !cb)) fail(CPM_ERR_ARG, "null argument");
    *out = nullptr;
    if (surface && cb) fail(CPM_ERR_ARG, "give a surface or a callback, not both");
    if (d != 2 && d != 3) fail(CPM_ERR_ARG, "d must be 2 or 3");
    if (p < 1 || p > 5) fail(CPM_ERR_ARG, "p must be in 1..5");
    if (reach != 1 && reach != 2) fail(CPM_ERR_ARG, "reach must be 1 or 2");
    if (!(h > 0) || !std::isfinite(h)) fail(CPM_ERR_ARG, "h must be positive");
    Surface S;
    CpSource src;
    src.d = d;
    if (surface) {
      S.kind = surface->kind;
      std::memcpy(S.params, surface->params, sizeof(S.params));
      std::memcpy(S.center, surface->center, sizeof(S.center));
      if ((S.kind == CPM_SURF_CIRCLE) != (d == 2)) fail(CPM_ERR_ARG, "circle is the only 2-D surface");
      if (S.kind < 0 || S.kind > 3) fail(CPM_ERR_ARG, "unknown surface kind");
      for (int k = 0; k < 3; ++k)
        if (!std::isfinite(S.params[k]) || !std::isfinite(S.center[k])) fail(CPM_ERR_ARG, "non-finite surface");
      if (S.params[0] <= 0) fail(CPM_ERR_ARG, "surface size must be positive");
      if (S.kind == CPM_SURF_TORUS && !(S.params[1] > 0 && S.params[1] < S.params[0]))
        fail(CPM_ERR_ARG, "torus needs 0 < r < R");
      if (S.kind == CPM_SURF_ELLIPSOID && !(S.params[1] > 0 && S.params[2] > 0))
        fail(CPM_ERR_ARG, "ellipsoid semi-axes must be positive");
      src.S = &S;
    } else {
      src.cb = cb;
      src.ctx = ctx;
    }
    *out = build_band_impl(src, d, h, p, lo, hi, gamma, reach);
    return CPM_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error(std::string("host allocation failed in ") + who);
    return CPM_ERR_OOM;
  } catch (...) {
    set_error(std::string("unexpected failure in ") + who);
    return CPM_ERR_DEVICE;
  }
}

}  // namespace

cpm_status cpm_band_build(const cpm_surface* surface, int32_t d, double h, int32_t p,
                          const double* lo, const double* hi, double gamma, cpm_band** out) {
  if (!surface) {
    set_error("null argument");
    return CPM_ERR_ARG;
  }
  return band_build_any("cpm_band_build", surface, nullptr, nullptr, d, h, p, lo, hi, gamma, 1, out);
}

cpm_status cpm_band_build_user(cpm_cp_callback cp, void* ctx, int32_t d, double h, int32_t p, const double* lo,
                               const double* hi, double gamma, cpm_band** out) {
  if (!cp) {
    set_error("null argument");
    return CPM_ERR_ARG;
  }
  return band_build_any("cpm_band_build_user", nullptr, cp, ctx, d, h, p, lo, hi, gamma, 1, out);
}

cpm_status cpm_band_build_reach(const cpm_surface* surface, cpm_cp_callback cp, void* ctx, int32_t d, double h,
                                int32_t p, const double* lo, const double* hi, double gamma, int32_t reach,
                                cpm_band** out) {
  return band_build_any("cpm_band_build_reach", surface, cp, ctx, d, h, p, lo, hi, gamma, reach, out);
}

cpm_status cpm_band_get_info(const cpm_band* band, cpm_band_info* info) {
  if (!band || !info) { set_error("null argument"); return CPM_ERR_ARG; }
  std::memset(info, 0, sizeof(*info));
  info->n_active = band->nA;
  info->n_ghost = band->nG;
  info->n_band = band->nBand;
  info->d = band->d;
  info->p = band->p;
  info->h = band->h;
  info->gamma = band->gamma;
  for (int k = 0; k < 3; ++k) { info->lo[k] = band->lo[k]; info->shape[k] = band->shape[k]; }
  info->n_bricks = band->nbricks();
  info->closure_iterations = band->closure_iterations;
  info->reach = band->reach;
  return CPM_OK;
}

cpm_status cpm_band_export(const cpm_band* band, int32_t* gidx, double* cp, uint8_t* kind) {
  if (!band) { set_error("null band"); return CPM_ERR_ARG; }
  const int64_t n = band->nodes();
  if (gidx) std::memcpy(gidx, band->gidx.data(), sizeof(int32_t) * n * band->d);
  if (cp) std::memcpy(cp, band->cp.data(), sizeof(double) * n * band->d);
  if (kind)
    for (int64_t i = 0; i < n; ++i) kind[i] = i < band->nA ? 0 : 1;
  return CPM_OK;
}

cpm_status cpm_band_export_interp(const cpm_band* band, double* ip, double* sign) {
  if (!band) { set_error("null band"); return CPM_ERR_ARG; }
  const int64_t n = band->nodes();
  if (ip) std::memcpy(ip, band->ip.data(), sizeof(double) * n * band->d);
  if (sign) {
    if (band->sgn.empty()) std::fill(sign, sign + n, 1.0);
    else std::memcpy(sign, band->sgn.data(), sizeof(double) * n);
  }
  return CPM_OK;
}

void cpm_band_destroy(cpm_band* band) { delete band; }
