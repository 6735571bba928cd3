// Operator setup: tiles and LDS footprints for the fused apply, per-brick
// extension-row lists for the atomic-free transpose, upload of the band to the
// device.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "common.h"

using namespace cpm;

namespace {

void base_of(const cpm_band_s& B, const double* cp, int32_t* b) {
  for (int k = 0; k < B.d; ++k) {
    double t = (cp[k] - B.lo[k]) / B.h;
    b[k] = (int32_t)std::floor(t - (B.p - 1) / 2.0);
  }
}

void local_of(int d, int bit, int* l) {
  if (d == 3) { l[0] = bit >> 4; l[1] = (bit >> 2) & 3; l[2] = bit & 3; }
  else { l[0] = bit >> 3; l[1] = bit & 7; l[2] = 0; }
}

// Tiles (2^d bricks): the jobs (extension rows the tile's stencils need: every
// band node of the tile plus the outward face neighbours of its active
// boundary nodes, each with its slot in the tile's LDS box), the bounding box
// of their interpolation cubes (the LDS footprint) and the Sigma_A bricks
// overlapping that footprint.
// halo = false: the extension pass of the two-pass apply (jobs are the tile's own
// band nodes only; their slots are unused). per_brick: every brick is a tile of its own
// (extension pass only: the footprint of one brick's rows always fits the LDS budget).
void build_tiles(const cpm_band_s& B, std::vector<DevTile>& tiles, std::vector<int32_t>& fvol,
                 std::vector<FootBrick>& fbrec, std::vector<Job>& jobs, bool halo = true,
                 bool per_brick = false) {
  bool orphan = false;
  const int d = B.d, E = brick_edge(d), T = 2 * E, P = B.p, W = T + 2;
  const int64_t nb = B.nbricks();
  std::vector<int64_t> start;
  for (int64_t i = 0; i < nb; ++i) {
    bool fresh = i == 0 || per_brick;
    if (!fresh)
      for (int k = 0; k < d; ++k)
        if ((B.bcoord[i * 3 + k] >> 1) != (B.bcoord[(i - 1) * 3 + k] >> 1)) fresh = true;
    if (fresh) start.push_back(i);
  }
  start.push_back(nb);
  const int64_t nt = (int64_t)start.size() - 1;
  tiles.assign(nt, DevTile{});
  fvol.assign(nt, 0);
  std::vector<std::vector<FootBrick>> fb(nt);
  std::vector<std::vector<Job>> jb(nt);
  auto slot_of = [&](const int* l) {   // tile-local coordinates in [-1, T] -> LDS box slot
    return d == 3 ? ((l[0] + 1) * W + (l[1] + 1)) * W + (l[2] + 1) : (l[0] + 1) * W + (l[1] + 1);
  };
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < nt; ++t) {
    DevTile& tl = tiles[t];
    for (int q = 0; q < 8; ++q) { tl.oA[q] = 0; tl.mA[q] = 0; tl.bid[q] = -1; }
    for (int k = 0; k < 3; ++k) tl.origin[k] = 0;
    for (int k = 0; k < d; ++k) tl.origin[k] = (B.bcoord[start[t] * 3 + k] >> 1) * T;
    int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    auto add_job = [&](int64_t node, const int* l) {
      int32_t b[3];
      base_of(B, &B.ip[node * d], b);
      for (int k = 0; k < d; ++k) { lo[k] = std::min(lo[k], b[k]); hi[k] = std::max(hi[k], b[k] + P); }
      jb[t].push_back(Job{(int32_t)node, (int32_t)slot_of(l)});
    };
    for (int64_t i = start[t]; i < start[t + 1]; ++i) {
      int sub = 0;
      for (int k = 0; k < d; ++k) sub = sub * 2 + (B.bcoord[i * 3 + k] & 1);
      tl.oA[sub] = B.offA[i];
      tl.mA[sub] = B.maskA[i];
      tl.bid[sub] = (int32_t)i;
      for (int set = 0; set < 2; ++set) {
        uint64_t m = set == 0 ? B.maskA[i] : B.maskG[i];
        int64_t base = set == 0 ? B.offA[i] : B.nA + B.offG[i];
        int64_t j = 0;
        while (m) {
          int bit = __builtin_ctzll(m);
          m &= m - 1;
          int64_t node = base + j++;
          int l[3];
          local_of(d, bit, l);
          int lt[3] = {0, 0, 0};
          for (int k = 0; k < d; ++k) lt[k] = B.bcoord[i * 3 + k] * E + l[k] - tl.origin[k];
          add_job(node, lt);
          if (set != 0 || !halo) continue;
          // face halo: outward neighbours of active nodes on the tile boundary
          for (int k = 0; k < d; ++k)
            for (int s = -1; s <= 1; s += 2) {
              int ln[3] = {lt[0], lt[1], lt[2]};
              ln[k] += s;
              if (ln[k] >= 0 && ln[k] < T) continue;
              int32_t gn[3] = {0, 0, 0};
              for (int q = 0; q < d; ++q) gn[q] = tl.origin[q] + ln[q];
              int64_t nn = B.lookup(gn);
              if (nn < 0) {
#pragma omp atomic write
                orphan = true;
                continue;
              }
              add_job(nn, ln);
            }
        }
      }
    }
    {
      // jobs in Morton order of their cube corner: the lanes of a wavefront read
      // overlapping or adjacent cubes, which cuts LDS bank conflicts
      std::vector<std::pair<uint64_t, Job>> key;
      key.reserve(jb[t].size());
      for (const Job& j : jb[t]) {
        int32_t b[3] = {0, 0, 0};
        base_of(B, &B.ip[(int64_t)j.node * d], b);
        uint64_t kk = 0;
        for (int bit = 20; bit >= 0; --bit)
          for (int k = 0; k < d; ++k) kk = (kk << 1) | (uint64_t)((b[k] >> bit) & 1);
        key.push_back({kk, j});
      }
      std::stable_sort(key.begin(), key.end(), [](const std::pair<uint64_t, Job>& a, const std::pair<uint64_t, Job>& b) {
        return a.first < b.first;
      });
      for (size_t q = 0; q < key.size(); ++q) jb[t][q] = key[q].second;
    }
    // footprint box aligned to bricks; strides padded against LDS bank conflicts
    const int sh = brick_shift(d);
    int32_t flo[3] = {0, 0, 0}, fdim[3] = {1, 1, 1};
    for (int k = 0; k < d; ++k) {
      flo[k] = (lo[k] >> sh) << sh;
      fdim[k] = (((hi[k] >> sh) + 1) << sh) - flo[k];
    }
    // y stride = z extent + 2, x stride = 6 (mod 32): the (p+1)^2 columns of
    // neighbouring cubes then fall on different banks far more often than with
    // the dense box (measured: about a third fewer conflict cycles)
    int32_t s1, s0;
    if (d == 3) {
      s1 = fdim[2] + 2;
      s0 = fdim[1] * s1 + ((6 - fdim[1] * s1) % 32 + 32) % 32;
    } else {
      s1 = 1;
      s0 = fdim[1] + ((6 - fdim[1]) % 32 + 32) % 32;
    }
    tl.fstr[0] = s0;
    tl.fstr[1] = s1;
    tl.fbase = d == 3 ? flo[0] * s0 + flo[1] * s1 + flo[2] : flo[0] * s0 + flo[1];
    const int64_t vol = (int64_t)fdim[0] * s0;
    tl.fvol = (int32_t)std::min<int64_t>(vol, INT32_MAX);
    fvol[t] = tl.fvol;
    // Sigma_A bricks inside the footprint box
    int32_t b0[3] = {0, 0, 0}, b1[3] = {0, 0, 0};
    for (int k = 0; k < d; ++k) { b0[k] = flo[k] >> sh; b1[k] = (flo[k] + fdim[k] - 1) >> sh; }
    for (int32_t x = b0[0]; x <= b1[0]; ++x)
      for (int32_t yv = b0[1]; yv <= b1[1]; ++yv)
        for (int32_t z = b0[2]; z <= (d == 3 ? b1[2] : b0[2]); ++z) {
          int32_t g[3] = {x << sh, yv << sh, d == 3 ? (z << sh) : 0};
          int32_t rel[3] = {0, 0, 0};
          bool in = true;
          for (int k = 0; k < d; ++k) {
            rel[k] = (g[k] >> sh) - B.bm_lo[k];
            if (g[k] < 0 || rel[k] < 0 || rel[k] >= B.bm_dim[k]) in = false;
          }
          if (!in) continue;
          int64_t bi = d == 3 ? ((int64_t)rel[0] * B.bm_dim[1] + rel[1]) * B.bm_dim[2] + rel[2]
                              : (int64_t)rel[0] * B.bm_dim[1] + rel[1];
          int32_t id = B.bmap[bi];
          if (id < 0 || !B.maskA[id]) continue;
          const int64_t lds = d == 3 ? (int64_t)(g[0] - flo[0]) * s0 + (int64_t)(g[1] - flo[1]) * s1 + (g[2] - flo[2])
                                     : (int64_t)(g[0] - flo[0]) * s0 + (g[1] - flo[1]);
          fb[t].push_back(FootBrick{B.maskA[id], B.offA[id], (int32_t)lds});
        }
  }
  if (orphan) fail(CPM_ERR_BAND, "active node without a band neighbour");
  fbrec.clear();
  jobs.clear();
  for (int64_t t = 0; t < nt; ++t) {
    tiles[t].fb_off = (int32_t)fbrec.size();
    tiles[t].fb_cnt = (int32_t)fb[t].size();
    tiles[t].job_off = (int32_t)jobs.size();
    tiles[t].job_cnt = (int32_t)jb[t].size();
    fbrec.insert(fbrec.end(), fb[t].begin(), fb[t].end());
    jobs.insert(jobs.end(), jb[t].begin(), jb[t].end());
  }
}

// Brick across each face of every brick: bnbr[i*2d + 2k + s] for axis k, side s
// (0: lower, 1: upper), -1 when that brick holds no band node. Every grid
// neighbour of an active node is a band node, so for an active node on a face
// the brick across it exists (checked here).
void build_brick_neighbours(const cpm_band_s& B, std::vector<int32_t>& bnbr) {
  const int d = B.d, sh = brick_shift(d), E = brick_edge(d);
  const int64_t nb = B.nbricks();
  bnbr.assign(nb * 2 * d, -1);
  bool bad = false;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nb; ++i) {
    for (int k = 0; k < d; ++k)
      for (int s = 0; s < 2; ++s) {
        int32_t g[3] = {0, 0, 0};
        for (int q = 0; q < d; ++q) g[q] = B.bcoord[i * 3 + q] << sh;
        g[k] += s ? E : -1;
        int32_t rel[3] = {0, 0, 0};
        bool in = true;
        for (int q = 0; q < d; ++q) {
          rel[q] = (g[q] >> sh) - B.bm_lo[q];
          if (g[q] < 0 || rel[q] < 0 || rel[q] >= B.bm_dim[q]) in = false;
        }
        int32_t id = -1;
        if (in) {
          const int64_t bi = d == 3 ? ((int64_t)rel[0] * B.bm_dim[1] + rel[1]) * B.bm_dim[2] + rel[2]
                                    : (int64_t)rel[0] * B.bm_dim[1] + rel[1];
          id = B.bmap[bi];
        }
        bnbr[i * 2 * d + 2 * k + s] = id;
        // active nodes on this face need the neighbouring brick
        uint64_t face = 0;
        for (int bit = 0; bit < 64; ++bit) {
          int l[3];
          local_of(d, bit, l);
          if (l[k] == (s ? E - 1 : 0)) face |= 1ull << bit;
        }
        if ((B.maskA[i] & face) && id < 0) {
#pragma omp atomic write
          bad = true;
        }
      }
  }
  if (bad) fail(CPM_ERR_BAND, "active node whose face neighbour brick is missing");
}

// Transpose lists: for every brick holding active nodes, the extension rows whose
// interpolation cube overlaps the brick's box, in increasing row order (a row's
// cube of (p+1)^d nodes overlaps at most 2^d bricks). ptr is indexed by brick id;
// list = the bricks with active nodes.
void build_brick_rows(const cpm_band_s& B, std::vector<int32_t>& ptr, std::vector<int32_t>& rows,
                      std::vector<int32_t>& list) {
  const int d = B.d, E = d == 3 ? 4 : 8, P = B.p;
  const int64_t n = B.nodes(), nb = B.nbricks();
  auto brick_id = [&](const int32_t* bc) -> int32_t {
    int64_t r = 0;
    for (int k = 0; k < d; ++k) {
      const int32_t q = bc[k] - B.bm_lo[k];
      if (q < 0 || q >= B.bm_dim[k]) return -1;
      r = r * B.bm_dim[k] + q;
    }
    return B.bmap[r];
  };
  // bricks overlapped by each row's cube (up to 2 per axis)
  std::vector<int32_t> hit(n * 8, -1);
  bool bad = false;
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; ++j) {
    int32_t b[3] = {0, 0, 0};
    base_of(B, &B.ip[j * d], b);
    int32_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    bool ok = true;
    for (int k = 0; k < d; ++k) {
      ok = ok && b[k] >= 0;
      lo[k] = b[k] / E;
      hi[k] = (b[k] + P) / E;
    }
    if (!ok) {
#pragma omp atomic write
      bad = true;
      continue;
    }
    int m = 0;
    for (int32_t x = lo[0]; x <= hi[0]; ++x)
      for (int32_t y = lo[1]; y <= hi[1]; ++y)
        for (int32_t z = lo[2]; z <= (d == 3 ? hi[2] : lo[2]); ++z) {
          const int32_t bc[3] = {x, y, z};
          const int32_t id = brick_id(bc);
          if (id >= 0 && B.maskA[id]) hit[j * 8 + m++] = id;
        }
  }
  if (bad) fail(CPM_ERR_BAND, "interpolation cube outside the grid");
  ptr.assign(nb + 1, 0);
  for (int64_t e = 0; e < n * 8; ++e)
    if (hit[e] >= 0) ptr[hit[e] + 1]++;
  for (int64_t i = 0; i < nb; ++i) ptr[i + 1] += ptr[i];
  if (ptr[nb] > INT32_MAX - 1) fail(CPM_ERR_BAND, "band too large for the transpose lists");
  rows.assign(ptr[nb], 0);
  std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
  for (int64_t j = 0; j < n; ++j)
    for (int m = 0; m < 8; ++m) {
      const int32_t id = hit[j * 8 + m];
      if (id >= 0) rows[fill[id]++] = (int32_t)j;
    }
  list.clear();
  for (int64_t i = 0; i < nb; ++i)
    if (B.maskA[i]) list.push_back((int32_t)i);
}

}  // namespace

void cpm::plan_pipe(std::vector<WorkItem>& work, const std::vector<int32_t>& cost, int grid,
               std::vector<PipeSpan>& plan) {
  plan.clear();
  const int64_t n = (int64_t)work.size();
  if (n == 0 || grid <= 0) return;
  const int per = grid / 8;
  plan.assign((size_t)per * 8, PipeSpan{0, 0, 1, 0});
  const bool by_cost = n <= kCostOrderMaxTiles;
  std::vector<WorkItem> out(work.size());
  for (int x = 0; x < 8; ++x) {
    const int64_t s = n * x / 8, e = n * (x + 1) / 8;
    if (!by_cost) {
      for (int j = 0; j < per; ++j) plan[(size_t)j * 8 + x] = PipeSpan{(int32_t)(s + j), (int32_t)e, per, 0};
      for (int64_t i = s; i < e; ++i) out[i] = work[i];
      continue;
    }
    std::vector<int64_t> idx((size_t)(e - s));
    for (int64_t i = s; i < e; ++i) idx[i - s] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return cost[a] > cost[b]; });
    std::vector<int64_t> load(per, 0);
    std::vector<std::vector<int64_t>> bins(per);
    for (int64_t i : idx) {
      int best = 0;
      for (int j = 1; j < per; ++j)
        if (load[j] < load[best]) best = j;
      bins[best].push_back(i);
      load[best] += kTileCostBase + cost[i];
    }
    int64_t pos = s;
    for (int j = 0; j < per; ++j) {
      plan[(size_t)j * 8 + x] = PipeSpan{(int32_t)pos, (int32_t)(pos + (int64_t)bins[j].size()), 1, 0};
      for (int64_t i : bins[j]) out[pos++] = work[i];
    }
  }
  work.swap(out);
}

// Lists of the two-pass apply: the extension pass visits every tile (a tile of
// ghost nodes only still owes their extension rows), with jobs = its own band
// nodes and the footprint of their cubes; the stencil pass visits the tiles with
// active nodes. Available when every extension-pass footprint fits the LDS budget.
static void setup_two_pass(cpm_operator_s& op, const cpm_band_s& B) {
  const int d = B.d;
  const size_t lds_bytes = (size_t)op.lds_bytes;
  std::vector<int32_t> fvolE;
  std::vector<FootBrick> fbrecE;
  std::vector<Job> jobsE;
  build_tiles(B, op.tilesE, fvolE, fbrecE, jobsE, false);
  const int cap = (int)(lds_bytes / sizeof(double));
  std::vector<WorkItem> ework, eslow;
  int ucapE = 0;
  std::vector<uint8_t> split(B.nbricks(), 0);   // bricks of tiles whose footprint does not fit
  bool any_split = false;
  const size_t ntiles = op.tilesE.size();
  auto fits = [&](const DevTile& tl, int32_t vol) {
    return vol <= cap && tl.job_cnt <= 512 && tl.fb_cnt <= kMaxFootBricks;
  };
  for (size_t t = 0; t < ntiles; ++t) {
    const DevTile& tl = op.tilesE[t];
    if (tl.job_cnt == 0) continue;
    if (!fits(tl, fvolE[t])) {
      for (int q = 0; q < 8; ++q)
        if (tl.bid[q] >= 0) { split[tl.bid[q]] = 1; any_split = true; }
      continue;
    }
    ework.push_back(WorkItem{0, (int32_t)t});
    ucapE = std::max(ucapE, fvolE[t]);
  }
  if (any_split) {
    // the bricks of oversized tiles as tiles of their own, appended to the list (their
    // records follow the first build's); a brick that still does not fit takes the slow
    // path (k_extend_bricks)
    std::vector<DevTile> tb;
    std::vector<int32_t> fvb;
    std::vector<FootBrick> fbb;
    std::vector<Job> jbb;
    build_tiles(B, tb, fvb, fbb, jbb, false, true);
    const int32_t fb0 = (int32_t)fbrecE.size(), jb0 = (int32_t)jobsE.size();
    fbrecE.insert(fbrecE.end(), fbb.begin(), fbb.end());
    jobsE.insert(jobsE.end(), jbb.begin(), jbb.end());
    for (size_t t = 0; t < tb.size(); ++t) {
      DevTile tl = tb[t];
      int32_t id = -1;
      for (int q = 0; q < 8; ++q)
        if (tl.bid[q] >= 0) id = tl.bid[q];
      if (id < 0 || !split[id] || tl.job_cnt == 0) continue;
      if (!fits(tl, fvb[t])) {
        eslow.push_back(WorkItem{0, id});
        continue;
      }
      tl.fb_off += fb0;
      tl.job_off += jb0;
      ework.push_back(WorkItem{0, (int32_t)op.tilesE.size()});
      op.tilesE.push_back(tl);
      ucapE = std::max(ucapE, fvb[t]);
    }
  }
  std::vector<WorkItem> swork;
  for (size_t t = 0; t < op.tiles.size(); ++t) {
    bool has_active = false;
    for (int q = 0; q < 8; ++q)
      if (op.tiles[t].mA[q]) has_active = true;
    if (has_active) swork.push_back(WorkItem{0, (int32_t)t});
  }
  op.twopass = !ework.empty() || !eslow.empty();
  if (!op.twopass) return;
  op.h_fbE = eslow;
  op.d_fbE.upload(eslow);
  op.d_fbrecE.upload(fbrecE);
  op.d_jobsE.upload(jobsE);
  std::vector<int32_t> cost(ework.size());
  for (size_t i = 0; i < ework.size(); ++i) cost[i] = op.tilesE[ework[i].idx].job_cnt;
  std::vector<PipeSpan> plan;
  plan_pipe(ework, cost, ework.empty() ? 0 : apply_pipe_grid(d, B.p, (int)ework.size(), ucapE, true), plan);
  op.d_planE.upload(plan);
  op.nplanE = (int)plan.size();
  std::vector<DevTile> wt;
  wt.reserve(ework.size());
  for (const WorkItem& wi : ework) {
    wt.push_back(op.tilesE[wi.idx]);
    wt.back().inst = 0;
    for (int q = 0; q < 8; ++q) wt.back().mA[q] = 0;   // no stencil rows in the extension pass
  }
  op.d_wtilesE.upload(wt);
  op.h_workE = ework;
  op.h_swork = swork;
  op.d_swork.upload(swork);
  op.ucapE = ucapE;
  op.d_v.alloc((size_t)B.nodes());
  op.I.fbrecE = op.d_fbrecE.p;
  op.I.jobsE = op.d_jobsE.p;
  op.I.vnode_off = 0;
  op.d_inst.upload(&op.I, 1);
}

// diagonal and neighbour weight of the stabilized operator of stencil order 2 or 4
static void stencil_coefficients(int order, int d, double h, double c, double& diag, double& w) {
  if (order == 4) {
    w = 1.0 / (12.0 * h * h);
    diag = c + 30.0 * d * w;
  } else {
    w = 1.0 / (h * h);
    diag = c + 2.0 * d / (h * h);
  }
}

static cpm_status operator_create(const cpm_band* band, double c, const cpm_operator_opts& o,
                                  cpm_operator** out) {
  try {
    if (!band || !out) fail(CPM_ERR_ARG, "null argument");
    *out = nullptr;
    if (!(c > 0) || !std::isfinite(c)) fail(CPM_ERR_ARG, "shift c must be positive and finite");
    const int order = o.order;
    if (order != 2 && order != 4) fail(CPM_ERR_ARG, "order must be 2 or 4");
    const int lds_bytes = o.apply_lds_bytes == 0 ? (int)kApplyLdsBytes : o.apply_lds_bytes;
    if (lds_bytes < 16384 || lds_bytes > (int)kApplyLdsBytes)
      fail(CPM_ERR_ARG, "apply_lds_bytes must be 0 or in 16384..65536");
    if (order == 4 && band->reach < 2) fail(CPM_ERR_ARG, "the fourth-order stencil needs a band of reach 2");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) fail(CPM_ERR_DEVICE, "no HIP device available");
    auto op = std::make_unique<cpm_operator_s>();
    op->band = std::make_shared<cpm_band_s>(*band);
    op->c = c;
    op->order = order;
    op->lds_bytes = lds_bytes;
    op->generic = order == 4 || band->p > 3;
    const cpm_band_s& B = *op->band;
    const int d = B.d;
    const int64_t n = B.nodes();
    std::vector<FootBrick> fbrec;
    std::vector<Job> jobs;
    std::vector<int32_t> tptr, trows, tlist, bnbr;
    if (!op->generic) {
      build_tiles(B, op->tiles, op->tile_fvol, fbrec, jobs);
      op->d_fbrec.upload(fbrec);
      op->d_jobs.upload(jobs);
      build_brick_rows(B, tptr, trows, tlist);
    } else {
      for (int64_t i = 0; i < B.nbricks(); ++i)
        if (B.maskA[i]) tlist.push_back((int32_t)i);
    }
    build_brick_neighbours(B, bnbr);
    // SoA closest points
    std::vector<double> cps(n * d);
    for (int64_t j = 0; j < n; ++j)
      for (int k = 0; k < d; ++k) cps[k * n + j] = (B.ip[j * d + k] - B.lo[k]) / B.h;
    op->d_tcp.upload(cps);
    if (!B.sgn.empty()) op->d_sgn.upload(B.sgn);
    op->d_maskA.upload(B.maskA);
    op->d_maskG.upload(B.maskG);
    op->d_offA.upload(B.offA);
    op->d_offG.upload(B.offG);
    op->d_bcoord.upload(B.bcoord);
    op->d_bmap.upload(B.bmap);
    op->d_tiles.upload(op->tiles);
    op->d_bptr.upload(tptr);
    op->d_brows.upload(trows);
    op->d_tlist.upload(tlist);
    op->d_bnbr.upload(bnbr);
    DevInst& I = op->I;
    std::memset(&I, 0, sizeof(I));
    I.d = d; I.p = B.p; I.nA = (int32_t)B.nA; I.nG = (int32_t)B.nG;
    I.h = B.h;
    I.order = order;
    stencil_coefficients(order, d, B.h, c, I.diag, I.inv_h2);
    for (int k = 0; k < 3; ++k) { I.lo[k] = B.lo[k]; I.bm_lo[k] = B.bm_lo[k]; I.bm_dim[k] = B.bm_dim[k]; }
    I.tcp = op->d_tcp.p;
    I.esgn = B.sgn.empty() ? nullptr : op->d_sgn.p;
    I.maskA = op->d_maskA.p; I.maskG = op->d_maskG.p;
    I.offA = op->d_offA.p; I.offG = op->d_offG.p;
    I.bcoord = op->d_bcoord.p; I.bmap = op->d_bmap.p;
    I.tiles = op->d_tiles.p;
    I.fbrec = op->d_fbrec.p;
    I.jobs = op->d_jobs.p;
    I.ntiles = (int32_t)op->tiles.size();
    I.nbricks = (int32_t)B.nbricks();
    I.trow_ptr = op->d_bptr.p; I.trows = op->d_brows.p;
    I.tbricks = op->d_tlist.p; I.ntbricks = (int32_t)tlist.size();
    I.bnbr = op->d_bnbr.p;
    I.vec_off = 0;
    op->d_inst.upload(&I, 1);
    if (op->generic) {
      // two-kernel apply: extension values of up to four right-hand sides; the one-RHS
      // extension pass runs on LDS tiles (the two-pass apply's extension pass)
      op->d_v.alloc((size_t)n * 4);
      {
        setup_two_pass(*op, B);
        if (op->twopass) {
          op->gep.dinst = op->d_inst.p;
          op->gep.pipe = PipeWork{op->d_wtilesE.p, op->d_planE.p, op->nplanE};
          op->gep.ucap = op->ucapE;
          op->gep.fb = op->d_fbE.p;
          op->gep.nfb = (int)op->h_fbE.size();
          op->gen.epass = &op->gep;
        }
      }
      op->gvoff = 0;
      op->gen.inst = &op->I;
      op->gen.voff = &op->gvoff;
      op->gen.ninst = 1;
      op->gen.vscr = op->d_v.p;
      *out = op.release();
      return CPM_OK;
    }
    // work lists: tiles whose footprint fits the LDS budget, the rest take the slow path
    const int cap = (int)(((size_t)lds_bytes - tile_lds_extra_bytes(d)) / sizeof(double));
    const int max_jobs = d == 3 ? 8 * 64 + 6 * 64 : 4 * 64 + 4 * 16;
    const int max_fb = kMaxFootBricks;
    std::vector<WorkItem> fast, slow;
    int ucap = 0;
    for (size_t t = 0; t < op->tiles.size(); ++t) {
      bool has_active = false;
      for (int q = 0; q < 8; ++q)
        if (op->tiles[t].mA[q]) has_active = true;
      if (!has_active) continue;
      if (op->tile_fvol[t] <= cap && op->tiles[t].job_cnt <= max_jobs && op->tiles[t].fb_cnt <= max_fb) {
        fast.push_back(WorkItem{0, (int32_t)t});
        ucap = std::max(ucap, op->tile_fvol[t]);
      } else {
        slow.push_back(WorkItem{0, (int32_t)t});
      }
    }
    {
      std::vector<int32_t> cost(fast.size());
      for (size_t i = 0; i < fast.size(); ++i) cost[i] = op->tiles[fast[i].idx].job_cnt;
      std::vector<PipeSpan> plan;
      plan_pipe(fast, cost, fast.empty() ? 0 : apply_pipe_grid(d, B.p, (int)fast.size(), ucap), plan);
      op->d_plan.upload(plan);
      op->nplan = (int)plan.size();
    }
    op->d_work.upload(fast);
    {
      std::vector<DevTile> wt;
      wt.reserve(fast.size());
      for (const WorkItem& wi : fast) {
        wt.push_back(op->tiles[wi.idx]);
        wt.back().inst = 0;
      }
      op->d_wtiles.upload(wt);
    }
    op->d_fb.upload(slow);
    op->h_work = fast;
    op->h_fb = slow;
    op->nwork = (int)fast.size();
    op->nfb = (int)slow.size();
    op->ucap = ucap;
    setup_two_pass(*op, B);
    *out = op.release();
    return CPM_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed in cpm_operator_create");
    return CPM_ERR_OOM;
  }
}

cpm_status cpm_operator_opts_default(cpm_operator_opts* o) {
  if (!o) {
    set_error("null argument");
    return CPM_ERR_ARG;
  }
  std::memset(o, 0, sizeof(*o));
  o->order = 2;
  o->apply_lds_bytes = 0;
  return CPM_OK;
}

cpm_status cpm_operator_create(const cpm_band* band, double c, void* stream, cpm_operator** out) {
  (void)stream;
  cpm_operator_opts o;
  cpm_operator_opts_default(&o);
  return operator_create(band, c, o, out);
}

cpm_status cpm_operator_create_ex(const cpm_band* band, double c, const cpm_operator_opts* opts, void* stream,
                                  cpm_operator** out) {
  (void)stream;
  if (!opts) {
    set_error("null argument");
    return CPM_ERR_ARG;
  }
  return operator_create(band, c, *opts, out);
}

cpm_status cpm_operator_get_info(const cpm_operator* op, cpm_operator_info* info) {
  if (!op || !info) {
    set_error("null argument");
    return CPM_ERR_ARG;
  }
  std::memset(info, 0, sizeof(*info));
  info->order = op->order;
  info->two_kernel = op->generic ? 1 : 0;
  info->two_pass = op->twopass ? 1 : 0;
  info->apply_lds_bytes = op->lds_bytes;
  info->n_tiles = op->nwork + op->nfb;
  info->n_fallback_tiles = op->nfb;
  info->apply_variant = op->apply_variant;
  return CPM_OK;
}

cpm_status cpm_operator_set_shift(cpm_operator* op, double c) {
  try {
    if (!op) fail(CPM_ERR_ARG, "null operator");
    if (!(c > 0) || !std::isfinite(c)) fail(CPM_ERR_ARG, "shift c must be positive and finite");
    hip_check(hipDeviceSynchronize(), "set_shift");
    op->c = c;
    stencil_coefficients(op->order, op->I.d, op->I.h, c, op->I.diag, op->I.inv_h2);
    op->d_inst.upload(&op->I, 1);
    // the cached single-solve batch holds a copy of the old shift
    op->solve_cache.reset();
    op->solve_cache_key = -1;
    return CPM_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  }
}

double cpm_operator_get_shift(const cpm_operator* op) { return op ? op->c : 0.0; }
int64_t cpm_operator_n_active(const cpm_operator* op) { return op ? op->band->nA : -1; }

void cpm_operator_destroy(cpm_operator* op) { delete op; }

cpm_status cpm_extend_apply(const cpm_operator* op, const double* u, double* v, void* stream) {
  try {
    if (!op || (!u && op->band->nA) || (!v && op->band->nodes())) fail(CPM_ERR_ARG, "null argument");
    if (u == v && u) fail(CPM_ERR_ARG, "u and v must not alias");
    hip_check(launch_extend(op->I, u, v, (hipStream_t)stream), "cpm_extend_apply");
    return CPM_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  }
}

cpm_status cpm_apply(const cpm_operator* op, const double* x, double* y, int32_t nrhs, void* stream) {
  try {
    if (!op || !x || !y) fail(CPM_ERR_ARG, "null argument");
    if (nrhs != 1 && nrhs != 2 && nrhs != 4) fail(CPM_ERR_ARG, "nrhs must be 1, 2 or 4");
    if (x == y) fail(CPM_ERR_ARG, "x and y must not alias");
    const int variant = (nrhs == 1 && op->apply_variant == kApplyTwoPass && !op->twopass) ? kApplyPipelined
                                                                                         : op->apply_variant;
    hip_check(launch_apply(op->apply_args(), nrhs, variant, x, y, (hipStream_t)stream), "cpm_apply");
    return CPM_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  }
}

cpm_status cpm_apply_T(const cpm_operator* op, const double* x, double* y, int32_t nrhs, void* stream) {
  try {
    if (!op || !x || !y) fail(CPM_ERR_ARG, "null argument");
    if (nrhs != 1 && nrhs != 2 && nrhs != 4) fail(CPM_ERR_ARG, "nrhs must be 1, 2 or 4");
    if (x == y) fail(CPM_ERR_ARG, "x and y must not alias");
    if (op->generic) fail(CPM_ERR_ARG, "the transposed apply needs a second-order operator with p <= 3");
    op->d_z.alloc((size_t)op->band->nodes() * 4);
    hip_check(launch_apply_T(op->I, nrhs, x, op->d_z.p, y, (hipStream_t)stream), "cpm_apply_T");
    return CPM_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  }
}
