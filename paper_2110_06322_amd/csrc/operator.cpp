// Operator setup: tiles and LDS footprints for the fused apply, extension-row
// buckets for the atomic-free transpose, upload of the band to the device.
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
void build_tiles(const cpm_band_s& B, std::vector<DevTile>& tiles, std::vector<int32_t>& fvol,
                 std::vector<FootBrick>& fbrec, std::vector<Job>& jobs) {
  bool orphan = false;
  const int d = B.d, E = brick_edge(d), T = 2 * E, P = B.p, W = T + 2;
  const int64_t nb = B.nbricks();
  std::vector<int64_t> start;
  for (int64_t i = 0; i < nb; ++i) {
    bool fresh = i == 0;
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
    for (int q = 0; q < 8; ++q) { tl.oA[q] = 0; tl.mA[q] = 0; }
    for (int k = 0; k < 3; ++k) tl.origin[k] = 0;
    for (int k = 0; k < d; ++k) tl.origin[k] = (B.bcoord[start[t] * 3 + k] >> 1) * T;
    int32_t lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    auto add_job = [&](int64_t node, const int* l) {
      int32_t b[3];
      base_of(B, &B.cp[node * d], b);
      for (int k = 0; k < d; ++k) { lo[k] = std::min(lo[k], b[k]); hi[k] = std::max(hi[k], b[k] + P); }
      jb[t].push_back(Job{(int32_t)node, (int32_t)slot_of(l)});
    };
    for (int64_t i = start[t]; i < start[t + 1]; ++i) {
      int sub = 0;
      for (int k = 0; k < d; ++k) sub = sub * 2 + (B.bcoord[i * 3 + k] & 1);
      tl.oA[sub] = B.offA[i];
      tl.mA[sub] = B.maskA[i];
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
          if (set != 0) continue;
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
        base_of(B, &B.cp[(int64_t)j.node * d], b);
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

// Extension rows bucketed by their cube's lower corner (an active node).
void build_buckets(const cpm_band_s& B, std::vector<int32_t>& ptr, std::vector<int32_t>& rows) {
  const int64_t n = B.nodes();
  std::vector<int32_t> corner(n);
  bool bad = false;
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < n; ++j) {
    int32_t b[3] = {0, 0, 0};
    base_of(B, &B.cp[j * B.d], b);
    int64_t c = B.lookup(b);
    if (c < 0 || c >= B.nA) {
#pragma omp atomic write
      bad = true;
      corner[j] = 0;
    } else {
      corner[j] = (int32_t)c;
    }
  }
  if (bad) fail(CPM_ERR_BAND, "interpolation cube corner outside Sigma_A");
  ptr.assign(B.nA + 1, 0);
  for (int64_t j = 0; j < n; ++j) ptr[corner[j] + 1]++;
  for (int64_t i = 0; i < B.nA; ++i) ptr[i + 1] += ptr[i];
  rows.assign(n, 0);
  std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
  for (int64_t j = 0; j < n; ++j) rows[fill[corner[j]]++] = (int32_t)j;
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

cpm_status cpm_operator_create(const cpm_band* band, double c, void* stream, cpm_operator** out) {
  (void)stream;
  try {
    if (!band || !out) fail(CPM_ERR_ARG, "null argument");
    *out = nullptr;
    if (!(c > 0) || !std::isfinite(c)) fail(CPM_ERR_ARG, "shift c must be positive and finite");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) fail(CPM_ERR_DEVICE, "no HIP device available");
    auto op = std::make_unique<cpm_operator_s>();
    op->band = std::make_shared<cpm_band_s>(*band);
    op->c = c;
    const cpm_band_s& B = *op->band;
    const int d = B.d;
    const int64_t n = B.nodes();
    std::vector<FootBrick> fbrec;
    std::vector<Job> jobs;
    build_tiles(B, op->tiles, op->tile_fvol, fbrec, jobs);
    op->d_fbrec.upload(fbrec);
    op->d_jobs.upload(jobs);
    std::vector<int32_t> bptr, brows;
    build_buckets(B, bptr, brows);
    // SoA closest points
    std::vector<double> cps(n * d);
    for (int64_t j = 0; j < n; ++j)
      for (int k = 0; k < d; ++k) cps[k * n + j] = (B.cp[j * d + k] - B.lo[k]) / B.h;
    op->d_tcp.upload(cps);
    op->d_maskA.upload(B.maskA);
    op->d_maskG.upload(B.maskG);
    op->d_offA.upload(B.offA);
    op->d_offG.upload(B.offG);
    op->d_bcoord.upload(B.bcoord);
    op->d_bmap.upload(B.bmap);
    op->d_tiles.upload(op->tiles);
    op->d_bptr.upload(bptr);
    op->d_brows.upload(brows);
    DevInst& I = op->I;
    std::memset(&I, 0, sizeof(I));
    I.d = d; I.p = B.p; I.nA = (int32_t)B.nA; I.nG = (int32_t)B.nG;
    I.h = B.h;
    I.inv_h2 = 1.0 / (B.h * B.h);
    I.diag = c + 2.0 * d / (B.h * B.h);
    for (int k = 0; k < 3; ++k) { I.lo[k] = B.lo[k]; I.bm_lo[k] = B.bm_lo[k]; I.bm_dim[k] = B.bm_dim[k]; }
    I.tcp = op->d_tcp.p;
    I.maskA = op->d_maskA.p; I.maskG = op->d_maskG.p;
    I.offA = op->d_offA.p; I.offG = op->d_offG.p;
    I.bcoord = op->d_bcoord.p; I.bmap = op->d_bmap.p;
    I.tiles = op->d_tiles.p;
    I.fbrec = op->d_fbrec.p;
    I.jobs = op->d_jobs.p;
    I.ntiles = (int32_t)op->tiles.size();
    I.nbricks = (int32_t)B.nbricks();
    I.bucket_ptr = op->d_bptr.p; I.bucket_rows = op->d_brows.p;
    I.vec_off = 0;
    op->d_inst.upload(&I, 1);
    // work lists: tiles whose footprint fits the LDS budget, the rest take the slow path
    const int cap = (int)((kApplyLdsBytes - tile_lds_extra_bytes(d)) / sizeof(double));
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

cpm_status cpm_operator_set_shift(cpm_operator* op, double c) {
  try {
    if (!op) fail(CPM_ERR_ARG, "null operator");
    if (!(c > 0) || !std::isfinite(c)) fail(CPM_ERR_ARG, "shift c must be positive and finite");
    hip_check(hipDeviceSynchronize(), "set_shift");
    op->c = c;
    op->I.diag = c + 2.0 * op->I.d / (op->I.h * op->I.h);
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
    hip_check(launch_apply(op->I.d, op->I.p, nrhs, op->apply_variant, op->d_inst.p, op->d_work.p, op->pipe(), op->nwork, op->ucap,
                           op->d_fb.p, op->nfb, x, y, (hipStream_t)stream),
              "cpm_apply");
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
    op->d_z.alloc((size_t)op->band->nodes() * 4);
    hip_check(launch_apply_T(op->I, nrhs, x, op->d_z.p, y, (hipStream_t)stream), "cpm_apply_T");
    return CPM_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  }
}
