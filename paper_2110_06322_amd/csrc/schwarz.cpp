// Restricted / optimized restricted additive Schwarz setup (paper Sec. 2.2;
// Sec. 4.1.1 for the defaults alpha = 4, alpha_cross = 20 and incomplete LU
// local solves).
//
//   partition : recursive coordinate bisection of Sigma_A by closest point:
//               axis of largest cp extent, split value s = floor(n/2)-th
//               smallest coordinate, cp < s to the first child;
//   overlap   : Omega_j = {i : box_lo_j - N_O h <= cp_i <= box_hi_j + N_O h};
//   local     : rows/columns of A in Omega_j, ascending grid key, on A's
//               structural pattern (every cube node of every neighbour);
//   ORAS      : a_ii += s_i / (1 + alpha_i h), s_i = sum of the couplings of
//               row i to nodes outside Omega_j, alpha_i = alpha_cross when
//               those nodes belong to two or more other subdomains;
//   factors   : ILU(0) (IKJ order) or dense LU with partial pivoting, in FP64,
//               stored as CSR with 16-bit local columns, FP64 or FP32 values.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "schwarz.h"

using namespace cpm;

namespace {

struct KdNode {
  int axis = -1;
  double split = 0;
  int left = -1, right = -1, leaf = -1;
};

// Lagrange basis on 0..p at s (product form)
inline void lagrange(int p, double s, double* w) {
  for (int j = 0; j <= p; ++j) {
    double v = 1.0;
    for (int m = 0; m <= p; ++m)
      if (m != j) v *= (s - m) / (double)(j - m);
    w[j] = v;
  }
}

struct Rcb {
  std::vector<KdNode> tree;
  std::vector<std::array<double, 3>> lo, hi;   // leaf boxes
  std::vector<int32_t> owner;
};

Rcb rcb(const cpm_band_s& B, int nparts) {
  const int d = B.d;
  const int64_t n = B.nA;
  Rcb R;
  R.owner.assign(n, 0);
  struct Part { std::vector<int32_t> idx; std::array<double, 3> lo, hi; int node; };
  std::vector<Part> parts(1);
  parts[0].idx.resize(n);
  std::iota(parts[0].idx.begin(), parts[0].idx.end(), 0);
  for (int k = 0; k < 3; ++k) { parts[0].lo[k] = 0; parts[0].hi[k] = 0; }
  for (int k = 0; k < d; ++k) {
    double mn = INFINITY, mx = -INFINITY;
    for (int64_t i = 0; i < n; ++i) { mn = std::min(mn, B.cp[i * d + k]); mx = std::max(mx, B.cp[i * d + k]); }
    parts[0].lo[k] = mn;
    parts[0].hi[k] = mx;
  }
  R.tree.push_back(KdNode{});
  parts[0].node = 0;
  while ((int)parts.size() < nparts) {
    std::vector<Part> next;
    for (auto& P : parts) {
      double ext[3] = {0, 0, 0};
      for (int k = 0; k < d; ++k) {
        double mn = INFINITY, mx = -INFINITY;
        for (int32_t i : P.idx) { mn = std::min(mn, B.cp[(int64_t)i * d + k]); mx = std::max(mx, B.cp[(int64_t)i * d + k]); }
        ext[k] = mx - mn;
      }
      int axis = 0;
      for (int k = 1; k < d; ++k)
        if (ext[k] > ext[axis]) axis = k;
      std::vector<double> vals(P.idx.size());
      for (size_t q = 0; q < P.idx.size(); ++q) vals[q] = B.cp[(int64_t)P.idx[q] * d + axis];
      std::vector<double> tmp(vals);
      size_t m = P.idx.size() / 2;
      std::nth_element(tmp.begin(), tmp.begin() + m, tmp.end());
      double s = tmp[m];
      Part L, U;
      for (size_t q = 0; q < P.idx.size(); ++q) (vals[q] < s ? L : U).idx.push_back(P.idx[q]);
      if (L.idx.empty() || U.idx.empty()) fail(CPM_ERR_ARG, "partition produced an empty subdomain");
      L.lo = P.lo; L.hi = P.hi; L.hi[axis] = s;
      U.lo = P.lo; U.hi = P.hi; U.lo[axis] = s;
      const int li = (int)R.tree.size();
      R.tree.push_back(KdNode{});
      const int ri = (int)R.tree.size();
      R.tree.push_back(KdNode{});
      R.tree[P.node].axis = axis;
      R.tree[P.node].split = s;
      R.tree[P.node].left = li;
      R.tree[P.node].right = ri;
      L.node = li;
      U.node = ri;
      next.push_back(std::move(L));
      next.push_back(std::move(U));
    }
    parts.swap(next);
  }
  R.lo.resize(parts.size());
  R.hi.resize(parts.size());
  for (size_t j = 0; j < parts.size(); ++j) {
    R.tree[parts[j].node].leaf = (int)j;
    R.lo[j] = parts[j].lo;
    R.hi[j] = parts[j].hi;
    for (int32_t i : parts[j].idx) R.owner[i] = (int32_t)j;
  }
  return R;
}

// leaves whose grown box holds point c (exact test at the leaves, safe pruning above)
void query(const Rcb& R, int node, const double* c, double delta, int d, std::vector<int>& out) {
  const KdNode& nd = R.tree[node];
  if (nd.leaf >= 0) {
    int j = nd.leaf;
    for (int k = 0; k < d; ++k)
      if (!(c[k] >= R.lo[j][k] - delta && c[k] <= R.hi[j][k] + delta)) return;
    out.push_back(j);
    return;
  }
  if (c[nd.axis] <= nd.split + delta) query(R, nd.left, c, delta, d, out);
  if (c[nd.axis] >= nd.split - delta) query(R, nd.right, c, delta, d, out);
}

int64_t grid_key(const cpm_band_s& B, int64_t node) {
  int64_t key = 0;
  for (int k = 0; k < B.d; ++k) key = key * B.shape[k] + B.gidx[node * B.d + k];
  return key;
}

}  // namespace

namespace cpm {

// Extension row of node n: global active indices and weights of its cube. Bands of degree
// p > 3 use degree 3 here: the preconditioner approximates the operator with cubic
// interpolation (the cubic cube lies inside the degree-p one, hence in Sigma_A).
void extension_row(const cpm_band_s& B, int64_t n, std::vector<int32_t>& cols, std::vector<double>& w) {
  const int d = B.d, p = std::min(B.p, 3), P1 = p + 1;
  int32_t b[3] = {0, 0, 0};
  double wk[3][4];
  for (int k = 0; k < d; ++k) {
    double t = (B.ip[n * d + k] - B.lo[k]) / B.h;
    double bf = std::floor(t - (p - 1) / 2.0);
    b[k] = (int32_t)bf;
    lagrange(p, t - bf, wk[k]);
  }
  const int nc = d == 3 ? P1 * P1 * P1 : P1 * P1;
  cols.resize(nc);
  w.resize(nc);
  for (int q = 0; q < nc; ++q) {
    int a[3] = {0, 0, 0}, r = q;
    for (int k = d - 1; k >= 0; --k) { a[k] = r % P1; r /= P1; }
    int32_t g[3] = {b[0] + a[0], b[1] + a[1], d == 3 ? b[2] + a[2] : 0};
    int64_t j = B.lookup(g);
    if (j < 0 || j >= B.nA) fail(CPM_ERR_BAND, "interpolation cube outside Sigma_A");
    cols[q] = (int32_t)j;
    double v = 1.0;
    for (int k = 0; k < d; ++k) v *= wk[k][a[k]];
    w[q] = B.sgn.empty() ? v : B.sgn[n] * v;
  }
}

// Row i of A restricted to its structural pattern: sorted global columns and values.
void operator_row(const cpm_band_s& B, double c, int64_t i, std::vector<int32_t>& cols, std::vector<double>& vals,
                  std::vector<int32_t>& scratch_c, std::vector<double>& scratch_w) {
  const int d = B.d;
  const double inv_h2 = 1.0 / (B.h * B.h);
  cols.clear();
  vals.clear();
  std::vector<std::pair<int32_t, double>> ent;
  ent.reserve(8 * 64);
  ent.push_back({(int32_t)i, c + 2.0 * d * inv_h2});
  for (int k = 0; k < d; ++k)
    for (int s = -1; s <= 1; s += 2) {
      int32_t g[3] = {0, 0, 0};
      for (int q = 0; q < d; ++q) g[q] = B.gidx[i * d + q];
      g[k] += s;
      int64_t n = B.lookup(g);
      if (n < 0) fail(CPM_ERR_BAND, "active node without a band neighbour");
      extension_row(B, n, scratch_c, scratch_w);
      for (size_t q = 0; q < scratch_c.size(); ++q) ent.push_back({scratch_c[q], -inv_h2 * scratch_w[q]});
    }
  std::stable_sort(ent.begin(), ent.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
  for (auto& e : ent) {
    if (!cols.empty() && cols.back() == e.first) vals.back() += e.second;
    else { cols.push_back(e.first); vals.push_back(e.second); }
  }
}

}  // namespace cpm

namespace {

// ILU(0), IKJ order, on the stored pattern (sorted columns). Returns false on a zero pivot.
bool ilu0(int n, const std::vector<int64_t>& ptr, const std::vector<int32_t>& col, std::vector<double>& val,
          std::vector<int64_t>& dpos) {
  dpos.assign(n, -1);
  for (int i = 0; i < n; ++i)
    for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e)
      if (col[e] == i) dpos[i] = e;
  std::vector<int64_t> where(n, -1);
  for (int i = 0; i < n; ++i) {
    if (dpos[i] < 0) return false;
    for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) where[col[e]] = e;
    for (int64_t e = ptr[i]; e < ptr[i + 1] && col[e] < i; ++e) {
      int k = col[e];
      double piv = val[dpos[k]];
      if (piv == 0.0) return false;
      double l = val[e] / piv;
      val[e] = l;
      for (int64_t f = dpos[k] + 1; f < ptr[k + 1]; ++f) {
        int64_t t = where[col[f]];
        if (t >= 0) val[t] -= l * val[f];
      }
    }
    for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) where[col[e]] = -1;
    if (val[dpos[i]] == 0.0) return false;
  }
  return true;
}

// Dense LU with partial pivoting: P A = L U. Returns false if singular.
bool dense_lu(int n, std::vector<double>& a, std::vector<int32_t>& perm) {
  perm.resize(n);
  std::iota(perm.begin(), perm.end(), 0);
  for (int k = 0; k < n; ++k) {
    int pr = k;
    double best = std::fabs(a[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(a[(size_t)i * n + k]) > best) { best = std::fabs(a[(size_t)i * n + k]); pr = i; }
    if (best == 0.0) return false;
    if (pr != k) {
      for (int j = 0; j < n; ++j) std::swap(a[(size_t)k * n + j], a[(size_t)pr * n + j]);
      std::swap(perm[k], perm[pr]);
    }
    double piv = a[(size_t)k * n + k];
    for (int i = k + 1; i < n; ++i) {
      double l = a[(size_t)i * n + k] / piv;
      a[(size_t)i * n + k] = l;
      if (l != 0.0)
        for (int j = k + 1; j < n; ++j) a[(size_t)i * n + j] -= l * a[(size_t)k * n + j];
    }
  }
  return true;
}

// Reverse Cuthill-McKee order of the symmetrized pattern (George & Liu 1981):
// each component starts at its unvisited node of least (degree, index);
// unvisited neighbours are queued by (degree, index); the sequence is reversed.
// Local rows by decreasing distance |x - cp(x)| of their grid node from the
// surface, ties by local index (ascending grid key); perm[q] = row at q.
std::vector<int32_t> distance_order(const cpm_band_s& B, const std::vector<int32_t>& rows) {
  const int n = (int)rows.size(), d = B.d;
  std::vector<double> dist(n);
  for (int q = 0; q < n; ++q) {
    const int64_t i = rows[q];
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
      const double x = B.lo[k] + B.gidx[i * d + k] * B.h;
      const double e = x - B.cp[i * d + k];
      s += e * e;
    }
    dist[q] = std::sqrt(s);
  }
  std::vector<int32_t> perm(n);
  for (int q = 0; q < n; ++q) perm[q] = q;
  std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return dist[a] > dist[b]; });
  return perm;
}

std::vector<int32_t> rcm_order(int n, const std::vector<int64_t>& ptr, const std::vector<int32_t>& col) {
  std::vector<int64_t> cnt(n + 1, 0);
  for (int i = 0; i < n; ++i)
    for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e)
      if (col[e] != i) { cnt[i + 1]++; cnt[col[e] + 1]++; }
  for (int i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  std::vector<int32_t> adj(cnt[n]);
  std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
  for (int i = 0; i < n; ++i)
    for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e)
      if (col[e] != i) { adj[fill[i]++] = col[e]; adj[fill[col[e]]++] = i; }
  std::vector<int64_t> aptr(n + 1, 0);
  std::vector<int32_t> a2;
  a2.reserve(adj.size());
  for (int i = 0; i < n; ++i) {
    std::sort(adj.begin() + cnt[i], adj.begin() + cnt[i + 1]);
    auto last = std::unique(adj.begin() + cnt[i], adj.begin() + cnt[i + 1]);
    a2.insert(a2.end(), adj.begin() + cnt[i], last);
    aptr[i + 1] = (int64_t)a2.size();
  }
  std::vector<int64_t> deg(n);
  for (int i = 0; i < n; ++i) deg[i] = aptr[i + 1] - aptr[i];
  auto less = [&](int a, int b) { return deg[a] != deg[b] ? deg[a] < deg[b] : a < b; };
  std::vector<int32_t> by(n);
  std::iota(by.begin(), by.end(), 0);
  std::sort(by.begin(), by.end(), less);
  std::vector<char> vis(n, 0);
  std::vector<int32_t> order;
  order.reserve(n);
  size_t nxt = 0;
  std::vector<int32_t> nb;
  while ((int)order.size() < n) {
    while (vis[by[nxt]]) ++nxt;
    size_t head = order.size();
    order.push_back(by[nxt]);
    vis[by[nxt]] = 1;
    while (head < order.size()) {
      int v = order[head++];
      nb.clear();
      for (int64_t e = aptr[v]; e < aptr[v + 1]; ++e)
        if (!vis[a2[e]]) nb.push_back(a2[e]);
      std::sort(nb.begin(), nb.end(), less);
      for (int u : nb) { vis[u] = 1; order.push_back(u); }
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}

// rows in increasing dependency level (a topological order of the sweep)
// (levpos, when given, receives the level of the row at each schedule position;
// by_class orders the rows of a level by their packet length class first)
std::vector<uint16_t> schedule(int n, const std::vector<int64_t>& ptr, const std::vector<uint16_t>& col, bool lower,
                               int& nlev, std::vector<int32_t>* levpos = nullptr, bool by_class = false) {
  std::vector<int> lev(n, 0);
  nlev = 0;
  for (int t = 0; t < n; ++t) {
    int i = lower ? t : n - 1 - t;
    int l = 0;
    for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) l = std::max(l, lev[col[e]] + 1);
    lev[i] = l;
    nlev = std::max(nlev, l + 1);
  }
  std::vector<uint16_t> s(n);
  std::iota(s.begin(), s.end(), 0);
  std::stable_sort(s.begin(), s.end(), [&](uint16_t a, uint16_t b) {
    if (lev[a] != lev[b]) return lev[a] < lev[b];
    if (by_class) {
      const int ca = packet_class(ptr[a + 1] - ptr[a]), cb = packet_class(ptr[b + 1] - ptr[b]);
      if (ca != cb) return ca < cb;
    }
    return lower ? a < b : a > b;
  });
  if (levpos) {
    levpos->resize(n);
    for (int t = 0; t < n; ++t) (*levpos)[t] = lev[s[t]];
  }
  return s;
}

}  // namespace

namespace cpm {

void build_schwarz_host(const cpm_band_s& B, double c, const cpm_precond_opts& o, SchwarzHost& S) {
  const int d = B.d;
  const int64_t nA = B.nA;
  const int np = o.n_parts;
  if (np < 1 || (np & (np - 1))) fail(CPM_ERR_ARG, "n_parts must be a power of two");
  if (np > nA) fail(CPM_ERR_ARG, "more subdomains than unknowns");
  if (!(o.overlap >= 0) || !std::isfinite(o.overlap)) fail(CPM_ERR_ARG, "overlap must be >= 0");
  if (o.kind == CPM_PC_ORAS && !(o.alpha > 0 && o.alpha_cross > 0)) fail(CPM_ERR_ARG, "alpha must be > 0");
  Rcb R = rcb(B, np);
  S.owner = R.owner;
  S.nparts = np;
  // ---- overlap sets
  const double delta = o.overlap * B.h;
  std::vector<std::vector<int32_t>> omega(np);
  {
    std::vector<std::vector<int>> hits(nA);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t i = 0; i < nA; ++i) query(R, 0, &B.cp[i * d], delta, d, hits[i]);
    for (int64_t i = 0; i < nA; ++i)
      for (int j : hits[i]) omega[j].push_back((int32_t)i);
  }
  std::vector<int64_t> keys(nA);
  for (int64_t i = 0; i < nA; ++i) keys[i] = grid_key(B, i);
  for (int j = 0; j < np; ++j) {
    std::sort(omega[j].begin(), omega[j].end(), [&](int32_t a, int32_t b) { return keys[a] < keys[b]; });
    if (omega[j].size() > 65535) fail(CPM_ERR_ARG, "subdomain larger than 65535 rows; use more subdomains");
  }
  // ---- global CSR of A (or A^T) on the structural pattern
  std::vector<int64_t> gptr(nA + 1, 0);
  std::vector<int32_t> gcol;
  std::vector<double> gval;
  {
    const int nthreads = 64;
    std::vector<std::vector<int32_t>> tc(nthreads);
    std::vector<std::vector<double>> tv(nthreads);
    std::vector<int64_t> rowlen(nA, 0);
    bool bad = false;
    std::string msg;
#pragma omp parallel for schedule(static, 1)
    for (int t = 0; t < nthreads; ++t) {
      std::vector<int32_t> rc, sc;
      std::vector<double> rv, sw;
      int64_t a = nA * t / nthreads, b = nA * (t + 1) / nthreads;
      try {
        for (int64_t i = a; i < b; ++i) {
          operator_row(B, c, i, rc, rv, sc, sw);
          rowlen[i] = (int64_t)rc.size();
          tc[t].insert(tc[t].end(), rc.begin(), rc.end());
          tv[t].insert(tv[t].end(), rv.begin(), rv.end());
        }
      } catch (const Error& e) {
#pragma omp critical
        { bad = true; msg = e.msg; }
      }
    }
    if (bad) fail(CPM_ERR_BAND, msg);
    for (int64_t i = 0; i < nA; ++i) gptr[i + 1] = gptr[i] + rowlen[i];
    gcol.reserve(gptr[nA]);
    gval.reserve(gptr[nA]);
    for (int t = 0; t < nthreads; ++t) {
      gcol.insert(gcol.end(), tc[t].begin(), tc[t].end());
      gval.insert(gval.end(), tv[t].begin(), tv[t].end());
      std::vector<int32_t>().swap(tc[t]);
      std::vector<double>().swap(tv[t]);
    }
  }
  if (o.transpose) {
    std::vector<int64_t> tp(nA + 1, 0);
    for (int64_t e = 0; e < gptr[nA]; ++e) tp[gcol[e] + 1]++;
    for (int64_t i = 0; i < nA; ++i) tp[i + 1] += tp[i];
    std::vector<int32_t> tcol(gptr[nA]);
    std::vector<double> tval(gptr[nA]);
    std::vector<int64_t> fill(tp.begin(), tp.end() - 1);
    for (int64_t i = 0; i < nA; ++i)
      for (int64_t e = gptr[i]; e < gptr[i + 1]; ++e) {
        int64_t t = fill[gcol[e]]++;
        tcol[t] = (int32_t)i;
        tval[t] = gval[e];
      }
    gptr.swap(tp);
    gcol.swap(tcol);
    gval.swap(tval);
  }
  S.global_nnz = gptr[nA];
  // ---- local matrices and factors, one subdomain per task
  S.subs.assign(np, SchwarzHost::Sub{});
  bool pivot_fail = false, other_fail = false;
  std::string other_msg;
#pragma omp parallel
  {
    std::vector<int32_t> local(nA, -1);
#pragma omp for schedule(dynamic, 1)
    for (int j = 0; j < np; ++j) {
      try {
        const auto& om = omega[j];
        const int n = (int)om.size();
        for (int q = 0; q < n; ++q) local[om[q]] = q;
        SchwarzHost::Sub& sub = S.subs[j];
        sub.n = n;
        sub.rows.assign(om.begin(), om.end());
        std::vector<int64_t> ptr(n + 1, 0);
        std::vector<int32_t> col;
        std::vector<double> val;
        for (int q = 0; q < n; ++q) {
          const int64_t gi = om[q];
          double s_out = 0.0;
          int own1 = -1;
          bool cross = false;
          std::vector<std::pair<int32_t, double>> ent;
          for (int64_t e = gptr[gi]; e < gptr[gi + 1]; ++e) {
            int32_t lk = local[gcol[e]];
            if (lk >= 0) ent.push_back({lk, gval[e]});
            else {
              s_out += gval[e];
              int ow = R.owner[gcol[e]];
              if (own1 < 0) own1 = ow;
              else if (ow != own1) cross = true;
            }
          }
          if (o.kind == CPM_PC_ORAS && own1 >= 0) {
            double a = cross ? o.alpha_cross : o.alpha;
            for (auto& e : ent)
              if (e.first == q) e.second += s_out / (1.0 + a * B.h);
          }
          std::sort(ent.begin(), ent.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
          for (auto& e : ent) { col.push_back(e.first); val.push_back(e.second); }
          ptr[q + 1] = (int64_t)col.size();
        }
        sub.nnz = (int64_t)col.size();
        if (o.subsolver == CPM_SUB_ILU0) {
          // reverse Cuthill-McKee or distance order, then ILU(0) of the permuted matrix
          std::vector<int32_t> perm =
              o.ordering == CPM_ORDER_DISTANCE ? distance_order(B, sub.rows) : rcm_order(n, ptr, col);
          std::vector<int32_t> inv(n);
          for (int q = 0; q < n; ++q) inv[perm[q]] = q;
          std::vector<int64_t> pptr(n + 1, 0);
          std::vector<int32_t> pcol;
          std::vector<double> pval;
          pcol.reserve(col.size());
          pval.reserve(val.size());
          std::vector<std::pair<int32_t, double>> row;
          for (int q = 0; q < n; ++q) {
            const int src = perm[q];
            row.clear();
            for (int64_t e = ptr[src]; e < ptr[src + 1]; ++e) row.push_back({inv[col[e]], val[e]});
            std::sort(row.begin(), row.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
            for (auto& r : row) { pcol.push_back(r.first); pval.push_back(r.second); }
            pptr[q + 1] = (int64_t)pcol.size();
          }
          std::vector<int64_t> dpos;
          if (!ilu0(n, pptr, pcol, pval, dpos)) {
#pragma omp atomic write
            pivot_fail = true;
          }
          sub.perm = perm;
          sub.operm = perm;
          sub.lptr.assign(n + 1, 0);
          sub.uptr.assign(n + 1, 0);
          sub.dinv.assign(n, 0.0);
          for (int q = 0; q < n; ++q) {
            for (int64_t e = pptr[q]; e < pptr[q + 1]; ++e) {
              if (pcol[e] < q) { sub.lcol.push_back((uint16_t)pcol[e]); sub.lval.push_back(pval[e]); }
              else if (pcol[e] > q) { sub.ucol.push_back((uint16_t)pcol[e]); sub.uval.push_back(pval[e]); }
              else sub.dinv[q] = 1.0 / pval[e];
            }
            sub.lptr[q + 1] = (int64_t)sub.lcol.size();
            sub.uptr[q + 1] = (int64_t)sub.ucol.size();
          }
        } else {
          if ((int64_t)n * n > (int64_t)1 << 26) fail(CPM_ERR_ARG, "dense LU subsolver: subdomain too large");
          std::vector<double> a((size_t)n * n, 0.0);
          for (int q = 0; q < n; ++q)
            for (int64_t e = ptr[q]; e < ptr[q + 1]; ++e) a[(size_t)q * n + col[e]] = val[e];
          if (!dense_lu(n, a, sub.perm)) {
#pragma omp atomic write
            pivot_fail = true;
          }
          sub.operm.resize(n);
          std::iota(sub.operm.begin(), sub.operm.end(), 0);
          sub.lptr.assign(n + 1, 0);
          sub.uptr.assign(n + 1, 0);
          sub.dinv.assign(n, 0.0);
          for (int q = 0; q < n; ++q) {
            for (int k = 0; k < q; ++k) { sub.lcol.push_back((uint16_t)k); sub.lval.push_back(a[(size_t)q * n + k]); }
            for (int k = q + 1; k < n; ++k) { sub.ucol.push_back((uint16_t)k); sub.uval.push_back(a[(size_t)q * n + k]); }
            sub.dinv[q] = 1.0 / a[(size_t)q * n + q];
            sub.lptr[q + 1] = (int64_t)sub.lcol.size();
            sub.uptr[q + 1] = (int64_t)sub.ucol.size();
          }
        }
        int ll = 0, lu = 0;
        const bool by_class = o.ordering == CPM_ORDER_DISTANCE;   // rows are packed by length class
        sub.schedL = schedule(n, sub.lptr, sub.lcol, true, ll, &sub.levL, by_class);
        sub.schedU = schedule(n, sub.uptr, sub.ucol, false, lu, &sub.levU, by_class);
        sub.levels = std::max(ll, lu);
        for (int q = 0; q < n; ++q) local[om[q]] = -1;
      } catch (const Error& e) {
#pragma omp critical
        {
          other_fail = true;
          other_msg = e.msg;
        }
      }
    }
  }
  if (other_fail) fail(CPM_ERR_ARG, other_msg);
  if (pivot_fail) fail(CPM_ERR_PIVOT, "zero pivot in a local factorization");
}

}  // namespace cpm
