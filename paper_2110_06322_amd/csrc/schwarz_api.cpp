// C ABI of the (O)RAS preconditioner: setup on the host, packed upload, apply.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "schwarz.h"

using namespace cpm;

cpm_status cpm_precond_opts_default(cpm_precond_opts* o) {
  if (!o) { set_error("null argument"); return CPM_ERR_ARG; }
  o->kind = CPM_PC_ORAS;
  o->n_parts = 64;
  o->overlap = 2.0;
  o->alpha = 4.0;
  o->alpha_cross = 20.0;
  o->subsolver = CPM_SUB_ILU0;
  o->precision = CPM_PREC_FP64;
  o->transpose = 0;
  o->ordering = CPM_ORDER_RCM;
  o->coarse = CPM_COARSE_NONE;
  return CPM_OK;
}

namespace {

constexpr int kMaxCoarse = 4096;

// Dense inverse by Gauss-Jordan elimination with partial pivoting (row-major n x n);
// false when a pivot vanishes. a is overwritten.
bool dense_inverse(int n, std::vector<double>& a, std::vector<double>& inv) {
  inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int k = 0; k < n; ++k) {
    int piv = k;
    double best = std::fabs(a[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      const double v = std::fabs(a[(size_t)i * n + k]);
      if (v > best) { best = v; piv = i; }
    }
    if (!(best > 0.0) || !std::isfinite(best)) return false;
    if (piv != k)
      for (int j = 0; j < n; ++j) {
        std::swap(a[(size_t)k * n + j], a[(size_t)piv * n + j]);
        std::swap(inv[(size_t)k * n + j], inv[(size_t)piv * n + j]);
      }
    const double d = a[(size_t)k * n + k];
    for (int j = 0; j < n; ++j) {
      a[(size_t)k * n + j] /= d;
      inv[(size_t)k * n + j] /= d;
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      const double f = a[(size_t)i * n + k];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        a[(size_t)i * n + j] -= f * a[(size_t)k * n + j];
        inv[(size_t)i * n + j] -= f * inv[(size_t)k * n + j];
      }
    }
  }
  return true;
}

// Coarse level: owned-node lists, the Galerkin matrix A0 = R0 A R0^T (column
// block j0..j0+3 from A applied to four indicator vectors, then restricted),
// its inverse on the device.
void build_coarse(cpm_precond_s& pc) {
  const cpm_operator_s* op = pc.op;
  const auto& owner = pc.host.owner;
  const int n = pc.host.nparts;
  const int64_t nA = op->band->nA;
  std::vector<int32_t> ptr(n + 1, 0), idx(nA);
  for (int64_t i = 0; i < nA; ++i) ptr[owner[i] + 1]++;
  for (int j = 0; j < n; ++j) ptr[j + 1] += ptr[j];
  {
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (int64_t i = 0; i < nA; ++i) idx[fill[owner[i]]++] = (int32_t)i;
  }
  pc.d_own_ptr.upload(ptr);
  pc.d_own_idx.upload(idx);
  pc.d_owner.upload(owner);
  DevCoarse& C = pc.C;
  C.n = n;
  C.mode = pc.opts.coarse;
  C.nA = nA;
  C.own_ptr = pc.d_own_ptr.p;
  C.own_idx = pc.d_own_idx.p;
  C.owner = pc.d_owner.p;
  C.vec_off = 0;
  C.coff = 0;
  DevBuf<double> X, Y, col;
  X.alloc((size_t)nA * 4);
  Y.alloc((size_t)nA * 4);
  col.alloc((size_t)n * 4);
  std::vector<double> A0((size_t)n * n), h(4 * (size_t)n);
  const hipStream_t s = nullptr;
  const ApplyArgs args = op->apply_args();
  for (int j0 = 0; j0 < n; j0 += 4) {
    hip_check(coarse_indicators(C, j0, X.p, s), "coarse indicators");
    hip_check(launch_apply(args, 4, kApplyPerTile, X.p, Y.p, s), "coarse apply");
    hip_check(coarse_restrict(C, 4, Y.p, col.p, s), "coarse restrict");
    hip_check(hipMemcpy(h.data(), col.p, h.size() * sizeof(double), hipMemcpyDeviceToHost), "coarse column");
    for (int j = 0; j < n; ++j)
      for (int q = 0; q < 4 && j0 + q < n; ++q) A0[(size_t)j * n + j0 + q] = h[(size_t)j * 4 + q];
  }
  std::vector<double> inv;
  if (!dense_inverse(n, A0, inv)) fail(CPM_ERR_PIVOT, "singular coarse matrix");
  pc.d_ainv.upload(inv);
  C.ainv = pc.d_ainv.p;
}

template <class T>
void upload_values(cpm_precond_s* pc, const std::vector<double>& lval, const std::vector<double>& uval) {
  const auto& subs = pc->host.subs;
  std::vector<T> lv(lval.begin(), lval.end()), uv(uval.begin(), uval.end()), dv;
  for (auto& s : subs)
    for (double x : s.dinv) dv.push_back((T)x);
  pc->d_lval.upload(reinterpret_cast<const char*>(lv.data()), lv.size() * sizeof(T));
  pc->d_uval.upload(reinterpret_cast<const char*>(uv.data()), uv.size() * sizeof(T));
  pc->d_dinv.upload(reinterpret_cast<const char*>(dv.data()), dv.size() * sizeof(T));
}

}  // namespace

cpm_status cpm_precond_create(const cpm_operator* op, const cpm_precond_opts* opts, cpm_precond** out) {
  try {
    if (!op || !opts || !out) fail(CPM_ERR_ARG, "null argument");
    *out = nullptr;
    if (opts->kind != CPM_PC_RAS && opts->kind != CPM_PC_ORAS) fail(CPM_ERR_ARG, "kind must be RAS or ORAS");
    if (opts->subsolver != CPM_SUB_ILU0 && opts->subsolver != CPM_SUB_DENSE_LU) fail(CPM_ERR_ARG, "bad subsolver");
    if (opts->precision != CPM_PREC_FP64 && opts->precision != CPM_PREC_FP32) fail(CPM_ERR_ARG, "bad precision");
    if (opts->ordering != CPM_ORDER_RCM && opts->ordering != CPM_ORDER_DISTANCE) fail(CPM_ERR_ARG, "bad ordering");
    if (opts->coarse != CPM_COARSE_NONE && opts->coarse != CPM_COARSE_ADDITIVE && opts->coarse != CPM_COARSE_FIRST)
      fail(CPM_ERR_ARG, "bad coarse option");
    if (opts->coarse != CPM_COARSE_NONE && opts->transpose) fail(CPM_ERR_ARG, "no coarse level with transpose = 1");
    if (opts->coarse != CPM_COARSE_NONE && opts->n_parts > kMaxCoarse)
      fail(CPM_ERR_ARG, "coarse level limited to 4096 subdomains");
    auto pc = std::make_unique<cpm_precond_s>();
    pc->op = op;
    pc->opts = *opts;
    build_schwarz_host(*op->band, op->c, *opts, pc->host);
    SchwarzHost& H = pc->host;
    const int np = H.nparts;
    std::vector<DevSub> subs(np);
    std::vector<int32_t> in_idx, out_idx, gL;
    std::vector<uint64_t> recL, recU;
    std::vector<uint32_t> pk;
    // the distance order's levels are wide: pack same-level rows for the packet kernel
    const bool want_packets = opts->ordering == CPM_ORDER_DISTANCE && opts->subsolver == CPM_SUB_ILU0;
    std::vector<uint16_t> lcol, ucol;
    std::vector<double> lval, uval;
    int64_t row_off = 0;
    for (int j = 0; j < np; ++j) {
      const auto& s = H.subs[j];
      subs[j].row_off = row_off;
      subs[j].lbase = (int64_t)lcol.size();
      subs[j].ubase = (int64_t)ucol.size();
      subs[j].n = s.n;
      subs[j].pk_off = (int64_t)pk.size();
      subs[j].npkL = subs[j].npkU = 0;
      subs[j].pad = 0;
      for (int q = 0; q < s.n; ++q) {
        in_idx.push_back(s.rows[s.perm[q]]);
        int32_t g = s.rows[s.operm[q]];
        out_idx.push_back(H.owner[g] == j ? (int32_t)(g | 0x80000000u) : g);
      }
      // entries re-stored in schedule order, one 64-bit record per scheduled row
      for (int lower = 1; lower >= 0; --lower) {
        const auto& sched = lower ? s.schedL : s.schedU;
        const auto& ptr = lower ? s.lptr : s.uptr;
        const auto& cs = lower ? s.lcol : s.ucol;
        const auto& vs = lower ? s.lval : s.uval;
        auto& oc = lower ? lcol : ucol;
        auto& ov = lower ? lval : uval;
        auto& rec = lower ? recL : recU;
        const int64_t base = lower ? subs[j].lbase : subs[j].ubase;
        for (int t = 0; t < s.n; ++t) {
          const int row = sched[t];
          const int64_t b = ptr[row], e = ptr[row + 1];
          if (e - b > 65535) fail(CPM_ERR_ARG, "row too long for the sweep record");
          pc->max_len = std::max<int>(pc->max_len, (int)(e - b));
          if (lower) gL.push_back(s.rows[s.perm[row]]);
          const uint64_t off = (uint64_t)((int64_t)oc.size() - base);
          if (off > 0xffffffffull) fail(CPM_ERR_ARG, "subdomain factors too large");
          rec.push_back(((uint64_t)row << 48) | ((uint64_t)(e - b) << 32) | off);
          oc.insert(oc.end(), cs.begin() + b, cs.begin() + e);
          ov.insert(ov.end(), vs.begin() + b, vs.begin() + e);
        }
      }
      if (want_packets) {
        for (int lower = 1; lower >= 0; --lower) {
          const auto& lev = lower ? s.levL : s.levU;
          const auto& sched = lower ? s.schedL : s.schedU;
          const auto& ptr = lower ? s.lptr : s.uptr;
          auto cls = [&](int t) { return packet_class(ptr[sched[t] + 1] - ptr[sched[t]]); };
          int32_t& count = lower ? subs[j].npkL : subs[j].npkU;
          int level_start = 0;   // schedule position of the first row of the current level
          for (int t = 0; t < s.n;) {
            const int k = cls(t);
            if (t > 0 && lev[t] != lev[t - 1]) level_start = t;
            int c = 1;
            while (c < kPacketRows && t + c < s.n && lev[t + c] == lev[t] && cls(t + c) == k) ++c;
            const uint32_t back = (uint32_t)std::min(t - level_start, 4095);
            pk.push_back((back << 20) | ((uint32_t)t << 4) | ((uint32_t)k << 2) | (uint32_t)(c - 1));
            ++count;
            t += c;
          }
        }
      }
      row_off += s.n;
      pc->max_rows = std::max(pc->max_rows, s.n);
      pc->max_levels = std::max(pc->max_levels, s.levels);
      pc->total_nnz += s.nnz;
    }
    pc->total_rows = row_off;
    // zero entries past the end: the row sweeps clamp their loads into the arrays,
    // the packet sweeps read up to a packet row's span past a row's first entry
    const int pad = kPacketLanes * kPacketEntries;
    lcol.insert(lcol.end(), pad, 0);
    ucol.insert(ucol.end(), pad, 0);
    lval.insert(lval.end(), pad, 0.0);
    uval.insert(uval.end(), pad, 0.0);
    pc->d_subs.upload(subs);
    pc->d_in.upload(in_idx);
    pc->d_gL.upload(gL);
    pc->d_out.upload(out_idx);
    pc->d_recL.upload(recL);
    pc->d_recU.upload(recU);
    pc->packets = want_packets && pc->max_len <= kPacketLanes * kPacketEntries;
    if (pc->packets) {
      pc->d_pk.upload(pk);
      pc->cfg.variant = kSchwarzPacket;
      pc->cfg.threads = 512;
    }
    pc->d_lcol.upload(lcol);
    pc->d_ucol.upload(ucol);
    const bool fp32 = opts->precision == CPM_PREC_FP32;
    if (fp32) upload_values<float>(pc.get(), lval, uval);
    else upload_values<double>(pc.get(), lval, uval);
    int32_t zero = 0;
    pc->d_err.upload(&zero, 1);
    // release the host factors; keep partition and row lists for export
    for (auto& s : H.subs) {
      std::vector<int64_t>().swap(s.lptr);
      std::vector<int64_t>().swap(s.uptr);
      std::vector<uint16_t>().swap(s.lcol);
      std::vector<uint16_t>().swap(s.ucol);
      std::vector<double>().swap(s.lval);
      std::vector<double>().swap(s.uval);
      std::vector<double>().swap(s.dinv);
      std::vector<int32_t>().swap(s.perm);
      std::vector<int32_t>().swap(s.operm);
      std::vector<uint16_t>().swap(s.schedL);
      std::vector<uint16_t>().swap(s.schedU);
      std::vector<int32_t>().swap(s.levL);
      std::vector<int32_t>().swap(s.levU);
    }
    DevPC& P = pc->P;
    std::memset(&P, 0, sizeof(P));
    P.nparts = np;
    P.fp32 = fp32 ? 1 : 0;
    P.subs = pc->d_subs.p;
    P.in_idx = pc->d_in.p;
    P.out_idx = pc->d_out.p;
    P.gL = pc->d_gL.p;
    P.recL = pc->d_recL.p;
    P.recU = pc->d_recU.p;
    P.pk = pc->packets ? pc->d_pk.p : nullptr;
    P.lcol = pc->d_lcol.p;
    P.ucol = pc->d_ucol.p;
    P.lval = pc->d_lval.p;
    P.uval = pc->d_uval.p;
    P.dinv = pc->d_dinv.p;
    P.error_flag = pc->d_err.p;
    P.vec_off = 0;
    pc->d_pc.upload(&P, 1);
    // largest subdomains first
    std::vector<int> order(np);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return H.subs[a].n > H.subs[b].n; });
    std::vector<WorkItem> work(np);
    for (int j = 0; j < np; ++j) work[j] = WorkItem{0, order[j]};
    pc->d_work.upload(work);
    pc->h_work = work;
    if (opts->coarse != CPM_COARSE_NONE) build_coarse(*pc);
    pc->serial = next_serial();
    *out = pc.release();
    return CPM_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed in cpm_precond_create");
    return CPM_ERR_OOM;
  }
}

cpm_status cpm_precond_get_info(const cpm_precond* pc, cpm_precond_info* info) {
  if (!pc || !info) { set_error("null argument"); return CPM_ERR_ARG; }
  std::memset(info, 0, sizeof(*info));
  info->n_parts = pc->host.nparts;
  info->total_rows = pc->total_rows;
  info->total_nnz = pc->total_nnz;
  info->max_rows = pc->max_rows;
  info->max_levels = pc->max_levels;
  info->precision = pc->opts.precision;
  info->kind = pc->opts.kind;
  return CPM_OK;
}

cpm_status cpm_precond_export_partition(const cpm_precond* pc, int32_t* owner, int64_t* ovl_ptr, int32_t* ovl_idx) {
  if (!pc) { set_error("null argument"); return CPM_ERR_ARG; }
  const auto& H = pc->host;
  if (owner) std::memcpy(owner, H.owner.data(), H.owner.size() * sizeof(int32_t));
  int64_t o = 0;
  for (int j = 0; j < H.nparts; ++j) {
    if (ovl_ptr) ovl_ptr[j] = o;
    if (ovl_idx) std::memcpy(ovl_idx + o, H.subs[j].rows.data(), H.subs[j].rows.size() * sizeof(int32_t));
    o += (int64_t)H.subs[j].rows.size();
  }
  if (ovl_ptr) ovl_ptr[H.nparts] = o;
  return CPM_OK;
}

namespace cpm {
// z = M^-1 r for one preconditioner (also used by the solver)
hipError_t precond_apply_raw(const cpm_precond_s* pc, const double* r, double* z, int nrhs, hipStream_t s) {
  auto one_level = [&](const double* rr) {
    return launch_schwarz(pc->cfg, pc->d_pc.p, pc->d_work.p, pc->host.nparts, pc->max_rows, pc->max_len, pc->P.fp32,
                          nrhs, rr, z, s);
  };
  if (pc->C.n == 0) return one_level(r);
  const DevCoarse& C = pc->C;
  const int64_t nv = C.nA * nrhs;
  pc->d_cv.alloc((size_t)C.n * 4);
  pc->d_ev.alloc((size_t)C.n * 4);
  hipError_t e;
  if ((e = coarse_restrict(C, nrhs, r, pc->d_cv.p, s)) != hipSuccess) return e;
  if ((e = coarse_solve(C, nrhs, pc->d_cv.p, pc->d_ev.p, s)) != hipSuccess) return e;
  if (C.mode == CPM_COARSE_ADDITIVE) {
    if ((e = one_level(r)) != hipSuccess) return e;
    return coarse_prolong(C, nrhs, pc->d_ev.p, z, true, s);
  }
  // coarse first: r' = r - A R0^T e, z = M1^-1 r' + R0^T e
  pc->d_tz.alloc((size_t)C.nA * 4);
  pc->d_tr.alloc((size_t)C.nA * 4);
  if ((e = coarse_prolong(C, nrhs, pc->d_ev.p, pc->d_tz.p, false, s)) != hipSuccess) return e;
  const int variant = (nrhs == 1 && pc->op->apply_variant == kApplyTwoPass && !pc->op->twopass) ? kApplyPipelined
                                                                                                : pc->op->apply_variant;
  if ((e = launch_apply(pc->op->apply_args(), nrhs, variant, pc->d_tz.p, pc->d_tr.p, s)) != hipSuccess) return e;
  if ((e = coarse_sub(nv, r, pc->d_tr.p, pc->d_tr.p, s)) != hipSuccess) return e;
  if ((e = one_level(pc->d_tr.p)) != hipSuccess) return e;
  return coarse_prolong(C, nrhs, pc->d_ev.p, z, true, s);
}
// error flag of the bounded waits (0 = fine); resets it
int precond_take_error(const cpm_precond_s* pc) {
  int32_t v = 0;
  if (hipMemcpy(&v, pc->d_err.p, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return 1;
  if (v) {
    int32_t zero = 0;
    (void)hipMemcpy(pc->d_err.p, &zero, sizeof(zero), hipMemcpyHostToDevice);
  }
  return v;
}
}  // namespace cpm

cpm_status cpm_precond_apply(const cpm_precond* pc, const double* r, double* z, int32_t nrhs, void* stream) {
  try {
    if (!pc || !r || !z) fail(CPM_ERR_ARG, "null argument");
    if (nrhs != 1 && nrhs != 2 && nrhs != 4) fail(CPM_ERR_ARG, "nrhs must be 1, 2 or 4");
    if (r == z) fail(CPM_ERR_ARG, "r and z must not alias");
    hipError_t e = precond_apply_raw(pc, r, z, nrhs, (hipStream_t)stream);
    if (e == hipErrorInvalidConfiguration)
      fail(CPM_ERR_ARG, "subdomains too large for the local-memory budget at this nrhs/precision");
    hip_check(e, "cpm_precond_apply");
    return CPM_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  }
}

void cpm_precond_destroy(cpm_precond* pc) { delete pc; }
