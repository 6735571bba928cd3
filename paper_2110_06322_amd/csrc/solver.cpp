// Restarted right-preconditioned FGMRES on the GPU for one or many systems
// (Sec. 4.1.1: GMRES with the DD preconditioners), with CGS2 orthogonalisation,
// device-side Givens rotations, one host synchronisation per restart cycle and
// a one-step-lagged convergence poll inside a cycle. GMRES-based iterative
// refinement (Carson & Higham 2017) reuses the same cycle: every restart
// recomputes r = f - A u in FP64 and solves the correction to inner_rtol with
// the FP32 preconditioner.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>

#include "krylov.h"
#include "schwarz.h"
#include "tune.h"

using namespace cpm;

namespace cpm {
hipError_t precond_apply_raw(const cpm_precond_s* pc, const double* r, double* z, int nrhs, hipStream_t s);
int precond_take_error(const cpm_precond_s* pc);
}  // namespace cpm

struct cpm_batch_s {
  int ni = 0, R = 1, ns = 0, d = 3, p = 3;
  std::vector<const cpm_operator_s*> ops;
  std::vector<const cpm_precond_s*> pcs;
  std::vector<int64_t> off;
  int64_t Ntot = 0;
  // operator apply over all instances
  std::vector<DevInst> hinst;
  DevBuf<DevInst> d_insts;
  // two-kernel apply (operators of stencil order 4 or degree p > 3): per-instance launches
  bool generic = false;
  std::vector<int64_t> gvoff;
  std::vector<GenericEPass> gep;
  DevBuf<double> gv;
  GenericPlan gen;
  DevBuf<WorkItem> d_work, d_fb;
  DevBuf<DevTile> d_wtiles;   // tiles of d_work in work order, with their instance
  DevBuf<PipeSpan> d_plan;     // spans of the persistent apply's workgroups
  int nplan = 0;
  int nwork = 0, nfb = 0, ucap = 0;
  PipeWork pipe() const { return PipeWork{d_wtiles.p, d_plan.p, nplan}; }
  int apply_variant = kApplyPipelined;
  // two-pass apply over all instances (when every operator has it)
  bool twopass = false;
  DevBuf<DevTile> d_wtilesE;
  DevBuf<PipeSpan> d_planE;
  DevBuf<WorkItem> d_swork, d_fbE;
  DevBuf<double> vscr;
  int nplanE = 0, ucapE = 0, nswork = 0, nfbE = 0;
  ApplyArgs apply_args() const {
    ApplyArgs A;
    A.gen = generic ? &gen : nullptr;
    A.d = d; A.p = p; A.insts = d_insts.p;
    A.work = d_work.p; A.nwork = nwork; A.pipe = pipe(); A.ucap = ucap;
    A.fb = d_fb.p; A.nfb = nfb;
    A.twopass = twopass;
    A.pipeE = PipeWork{d_wtilesE.p, d_planE.p, nplanE};
    A.ucapE = ucapE;
    A.swork = d_swork.p; A.nswork = nswork;
    A.fbE = d_fbE.p; A.nfbE = nfbE;
    A.vscr = vscr.p;
    return A;
  }
  SchwarzCfg pc_cfg;
  // operator algebra of the current solve: the operator is P(L) = sum_k poly_coef[k] L^k with
  // L = c_i I - A_i (poly_n = 0: A itself), the preconditioner is applied pc_power times
  std::vector<double> shift;   // c_i of every instance at creation
  DevBuf<double> d_shift;
  int poly_n = 0, pc_power = 1;
  double poly_coef[kMaxPoly] = {};
  DevBuf<double> pbuf, pctmp;
  // inner solves as the preconditioner: each application of M^-1 becomes an FGMRES solve of
  // the instances' own operators A w = v to pc_inner_rtol (at most pc_inner_max_it steps),
  // preconditioned by the batch's preconditioners; inner is a batch of the same operators
  double pc_inner_rtol = 0.0;
  int pc_inner_max_it = 0;
  std::shared_ptr<cpm_batch_s> inner;
  // coarse levels (two-level Schwarz): each instance's view with batch offsets
  std::vector<DevCoarse> coarse;
  bool any_coarse = false, any_coarse_first = false;
  bool all_coarse_first = false;   // every instance coarse-first: r - A z_c overwrites all of ctr
  DevBuf<double> cvec, evec, ctz, ctr;
  // preconditioners
  bool any_pc = false, all_pc = true, pc_packets = false;
  int pc_fp32 = 0, pc_transpose = -1, max_rows = 0, max_len = 0, npcwork = 0;
  DevBuf<DevPC> d_pcs;
  DevBuf<WorkItem> d_pcwork;
  DevBuf<int32_t> d_copy_inst;
  // reduction chunks
  std::vector<Chunk> chunks;
  DevBuf<Chunk> d_chunks;
  std::vector<int32_t> cbeg;
  DevBuf<int32_t> d_cbeg;
  int nchunks = 0;
  // workspace
  int m_alloc = 0;
  DevBuf<double> V, Z, w, r, t, f, x, part, partn, zT;
  DevBuf<double> H, g, cs, sn, y, hcol, hv, nrm2, beta, scale, tol_in, est;
  DevBuf<int32_t> act, steps, bad, budget, n_active;
  int32_t* h_nact = nullptr;   // pinned [2]
  hipEvent_t ev[2] = {nullptr, nullptr};
  int ws_gen = 0;               // bumped when the Krylov bases are reallocated
  // one restart cycle captured as a graph, replayed on a private stream
  hipStream_t gstream = nullptr;
  hipGraphExec_t gexec = nullptr;
  hipEvent_t gev[2] = {nullptr, nullptr};
  int g_m = -1, g_tr = -1, g_gen = -1;
  ~cpm_batch_s() {
    if (h_nact) (void)hipHostFree(h_nact);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    for (auto& e : gev)
      if (e) (void)hipEventDestroy(e);
    if (gstream) (void)hipStreamDestroy(gstream);
  }
};

namespace {

void build_batch(cpm_batch_s& Bt, int n, const cpm_operator_s* const* ops, const cpm_precond_s* const* pcs, int R) {
  if (n < 1) fail(CPM_ERR_ARG, "empty batch");
  if (R != 1 && R != 2 && R != 4) fail(CPM_ERR_ARG, "nrhs must be 1, 2 or 4");
  if ((int64_t)n * R > kMaxSystems) fail(CPM_ERR_ARG, "too many systems in one batch (max 1024)");
  Bt.ni = n;
  Bt.R = R;
  Bt.ns = n * R;
  Bt.d = ops[0]->I.d;
  Bt.p = ops[0]->I.p;
  Bt.off.assign(n + 1, 0);
  std::vector<WorkItem> fast, slow, pcw, ework, swork, eslow;
  Bt.twopass = true;
  int64_t vnodes = 0;
  std::vector<DevPC> hpcs(n);
  std::vector<int32_t> copy_inst(n, 0);
  for (int i = 0; i < n; ++i) {
    const cpm_operator_s* op = ops[i];
    if (!op) fail(CPM_ERR_ARG, "null operator in batch");
    if (op->I.d != Bt.d || op->I.p != Bt.p) fail(CPM_ERR_ARG, "all operators of a batch need the same d and p");
    if (i == 0) Bt.generic = op->generic;
    if (op->generic != Bt.generic)
      fail(CPM_ERR_ARG, "a batch cannot mix fused (second order, p <= 3) and two-kernel operators");
    Bt.ops.push_back(op);
    Bt.off[i + 1] = Bt.off[i] + op->band->nA;
    DevInst I = op->I;
    I.vec_off = Bt.off[i];
    I.vnode_off = vnodes;
    vnodes += op->band->nodes();
    Bt.hinst.push_back(I);
    Bt.shift.push_back(op->c);
    for (const WorkItem& wi : op->h_work) fast.push_back(WorkItem{i, wi.idx});
    for (const WorkItem& wi : op->h_fb) slow.push_back(WorkItem{i, wi.idx});
    Bt.ucap = std::max(Bt.ucap, op->ucap);
    if (!op->twopass) Bt.twopass = false;
    for (const WorkItem& wi : op->h_workE) ework.push_back(WorkItem{i, wi.idx});
    for (const WorkItem& wi : op->h_swork) swork.push_back(WorkItem{i, wi.idx});
    for (const WorkItem& wi : op->h_fbE) eslow.push_back(WorkItem{i, wi.idx});
    Bt.ucapE = std::max(Bt.ucapE, op->ucapE);
    if (i == 0) Bt.apply_variant = op->apply_variant;
    const cpm_precond_s* pc = pcs ? pcs[i] : nullptr;
    Bt.pcs.push_back(pc);
    if (pc) {
      if (pc->op != op) fail(CPM_ERR_ARG, "preconditioner built for another operator");
      if (Bt.any_pc && pc->P.fp32 != Bt.pc_fp32) fail(CPM_ERR_ARG, "mixed preconditioner precisions in one batch");
      if (Bt.pc_transpose >= 0 && pc->opts.transpose != Bt.pc_transpose)
        fail(CPM_ERR_ARG, "mixed transposed / plain preconditioners in one batch");
      if (Bt.any_pc && pc->packets != Bt.pc_packets)
        fail(CPM_ERR_ARG, "mixed row orderings (packet and row layouts) in one batch");
      if (!Bt.any_pc) Bt.pc_cfg = pc->cfg;
      Bt.pc_packets = pc->packets;
      Bt.pc_fp32 = pc->P.fp32;
      Bt.pc_transpose = pc->opts.transpose;
      Bt.any_pc = true;
      DevPC P = pc->P;
      P.vec_off = Bt.off[i];
      hpcs[i] = P;
      for (const WorkItem& wi : pc->h_work) pcw.push_back(WorkItem{i, wi.idx});
      Bt.max_rows = std::max(Bt.max_rows, pc->max_rows);
      Bt.max_len = std::max(Bt.max_len, pc->max_len);
    } else {
      Bt.all_pc = false;
      copy_inst[i] = 1;
      std::memset(&hpcs[i], 0, sizeof(DevPC));
    }
  }
  Bt.Ntot = Bt.off[n];
  Bt.d_insts.upload(Bt.hinst);
  if (Bt.generic) {
    Bt.gvoff.assign(n, 0);
    int64_t tot = 0;
    for (int i = 0; i < n; ++i) {
      Bt.gvoff[i] = tot;
      tot += ops[i]->band->nodes();
    }
    Bt.gv.alloc((size_t)tot * R);
    Bt.gen.inst = Bt.hinst.data();
    Bt.gen.voff = Bt.gvoff.data();
    Bt.gen.ninst = n;
    Bt.gen.vscr = Bt.gv.p;
    // LDS extension passes of the instances that have them (their tiles name instance 0:
    // point each at its own record of the batch)
    Bt.gep.assign(n, GenericEPass{});
    bool any = false;
    for (int i = 0; i < n; ++i) {
      if (Bt.hinst[i].vnode_off != Bt.gvoff[i]) fail(CPM_ERR_STATE, "batch node offsets disagree");
      if (!ops[i]->gen.epass) continue;
      Bt.gep[i] = ops[i]->gep;
      Bt.gep[i].dinst = Bt.d_insts.p + i;
      any = true;
    }
    Bt.gen.epass = any ? Bt.gep.data() : nullptr;
  }
  Bt.d_shift.upload(Bt.shift);
  {
    std::vector<int32_t> cost(fast.size());
    for (size_t i = 0; i < fast.size(); ++i) cost[i] = ops[fast[i].inst]->tiles[fast[i].idx].job_cnt;
    std::vector<PipeSpan> plan;
    plan_pipe(fast, cost, fast.empty() ? 0 : apply_pipe_grid(Bt.d, Bt.p, (int)fast.size(), Bt.ucap), plan);
    Bt.d_plan.upload(plan);
    Bt.nplan = (int)plan.size();
  }
  Bt.d_work.upload(fast);
  {
    std::vector<DevTile> wt;
    wt.reserve(fast.size());
    for (const WorkItem& wi : fast) {
      wt.push_back(ops[wi.inst]->tiles[wi.idx]);
      wt.back().inst = wi.inst;
    }
    Bt.d_wtiles.upload(wt);
  }
  Bt.d_fb.upload(slow);
  Bt.nwork = (int)fast.size();
  Bt.nfb = (int)slow.size();
  if (Bt.twopass && (!ework.empty() || !eslow.empty())) {
    std::vector<int32_t> cost(ework.size());
    for (size_t i = 0; i < ework.size(); ++i) cost[i] = ops[ework[i].inst]->tilesE[ework[i].idx].job_cnt;
    std::vector<PipeSpan> plan;
    plan_pipe(ework, cost, ework.empty() ? 0 : apply_pipe_grid(Bt.d, Bt.p, (int)ework.size(), Bt.ucapE, true), plan);
    Bt.d_fbE.upload(eslow);
    Bt.nfbE = (int)eslow.size();
    Bt.d_planE.upload(plan);
    Bt.nplanE = (int)plan.size();
    std::vector<DevTile> wt;
    wt.reserve(ework.size());
    for (const WorkItem& wi : ework) {
      wt.push_back(ops[wi.inst]->tilesE[wi.idx]);
      wt.back().inst = wi.inst;
      for (int q = 0; q < 8; ++q) wt.back().mA[q] = 0;
    }
    Bt.d_wtilesE.upload(wt);
    Bt.d_swork.upload(swork);
    Bt.nswork = (int)swork.size();
    Bt.vscr.alloc((size_t)vnodes * Bt.R);
  } else {
    Bt.twopass = false;
  }
  if (Bt.apply_variant == kApplyTwoPass && !Bt.twopass) Bt.apply_variant = kApplyPipelined;
  {
    int64_t coff = 0;
    int nfirst = 0;
    Bt.coarse.assign(n, DevCoarse{});
    for (int i = 0; i < n; ++i) {
      const cpm_precond_s* pc = pcs ? pcs[i] : nullptr;
      if (!pc || pc->C.n == 0) continue;
      DevCoarse C = pc->C;
      C.vec_off = Bt.off[i];
      C.coff = coff;
      coff += C.n;
      Bt.coarse[i] = C;
      Bt.any_coarse = true;
      if (C.mode == CPM_COARSE_FIRST) {
        Bt.any_coarse_first = true;
        ++nfirst;
      }
    }
    Bt.all_coarse_first = nfirst == n;
    if (Bt.any_coarse) {
      Bt.cvec.alloc((size_t)coff * R);
      Bt.evec.alloc((size_t)coff * R);
      if (Bt.any_coarse_first) {
        Bt.ctz.alloc((size_t)Bt.Ntot * R);
        Bt.ctr.alloc((size_t)Bt.Ntot * R);
      }
    }
  }
  // largest subdomains first across the whole batch
  if (Bt.any_pc) {
    std::stable_sort(pcw.begin(), pcw.end(), [&](const WorkItem& a, const WorkItem& b) {
      return pcs[a.inst]->host.subs[a.idx].n > pcs[b.inst]->host.subs[b.idx].n;
    });
    Bt.d_pcs.upload(hpcs);
    Bt.d_pcwork.upload(pcw);
    Bt.npcwork = (int)pcw.size();
  }
  Bt.d_copy_inst.upload(copy_inst);
  Bt.cbeg.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    const int64_t nA = ops[i]->band->nA;
    for (int64_t a = 0; a < nA; a += kChunkNodes)
      Bt.chunks.push_back(Chunk{i, 0, Bt.off[i] + a, std::min<int64_t>(kChunkNodes, nA - a)});
    Bt.cbeg[i + 1] = (int32_t)Bt.chunks.size();
  }
  Bt.nchunks = (int)Bt.chunks.size();
  Bt.d_chunks.upload(Bt.chunks);
  Bt.d_cbeg.upload(Bt.cbeg);
  hip_check(hipHostMalloc((void**)&Bt.h_nact, 2 * sizeof(int32_t)), "hipHostMalloc");
  for (auto& e : Bt.ev) hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
}

void ensure_workspace(cpm_batch_s& Bt, int m) {
  const size_t Ns = (size_t)Bt.Ntot * Bt.R;
  if (Bt.m_alloc < m) {
    Bt.V.alloc(Ns * (m + 1));
    Bt.Z.alloc(Ns * m);
    Bt.part.alloc((size_t)(m + 1) * Bt.nchunks * Bt.R);
    const size_t ns = Bt.ns;
    Bt.H.alloc(ns * (m + 1) * m);
    Bt.g.alloc(ns * (m + 1));
    Bt.cs.alloc(ns * m);
    Bt.sn.alloc(ns * m);
    Bt.y.alloc(ns * m);
    Bt.hcol.alloc(ns * (m + 1));
    Bt.hv.alloc(ns * (m + 1));
    Bt.m_alloc = m;
    ++Bt.ws_gen;
  }
  Bt.w.alloc(Ns);
  Bt.r.alloc(Ns);
  Bt.t.alloc(Ns);
  Bt.f.alloc(Ns);
  Bt.x.alloc(Ns);
  Bt.partn.alloc((size_t)Bt.nchunks * Bt.R);
  const size_t ns = Bt.ns;
  Bt.nrm2.alloc(ns);
  Bt.beta.alloc(ns);
  Bt.scale.alloc(ns);
  Bt.tol_in.alloc(ns);
  Bt.est.alloc(ns);
  Bt.act.alloc(ns);
  Bt.steps.alloc(ns);
  Bt.bad.alloc(ns);
  Bt.budget.alloc(ns);
  Bt.n_active.alloc(1);
}

GmresState state_of(cpm_batch_s& Bt, int m) {
  GmresState S;
  std::memset(&S, 0, sizeof(S));
  S.m = m;
  S.H = Bt.H.p; S.g = Bt.g.p; S.cs = Bt.cs.p; S.sn = Bt.sn.p; S.y = Bt.y.p;
  S.hcol = Bt.hcol.p; S.hv = Bt.hv.p; S.nrm2 = Bt.nrm2.p; S.beta = Bt.beta.p; S.scale = Bt.scale.p;
  S.tol_in = Bt.tol_in.p; S.est = Bt.est.p; S.act = Bt.act.p; S.steps = Bt.steps.p; S.bad = Bt.bad.p;
  S.budget = Bt.budget.p;
  S.n_active = Bt.n_active.p;
  return S;
}

// y = A x (or A^T x) over all instances of the batch, packed layout
void batch_apply(cpm_batch_s& Bt, const double* x, double* y, bool transpose, hipStream_t s,
                 const Gate& gate = Gate{}) {
  if (!transpose && Bt.poly_n > 0) {
    // y = a_0 x; v_0 = x; v_k = c v_{k-1} - A v_{k-1}; y += a_k v_k (v_k in buffer (k-1) mod 2)
    const size_t Ns = (size_t)Bt.Ntot * Bt.R;
    hip_check(poly_scale((int64_t)Ns, Bt.poly_coef[0], x, y, s), "polynomial apply");
    const double* v = x;
    for (int k = 1; k < Bt.poly_n; ++k) {
      double* buf = Bt.pbuf.p + (size_t)((k - 1) & 1) * Ns;
      hip_check(launch_apply(Bt.apply_args(), Bt.R, Bt.apply_variant, v, buf, s, gate), "operator apply");
      hip_check(poly_step_chunks(Bt.R, Bt.d_chunks.p, Bt.nchunks, Bt.d_shift.p, Bt.poly_coef[k], v, buf, buf, y, s),
                "polynomial apply");
      v = buf;
    }
    return;
  }
  if (!transpose) {
    hip_check(launch_apply(Bt.apply_args(), Bt.R, Bt.apply_variant, x, y, s, gate), "operator apply");
    return;
  }
  int64_t mx = 0;
  for (auto* op : Bt.ops) mx = std::max<int64_t>(mx, op->band->nodes());
  Bt.zT.alloc((size_t)mx * Bt.R);
  for (int i = 0; i < Bt.ni; ++i)
    hip_check(launch_apply_T(Bt.hinst[i], Bt.R, x, Bt.zT.p, y, s, gate, i), "transposed operator apply");
}

void batch_precond_once(cpm_batch_s& Bt, const double* v, double* z, hipStream_t s, const Gate& gate) {
  // coarse levels: coarse-first instances solve their one-level problem on r - A z_c
  const double* vin = v;
  if (Bt.any_coarse) {
    for (int i = 0; i < Bt.ni; ++i) {
      const DevCoarse& C = Bt.coarse[i];
      if (C.n == 0) continue;
      hip_check(coarse_restrict(C, Bt.R, v, Bt.cvec.p, s), "coarse restrict");
      hip_check(coarse_solve(C, Bt.R, Bt.cvec.p, Bt.evec.p, s), "coarse solve");
    }
    if (Bt.any_coarse_first) {
      // instances without a coarse-first level precondition v itself
      if (!Bt.all_coarse_first)
        hip_check(hipMemcpyAsync(Bt.ctr.p, v, (size_t)Bt.Ntot * Bt.R * sizeof(double), hipMemcpyDeviceToDevice, s),
                  "copy");
      for (int i = 0; i < Bt.ni; ++i) {
        const DevCoarse& C = Bt.coarse[i];
        if (C.n == 0 || C.mode != CPM_COARSE_FIRST) continue;
        const cpm_operator_s* op = Bt.ops[i];
        const int64_t o = Bt.off[i] * Bt.R;
        DevCoarse L = C;   // the operator's own (unpacked) view of the instance's vectors
        L.vec_off = 0;
        hip_check(coarse_prolong(L, Bt.R, Bt.evec.p, Bt.ctz.p + o, false, s), "coarse prolong");
        const int variant = (Bt.R == 1 && op->apply_variant == kApplyTwoPass && !op->twopass) ? kApplyPipelined
                                                                                              : op->apply_variant;
        hip_check(launch_apply(op->apply_args(), Bt.R, variant, Bt.ctz.p + o, Bt.ctr.p + o, s), "coarse apply");
        hip_check(coarse_sub(op->band->nA * Bt.R, v + o, Bt.ctr.p + o, Bt.ctr.p + o, s), "coarse residual");
      }
      vin = Bt.ctr.p;
    }
  }
  if (Bt.any_pc) {
    hipError_t e = launch_schwarz(Bt.pc_cfg, Bt.d_pcs.p, Bt.d_pcwork.p, Bt.npcwork, Bt.max_rows, Bt.max_len,
                                  Bt.pc_fp32, Bt.R, vin, z, s, gate);
    if (e == hipErrorInvalidConfiguration)
      fail(CPM_ERR_ARG, "subdomains too large for the local-memory budget at this nrhs/precision");
    hip_check(e, "preconditioner apply");
  }
  if (!Bt.all_pc) hip_check(vec_copy(Bt.R, v, z, Bt.d_chunks.p, Bt.nchunks, Bt.d_copy_inst.p, s), "copy");
  if (Bt.any_coarse)
    for (int i = 0; i < Bt.ni; ++i)
      if (Bt.coarse[i].n) hip_check(coarse_prolong(Bt.coarse[i], Bt.R, Bt.evec.p, z, true, s), "coarse prolong");
}

cpm_status solve_impl(cpm_batch_s& Bt, const double* const* fin, double* const* uin, const cpm_solve_opts& o,
                      cpm_solve_stats* stats, hipStream_t st);

// z = A^-1 v approximately: an FGMRES solve from zero of every instance's own operator,
// preconditioned by its (O)RAS, to the inner tolerance (host-synchronizing)
void inner_solve(cpm_batch_s& Bt, const double* v, double* z, hipStream_t s) {
  if (!Bt.inner) {
    Bt.inner = std::make_shared<cpm_batch_s>();
    build_batch(*Bt.inner, Bt.ni, Bt.ops.data(), Bt.pcs.data(), Bt.R);
  }
  cpm_solve_opts io;
  std::memset(&io, 0, sizeof io);
  io.restart = 30;
  io.rtol = Bt.pc_inner_rtol;
  io.max_it = Bt.pc_inner_max_it;
  io.mode = CPM_MODE_FP64;
  io.inner_rtol = 1e-4;
  io.stagnation_cycles = 50;
  io.pc_power = 1;
  std::vector<const double*> f(Bt.ni);
  std::vector<double*> u(Bt.ni);
  for (int i = 0; i < Bt.ni; ++i) {
    f[i] = v + Bt.off[i] * Bt.R;
    u[i] = z + Bt.off[i] * Bt.R;
  }
  hip_check(hipMemsetAsync(z, 0, (size_t)Bt.Ntot * Bt.R * sizeof(double), s), "zero");
  const cpm_status e = solve_impl(*Bt.inner, f.data(), u.data(), io, nullptr, s);
  if (e != CPM_OK && e != CPM_NOT_CONVERGED) fail(e, "inner preconditioner solve failed");
}

// z = M^-k v with k = pc_power (the intermediate results alternate between pctmp and z)
void batch_precond(cpm_batch_s& Bt, const double* v, double* z, hipStream_t s, const Gate& gate = Gate{}) {
  const int k = Bt.pc_power;
  const bool inner = Bt.pc_inner_rtol > 0.0;
  if (k <= 1) {
    if (inner) return inner_solve(Bt, v, z, s);
    return batch_precond_once(Bt, v, z, s, gate);
  }
  const double* in = v;
  for (int q = 0; q < k; ++q) {
    double* out = ((k - 1 - q) & 1) ? Bt.pctmp.p : z;
    if (inner) inner_solve(Bt, in, out, s);
    else batch_precond_once(Bt, in, out, s, gate);
    in = out;
  }
}

// One Arnoldi step j of every active system (preconditioner, operator, CGS2,
// Givens, next basis vector). The preconditioner and operator skip instances
// whose systems have all stopped (device activity flags); graph-captured
// cycles also pass the active-system count, so that steps after convergence
// are no-ops.
// pe / ae (optional): event pairs recorded around the preconditioner and the operator.
void issue_step(cpm_batch_s& Bt, const GmresState& S, int m, int j, bool tr, hipStream_t st, const Gate& gate,
                hipEvent_t* pe = nullptr, hipEvent_t* ae = nullptr) {
  const int R = Bt.R, ns = Bt.ns;
  const size_t Ns = (size_t)Bt.Ntot * R;
  double* Vj = Bt.V.p + (size_t)j * Ns;
  double* Zj = Bt.any_pc ? Bt.Z.p + (size_t)j * Ns : Vj;
  if (pe) hip_check(hipEventRecord(pe[0], st), "event");
  if (Bt.any_pc) batch_precond(Bt, Vj, Zj, st, gate);
  if (pe) hip_check(hipEventRecord(pe[1], st), "event");
  if (ae) hip_check(hipEventRecord(ae[0], st), "event");
  batch_apply(Bt, Zj, Bt.w.p, tr, st, gate);
  if (ae) hip_check(hipEventRecord(ae[1], st), "event");
  for (int pass = 0; pass < 2; ++pass) {
    hip_check(vec_dots(R, Bt.V.p, Ns, j + 1, Bt.w.p, Bt.d_chunks.p, Bt.nchunks, Bt.act.p, Bt.part.p, st), "dots");
    hip_check(vec_reduce(R, Bt.part.p, j + 1, Bt.nchunks, Bt.d_cbeg.p, ns, Bt.hv.p, m + 1, Bt.hcol.p, m + 1, st),
              "reduce");
    hip_check(vec_update(R, Bt.V.p, Ns, j + 1, Bt.w.p, Bt.d_chunks.p, Bt.nchunks, Bt.act.p, Bt.hv.p, m + 1,
                         pass == 1 ? Bt.partn.p : nullptr, st),
              "update");
  }
  hip_check(vec_reduce(R, Bt.partn.p, 1, Bt.nchunks, Bt.d_cbeg.p, ns, Bt.nrm2.p, 1, nullptr, 0, st), "reduce");
  hip_check(gmres_givens(S, j, ns, st), "givens");
  hip_check(vec_scale(R, Bt.w.p, Bt.V.p + (size_t)(j + 1) * Ns, Bt.d_chunks.p, Bt.nchunks, Bt.act.p, Bt.scale.p, st),
            "scale");
}

// end of a cycle: x += Z y, t = A x, r = f - t and |r|^2 per system into nrm2
void issue_cycle_end(cpm_batch_s& Bt, const GmresState& S, int m, bool tr, hipStream_t st) {
  const int R = Bt.R, ns = Bt.ns;
  const size_t Ns = (size_t)Bt.Ntot * R;
  const double* Zb = Bt.any_pc ? Bt.Z.p : Bt.V.p;
  hip_check(gmres_hsolve(S, ns, st), "hsolve");
  hip_check(vec_xupdate(R, Bt.x.p, Zb, Ns, Bt.d_chunks.p, Bt.nchunks, Bt.steps.p, Bt.y.p, m, st), "xupdate");
  batch_apply(Bt, Bt.x.p, Bt.t.p, tr, st);
  hip_check(vec_residual(R, Bt.f.p, Bt.t.p, Bt.r.p, Bt.d_chunks.p, Bt.nchunks, Bt.partn.p, st), "norm");
  hip_check(vec_reduce(R, Bt.partn.p, 1, Bt.nchunks, Bt.d_cbeg.p, ns, Bt.nrm2.p, 1, nullptr, 0, st), "reduce");
}

// the whole restart cycle as a graph (captured once per batch, restart length and direction)
void ensure_cycle_graph(cpm_batch_s& Bt, const GmresState& S, int m, bool tr) {
  if (Bt.gexec && Bt.g_m == m && Bt.g_tr == (int)tr && Bt.g_gen == Bt.ws_gen) return;
  if (Bt.gexec) {
    (void)hipGraphExecDestroy(Bt.gexec);
    Bt.gexec = nullptr;
  }
  if (!Bt.gstream) hip_check(hipStreamCreateWithFlags(&Bt.gstream, hipStreamNonBlocking), "graph stream");
  for (auto& e : Bt.gev)
    if (!e) hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "graph event");
  const int R = Bt.R, ns = Bt.ns;
  const size_t Ns = (size_t)Bt.Ntot * R;
  hipStream_t gs = Bt.gstream;
  hipGraph_t graph = nullptr;
  hip_check(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal), "begin capture");
  try {
    hip_check(gmres_cycle_init(S, ns, gs), "cycle init");
    hip_check(vec_scale(R, Bt.r.p, Bt.V.p, Bt.d_chunks.p, Bt.nchunks, Bt.act.p, Bt.scale.p, gs), "v0");
    for (int j = 0; j < m; ++j) issue_step(Bt, S, m, j, tr, gs, Gate{Bt.n_active.p, Bt.act.p, Bt.R});
    issue_cycle_end(Bt, S, m, tr, gs);
  } catch (...) {
    hipGraph_t dead = nullptr;
    (void)hipStreamEndCapture(gs, &dead);
    if (dead) (void)hipGraphDestroy(dead);
    throw;
  }
  hip_check(hipStreamEndCapture(gs, &graph), "end capture");
  hipError_t e = hipGraphInstantiate(&Bt.gexec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  hip_check(e, "graph instantiate");
  Bt.g_m = m;
  Bt.g_tr = (int)tr;
  Bt.g_gen = Bt.ws_gen;
  (void)Ns;
}

// |v|^2 per system (packed v) into host array
void norms2(cpm_batch_s& Bt, const double* v, const double* t, double* r, std::vector<double>& out, hipStream_t s) {
  hip_check(vec_residual(Bt.R, v, t, r, Bt.d_chunks.p, Bt.nchunks, Bt.partn.p, s), "norm");
  hip_check(vec_reduce(Bt.R, Bt.partn.p, 1, Bt.nchunks, Bt.d_cbeg.p, Bt.ns, Bt.nrm2.p, 1, nullptr, 0, s), "reduce");
  out.resize(Bt.ns);
  hip_check(hipMemcpyAsync(out.data(), Bt.nrm2.p, Bt.ns * sizeof(double), hipMemcpyDeviceToHost, s), "copy");
  hip_check(hipStreamSynchronize(s), "sync");
}

cpm_status solve_impl(cpm_batch_s& Bt, const double* const* fin, double* const* uin, const cpm_solve_opts& o,
                      cpm_solve_stats* stats, hipStream_t st) {
  const int m = o.restart;
  if (m < 1 || m > kMaxRestart) fail(CPM_ERR_ARG, "restart must be in 1..64");
  if (!(o.rtol >= 0) || !(o.atol >= 0)) fail(CPM_ERR_ARG, "tolerances must be >= 0");
  if (o.max_it < 1) fail(CPM_ERR_ARG, "max_it must be >= 1");
  if (o.mode != CPM_MODE_FP64 && o.mode != CPM_MODE_MIXED_IR) fail(CPM_ERR_ARG, "bad mode");
  if (o.mode == CPM_MODE_MIXED_IR && Bt.any_pc && !Bt.pc_fp32)
    fail(CPM_ERR_ARG, "MIXED_IR needs FP32 preconditioners");
  if (o.mode == CPM_MODE_MIXED_IR && !(o.inner_rtol > 0 && o.inner_rtol < 1)) fail(CPM_ERR_ARG, "inner_rtol in (0,1)");
  if (Bt.any_pc && (Bt.pc_transpose != 0) != (o.transpose != 0))
    fail(CPM_ERR_ARG, "preconditioner transpose flag does not match the solve");
  if (o.transpose && Bt.generic)
    fail(CPM_ERR_ARG, "transposed solves need second-order operators with p <= 3");
  for (int i = 0; i < Bt.ni; ++i)
    if (!fin[i] || !uin[i]) fail(CPM_ERR_ARG, "null vector");
  if (o.poly_n < 0 || o.poly_n > kMaxPoly) fail(CPM_ERR_ARG, "poly_n must be in 0..5");
  if (o.pc_power < 0 || o.pc_power > 4) fail(CPM_ERR_ARG, "pc_power must be in 1..4 (0 = 1)");
  if (o.poly_n > 0) {
    if (o.transpose) fail(CPM_ERR_ARG, "polynomial operators cannot be solved transposed");
    if (o.use_graph) fail(CPM_ERR_ARG, "polynomial operators cannot be combined with use_graph");
    bool nz = false;
    for (int k = 0; k < o.poly_n; ++k) {
      if (!std::isfinite(o.poly_coef[k])) fail(CPM_ERR_ARG, "non-finite polynomial coefficient");
      nz = nz || o.poly_coef[k] != 0.0;
    }
    if (!nz) fail(CPM_ERR_ARG, "all polynomial coefficients are zero");
  }
  if (o.pc_power > 1 && o.use_graph) fail(CPM_ERR_ARG, "pc_power > 1 cannot be combined with use_graph");
  if (!(o.pc_inner_rtol >= 0.0 && o.pc_inner_rtol < 1.0)) fail(CPM_ERR_ARG, "pc_inner_rtol must be in [0, 1)");
  if (o.pc_inner_rtol > 0.0) {
    if (!Bt.any_pc) fail(CPM_ERR_ARG, "inner preconditioner solves need preconditioners");
    if (o.use_graph) fail(CPM_ERR_ARG, "inner preconditioner solves cannot be combined with use_graph");
    if (o.transpose) fail(CPM_ERR_ARG, "inner preconditioner solves are not transposed");
    if (o.pc_inner_max_it < 1) fail(CPM_ERR_ARG, "pc_inner_max_it must be >= 1");
  }
  ensure_workspace(Bt, m);
  // the operator algebra holds for this solve only
  struct PolyScope {
    cpm_batch_s& B;
    ~PolyScope() { B.poly_n = 0; B.pc_power = 1; B.pc_inner_rtol = 0.0; B.pc_inner_max_it = 0; }
  } poly_scope{Bt};
  Bt.pc_inner_rtol = o.pc_inner_rtol;
  Bt.pc_inner_max_it = o.pc_inner_max_it;
  Bt.poly_n = o.poly_n;
  for (int k = 0; k < kMaxPoly; ++k) Bt.poly_coef[k] = k < o.poly_n ? o.poly_coef[k] : 0.0;
  Bt.pc_power = std::max(1, (int)o.pc_power);
  if (Bt.poly_n > 1) Bt.pbuf.alloc((size_t)Bt.Ntot * Bt.R * 2);
  if (Bt.pc_power > 1 && Bt.any_pc) Bt.pctmp.alloc((size_t)Bt.Ntot * Bt.R);
  const int R = Bt.R, ns = Bt.ns;
  const bool tr = o.transpose != 0;
  hipEvent_t e0, e1;
  hip_check(hipEventCreate(&e0), "event");
  hip_check(hipEventCreate(&e1), "event");
  hip_check(hipEventRecord(e0, st), "event");
  for (int i = 0; i < Bt.ni; ++i) {
    const size_t bytes = (size_t)(Bt.off[i + 1] - Bt.off[i]) * R * sizeof(double);
    hip_check(hipMemcpyAsync(Bt.f.p + Bt.off[i] * R, fin[i], bytes, hipMemcpyDeviceToDevice, st), "copy f");
    hip_check(hipMemcpyAsync(Bt.x.p + Bt.off[i] * R, uin[i], bytes, hipMemcpyDeviceToDevice, st), "copy u");
  }
  std::vector<double> fn2, b2;
  norms2(Bt, Bt.f.p, nullptr, nullptr, fn2, st);
  batch_apply(Bt, Bt.x.p, Bt.t.p, tr, st);
  norms2(Bt, Bt.f.p, Bt.t.p, Bt.r.p, b2, st);
  std::vector<double> fn(ns), beta(ns), tol(ns), best(ns);
  std::vector<int> done(ns, 0), its(ns, 0), cycles(ns, 0), stall(ns, 0), stat(ns, CPM_OK);
  std::vector<int32_t> zero_sys(ns, 0);
  bool any_zero = false;
  for (int s = 0; s < ns; ++s) {
    fn[s] = std::sqrt(fn2[s]);
    beta[s] = std::sqrt(b2[s]);
    tol[s] = std::max(o.rtol * fn[s], o.atol);
    best[s] = beta[s];
    if (!std::isfinite(beta[s]) || !std::isfinite(fn[s])) { done[s] = 1; stat[s] = CPM_NOT_CONVERGED; }
    else if (fn[s] == 0.0) { done[s] = 1; zero_sys[s] = 1; any_zero = true; beta[s] = 0; }
    else if (beta[s] <= tol[s]) done[s] = 1;
  }
  if (any_zero) {  // f = 0: the solution is 0
    std::vector<double> zs(ns, 0.0);
    hip_check(hipMemcpy(Bt.scale.p, zs.data(), ns * sizeof(double), hipMemcpyHostToDevice), "upload");
    hip_check(hipMemcpy(Bt.act.p, zero_sys.data(), ns * sizeof(int32_t), hipMemcpyHostToDevice), "upload");
    hip_check(vec_scale(R, Bt.x.p, Bt.x.p, Bt.d_chunks.p, Bt.nchunks, Bt.act.p, Bt.scale.p, st), "zero");
  }
  GmresState S = state_of(Bt, m);
  const bool graph = o.use_graph != 0;
  if (graph) {
    if (o.profile) fail(CPM_ERR_ARG, "profile cannot be combined with use_graph");
    if (Bt.any_pc) batch_precond(Bt, Bt.r.p, Bt.w.p, st);   // kernel attributes set outside the capture
    hip_check(hipStreamSynchronize(st), "sync");
    ensure_cycle_graph(Bt, S, m, tr);
  }
  double ms_pc = 0, ms_ap = 0;
  int n_pc = 0, n_ap = 2, n_pc_t = 0, n_ap_t = 0;
  std::vector<hipEvent_t> pev, aev;
  if (o.profile) {
    pev.resize(2 * m);
    aev.resize(2 * m);
    for (auto& e : pev) hip_check(hipEventCreate(&e), "event");
    for (auto& e : aev) hip_check(hipEventCreate(&e), "event");
  }
  std::vector<int32_t> act(ns), steps(ns), bad(ns), budget(ns);
  std::vector<double> tin(ns);
  for (;;) {
    int nact = 0;
    for (int s = 0; s < ns; ++s) {
      act[s] = (!done[s] && its[s] < o.max_it) ? 1 : 0;
      nact += act[s];
      double t = tol[s];
      if (o.mode == CPM_MODE_MIXED_IR) t = std::max(tol[s], o.inner_rtol * beta[s]);
      tin[s] = t;
      budget[s] = std::max(0, o.max_it - its[s]);
    }
    if (nact == 0) break;
    hip_check(hipMemcpyAsync(Bt.budget.p, budget.data(), ns * sizeof(int32_t), hipMemcpyHostToDevice, st), "upload");
    hip_check(hipMemcpyAsync(Bt.act.p, act.data(), ns * sizeof(int32_t), hipMemcpyHostToDevice, st), "upload");
    hip_check(hipMemcpyAsync(Bt.tol_in.p, tin.data(), ns * sizeof(double), hipMemcpyHostToDevice, st), "upload");
    hip_check(hipMemcpyAsync(Bt.beta.p, beta.data(), ns * sizeof(double), hipMemcpyHostToDevice, st), "upload");
    hip_check(hipMemsetAsync(Bt.bad.p, 0, ns * sizeof(int32_t), st), "memset");
    int jdone = 0;
    if (graph) {
      // the gate of the captured steps starts at the number of active systems
      Bt.h_nact[0] = nact;
      hip_check(hipMemcpyAsync(Bt.n_active.p, &Bt.h_nact[0], sizeof(int32_t), hipMemcpyHostToDevice, st), "upload");
      hip_check(hipEventRecord(Bt.gev[0], st), "event");
      hip_check(hipStreamWaitEvent(Bt.gstream, Bt.gev[0], 0), "wait");
      hip_check(hipGraphLaunch(Bt.gexec, Bt.gstream), "graph launch");
      hip_check(hipEventRecord(Bt.gev[1], Bt.gstream), "event");
      hip_check(hipStreamWaitEvent(st, Bt.gev[1], 0), "wait");
      jdone = m;
      n_pc += Bt.any_pc ? m : 0;
      n_ap += m + 1;
    } else {
      hip_check(gmres_cycle_init(S, ns, st), "cycle init");
      hip_check(vec_scale(R, Bt.r.p, Bt.V.p, Bt.d_chunks.p, Bt.nchunks, Bt.act.p, Bt.scale.p, st), "v0");
      for (int j = 0; j < m; ++j) {
        issue_step(Bt, S, m, j, tr, st, Gate{nullptr, Bt.act.p, Bt.R}, o.profile ? &pev[2 * j] : nullptr,
                   o.profile ? &aev[2 * j] : nullptr);
        if (Bt.any_pc) ++n_pc;
        ++n_ap;
        hip_check(hipMemcpyAsync(&Bt.h_nact[j & 1], Bt.n_active.p, sizeof(int32_t), hipMemcpyDeviceToHost, st),
                  "poll");
        hip_check(hipEventRecord(Bt.ev[j & 1], st), "event");
        jdone = j + 1;
        if (j >= 1) {
          hip_check(hipEventSynchronize(Bt.ev[(j - 1) & 1]), "poll");
          if (Bt.h_nact[(j - 1) & 1] == 0) break;
        }
      }
      issue_cycle_end(Bt, S, m, tr, st);
      ++n_ap;
    }
    b2.resize(ns);
    hip_check(hipMemcpyAsync(b2.data(), Bt.nrm2.p, ns * sizeof(double), hipMemcpyDeviceToHost, st), "copy");
    hip_check(hipStreamSynchronize(st), "sync");
    hip_check(hipMemcpy(steps.data(), Bt.steps.p, ns * sizeof(int32_t), hipMemcpyDeviceToHost), "steps");
    hip_check(hipMemcpy(bad.data(), Bt.bad.p, ns * sizeof(int32_t), hipMemcpyDeviceToHost), "bad");
    if (o.profile) {
      for (int j = 0; j < jdone; ++j) {
        float a = 0, b = 0;
        if (Bt.any_pc && hipEventElapsedTime(&a, pev[2 * j], pev[2 * j + 1]) == hipSuccess) { ms_pc += a; ++n_pc_t; }
        if (hipEventElapsedTime(&b, aev[2 * j], aev[2 * j + 1]) == hipSuccess) { ms_ap += b; ++n_ap_t; }
      }
    }
    for (int s = 0; s < ns; ++s) {
      if (!act[s]) continue;
      its[s] += steps[s];
      cycles[s]++;
      beta[s] = std::sqrt(b2[s]);
      if (bad[s] || !std::isfinite(beta[s])) { done[s] = 1; stat[s] = CPM_NOT_CONVERGED; continue; }
      if (beta[s] <= tol[s]) { done[s] = 1; continue; }
      if (beta[s] < 0.99 * best[s]) { best[s] = beta[s]; stall[s] = 0; }
      else if (++stall[s] >= std::max(1, o.stagnation_cycles)) { done[s] = 1; stat[s] = CPM_NOT_CONVERGED; }
      if (!done[s] && its[s] >= o.max_it) { done[s] = 1; stat[s] = CPM_NOT_CONVERGED; }
    }
  }
  for (int i = 0; i < Bt.ni; ++i) {
    const size_t bytes = (size_t)(Bt.off[i + 1] - Bt.off[i]) * R * sizeof(double);
    hip_check(hipMemcpyAsync(uin[i], Bt.x.p + Bt.off[i] * R, bytes, hipMemcpyDeviceToDevice, st), "copy u");
  }
  hip_check(hipEventRecord(e1, st), "event");
  hip_check(hipEventSynchronize(e1), "sync");
  float ms = 0;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (auto& e : pev) (void)hipEventDestroy(e);
  for (auto& e : aev) (void)hipEventDestroy(e);
  bool pc_err = false;
  for (auto* pc : Bt.pcs)
    if (pc && precond_take_error(pc)) pc_err = true;
  if (pc_err) fail(CPM_ERR_DEVICE, "preconditioner wait limit expired (dependency schedule broken)");
  cpm_status ret = CPM_OK;
  for (int s = 0; s < ns; ++s) {
    if (!done[s] || stat[s] != CPM_OK) { stat[s] = CPM_NOT_CONVERGED; ret = CPM_NOT_CONVERGED; }
    if (stats) {
      cpm_solve_stats& q = stats[s];
      std::memset(&q, 0, sizeof(q));
      q.iterations = its[s];
      q.restarts = cycles[s];
      q.converged = stat[s] == CPM_OK ? 1 : 0;
      q.status = stat[s];
      q.relres = fn[s] > 0 ? beta[s] / fn[s] : 0.0;
      q.ms_total = ms;
      q.ms_precond = ms_pc;
      q.ms_apply = ms_ap;
      q.n_precond = o.profile ? n_pc_t : n_pc;
      q.n_apply = o.profile ? n_ap_t : n_ap;
    }
  }
  if (ret != CPM_OK) set_error("solver stopped before reaching the tolerance");
  return ret;
}

std::atomic<int64_t> g_serial{1};

}  // namespace

namespace cpm {
int64_t next_serial() { return g_serial.fetch_add(1); }
}  // namespace cpm

cpm_status cpm_solve_opts_default(cpm_solve_opts* o) {
  if (!o) { set_error("null argument"); return CPM_ERR_ARG; }
  std::memset(o, 0, sizeof(*o));
  o->restart = 30;
  o->rtol = 1e-10;
  o->atol = 0.0;
  o->max_it = 10000;
  o->mode = CPM_MODE_FP64;
  o->inner_rtol = 1e-4;
  o->stagnation_cycles = 50;
  o->poly_n = 0;
  o->pc_power = 1;
  o->pc_inner_rtol = 0.0;
  o->pc_inner_max_it = 30;
  return CPM_OK;
}

cpm_status cpm_solve(const cpm_operator* op, const cpm_precond* pc, const double* f, double* u, int32_t nrhs,
                     const cpm_solve_opts* opts, cpm_solve_stats* stats, void* stream) {
  try {
    if (!op || !f || !u || !opts) fail(CPM_ERR_ARG, "null argument");
    if (f == u) fail(CPM_ERR_ARG, "f and u must not alias");
    auto& cache = op->solve_cache;
    const int64_t key = pc ? pc->serial : 0;
    if (!cache || cache->R != nrhs || op->solve_cache_key != key) {
      cache.reset();
      auto Bt = std::make_shared<cpm_batch_s>();
      const cpm_operator_s* o1 = op;
      const cpm_precond_s* p1 = pc;
      build_batch(*Bt, 1, &o1, &p1, nrhs);
      cache = Bt;
      op->solve_cache_key = key;
    }
    const double* fa[1] = {f};
    double* ua[1] = {u};
    std::vector<cpm_solve_stats> st(nrhs);
    cpm_status r = solve_impl(*cache, fa, ua, *opts, st.data(), (hipStream_t)stream);
    if (stats) {
      // one stats record per call: the worst right-hand side
      int w = 0;
      for (int q = 1; q < nrhs; ++q)
        if (st[q].relres > st[w].relres || !st[q].converged) w = q;
      *stats = st[w];
      for (int q = 0; q < nrhs; ++q) stats->iterations = std::max(stats->iterations, st[q].iterations);
    }
    return r;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed in cpm_solve");
    return CPM_ERR_OOM;
  }
}

cpm_status cpm_batch_create(int32_t n, const cpm_operator* const* ops, const cpm_precond* const* pcs,
                            const int32_t* nrhs, cpm_batch** out) {
  try {
    if (!ops || !out || n < 1) fail(CPM_ERR_ARG, "bad argument");
    *out = nullptr;
    int R = nrhs ? nrhs[0] : 1;
    for (int i = 0; i < n; ++i)
      if (nrhs && nrhs[i] != R) fail(CPM_ERR_ARG, "all instances of a batch need the same nrhs");
    auto Bt = std::make_unique<cpm_batch_s>();
    build_batch(*Bt, n, ops, pcs, R);
    *out = Bt.release();
    return CPM_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed in cpm_batch_create");
    return CPM_ERR_OOM;
  }
}

cpm_status cpm_batch_autotune(cpm_batch* b, const char* cache_path, int32_t force, void* stream,
                              cpm_tune_result* out) {
  try {
    if (!b || !out) fail(CPM_ERR_ARG, "null argument");
    std::memset(out, 0, sizeof(*out));
    cpm_batch_s& Bt = *b;
    hipStream_t s = (hipStream_t)stream;
    const int reps = 5;
    ensure_workspace(Bt, 1);
    const size_t Ns = (size_t)Bt.Ntot * Bt.R;
    hip_check(hipMemsetD32Async((hipDeviceptr_t)Bt.r.p, 0x3ff00000, Ns * 2, s), "tune fill");
    tune::Cache cache = tune::read_cache(cache_path);
    bool dirty = false, all_cached = true;
    const std::string dev = tune::device_tag();
    {
      char key[200];
      std::snprintf(key, sizeof key, "batch-apply|%s|d%dp%dr%d|inst2^%d|nodes2^%d", dev.c_str(), Bt.d, Bt.p, Bt.R,
                    tune::log2i(Bt.ni), tune::log2i((double)Bt.Ntot));
      auto it = cache.find(key);
      if (!force && it != cache.end() && it->second.size() == 1 &&
          (it->second[0] == kApplyPipelined || it->second[0] == kApplyPerTile ||
           (it->second[0] == kApplyTwoPass && Bt.twopass && Bt.R == 1))) {
        Bt.apply_variant = it->second[0];
      } else {
        all_cached = false;
        double best = 1e30;
        int bestv = kApplyPipelined;
        for (int v : {kApplyPipelined, kApplyPerTile, kApplyTwoPass}) {
          if ((v == kApplyPipelined || v == kApplyTwoPass) && Bt.R != 1) continue;
          if (v == kApplyTwoPass && !Bt.twopass) continue;
          Bt.apply_variant = v;
          const double ms = tune::time_ms(
              [&] { return launch_apply(Bt.apply_args(), Bt.R, v, Bt.r.p, Bt.w.p, s); }, reps, s);
          if (ms < best) { best = ms; bestv = v; }
        }
        Bt.apply_variant = bestv;
        cache[key] = {bestv};
        dirty = true;
      }
      out->apply_variant = Bt.apply_variant;
      out->apply_ms = tune::time_ms(
          [&] { return launch_apply(Bt.apply_args(), Bt.R, Bt.apply_variant, Bt.r.p, Bt.w.p, s); }, reps, s);
    }
    if (Bt.any_pc) {
      int max_levels = 0;
      for (auto* pc : Bt.pcs)
        if (pc) max_levels = std::max(max_levels, pc->max_levels);
      char key[220];
      std::snprintf(key, sizeof key, "batch-schwarz|%s|%s%s|r%d|rows2^%d|levels2^%d|parts2^%d", dev.c_str(),
                    Bt.pc_fp32 ? "fp32" : "fp64", Bt.pc_packets ? "|packets" : "", Bt.R, tune::log2i(Bt.max_rows), tune::log2i(max_levels),
                    tune::log2i(Bt.npcwork));
      auto it = cache.find(key);
      auto run = [&] {
        return launch_schwarz(Bt.pc_cfg, Bt.d_pcs.p, Bt.d_pcwork.p, Bt.npcwork, Bt.max_rows, Bt.max_len, Bt.pc_fp32,
                              Bt.R, Bt.r.p, Bt.w.p, s);
      };
      if (!force && it != cache.end() && tune::valid_schwarz(it->second, Bt.pc_packets, Bt.pc_fp32 != 0, Bt.R)) {
        Bt.pc_cfg.variant = it->second[0];
        Bt.pc_cfg.threads = it->second[1];
        Bt.pc_cfg.sleep = it->second[2];
      } else {
        all_cached = false;
        double best = 1e30;
        SchwarzCfg bestc = Bt.pc_cfg;
        for (const SchwarzCfg& c : tune::schwarz_candidates(Bt.pc_packets, Bt.pc_fp32 != 0, Bt.R)) {
          Bt.pc_cfg = c;
          if (!tune::launchable(run)) continue;
          const double ms = tune::time_ms(run, reps, s);
          if (ms < best) { best = ms; bestc = c; }
        }
        if (best >= 1e30) {
          Bt.pc_cfg = bestc;
          fail(CPM_ERR_ARG, "subdomains too large for the local-memory budget at this nrhs/precision");
        }
        Bt.pc_cfg = bestc;
        cache[key] = {bestc.variant, bestc.threads, bestc.sleep};
        dirty = true;
      }
      out->schwarz_variant = Bt.pc_cfg.variant;
      out->schwarz_threads = Bt.pc_cfg.threads;
      out->schwarz_sleep = Bt.pc_cfg.sleep;
      out->precond_ms = tune::time_ms(run, reps, s);
      bool pc_err = false;
      for (auto* pc : Bt.pcs)
        if (pc && precond_take_error(pc)) pc_err = true;
      if (pc_err) fail(CPM_ERR_DEVICE, "a subdomain solve timed out while tuning");
    }
    hip_check(hipStreamSynchronize(s), "tune");
    Bt.g_gen = -1;   // a captured cycle holds the old kernel choices
    out->from_cache = all_cached ? 1 : 0;
    if (dirty) tune::write_cache(cache_path, cache);
    return CPM_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed in cpm_batch_autotune");
    return CPM_ERR_OOM;
  }
}

cpm_status cpm_batch_solve(cpm_batch* b, const double* const* f, double* const* u, const cpm_solve_opts* opts,
                           cpm_solve_stats* stats, void* stream) {
  try {
    if (!b || !f || !u || !opts) fail(CPM_ERR_ARG, "null argument");
    return solve_impl(*b, f, u, *opts, stats, (hipStream_t)stream);
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed in cpm_batch_solve");
    return CPM_ERR_OOM;
  }
}

cpm_status cpm_batch_apply(cpm_batch* b, const double* const* x, double* const* y, void* stream) {
  try {
    if (!b || !x || !y) fail(CPM_ERR_ARG, "null argument");
    hipStream_t st = (hipStream_t)stream;
    ensure_workspace(*b, 1);
    for (int i = 0; i < b->ni; ++i) {
      if (!x[i] || !y[i]) fail(CPM_ERR_ARG, "null vector");
      const size_t bytes = (size_t)(b->off[i + 1] - b->off[i]) * b->R * sizeof(double);
      hip_check(hipMemcpyAsync(b->x.p + b->off[i] * b->R, x[i], bytes, hipMemcpyDeviceToDevice, st), "copy");
    }
    batch_apply(*b, b->x.p, b->t.p, false, st);
    for (int i = 0; i < b->ni; ++i) {
      const size_t bytes = (size_t)(b->off[i + 1] - b->off[i]) * b->R * sizeof(double);
      hip_check(hipMemcpyAsync(y[i], b->t.p + b->off[i] * b->R, bytes, hipMemcpyDeviceToDevice, st), "copy");
    }
    return CPM_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  }
}

void cpm_batch_destroy(cpm_batch* b) { delete b; }
