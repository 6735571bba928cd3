// Additive Runge-Kutta IMEX time stepping of surface reaction-diffusion
// systems (Sec. 1, eq. rdsys; Sec. 4.1.3 eq. heat; Sec. 4.1.5 eq. grayscott,
// whose default integrator is a third-order additive Runge-Kutta IMEX
// method). For w_t = F_E(t, w) + mu Lap_S w with the diffusion implicit:
//   W_1 = w^n
//   (I - dt gamma mu Lap) W_i = w^n + dt sum_{j<i} (aE_ij KE_j + aI_ij KI_j)
//   KE_j = F_E(t + c_j dt, W_j),  KI_j = mu Lap_S^h W_j
//   w^{n+1} = w^n + dt sum_j (bE_j KE_j + bI_j KI_j).
// With A(c) = c I - Lap_S^h (eq. lapBel) each stage solve is A(c_w) W_i =
// rhs / (dt gamma mu_w), c_w = 1/(dt gamma mu_w), and Lap_S^h x = c_w x - A x.
// The species' stage solves run as one batch (shared launches).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "common.h"

#pragma clang fp contract(off)

namespace cpm {

constexpr int kImexMaxTerms = 8;
constexpr int kImexMaxStages = 4;

struct CombineTerms {
  const double* v[kImexMaxTerms];
  double a[kImexMaxTerms];
  int n;
};

// out = scale * (w0 + sum_k a_k v_k), terms added in order (out may alias w0)
__global__ void k_imex_combine(int64_t n, const double* w0, CombineTerms T, double scale, double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = w0[i];
  for (int k = 0; k < T.n; ++k) acc += T.a[k] * T.v[k][i];
  out[i] = scale * acc;
}

// out = mu (c x - (A x)) = mu Lap_S^h x
__global__ void k_imex_lap(int64_t n, double c, double mu, const double* __restrict__ x,
                           const double* __restrict__ ax, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = mu * (c * x[i] - ax[i]);
}

// Gray-Scott reaction (eq. grayscott): eu = -u v^2 + F (1 - u), ev = u v^2 - (F + k) v
__global__ void k_imex_gray_scott(int64_t n, double F, double k, const double* __restrict__ u,
                                  const double* __restrict__ v, double* __restrict__ eu, double* __restrict__ ev) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = u[i], b = v[i];
  const double abb = a * b * b;
  eu[i] = -abb + F * (1.0 - a);
  ev[i] = abb - (F + k) * b;
}

// FitzHugh-Nagumo reaction (eq. fitznag): eu = (a - u)(u - 1) u - v, ev = eps (beta u - v)
__global__ void k_imex_fhn(int64_t n, double a, double eps, double beta, const double* __restrict__ u,
                           const double* __restrict__ v, double* __restrict__ eu, double* __restrict__ ev) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = u[i], y = v[i];
  eu[i] = (a - x) * (x - 1.0) * x - y;
  ev[i] = eps * (beta * x - y);
}

// Schnackenberg reaction (eq. schnack): eu = d1 - u + u^2 v + lam v, ev = d2 - u^2 v - lam v
__global__ void k_imex_schnack(int64_t n, double d1, double d2, double lam, const double* __restrict__ u,
                               const double* __restrict__ v, double* __restrict__ eu, double* __restrict__ ev) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = u[i], y = v[i];
  const double xxy = x * x * y;
  eu[i] = d1 - x + xxy + lam * y;
  ev[i] = d2 - xxy - lam * y;
}

// forced heat equation (eq. heat): e = cos(t) g1 + sin(t) g2
__global__ void k_imex_forcing(int64_t n, double ct, double st, const double* __restrict__ g1,
                               const double* __restrict__ g2, double* __restrict__ e) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  e[i] = ct * g1[i] + st * g2[i];
}

static dim3 grid_for(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

// Butcher tableaux of the IMEX schemes (exact rationals of the publications,
// rounded to double): ARK3(2)4L[2]SA of Kennedy & Carpenter (Appl. Numer.
// Math. 44, 2003) and IMEX Euler.
struct Tableau {
  int s;
  double c[kImexMaxStages], AE[kImexMaxStages][kImexMaxStages], AI[kImexMaxStages][kImexMaxStages];
  double bE[kImexMaxStages], bI[kImexMaxStages];
};

static Tableau make_tableau(int scheme) {
  Tableau T;
  std::memset(&T, 0, sizeof T);
  if (scheme == CPM_IMEX_EULER) {
    T.s = 2;
    T.c[1] = 1.0;
    T.AE[1][0] = 1.0;
    T.AI[1][1] = 1.0;
    T.bE[0] = 1.0;
    T.bI[1] = 1.0;
    return T;
  }
  const double g = 1767732205903.0 / 4055673282236.0;
  T.s = 4;
  T.c[1] = 1767732205903.0 / 2027836641118.0;
  T.c[2] = 3.0 / 5.0;
  T.c[3] = 1.0;
  T.AI[1][0] = g;
  T.AI[1][1] = g;
  T.AI[2][0] = 2746238789719.0 / 10658868560708.0;
  T.AI[2][1] = -640167445237.0 / 6845629431997.0;
  T.AI[2][2] = g;
  const double b[4] = {1471266399579.0 / 7840856788654.0, -4482444167858.0 / 7529755066697.0,
                       11266239266428.0 / 11593286722821.0, g};
  for (int j = 0; j < 4; ++j) {
    T.AI[3][j] = b[j];
    T.bE[j] = b[j];
    T.bI[j] = b[j];
  }
  T.AE[1][0] = 1767732205903.0 / 2027836641118.0;
  T.AE[2][0] = 5535828885825.0 / 10492691773637.0;
  T.AE[2][1] = 788022342437.0 / 10882634858940.0;
  T.AE[3][0] = 6485989280629.0 / 16251701735622.0;
  T.AE[3][1] = -4246266847089.0 / 9704473918619.0;
  T.AE[3][2] = 10755448449292.0 / 10357097424841.0;
  return T;
}

}  // namespace cpm

using namespace cpm;

struct cpm_imex_s {
  cpm_imex_opts o{};
  Tableau T{};
  int ns = 1;
  int64_t n = 0;
  const cpm_operator* ops[2] = {nullptr, nullptr};
  double shift[2] = {0, 0};
  cpm_batch* batch = nullptr;
  DevBuf<double> KE, KI, rhs, W, ax, g;   // KE/KI: [stage][species][n]; rhs/W: [species][n]; g: forcing [2][n]
  ~cpm_imex_s() {
    if (batch) cpm_batch_destroy(batch);
  }
  double* ke(int i, int sp) { return KE.p + ((size_t)i * ns + sp) * n; }
  double* ki(int i, int sp) { return KI.p + ((size_t)i * ns + sp) * n; }
};

namespace {

double imex_gamma(const Tableau& T) { return T.AI[T.s - 1][T.s - 1]; }

void explicit_terms(cpm_imex_s& M, double t, const double* const* w, int stage, hipStream_t s) {
  if (M.o.kind == CPM_RD_GRAY_SCOTT) {
    hipLaunchKernelGGL(k_imex_gray_scott, grid_for(M.n), dim3(256), 0, s, M.n, M.o.F, M.o.k, w[0], w[1],
                       M.ke(stage, 0), M.ke(stage, 1));
  } else if (M.o.kind == CPM_RD_FITZHUGH_NAGUMO) {
    hipLaunchKernelGGL(k_imex_fhn, grid_for(M.n), dim3(256), 0, s, M.n, M.o.rd[0], M.o.rd[1], M.o.rd[2], w[0], w[1],
                       M.ke(stage, 0), M.ke(stage, 1));
  } else if (M.o.kind == CPM_RD_SCHNACKENBERG) {
    hipLaunchKernelGGL(k_imex_schnack, grid_for(M.n), dim3(256), 0, s, M.n, M.o.rd[0], M.o.rd[1], M.o.rd[2], w[0],
                       w[1], M.ke(stage, 0), M.ke(stage, 1));
  } else {
    hipLaunchKernelGGL(k_imex_forcing, grid_for(M.n), dim3(256), 0, s, M.n, std::cos(t), std::sin(t), M.g.p,
                       M.g.p + M.n, M.ke(stage, 0));
  }
  hip_check(hipGetLastError(), "imex explicit terms");
}

void implicit_terms(cpm_imex_s& M, const double* const* w, int stage, hipStream_t s) {
  for (int sp = 0; sp < M.ns; ++sp) {
    cpm_status st = cpm_apply(M.ops[sp], w[sp], M.ax.p, 1, s);
    if (st != CPM_OK) fail(st, std::string("imex: ") + cpm_last_error());
    hipLaunchKernelGGL(k_imex_lap, grid_for(M.n), dim3(256), 0, s, M.n, M.shift[sp], M.o.mu[sp], w[sp], M.ax.p,
                       M.ki(stage, sp));
    hip_check(hipGetLastError(), "imex implicit terms");
  }
}

// out = scale (w0 + dt sum_{j<upto} (aE_j KE_j + aI_j KI_j)) for species sp
void combine(cpm_imex_s& M, int sp, const double* w0, const double* aE, const double* aI, int upto, double scale,
             double* out, hipStream_t s) {
  CombineTerms C;
  std::memset(&C, 0, sizeof C);
  const double dt = M.o.dt;
  for (int j = 0; j < upto; ++j) {
    if (aE[j] != 0.0) { C.v[C.n] = M.ke(j, sp); C.a[C.n] = dt * aE[j]; ++C.n; }
    if (aI[j] != 0.0) { C.v[C.n] = M.ki(j, sp); C.a[C.n] = dt * aI[j]; ++C.n; }
  }
  hipLaunchKernelGGL(k_imex_combine, grid_for(M.n), dim3(256), 0, s, M.n, w0, C, scale, out);
  hip_check(hipGetLastError(), "imex combine");
}

}  // namespace

cpm_status cpm_imex_opts_default(cpm_imex_opts* o) {
  if (!o) {
    set_error("null argument");
    return CPM_ERR_ARG;
  }
  std::memset(o, 0, sizeof(*o));
  o->scheme = CPM_IMEX_ARK3;
  o->kind = CPM_RD_GRAY_SCOTT;
  o->nspecies = 2;
  o->dt = 1.0;
  o->mu[0] = 2e-5;
  o->mu[1] = 1e-5;
  o->F = 0.04;
  o->k = 0.06;
  o->tune = 0;
  return CPM_OK;
}

double cpm_imex_shift(const cpm_imex_opts* o, int32_t species) {
  if (!o || species < 0 || species > 1 || !(o->dt > 0) || !(o->mu[species] > 0)) return 0.0;
  const Tableau T = make_tableau(o->scheme == CPM_IMEX_EULER ? CPM_IMEX_EULER : CPM_IMEX_ARK3);
  return 1.0 / (o->dt * imex_gamma(T) * o->mu[species]);
}

cpm_status cpm_imex_create(const cpm_operator* const* ops, const cpm_precond* const* pcs, const cpm_imex_opts* opts,
                           const double* const* forcing, cpm_imex** out) {
  try {
    if (!ops || !opts || !out) fail(CPM_ERR_ARG, "null argument");
    *out = nullptr;
    const cpm_imex_opts& o = *opts;
    if (o.scheme != CPM_IMEX_EULER && o.scheme != CPM_IMEX_ARK3) fail(CPM_ERR_ARG, "unknown IMEX scheme");
    if (o.kind < CPM_RD_GRAY_SCOTT || o.kind > CPM_RD_SCHNACKENBERG) fail(CPM_ERR_ARG, "unknown reaction-diffusion kind");
    const int ns = o.kind == CPM_RD_HEAT ? 1 : 2;
    if (o.nspecies != ns) fail(CPM_ERR_ARG, "nspecies must be 1 for the heat equation and 2 otherwise");
    for (int q = 0; q < 3; ++q)
      if (!std::isfinite(o.rd[q])) fail(CPM_ERR_ARG, "non-finite reaction parameter");
    if (!(o.dt > 0) || !std::isfinite(o.dt)) fail(CPM_ERR_ARG, "dt must be positive");
    auto M = std::make_unique<cpm_imex_s>();
    M->o = o;
    M->T = make_tableau(o.scheme);
    M->ns = ns;
    for (int sp = 0; sp < ns; ++sp) {
      if (!(o.mu[sp] > 0) || !std::isfinite(o.mu[sp])) fail(CPM_ERR_ARG, "diffusion coefficients must be positive");
      if (!ops[sp]) fail(CPM_ERR_ARG, "null operator");
      M->ops[sp] = ops[sp];
      M->shift[sp] = cpm_imex_shift(&o, sp);
      const double c = cpm_operator_get_shift(ops[sp]);
      if (!(std::fabs(c - M->shift[sp]) <= 1e-12 * M->shift[sp]))
        fail(CPM_ERR_ARG, "operator " + std::to_string(sp) + " has shift " + std::to_string(c) +
                              "; the scheme's stage solves need 1/(dt gamma mu) = " + std::to_string(M->shift[sp]));
      M->shift[sp] = c;
      if (sp > 0 && cpm_operator_n_active(ops[sp]) != cpm_operator_n_active(ops[0]))
        fail(CPM_ERR_ARG, "the species' operators must share one band");
    }
    M->n = cpm_operator_n_active(ops[0]);
    if (o.kind == CPM_RD_HEAT) {
      if (!forcing || !forcing[0] || !forcing[1]) fail(CPM_ERR_ARG, "the heat equation needs two forcing fields");
      M->g.alloc((size_t)2 * M->n);
      for (int q = 0; q < 2; ++q)
        hip_check(hipMemcpy(M->g.p + q * M->n, forcing[q], (size_t)M->n * sizeof(double), hipMemcpyDeviceToDevice),
                  "copy forcing");
    }
    const int32_t nr[2] = {1, 1};
    cpm_status st = cpm_batch_create(ns, ops, pcs, nr, &M->batch);
    if (st != CPM_OK) fail(st, std::string("imex: ") + cpm_last_error());
    if (o.tune) {
      cpm_tune_result tr;
      st = cpm_batch_autotune(M->batch, nullptr, 0, nullptr, &tr);
      if (st != CPM_OK) fail(st, std::string("imex tune: ") + cpm_last_error());
    }
    const size_t per = (size_t)M->T.s * ns * M->n;
    M->KE.alloc(per);
    M->KI.alloc(per);
    M->rhs.alloc((size_t)ns * M->n);
    M->W.alloc((size_t)ns * M->n);
    M->ax.alloc((size_t)M->n);
    *out = M.release();
    return CPM_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed in cpm_imex_create");
    return CPM_ERR_OOM;
  }
}

cpm_status cpm_imex_step(cpm_imex* im, double t, double* const* w, int32_t nsteps, const cpm_solve_opts* sopts,
                         cpm_solve_stats* stats, void* stream) {
  try {
    if (!im || !w || !sopts) fail(CPM_ERR_ARG, "null argument");
    if (nsteps < 0) fail(CPM_ERR_ARG, "nsteps must be >= 0");
    cpm_imex_s& M = *im;
    for (int sp = 0; sp < M.ns; ++sp)
      if (!w[sp] && M.n) fail(CPM_ERR_ARG, "null state vector");
    if (sopts->transpose) fail(CPM_ERR_ARG, "stage solves are not transposed");
    if (sopts->poly_n != 0) fail(CPM_ERR_ARG, "stage solves use the shifted operator itself (poly_n = 0)");
    hipStream_t s = (hipStream_t)stream;
    std::vector<cpm_solve_stats> acc(M.ns);
    for (auto& a : acc) {
      std::memset(&a, 0, sizeof a);
      a.converged = 1;
    }
    const Tableau& T = M.T;
    const double gam = imex_gamma(T);
    cpm_status result = CPM_OK;
    double* Wp[2] = {M.W.p, M.W.p + M.n};
    const double* Wc[2] = {Wp[0], Wp[1]};
    const double* wc[2] = {w[0], M.ns > 1 ? w[1] : nullptr};
    double* rp[2] = {M.rhs.p, M.rhs.p + M.n};
    const double* rc[2] = {rp[0], rp[1]};
    for (int step = 0; step < nsteps && result == CPM_OK; ++step) {
      const double tn = t + step * M.o.dt;
      explicit_terms(M, tn, wc, 0, s);
      implicit_terms(M, wc, 0, s);
      for (int sp = 0; sp < M.ns; ++sp)   // warm start of the first stage solve: w^n
        hip_check(hipMemcpyAsync(Wp[sp], w[sp], (size_t)M.n * sizeof(double), hipMemcpyDeviceToDevice, s), "copy");
      for (int i = 1; i < T.s; ++i) {
        for (int sp = 0; sp < M.ns; ++sp)
          combine(M, sp, w[sp], T.AE[i], T.AI[i], i, 1.0 / (M.o.dt * gam * M.o.mu[sp]), rp[sp], s);
        std::vector<cpm_solve_stats> st(M.ns);
        cpm_status e = cpm_batch_solve(M.batch, rc, Wp, sopts, st.data(), s);
        for (int sp = 0; sp < M.ns; ++sp) {
          acc[sp].iterations += st[sp].iterations;
          acc[sp].restarts += st[sp].restarts;
          acc[sp].converged = acc[sp].converged && st[sp].converged;
          acc[sp].relres = std::max(acc[sp].relres, st[sp].relres);
          acc[sp].ms_total += st[sp].ms_total;
          acc[sp].n_precond += st[sp].n_precond;
          acc[sp].n_apply += st[sp].n_apply;
          if (st[sp].status != CPM_OK) acc[sp].status = st[sp].status;
        }
        if (e != CPM_OK) {
          if (e != CPM_NOT_CONVERGED) fail(e, std::string("imex stage solve: ") + cpm_last_error());
          result = CPM_NOT_CONVERGED;
          break;
        }
        explicit_terms(M, tn + T.c[i] * M.o.dt, Wc, i, s);
        implicit_terms(M, Wc, i, s);
      }
      if (result != CPM_OK) break;
      for (int sp = 0; sp < M.ns; ++sp) combine(M, sp, w[sp], T.bE, T.bI, T.s, 1.0, w[sp], s);
    }
    hip_check(hipStreamSynchronize(s), "imex step");
    if (stats)
      for (int sp = 0; sp < M.ns; ++sp) stats[sp] = acc[sp];
    if (result != CPM_OK) set_error("an IMEX stage solve did not converge");
    return result;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed in cpm_imex_step");
    return CPM_ERR_OOM;
  }
}

void cpm_imex_destroy(cpm_imex* im) { delete im; }
