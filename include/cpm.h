/*
 * cpm.h - C ABI of the MI355X closest point method (CPM) solver hot path.
 *
 * Method: May, Haynes & Ruuth, "A closest point method library for PDEs on
 * surfaces with parallel domain decomposition solvers and preconditioners"
 * (arXiv 2110.06322). The library discretizes the shifted surface Poisson
 * problem (c - Lap_S) u = f (Sec. 1, eq. shiftPoisson) with the stabilized
 * CPM operator (Sec. 2.1, eq. lapBel)
 *
 *     A = c I - Delta_S^h = (c + 2d/h^2) I - h^-2 O E,
 *
 * E the tensor-product degree-p Lagrange extension from the active nodes
 * Sigma_A to Sigma_A u Sigma_G, O the sum over the 2d grid neighbours, and
 * solves it with right-preconditioned GMRES (Sec. 4.1.1) and restricted /
 * optimized restricted additive Schwarz preconditioners (Sec. 2.2).
 *
 * Conventions for every entry point:
 *   - All functions return cpm_status; CPM_OK is 0. On failure a message is
 *     available from cpm_last_error() (thread-local, valid until the next
 *     call on the same thread). No C++ exception crosses this interface.
 *   - Arguments are validated before any device work is queued.
 *   - Handles are opaque and owned by the library; *_destroy releases their
 *     host and device memory (destroy(NULL) is a no-op).
 *   - "device" pointers are HIP device pointers (e.g. torch tensor
 *     data_ptr()); "host" pointers are ordinary CPU memory. The library never
 *     keeps a caller pointer after the call returns. Calls taking a `stream`
 *     (a hipStream_t passed as void*, NULL = default stream) are
 *     asynchronous on that stream unless stated otherwise: the caller keeps
 *     its buffers alive until the stream has passed the call.
 *   - Vectors over the unknowns are FP64, contiguous, in the library's node
 *     order (cpm_band_export); with nrhs > 1 they are interleaved
 *     [node][rhs].
 */
#ifndef CPM_H
#define CPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CPM_VERSION 1

typedef enum {
  CPM_OK = 0,
  CPM_ERR_ARG = 1,        /* invalid handle, size, option or pointer */
  CPM_ERR_BAND = 2,       /* band leaves the grid box or closure failed */
  CPM_ERR_PIVOT = 3,      /* zero pivot in a local factorization */
  CPM_ERR_DEVICE = 4,     /* HIP runtime error, or no usable GPU */
  CPM_ERR_OOM = 5,        /* host or device allocation failed */
  CPM_NOT_CONVERGED = 6,  /* solver stopped before reaching the tolerance */
  CPM_ERR_STATE = 7       /* object used in a state that does not allow it */
} cpm_status;

/* ---------------------------------------------------------------------
 * Surfaces and the computational band (Sec. 2.1: closest point function
 * eq. cpFunc; active nodes Sigma_A containing every (p+1)^d interpolation
 * cube; ghost nodes Sigma_G completing the finite-difference stencils).
 * ------------------------------------------------------------------- */
typedef enum {
  CPM_SURF_CIRCLE = 0,    /* d = 2: params[0] = R, centre[0..1] */
  CPM_SURF_SPHERE = 1,    /* d = 3: params[0] = R, centre[0..2] */
  CPM_SURF_TORUS = 2,     /* d = 3, axis z, centre 0: params = {R, r} */
  CPM_SURF_ELLIPSOID = 3  /* d = 3, centre 0, axis-aligned: params = {a, b, c} */
} cpm_surface_kind;

typedef struct {
  int32_t kind;           /* cpm_surface_kind */
  double params[3];
  double center[3];
} cpm_surface;

typedef struct cpm_band_s cpm_band;

typedef struct {
  int64_t n_active;       /* N_A = |Sigma_A|, the unknowns */
  int64_t n_ghost;        /* N_G = |Sigma_G| */
  int64_t n_band;         /* |B_gamma| */
  int32_t d, p;
  double h, gamma;
  double lo[3];
  int32_t shape[3];       /* grid points per axis */
  int64_t n_bricks;       /* 4x4x4 (d=3) or 8x8 (d=2) node bricks holding band nodes */
  int32_t closure_iterations;
  int32_t reach;          /* the ghost set's reach along an axis (1, or 2 for fourth-order stencils) */
} cpm_band_info;

/* Build the band on the host. Grid nodes x_i = lo + i h, i_k in
 * [0, floor((hi_k-lo_k)/h + 0.5)]. B_gamma = {x : |x - cp(x)| <= gamma(1+1e-10)};
 * Sigma_A = union over x in B_gamma of the cube b + {0..p}^d with
 * b = floor((cp(x)-lo)/h - (p-1)/2); Sigma_G = grid neighbours of Sigma_A not
 * in Sigma_A. gamma <= 0 selects h sqrt((d-1)((p+1)/2)^2 + (1+(p+1)/2)^2).
 * d in {2,3}, p in 1..5 (the fused second-order apply takes p <= 3; p = 4, 5
 * run the two-kernel path, see cpm_operator_opts). Errors: CPM_ERR_ARG (bad sizes / surface),
 * CPM_ERR_BAND (a cube or neighbour leaves the grid box, or closure needs
 * more than one extra pass). lo/hi: host arrays of d doubles. */
cpm_status cpm_band_build(const cpm_surface* surface, int32_t d, double h, int32_t p,
                          const double* lo, const double* hi, double gamma,
                          cpm_band** out);
/* Closest points supplied by the caller (Sec. 2.1: the library takes
 * user-defined closest point functions; Sec. 4.1.6: an open, user-defined
 * hemisphere with mixed boundary conditions). The callback receives n points
 * x [n][d] (host) and writes their closest points cp [n][d] and flags
 * flag [n]: 1 when the closest point lies on a part of the surface's boundary
 * carrying homogeneous Dirichlet conditions, else 0 (interior points, and
 * boundary points with the natural homogeneous Neumann treatment). It returns
 * 0 on success; anything else aborts the build with CPM_ERR_ARG. It is called
 * from the building thread only, with batches of up to 2^20 points.
 * A node x whose closest point c is flagged takes the extension
 * -(E u)(cp(2c - x)): interpolation at the closest point of its mirror image
 * through c, negated (second-order homogeneous Dirichlet). The band is then
 * built as by cpm_band_build with these interpolation points. */
typedef int32_t (*cpm_cp_callback)(int64_t n, const double* x, double* cp, int32_t* flag, void* ctx);
cpm_status cpm_band_build_user(cpm_cp_callback cp, void* ctx, int32_t d, double h, int32_t p, const double* lo,
                               const double* hi, double gamma, cpm_band** out);
/* Either builder with a wider ghost set (Sec. 3.1.2: the fourth-order
 * Laplace-Beltrami grid function's stencil reaches two nodes along each
 * axis): Sigma_G = the grid nodes within `reach` steps along an axis of
 * Sigma_A that are not in Sigma_A, reach in {1, 2}; gamma <= 0 selects
 * h sqrt((d-1)((p+1)/2)^2 + (reach+(p+1)/2)^2). Exactly one of surface and
 * cp is given (ctx goes with cp). Errors as for the builders above. */
cpm_status cpm_band_build_reach(const cpm_surface* surface, cpm_cp_callback cp, void* ctx, int32_t d, double h,
                                int32_t p, const double* lo, const double* hi, double gamma, int32_t reach,
                                cpm_band** out);
cpm_status cpm_band_get_info(const cpm_band* band, cpm_band_info* info);
/* Export the library's node order: Sigma_A first (indices 0..N_A-1, the
 * unknowns), then Sigma_G. Host arrays, caller-owned, any may be NULL:
 * gidx [(N_A+N_G) x d] int32 grid indices, cp [(N_A+N_G) x d] closest
 * points, kind [N_A+N_G] (0 active, 1 ghost). Row-major [node][axis]. */
cpm_status cpm_band_export(const cpm_band* band, int32_t* gidx, double* cp, uint8_t* kind);
/* The extension rows' interpolation points ip [(N_A+N_G) x d] and signs
 * sign [N_A+N_G] (+1, or -1 for mirrored Dirichlet rows), same order as
 * cpm_band_export; host arrays, either may be NULL. */
cpm_status cpm_band_export_interp(const cpm_band* band, double* ip, double* sign);
void cpm_band_destroy(cpm_band* band);

/* ---------------------------------------------------------------------
 * Operator A = (c + 2d/h^2) I - h^-2 O E (Sec. 2.1 eq. lapBel, Sec. 1 eq.
 * shiftPoisson), matrix-free on the GPU.
 * ------------------------------------------------------------------- */
typedef struct cpm_operator_s cpm_operator;

/* Uploads the band (closest points, brick map, tiles) to device memory
 * owned by the operator. The band may be destroyed afterwards. c > 0. */
cpm_status cpm_operator_create(const cpm_band* band, double c, void* stream, cpm_operator** out);
/* Operator options.
 * order: the stabilized operator's stencil order (Sec. 3.1.2: built-in
 *   second- and fourth-order Laplace-Beltrami grid functions):
 *   2: A = (c + 2d/h^2) I - h^-2 O1 E (as cpm_operator_create);
 *   4: A = (c + 30d/(12h^2)) I - (12h^2)^-1 (16 O1 - O2) E, with O1 the sum
 *      over the 2d nearest grid neighbours and O2 over the 2d nodes two steps
 *      away along an axis (the five-point fourth-order second difference per
 *      axis, the node's own term un-extended); needs a band of reach 2
 *      (cpm_band_build_reach).
 *   Order 2 with p <= 3 runs the fused apply; order 4, or p = 4 or 5, runs two
 *   kernels (every extension row into an operator-owned vector of
 *   (N_A+N_G) * 4 doubles, then the stencil). With degree-p interpolation the
 *   surface solution's error is O(h^order) + O(h^(p-1)): order 4 needs p = 5
 *   for fourth order. Two-kernel operators support everything but the
 *   transposed apply (and so transposed solves); a preconditioner built on
 *   them is the (O)RAS of the second-order operator with degree min(p, 3)
 *   interpolation at the same shift, a spectrally equivalent approximation.
 * apply_lds_bytes: LDS budget per tile of the fused apply, 16384..65536
 *   (0: 65536); tiles whose footprint does not fit are applied by a slower
 *   kernel that reads x from global memory (same results, bit for bit). */
typedef struct {
  int32_t order;            /* 2 (default) or 4 */
  int32_t apply_lds_bytes;  /* 0 (default) or 16384..65536 */
} cpm_operator_opts;

typedef struct {
  int32_t order;
  int32_t two_kernel;        /* 1: the two-kernel apply (order 4 or p > 3) */
  int32_t two_pass;          /* 1: the two-pass variant of the fused apply is available */
  int32_t apply_lds_bytes;
  int32_t n_tiles;           /* tiles of the fused apply with active nodes */
  int32_t n_fallback_tiles;  /* of which applied by the global-memory kernel */
  int32_t apply_variant;     /* one-RHS kernel in use (see cpm_tune_result) */
} cpm_operator_info;

cpm_status cpm_operator_opts_default(cpm_operator_opts* opts);
cpm_status cpm_operator_create_ex(const cpm_band* band, double c, const cpm_operator_opts* opts, void* stream,
                                  cpm_operator** out);
cpm_status cpm_operator_get_info(const cpm_operator* op, cpm_operator_info* info);
/* Changes the shift c (> 0) of A = (c + 2d/h^2) I - h^-2 O E. Synchronizes
 * the device. Later cpm_solve calls use the new shift; a batch takes its
 * operators' shifts when it is created, so create batches after this call. */
cpm_status cpm_operator_set_shift(cpm_operator* op, double c);
double cpm_operator_get_shift(const cpm_operator* op);
int64_t cpm_operator_n_active(const cpm_operator* op);
void cpm_operator_destroy(cpm_operator* op);

/* v = E u: the extension at every node of Sigma_A u Sigma_G (Sec. 2.1).
 * u: device [N_A], v: device [N_A+N_G]. Test hook; one right-hand side. */
cpm_status cpm_extend_apply(const cpm_operator* op, const double* u, double* v, void* stream);
/* y = A x (transpose = 0) or y = A^T x (transpose = 1).
 * x, y: device [N_A * nrhs], interleaved [node][rhs], must not alias;
 * nrhs in {1, 2, 4}. A^T x = (c + 2d/h^2) x - h^-2 E^T (O^T x) is evaluated
 * without atomics (each output gathers the extension rows that reach it). */
cpm_status cpm_apply(const cpm_operator* op, const double* x, double* y, int32_t nrhs, void* stream);
cpm_status cpm_apply_T(const cpm_operator* op, const double* x, double* y, int32_t nrhs, void* stream);
/* The same y = A^T x for callers that cannot allocate device memory (code
 * under HIP stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): cpm_apply_T allocates its (N_A+N_G) * nrhs intermediate sums on
 * first use, this call keeps them in a static device array of 4,194,304
 * doubles (32 MiB per GPU, held until the process ends) and calls no
 * allocator. Larger (N_A+N_G) * nrhs is refused with CPM_ERR_ARG before any
 * launch. All calls on one GPU share that array: calls that overlap on one GPU
 * (concurrent streams or threads) race and must be ordered by the caller.
 * The current device must be the operator's. Same arguments and results as
 * cpm_apply_T (identical bits). */
cpm_status cpm_apply_T_noalloc(const cpm_operator* op, const double* x, double* y, int32_t nrhs, void* stream);

/* dL/dc for u = A(c)^-1 f (Sec. 2.1, eq. lapBel: A(c) = c I + K with K
 * independent of c): with lambda the adjoint solution of A^T lambda = dL/du,
 * grad[0] = -sum_i lambda_i u_i over all N_A * nrhs entries (for nrhs > 1 the
 * right-hand sides share c, so their contributions add).
 * lambda, u: device [N_A * nrhs]; grad: device, one double (written
 * asynchronously on the stream). The sum is reduced in a fixed order, so
 * repeated calls give identical bits. Uses an operator-owned buffer of chunk
 * sums (allocated on first use): calls on one operator must not overlap.
 * nrhs in {1, 2, 4}. */
cpm_status cpm_shift_gradient(const cpm_operator* op, const double* lambda, const double* u, int32_t nrhs,
                              double* grad, void* stream);

/* ---------------------------------------------------------------------
 * Restricted (RAS) and optimized restricted (ORAS) additive Schwarz
 * preconditioners (Sec. 2.2, eq. ddIter and the restricted recombination;
 * Sec. 4.1.1: alpha = 4, alpha_cross = 20, ILU(0) local solves by default).
 *   partition : recursive coordinate bisection of Sigma_A by closest point
 *               (axis of largest extent, split value = floor(n/2)-th smallest
 *               coordinate, cp < split goes first); n_parts a power of two;
 *   overlap   : Omega_j = nodes whose cp lies in box_j grown by overlap*h;
 *   local     : rows/columns of A in Omega_j (ascending grid key), on A's
 *               structural pattern;
 *   ORAS      : a_ii += s_i/(1 + alpha_i h), s_i the sum of the dropped
 *               couplings of row i, alpha_i = alpha_cross when they belong
 *               to >= 2 other subdomains;
 *   subsolver : ILU(0) (default) or exact dense LU (tests, small parts);
 *   apply     : z = sum_j Rt_j^T A_j^-1 R_j r, written only at owned nodes.
 * ------------------------------------------------------------------- */
typedef enum { CPM_PC_NONE = 0, CPM_PC_RAS = 1, CPM_PC_ORAS = 2 } cpm_pc_kind;
typedef enum { CPM_SUB_ILU0 = 0, CPM_SUB_DENSE_LU = 1 } cpm_subsolver;
typedef enum { CPM_PREC_FP64 = 0, CPM_PREC_FP32 = 1 } cpm_precision;
/* local row order before ILU(0): reverse Cuthill-McKee of the symmetrised
 * local graph (default), or decreasing distance |x - cp(x)| of the row's grid
 * node from the surface (ties by grid key). The distance order cuts the
 * dependency chains of the triangular solves about tenfold (as long as the
 * band is thick rather than the subdomain), but the Krylov iteration count
 * grows by 50-85 % with ORAS on the sphere and torus workloads. Its wide
 * levels are stored as packets of up to four same-level rows, solved together
 * by one wavefront (16 lanes per row); this needs factor rows of at most 192
 * entries (3-D p = 3 rows have at most 176), else the rows are solved one per
 * wavefront. */
typedef enum { CPM_ORDER_RCM = 0, CPM_ORDER_DISTANCE = 1 } cpm_ordering;
/* Coarse level (two-level Schwarz; the one-level method's iteration count grows
 * with the number of subdomains, Sec. 5 Table 3): the piecewise-constant coarse
 * space of one vector per subdomain (1 on the nodes it owns, R0), the Galerkin
 * coarse matrix A0 = R0 A R0^T (built with the operator, inverted densely), and
 *   ADDITIVE:     z = M1^-1 r + R0^T A0^-1 R0 r,
 *   COARSE_FIRST: z_c = R0^T A0^-1 R0 r, z = z_c + M1^-1 (r - A z_c),
 * M1 the one-level (O)RAS. Not with transpose = 1. */
typedef enum { CPM_COARSE_NONE = 0, CPM_COARSE_ADDITIVE = 1, CPM_COARSE_FIRST = 2 } cpm_coarse;

typedef struct {
  int32_t kind;           /* cpm_pc_kind */
  int32_t n_parts;        /* N_S, power of two, >= 1 */
  double overlap;         /* N_O in units of h, >= 0 */
  double alpha;           /* Robin parameter (ORAS), > 0 */
  double alpha_cross;     /* Robin parameter at cross points (ORAS), > 0 */
  int32_t subsolver;      /* cpm_subsolver */
  int32_t precision;      /* cpm_precision of the factors and local solves */
  int32_t transpose;      /* 1: build on A^T (for adjoint solves) */
  int32_t ordering;       /* cpm_ordering (ILU(0) only) */
  int32_t coarse;         /* cpm_coarse (default NONE; n_parts <= 4096) */
} cpm_precond_opts;

typedef struct cpm_precond_s cpm_precond;

typedef struct {
  int32_t n_parts;
  int64_t total_rows;     /* sum_j |Omega_j| */
  int64_t total_nnz;      /* sum_j nnz(A_j) */
  int32_t max_rows;       /* max_j |Omega_j| */
  int32_t max_levels;     /* longest dependency chain of a triangular solve */
  int32_t precision;
  int32_t kind;
} cpm_precond_info;

/* Builds partition, local matrices and factors on the host, uploads them to
 * device memory owned by the preconditioner. Uses op's current shift c.
 * Errors: CPM_ERR_ARG, CPM_ERR_PIVOT (zero pivot), CPM_ERR_OOM. */
cpm_status cpm_precond_create(const cpm_operator* op, const cpm_precond_opts* opts,
                              cpm_precond** out);
cpm_status cpm_precond_get_info(const cpm_precond* pc, cpm_precond_info* info);
/* Host arrays: owner [N_A] (subdomain owning each node), ovl_ptr
 * [n_parts+1] int64, ovl_idx [total_rows] (node indices of each Omega_j in
 * local order). Any may be NULL. */
cpm_status cpm_precond_export_partition(const cpm_precond* pc, int32_t* owner,
                                        int64_t* ovl_ptr, int32_t* ovl_idx);
/* z = M^-1 r. r, z: device [N_A * nrhs], must not alias; nrhs in {1,2,4}. */
cpm_status cpm_precond_apply(const cpm_precond* pc, const double* r, double* z, int32_t nrhs,
                             void* stream);
void cpm_precond_destroy(cpm_precond* pc);

/* ---------------------------------------------------------------------
 * Solver: restarted right-preconditioned flexible GMRES in FP64 with
 * classical Gram-Schmidt twice (CGS2) and Givens rotations on the device.
 * mode FP64     : preconditioner as built (FP64 or FP32 factors);
 * mode MIXED_IR : GMRES-based iterative refinement: each restart cycle
 *                 solves the correction equation A d = r to inner_rtol
 *                 relative to its own residual, r = f - A u is recomputed
 *                 in FP64 at every restart (requires an FP32 preconditioner
 *                 or none).
 * Stopping: |f - A u|_2 <= max(rtol |f|_2, atol), checked on the true FP64
 * residual at every restart and at exit; x0 = contents of u (zero it for
 * x0 = 0). Blocks until the solution is in u and stats are final.
 * Returns CPM_NOT_CONVERGED (u = last iterate, stats filled) when max_it is
 * reached, on stagnation, or on a non-finite residual.
 * ------------------------------------------------------------------- */
typedef enum { CPM_MODE_FP64 = 0, CPM_MODE_MIXED_IR = 1 } cpm_solve_mode;

typedef struct {
  int32_t restart;        /* Krylov dimension per cycle, 1..64 (default 30) */
  double rtol;
  double atol;
  int32_t max_it;         /* cap on Arnoldi steps */
  int32_t mode;           /* cpm_solve_mode */
  int32_t transpose;      /* 1: solve A^T u = f (pc must be built with transpose=1) */
  int32_t use_graph;      /* 1: run each restart cycle as one captured hipGraph, replayed on a
                             library stream ordered after `stream`; all m steps are launched and
                             the operator and preconditioner kernels turn into no-ops once every
                             system has stopped (results equal those of the eager path); the
                             graph is captured on first use per batch and restart length.
                             Not combinable with profile. */
  double inner_rtol;      /* MIXED_IR: per-cycle reduction target (default 1e-4) */
  int32_t stagnation_cycles; /* cycles without 1% progress before giving up (default 50) */
  int32_t profile;        /* 1: time operator / preconditioner kernels with hipEvents (adds syncs) */
  /* Operator algebra (Sec. 3.1.2, grid functions added and composed; Sec. 4.1.2, the
   * shifted biharmonic equation): poly_n = 0 solves A u = f. poly_n in 1..5 solves
   * P(L) u = f instead, P(L) = sum_{k < poly_n} poly_coef[k] L^k, where L = c I - A(c)
   * is the second-order Laplace-Beltrami operator of each instance (c its shift; L
   * does not depend on c). The shifted biharmonic c0 + L^2 is poly_n = 3, poly_coef
   * = {c0, 0, 1}. One application of P(L) costs poly_n - 1 applies of A.
   * Not combinable with transpose or use_graph. */
  int32_t poly_n;
  double poly_coef[5];
  /* preconditioner applications per Arnoldi step, 1..4 (default 1): z = M^-k v. With
   * k = 2 and M the (O)RAS of A(sqrt(c0)), M^-2 approximates A(sqrt(c0))^-2, whose
   * inverse (sqrt(c0) - L)^2 is spectrally equivalent to c0 + L^2 (ratio within
   * [1, 2] for a negative semi-definite L). */
  int32_t pc_power;
  /* pc_inner_rtol in (0, 1): every preconditioner application becomes an inner
   * FGMRES solve of the instances' own operators A(c) w = v from zero, to
   * pc_inner_rtol relative, at most pc_inner_max_it steps (default 30),
   * preconditioned by the (O)RAS (the outer FGMRES is flexible, so an inexact
   * inner solve is a valid variable preconditioner). With pc_power 2 and the
   * operator at shift sqrt(c0) this applies A(sqrt(c0))^-2 almost exactly to
   * the shifted biharmonic c0 + L^2, whose iteration count then stays flat in
   * h, where squaring the (O)RAS itself does not. 0 (default): off.
   * Host-synchronizing; not combinable with use_graph or transpose. */
  double pc_inner_rtol;
  int32_t pc_inner_max_it;
} cpm_solve_opts;

typedef struct {
  int32_t iterations;     /* Arnoldi steps */
  int32_t restarts;       /* restart cycles */
  int32_t converged;
  int32_t status;         /* cpm_status of this system */
  double relres;          /* true |f - A u| / |f| at exit */
  double ms_total;        /* wall time of the solve (hipEvent) */
  double ms_precond;      /* profiled: total time of the timed preconditioner launches, else 0 */
  double ms_apply;        /* profiled: total time of the timed operator launches, else 0 */
  int32_t n_precond;      /* preconditioner applications (profiled: the timed ones; use_graph:
                             launches, some of which may have been no-ops) */
  int32_t n_apply;        /* operator applications (profiled: the timed ones, one per Arnoldi step) */
} cpm_solve_stats;

cpm_status cpm_solve_opts_default(cpm_solve_opts* opts);
cpm_status cpm_precond_opts_default(cpm_precond_opts* opts);

/* y = P(L) x = sum_{k < ncoef} coef[k] L^k x with L = c I - A(c) the operator's
 * Laplace-Beltrami operator (Sec. 3.1.2: grid functions added and composed;
 * the biharmonic is L L). ncoef in 1..5, coef: host [ncoef], finite.
 * x, y: device [N_A * nrhs], nrhs in {1,2,4}, must not alias. Stream-ordered;
 * allocates a workspace of 2 N_A nrhs doubles on first use per size (not under
 * graph capture then). CPM_ERR_ARG on bad arguments. */
cpm_status cpm_poly_apply(const cpm_operator* op, int32_t ncoef, const double* coef, const double* x,
                          double* y, int32_t nrhs, void* stream);

/* f, u: device [N_A * nrhs]; pc may be NULL (no preconditioner). stats may be NULL. */
cpm_status cpm_solve(const cpm_operator* op, const cpm_precond* pc, const double* f, double* u,
                     int32_t nrhs, const cpm_solve_opts* opts, cpm_solve_stats* stats,
                     void* stream);

/* ---------------------------------------------------------------------
 * Batched solves: many surfaces (operators of different sizes, shifts and
 * preconditioners) and many right-hand sides, advanced together: every
 * kernel of an Arnoldi step is one launch over all instances' tiles,
 * subdomains and vector chunks. Instances finish independently.
 * ------------------------------------------------------------------- */
typedef struct cpm_batch_s cpm_batch;

/* ops[i], pcs[i] (pcs may be NULL or hold NULLs): borrowed, must outlive
 * the batch; nrhs[i] in {1,2,4}. Each operator's shift is copied at
 * creation (see cpm_operator_set_shift). */
cpm_status cpm_batch_create(int32_t n, const cpm_operator* const* ops,
                            const cpm_precond* const* pcs, const int32_t* nrhs,
                            cpm_batch** out);
/* f[i], u[i]: device [N_A(i) * nrhs(i)]. stats: host array of
 * sum_i nrhs(i) entries (system order: instance-major) or NULL. Returns
 * CPM_NOT_CONVERGED if any system did not converge. */
cpm_status cpm_batch_solve(cpm_batch* batch, const double* const* f, double* const* u,
                           const cpm_solve_opts* opts, cpm_solve_stats* stats, void* stream);
/* y[i] = A_i x[i] for every instance in one launch. */
cpm_status cpm_batch_apply(cpm_batch* batch, const double* const* x, double* const* y,
                           void* stream);
void cpm_batch_destroy(cpm_batch* batch);

/* ---------------------------------------------------------------------
 * Autotuning. Times the candidate kernel configurations of the operator's
 * apply (one right-hand side: persistent pipelined kernel or one workgroup
 * per tile) and, when pc is given, of its subdomain solves (completion flags
 * or values-as-flags; 256, 512 or 1024 threads per subdomain, for packet
 * factors 256 or 512, or 768 with FP32 factors and 1-2 right-hand sides;
 * with or without back-off while waiting) on library-allocated scratch
 * vectors, and keeps the fastest. All candidates for one factor layout
 * compute bit-identical results; only
 * speed differs. Choices are cached per shape class (device, d, p, nrhs and
 * power-of-two size classes) in the JSON file cache_path (NULL: no file; a
 * missing or unreadable file counts as empty; it is rewritten when a class is
 * added). force = 1 re-times classes found in the cache. Synchronizes the
 * stream; allocates device memory, so it must not run under graph capture.
 * Batches and solves created afterwards use the new choices.
 * ------------------------------------------------------------------- */
typedef struct {
  int32_t apply_variant;     /* 0 pipelined, 1 per tile */
  int32_t schwarz_variant;   /* rows one per wavefront: 0 completion flags, 1 values as flags;
                                packets (distance order): 2 values as flags, 3 completion flags */
  int32_t schwarz_threads;   /* threads per subdomain workgroup */
  int32_t schwarz_sleep;     /* 1 = back off while waiting on a dependency */
  double apply_ms;           /* mean time of one apply with the chosen kernel */
  double precond_ms;         /* mean time of one preconditioner apply (0 without pc) */
  int32_t from_cache;        /* 1 when every choice came from the cache file */
} cpm_tune_result;

cpm_status cpm_autotune(cpm_operator* op, cpm_precond* pc, int32_t nrhs, const char* cache_path,
                        int32_t force, void* stream, cpm_tune_result* out);

/* The same for a batch: times the batch's shared apply and subdomain-solve
 * launches over all its instances (so concurrency between subdomains of
 * different instances counts) and sets the batch's own choices; classes are
 * keyed by instance count and total size as well. Allocates the batch's
 * workspace if needed; synchronizes the stream. */
cpm_status cpm_batch_autotune(cpm_batch* batch, const char* cache_path, int32_t force, void* stream,
                              cpm_tune_result* out);

/* ---------------------------------------------------------------------
 * Reaction-diffusion (Sec. 1, eq. rdsys; Sec. 4.1.5, eq. grayscott):
 * IMEX-Euler right-hand sides of the Gray-Scott system, the reaction taken
 * explicitly and the diffusion implicitly:
 *   fu = (u/dt - u v^2 + F (1 - u)) / mu_u,  fv = (v/dt + u v^2 - (F + k) v) / mu_v,
 * so that (1/(mu dt) - Lap_S^h) w^{n+1} = fw advances each species.
 * u, v, fu, fv: device [n]; fu/fv may not alias u/v. Asynchronous on stream.
 * ------------------------------------------------------------------- */
cpm_status cpm_gray_scott_rhs(int64_t n, const double* u, const double* v, double F, double k, double dt,
                              double mu_u, double mu_v, double* fu, double* fv, void* stream);

/* ---------------------------------------------------------------------
 * Additive Runge-Kutta IMEX time stepping of surface reaction-diffusion
 * systems w_t = F_E(t, w) + mu Lap_S w (Sec. 1, eq. rdsys): the diffusion
 * implicit, the rest explicit. Sec. 4.1.3 (heat equation, eq. heat) and
 * Sec. 4.1.5 (Gray-Scott, eq. grayscott) run with a third-order additive
 * Runge-Kutta IMEX integrator by default; CPM_IMEX_ARK3 is ARK3(2)4L[2]SA
 * (Kennedy & Carpenter, Appl. Numer. Math. 44, 2003: explicit tableau A^E,
 * L-stable stiffly accurate ESDIRK tableau A^I with diagonal gamma), and
 * CPM_IMEX_EULER is forward/backward Euler. A step computes
 *   W_1 = w^n,
 *   (I - dt gamma mu Lap) W_i = w^n + dt sum_{j<i} (aE_ij KE_j + aI_ij KI_j),
 *   KE_j = F_E(t + c_j dt, W_j), KI_j = mu Lap_S^h W_j,
 *   w^{n+1} = w^n + dt sum_j (bE_j KE_j + bI_j KI_j),
 * each stage solve being A(c_w) W_i = rhs/(dt gamma mu_w) with the species'
 * operator at shift c_w = 1/(dt gamma mu_w) (cpm_imex_shift), and
 * Lap_S^h x = c_w x - A(c_w) x. The species' stage solves run as one batch,
 * warm-started from the previous stage.
 *   kind GRAY_SCOTT: 2 species, F_E = (-u v^2 + F(1-u), u v^2 - (F+k) v);
 *   kind HEAT:       1 species, F_E = cos(t) g1 + sin(t) g2 (eq. htForce has
 *                    this form), g1, g2 given at create;
 *   kind FITZHUGH_NAGUMO (Sec. 4.1.4, eq. fitznag): 2 species,
 *                    F_E = ((a - u)(u - 1) u - v, eps (beta u - v)),
 *                    rd = {a, eps, beta} (the paper: 0.1, 0.01, 0.5);
 *   kind SCHNACKENBERG (Sec. 4.1.6, eq. schnack): 2 species,
 *                    F_E = (d1 - u + u^2 v + lam v, d2 - u^2 v - lam v),
 *                    rd = {d1, d2, lam} (the paper: 0.003, 0.7, 0.06).
 * ------------------------------------------------------------------- */
typedef enum { CPM_IMEX_EULER = 0, CPM_IMEX_ARK3 = 1 } cpm_imex_scheme;
typedef enum {
  CPM_RD_GRAY_SCOTT = 0,
  CPM_RD_HEAT = 1,
  CPM_RD_FITZHUGH_NAGUMO = 2,
  CPM_RD_SCHNACKENBERG = 3
} cpm_rd_kind;

typedef struct {
  int32_t scheme;         /* cpm_imex_scheme (default ARK3) */
  int32_t kind;           /* cpm_rd_kind (default GRAY_SCOTT) */
  int32_t nspecies;       /* 1 for the heat equation, else 2 */
  double dt;              /* time step, > 0 */
  double mu[2];           /* diffusion coefficient of each species, > 0 */
  double F, k;            /* Gray-Scott feed and kill rates */
  int32_t tune;           /* 1: autotune the stage solves' kernels at creation */
  double rd[3];           /* FitzHugh-Nagumo {a, eps, beta} or Schnackenberg {d1, d2, lam} */
} cpm_imex_opts;

typedef struct cpm_imex_s cpm_imex;

cpm_status cpm_imex_opts_default(cpm_imex_opts* opts);
/* The shift 1/(dt gamma mu_species) the species' operator must carry (0 on
 * bad arguments). */
double cpm_imex_shift(const cpm_imex_opts* opts, int32_t species);
/* ops[s] (and pcs[s], may be NULL or hold NULLs): borrowed, one per species,
 * on one band, shifts as cpm_imex_shift gives (else CPM_ERR_ARG); they must
 * outlive the integrator. forcing: HEAT only, device {g1, g2}, each [N_A],
 * copied at creation. Allocates stage buffers of 2 s nspecies N_A + 3 N_A
 * doubles (s stages). */
cpm_status cpm_imex_create(const cpm_operator* const* ops, const cpm_precond* const* pcs,
                           const cpm_imex_opts* opts, const double* const* forcing, cpm_imex** out);
/* Advances w[s] (device [N_A] each, in place) by nsteps steps from time t.
 * Stage solves use sopts (FP64 or MIXED_IR; not transposed). stats: host
 * array of nspecies entries or NULL (iterations, restarts, apply and
 * preconditioner counts, time summed over all stage solves; relres the
 * largest; converged only if all were). Blocks until done. Returns
 * CPM_NOT_CONVERGED (w holds the last completed step) when a stage solve
 * fails to converge. */
cpm_status cpm_imex_step(cpm_imex* im, double t, double* const* w, int32_t nsteps, const cpm_solve_opts* sopts,
                         cpm_solve_stats* stats, void* stream);
void cpm_imex_destroy(cpm_imex* im);

/* ---------------------------------------------------------------------
 * Misc
 * ------------------------------------------------------------------- */
const char* cpm_last_error(void);
int32_t cpm_version(void);
/* Number of HIP devices visible (0 when none); never fails. */
int32_t cpm_device_count(void);
/* sizeof of the public option / result structs, for bindings that declare
 * them by hand: 0 cpm_solve_opts, 1 cpm_solve_stats, 2 cpm_precond_opts,
 * 3 cpm_tune_result, 4 cpm_imex_opts, 5 cpm_band_info, 6 cpm_operator_opts,
 * 7 cpm_operator_info; -1 for any other value. Host only. */
int64_t cpm_abi_sizeof(int32_t which);

#ifdef __cplusplus
}
#endif
#endif /* CPM_H */
