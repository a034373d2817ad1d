/*
 * hsrom.h -- C ABI of the MI355X (gfx950) hybrid-snapshot adaptive ROM step.
 *
 * Method: Zucatti & Zahr, "An adaptive, training-free reduced-order model for
 * convection-dominated problems based on hybrid snapshots" (arXiv 2301.01718).
 * The four calls below follow the paper's problem statement:
 *   hdm_step        -- full HDM solve R_k(q) = 0 (Sec. 2.2, eq. hdm)
 *   sample_select   -- error ordering, G, sampled set and its neighbours
 *                      (Sec. 2.3.3, eq. rre; Alg. 1 set operations)
 *   rom_hybrid_step -- partial HDM + gappy-POD fit + subiterations +
 *                      reconstruction + residual-gated filter
 *                      (eq. hybrid, eq. partial_hdm2, eq. red_coord,
 *                      Sec. 2.3.2, Sec. 2.3.4; Alg. 1 hybrid branch)
 *   basis_update    -- window mean and POD basis (eq. pod, eq. mean;
 *                      Alg. 1 basis update)
 *
 * Conventions for every call
 * --------------------------
 * - All double / int32 / uint8 array arguments are DEVICE pointers on the
 *   context's device unless the comment says "host".  They are owned by the
 *   caller and never freed by the library.  Outputs must not alias inputs.
 * - State vectors are component-major: q[c * ncell + i + nx * j], length
 *   N = ncomp * ncell (ncomp = 1 for Burgers, 4 for Euler: rho, rho u,
 *   rho v, E).  Bases are column-major N x m: Phi[col * N + row].
 * - Work is enqueued on the stream given to hs_create.  Calls that must take
 *   a data-dependent decision (Newton convergence, subiteration and filter
 *   stopping, set sizes) read it back internally and return once every
 *   decision is taken and reported (info, counts, m_eff); unless a call says
 *   otherwise they also return only when their outputs are complete.
 *   rom_hybrid_step returns with the work after its last decision (the
 *   indicator, the final copies) still enqueued: its outputs are complete in
 *   the stream's order, so later work on that stream needs no wait, and a
 *   reader on the host or on another stream synchronises first (hs_sync).
 * - Return value: HS_OK (0) or a negative status.  Argument errors are
 *   reported before any work is enqueued.  Numerical failures
 *   (HS_ERR_NOT_CONVERGED, HS_ERR_RANK, HS_ERR_NONFINITE) leave the outputs
 *   undefined.  hs_last_error() gives a message for the last failure.
 * - No C++ exception crosses this interface.  One context per stream and
 *   host thread; a context is not thread-safe.
 * - Arithmetic is IEEE double throughout unless a precision field says
 *   otherwise; reductions use fixed orders, so identical inputs give
 *   bitwise-identical outputs.
 */
#ifndef HSROM_H
#define HSROM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
#define HS_OK                 0
#define HS_ERR_INVALID_ARG   -1   /* null pointer, bad enum, bad parameter */
#define HS_ERR_SHAPE         -2   /* size beyond the context's capacity */
#define HS_ERR_NOT_CONVERGED -3   /* Newton / linear iteration hit its limit */
#define HS_ERR_RANK          -4   /* empty basis or a rank-zero fit */
#define HS_ERR_NONFINITE     -5   /* NaN or Inf met in a residual */
#define HS_ERR_HIP           -6   /* HIP runtime failure */
#define HS_ERR_OOM           -7   /* device allocation failed */

/* --------------------------------------------------------- problem kinds */
#define HS_BURGERS_1D 0   /* u_t + (u^2/2)_x = 0 on (0,1) */
#define HS_BURGERS_2D 1   /* u_t + (u^2/2)_x + (u^2/2)_y = 0 on (0,1)^2 */
#define HS_EULER_2D   2   /* 2D Euler, ideal gas (Sec. 3.1, eq. euler) */

#define HS_BC_INFLOW_OUTFLOW 0 /* left ghost = inflow value, right ghost = last cell */
#define HS_BC_PERIODIC       1
#define HS_BC_TRANSMISSIVE   2 /* every ghost = its boundary cell */

/* Precision of the basis Phi.  HS_FP64: Phi is double.  HS_MIXED_FP32: Phi
 * is an FP32 master copy (float): every N-stream of the hybrid step that reads
 * the basis (fit gathers and projections, ring update, reconstruction,
 * indicator) moves half the bytes, while all arithmetic stays FP64 (products
 * of the float entries are formed and accumulated in double, and the fit is
 * refined in FP64).  basis_update works in FP64 in both modes: its cut
 * sigma_i > tau_pod sigma_0 (tau_pod = 1e-8) needs singular values resolved
 * to far below FP32 resolution. */
#define HS_FP64        0
#define HS_MIXED_FP32  1

typedef int32_t hs_status;
typedef struct hs_ctx hs_ctx;          /* opaque, library-owned */
typedef struct hs_samples hs_samples;  /* opaque, library-owned */

/* Problem description; copied at hs_create.  The spatial scheme is the
 * first-order finite-volume Rusanov flux with backward Euler in time
 * (eq. bdf with s = 1; eq. hdm). */
typedef struct hs_problem {
  int32_t kind;          /* HS_BURGERS_1D / HS_BURGERS_2D / HS_EULER_2D */
  int32_t nx, ny;        /* cells; ny = 1 for HS_BURGERS_1D */
  int32_t bc;            /* HS_BC_* */
  double  dx, dy, dt;    /* dy ignored in 1D */
  double  gamma;         /* ratio of specific heats (Euler) */
  double  inflow;        /* left Dirichlet value (HS_BC_INFLOW_OUTFLOW) */
  double  newton_rtol;   /* stop when ||R||_inf <= newton_rtol * max(1, ||q_prev||_inf); 0 -> 1e-13 */
  int32_t newton_maxit;  /* 0 -> 30 */
  double  lin_rtol;      /* relative accuracy of each Newton correction; 0 -> 1e-10 */
  int32_t lin_maxit;     /* cap on linear sweeps per Newton iteration; 0 -> 400 */
  int32_t m_max;         /* largest basis rank used with this context (<= 64) */
  int32_t w_max;         /* largest window length used with this context (<= 64) */
} hs_problem;

/* Per-call diagnostics, written to HOST memory when the pointer is non-null. */
typedef struct hs_step_info {
  int32_t newton_iters;    /* Newton iterations (summed over subiterations) */
  int32_t lin_sweeps;      /* linear relaxation sweeps (summed) */
  int32_t subiters;        /* J, the number of subiterations (hybrid step) */
  int32_t filter_passes;   /* filter passes over all orders */
  int32_t filter_kept;     /* cells whose filtered value was kept, summed */
  int32_t n_s, l;          /* sampled cells and neighbour cells */
  int32_t fit_rank;        /* rank kept by the truncated pseudo-inverse */
  double  residual_inf;    /* final ||R||_inf of the (restricted) Newton solve */
  double  dy_last;         /* last ||y^(j) - y^(j-1)||_2 */
  double  fit_cond;        /* sigma_max / sigma_min(kept) of the gathered basis */
} hs_step_info;

/* ------------------------------------------------------------ lifetime */
/* Create a context on the current HIP device.  hip_stream may be NULL (the
 * null stream).  Allocates all workspace for the problem size, m_max and
 * w_max. */
hs_status hs_create(const hs_problem* problem /* host */, void* hip_stream, hs_ctx** out /* host */);
hs_status hs_destroy(hs_ctx* ctx);
/* Wait for all work enqueued by this context. */
hs_status hs_sync(hs_ctx* ctx);
const char* hs_status_string(hs_status s);
const char* hs_last_error(const hs_ctx* ctx);

/* -------------------------------------------------------- A1/A2 kernels */
/* R = R_k(q) = q - q_prev + dt * div_h F(q), full mesh (eq. hdm, BDF1). */
hs_status hs_residual(hs_ctx* ctx, const double* q, const double* q_prev, double* R);
/* out = (dR/dq)(q) * v, the exact Jacobian of hs_residual at q. */
hs_status hs_jvp(hs_ctx* ctx, const double* q, const double* v, double* out);

/* ------------------------------------------------------------ hdm_step */
/* Full HDM step: Newton from the guess q_prev until
 * ||R_k(q_out)||_inf <= newton_rtol * max(1, ||q_prev||_inf) (eq. hdm).
 * Each correction solves the exact Jacobian system by (block-)Jacobi
 * relaxation to relative accuracy lin_rtol, with the sweep count set from a
 * computed contraction bound.  Errors: HS_ERR_NOT_CONVERGED,
 * HS_ERR_NONFINITE. */
hs_status hdm_step(hs_ctx* ctx, const double* q_prev, double* q_out, hs_step_info* info /* host, may be NULL */);

/* ------------------------------------------------- the paper's own HDM */
/* Sec. 3.1's full-order scheme on an HS_EULER_2D context (its nx, ny, dx, dy,
 * dt, gamma, newton_rtol, newton_maxit, lin_maxit): MUSCL reconstruction of
 * the primitive variables (rho, u, v, P) with the minmod limiter, slope
 * minmod(w_i - w_{i-1}, w_{i+1} - w_i) and face states w_i +- slope_i / 2;
 * Roe's approximate Riemann solver at every face (no entropy fix); BDF2 in
 * time (eq. bdf, a_0 = 1/3, a_1 = -4/3, a_2 = 1, beta = 2/3), BDF1 when
 * q_prev2 is NULL.  With ny = 1 the scheme is one-dimensional (no y fluxes).
 * Boundaries come with each call and replace the context's bc:
 *   HS_PAPER_BC_FIXED  two ghost layers hold the given conservative states
 *                      (Sec. 3.2: the initial boundary states), ghost[0..3]
 *                      outside the left, right, bottom, top boundary (bottom
 *                      and top ignored when ny = 1); density must be > 0;
 *   HS_PAPER_BC_WALL   reflective walls (Sec. 3.3): the ghosts mirror the
 *                      boundary cells with the normal momentum reversed; needs
 *                      nx >= 2.
 * State layout as everywhere: component-major (rho | rho u | rho v | E), cell
 * i + nx j; all vectors are device pointers of 4 nx ny doubles. */
#define HS_PAPER_BC_FIXED 0
#define HS_PAPER_BC_WALL  1
typedef struct hs_paper_hdm {
  int32_t bc;            /* HS_PAPER_BC_* */
  int32_t reserved;
  double  ghost[4][4];   /* FIXED: (rho, rho u, rho v, E) of the left, right, bottom, top ghosts */
} hs_paper_hdm;
/* R = a_2 q - beta dt f*(q) + a_0 q_prev2 + a_1 q_prev (eq. hdm with BDF2),
 * or q - dt f*(q) - q_prev when q_prev2 is NULL.  R must not alias an input.
 * Errors: HS_ERR_INVALID_ARG (not an Euler context, bad bc or ghosts). */
hs_status hs_paper_residual(hs_ctx* ctx, const hs_paper_hdm* hdm /* host */, const double* q, const double* q_prev,
                            const double* q_prev2 /* may be NULL */, double* R);
/* One step of the paper's scheme: q_out solves R(q_out) = 0 to
 * ||R||_inf <= newton_rtol * max(1, ||q_prev||_inf), from the guess q_prev,
 * by defect correction (each iteration relaxes the first-order Rusanov
 * Jacobian of the step against the second-order residual; at most
 * 4 newton_maxit iterations).  info->newton_iters counts the corrections,
 * info->lin_sweeps their relaxation sweeps.  q_out must not alias an input.
 * Errors: HS_ERR_INVALID_ARG, HS_ERR_NOT_CONVERGED, HS_ERR_NONFINITE (a
 * state without positive density or pressure). */
hs_status hdm_step_bdf2(hs_ctx* ctx, const hs_paper_hdm* hdm /* host */, const double* q_prev,
                        const double* q_prev2 /* may be NULL */, double* q_out, hs_step_info* info /* host, may be NULL */);

/* -------------------------------------------------------- sample_select */
#define HS_RULE_FRACTION 0   /* n_g = min(ceil(fraction * ncell), #{eps > 0}) */
#define HS_RULE_RRE      1   /* smallest n_g with RRE(n_g) >= delta (eq. rre) */

typedef struct hs_sample_params {
  int32_t rule;       /* HS_RULE_* */
  double  fraction;   /* HS_RULE_FRACTION */
  double  delta;      /* HS_RULE_RRE */
  int32_t halo;       /* Chebyshev dilation radius of G (0..8) */
} hs_sample_params;

hs_status hs_samples_create(hs_ctx* ctx, hs_samples** out /* host */);
hs_status hs_samples_destroy(hs_samples* s);
/* From the per-cell indicator eps (ncell doubles, >= 0) build G (the n_g
 * largest, ties to the lower cell index; Sec. 2.3.3), the sampled set
 * hat-S = dilate(G, halo), its face-neighbour ring tilde-S and the
 * complement (Alg. 1: union, setdiff, Neighbors).  The sets are stored in
 * the library-owned object; their sizes are known on return. */
hs_status sample_select(hs_ctx* ctx, const double* eps, const hs_sample_params* params /* host */,
                        hs_samples* out);
/* Set the sampled set directly from a sorted, duplicate-free cell list
 * (hat, n_s entries, device); tilde-S is derived as in sample_select. */
hs_status hs_samples_set(hs_ctx* ctx, hs_samples* s, const int32_t* hat, int32_t n_s);
/* counts[0..2] = n_g, n_s, l (host). */
hs_status hs_samples_counts(const hs_samples* s, int32_t* counts /* host, 3 */);
/* Copy the sorted lists and the mask out (any pointer may be NULL):
 * hat (n_s int32), tilde (l int32), mask (ncell uint8, 1 on hat-S). */
hs_status hs_samples_export(hs_ctx* ctx, const hs_samples* s, int32_t* hat, int32_t* tilde, uint8_t* mask);

/* ---------------------------------------------------- indicator (A4) */
/* eps_j = sum_c (gamma - psi - Phi y)^2 at cell j with y = Phi^T (gamma - psi)
 * (a snapshot known everywhere; Sec. 2.3.3).  Cells whose error norm is below
 * floor_rel * max(1, ||gamma||_inf) get eps = 0.  y_out (m doubles) may be NULL. */
hs_status hs_indicator_full(hs_ctx* ctx, const double* gamma, const void* Phi /* see precision */,
                            const double* psi, int32_t m, double floor_rel, int32_t precision, double* eps,
                            double* y_out);
/* hs_indicator_full for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no context, no allocation, no host synchronisation.  The
 * kernels are hs_indicator_full's (same results to the bit); their working
 * memory (projection partials, the m x m identity, y, the max-|gamma|
 * partials: 386 KiB) is one file-scope device array of the library, which
 * each GPU holds until the process ends.  Every call on a GPU uses that GPU's
 * array, so calls that overlap on one GPU (two streams, two threads) race;
 * consecutive calls on one stream are ordered.  Enqueued on hip_stream (NULL:
 * the null stream); returns after enqueueing.  ncell cells of ncomp (1 or 4)
 * components, gamma/psi/eps/y_out as in hs_indicator_full (device pointers,
 * y_out may be NULL).  HS_ERR_SHAPE: m outside 1..64 or ncomp * ncell >= 2^31
 * (the array's limits); HS_ERR_INVALID_ARG: a NULL pointer, ncomp not 1 or 4,
 * a precision other than HS_FP64 / HS_MIXED_FP32, floor_rel < 0; HS_ERR_HIP:
 * a launch or the array's address lookup failed. */
hs_status hs_indicator_full_noalloc(void* hip_stream, int32_t ncell, int32_t ncomp, const double* gamma,
                                    const void* Phi /* see precision */, const double* psi, int32_t m,
                                    double floor_rel, int32_t precision, double* eps, double* y_out);

/* ------------------------------------------------------ basis_update */
/* snaps: HOST array of nsnap DEVICE pointers to N-vectors, oldest first:
 * gamma_{k-w}..gamma_k (nsnap = w + 1) or gamma_0..gamma_{w-1} (nsnap = w,
 * the first update).  Centring state = mean of the first w snapshots (the
 * lagged reference state psi_k); psi_out = mean of the last w (psi_{k+1},
 * eq. mean).  Phi_out (N x m, column-major) = the first m_eff left singular
 * vectors of X = [snap - centre] over the last w snapshots (eq. pod), with
 * m_eff = #{i < m : sigma_i > tau_pod * sigma_0}; columns beyond m_eff are
 * left untouched.  sigma_out gets all w singular values (descending).
 * Sign: each right singular vector has its largest-magnitude entry positive.
 * The singular values come from a triangular factor of X (two window passes:
 * a Gram-based preconditioner, then the Gram of the preconditioned window),
 * accurate to about eps sigma_0 absolutely, so any tau_pod >= 1e-12 cuts at
 * a reproducible rank; Phi = X V_m diag(1/sigma_m) (third pass) spans the
 * POD subspace to rounding and is orthonormal to about eps sigma_0 / sigma_i.
 * precision: HS_FP64 (Phi_out is double*) or HS_MIXED_FP32 (Phi_out is
 * float*: the FP32 master copy, formed in FP64 and rounded once). */
hs_status basis_update(hs_ctx* ctx, const double* const* snaps /* host */, int32_t nsnap, int32_t w,
                       int32_t m, double tau_pod, int32_t precision,
                       void* Phi_out, double* psi_out, double* sigma_out, int32_t* m_eff /* host */);
/* The same update split in two: basis_update_async enqueues it on a stream
 * of the context's own (ordered after all work enqueued on the context's
 * stream so far) and returns; basis_update_finish waits for it and returns
 * m_eff.  In between, other calls on the context may run (the sampling step
 * of Alg. 1 overlaps the update this way) provided they do not read or write
 * the snapshots, Phi_out, psi_out or sigma_out; a second update, synchronous
 * or not, is rejected until the first is finished. */
hs_status basis_update_async(hs_ctx* ctx, const double* const* snaps /* host */, int32_t nsnap, int32_t w,
                             int32_t m, double tau_pod, int32_t precision, void* Phi_out, double* psi_out,
                             double* sigma_out);
hs_status basis_update_finish(hs_ctx* ctx, int32_t* m_eff /* host */);
/* m_eff of the last completed basis update (synchronous, finished, or
 * completed by a hybrid step given HS_BASIS_PENDING).  Error if an update is
 * still in flight. */
hs_status hs_basis_m_eff(hs_ctx* ctx, int32_t* m_eff /* host */);

/* --------------------------------------------------- rom_hybrid_step */
/* m = HS_BASIS_PENDING: Phi and psi are the outputs of an asynchronous
 * basis_update that is still in flight.  The step runs its first restricted
 * Newton solve (which does not read the basis) beside the update, then
 * completes the update as basis_update_finish would and uses its m_eff
 * (read it back with hs_basis_m_eff; on every return path the update has
 * been completed).  Results are those of finishing the update first. */
#define HS_BASIS_PENDING (-1)
typedef struct hs_hybrid_params {
  double  eps_y;            /* subiteration tolerance (paper: 1e-4) */
  int32_t jmax;             /* max subiterations (paper: 10) */
  int32_t n_orders;         /* number of filter orders applied (0..4) */
  int32_t filter_orders[4]; /* n of S_n = I - (-delta^2/4)^n: 1, 2, 3 = orders 2, 4, 6 */
  double  eps_f;            /* filter stop tolerance on the relative l1 decrease (paper: 1e-2) */
  int32_t jfmax;            /* max passes per filter order (paper: 10) */
  double  rcond_fit;        /* pseudo-inverse cutoff relative to sigma_max (1e-8); the fit
                               factorises the gathered Gram, so the cut is never
                               below sqrt(64 eps) = 1.2e-7 (kappa is reported) */
  double  floor_rel;        /* indicator floor (1e-14) */
  int32_t precision;        /* HS_FP64 (Phi double) or HS_MIXED_FP32 (Phi float) */
} hs_hybrid_params;

/* One hybrid snapshot from q_prev = gamma_{k-1} with basis (Phi, psi; m
 * columns) and the sampled sets s (eq. hybrid).  Writes gamma_k to q_out,
 * the reduced coordinates y^(J) to y_out (m, may be NULL) and the indicator
 * of the filtered snapshot to eps_out (ncell, may be NULL).  Returns before
 * the last kernels have run (see the conventions: outputs complete in
 * stream order).  Errors: HS_ERR_RANK (m = 0 or empty hat-S),
 * HS_ERR_NOT_CONVERGED. */
hs_status rom_hybrid_step(hs_ctx* ctx, const double* q_prev, const void* Phi, const double* psi,
                          int32_t m, const hs_samples* s, const hs_hybrid_params* params /* host */,
                          double* q_out, double* eps_out, double* y_out, hs_step_info* info /* host */);

/* One hybrid snapshot whose subiterations are Gauss-Newton steps on the
 * reduced coordinates (Sec. 2.3.2 with the sampled solution's dependence on
 * the ring values kept): minimise |Phi_S y - (v(y) - psi_S)| where v(y)
 * solves the partial HDM (eq. partial_hdm2) with the ring at psi + Phi y;
 * dv/dy = -J_S^-1 J_T Phi_T (J_S, J_T: the sampled rows of the Jacobian on
 * the sampled and ring columns), so each step takes m relaxed solves with
 * J_S into work and the pseudo-inverse of A^T A, A = Phi_S + J_S^-1 J_T Phi_T.
 * The first iterate is the paper's first subiteration; the loop stops when
 * ||dy||_2 < eps_y or after jmax iterations (info->subiters), and a final
 * partial solve makes the sampled values consistent with the last y.  The
 * reconstruction, filter and indicator are rom_hybrid_step's.  FP64 basis
 * (params->precision = HS_FP64) and the context's first-order scheme.
 * work: device, m N doubles (caller-owned scratch).  Errors as
 * rom_hybrid_step. */
hs_status rom_hybrid_step_gn(hs_ctx* ctx, const double* q_prev, const double* Phi, const double* psi, int32_t m,
                             const hs_samples* s, const hs_hybrid_params* params /* host */, double* work,
                             double* q_out, double* eps_out, double* y_out, hs_step_info* info /* host */);

/* One hybrid snapshot with the paper's own scheme (Sec. 3.1; see
 * hs_paper_hdm): rom_hybrid_step with the BDF residual (q_prev2 =
 * gamma_{k-2}; NULL: BDF1) in the partial solve (eq. partial_hdm2, by the
 * defect correction of hdm_step_bdf2 restricted to hat-S) and in the filter
 * gate.  The residual of a sampled cell reads two cells along each axis, so
 * after every fit every unsampled entry takes psi + Phi y (info->l reports
 * their count).  Needs an HS_EULER_2D context created with
 * HS_BC_TRANSMISSIVE (its filters extrapolate by zeroth order at the
 * boundaries); m >= 1 (no HS_BASIS_PENDING).  fit_points (device, n_fit
 * state entries in sampled cells, e.g. hs_odeim's points): the fit of
 * eq. red_coord uses those rows only (entries outside [0, N) add no row);
 * NULL / 0: every entry of the sampled cells.  Errors as rom_hybrid_step. */
hs_status rom_hybrid_step_bdf2(hs_ctx* ctx, const hs_paper_hdm* hdm /* host */, const double* q_prev,
                               const double* q_prev2 /* may be NULL */, const void* Phi, const double* psi,
                               int32_t m, const hs_samples* s, const int32_t* fit_points /* may be NULL */,
                               int32_t n_fit, const hs_hybrid_params* params /* host */,
                               double* q_out, double* eps_out, double* y_out, hs_step_info* info /* host */);

/* ODEIM points of a basis (eq. odeim): n_p entries of the state vector
 * (indices a ncell + cell into the component-major layout) written to
 * points (device, n_p int32, in the order taken).  The first m are QDEIM's:
 * step j takes the row phi_i of Phi whose component orthogonal to the rows
 * already taken is longest (the pivots of a column-pivoted QR of Phi^T).
 * Each further point maximises the lower bound (g + |phi|^2 - sqrt((g +
 * |phi|^2)^2 - 4 g (u_1^T phi)^2)) / 2 of the increase of the smallest
 * eigenvalue of the sampled Gram Phi_P^T Phi_P (l_1 <= l_2 its two smallest
 * eigenvalues, u_1 the eigenvector of l_1, g = l_2 - l_1; (u_1^T phi)^2 when
 * m = 1).  Ties go to the lowest index.  Phi: FP64, column-major (column j at
 * Phi + j N), orthonormal columns.  1 <= m <= min(16, m_max), m <= n_p <= N.
 * Uses the context's scratch (no call of the context may overlap).  Errors:
 * HS_ERR_INVALID_ARG. */
hs_status hs_odeim(hs_ctx* ctx, const double* Phi, int32_t m, int32_t n_p, int32_t* points);
/* Adds the cells of n_p state entries (as hs_odeim returns them) to the
 * sampled set s (Sec. 2.3.3: hat-S = G u P) and rebuilds its ring, lists and
 * neighbour table; n_g is kept; entries outside [0, N) are ignored.  The fit rows of rom_hybrid_step_bdf2 must
 * lie in sampled cells: pass the same points as its fit_points. */
hs_status hs_samples_add_points(hs_ctx* ctx, hs_samples* s, const int32_t* points, int32_t n_p);

/* rom_hybrid_step whose fit (eq. red_coord) uses the given n_fit state
 * entries (device int32, in sampled cells: e.g. hs_odeim's points after
 * hs_samples_add_points) instead of every entry of the sampled cells;
 * entries outside [0, N) add no row.  n_fit = 0 is rom_hybrid_step. */
hs_status rom_hybrid_step_fit(hs_ctx* ctx, const double* q_prev, const void* Phi, const double* psi, int32_t m,
                              const hs_samples* s, const int32_t* fit_points, int32_t n_fit,
                              const hs_hybrid_params* params /* host */, double* q_out, double* eps_out,
                              double* y_out, hs_step_info* info /* host */);

/* The residual-gated filter sequence alone (Sec. 2.3.4), on a full state. */
hs_status hs_filter(hs_ctx* ctx, const double* gamma_in, const double* q_prev,
                    const hs_hybrid_params* params /* host */, double* gamma_out, hs_step_info* info);

/* --------------------------------------------- adjoint (frozen decisions) */
/* The adjoint differentiates the trajectory map with every decision of the
 * forward run frozen: the step schedule, the sampled sets, the subiteration
 * count J, the filter masks and the bases (Phi_k, psi_k).  A hybrid step's
 * decisions are kept in a library-owned tape. */
typedef struct hs_htape hs_htape;
#define HS_TAPE_RECORD 0   /* normal hybrid step; copy its decisions into the tape */
#define HS_TAPE_REPLAY 1   /* rerun with the tape's decisions; record its internal states */

hs_status hs_htape_create(hs_ctx* ctx, hs_htape** out /* host */);
hs_status hs_htape_destroy(hs_htape* tape);
/* Inspect a recorded tape: J, the number of applied filter passes and their
 * orders (passes: host array of at least 64 entries, may be NULL) and their
 * kept-cell masks (device, npass x ncell bytes, may be NULL). */
hs_status hs_htape_info(const hs_htape* tape, int32_t* J /* host */, int32_t* npass /* host */,
                        int32_t* passes /* host */, uint8_t* masks /* device */);
/* The sampled set a tape holds (borrowed: owned and freed by the tape). */
hs_status hs_htape_samples(hs_htape* tape, hs_samples** out /* host */);
/* rom_hybrid_step with a tape.  HS_TAPE_RECORD: as rom_hybrid_step (s are the
 * sets to use), and the tape keeps a copy of the sampled set, J and every
 * applied filter pass (order and kept-cell mask).  HS_TAPE_REPLAY: s is
 * ignored; the step runs exactly the tape's J subiterations on its sets and
 * applies its filter passes and masks without gating, recording the state
 * after each subiteration's Newton solve and the fit's pseudo-inverse.  With
 * the same q_prev, Phi, psi and m, a replay reproduces the recorded output. */
hs_status rom_hybrid_step_taped(hs_ctx* ctx, const double* q_prev, const void* Phi, const double* psi,
                                int32_t m, const hs_samples* s, const hs_hybrid_params* params /* host */,
                                double* q_out, double* eps_out, hs_step_info* info /* host */,
                                hs_htape* tape, int32_t mode);
/* lam_out = (d gamma_k / d gamma_{k-1})^T lam_in for a full step whose output
 * is q_out: solves J(q_out)^T lam_out = lam_in (eq. hdm: dR/dq_prev = -I) by
 * transposed block-Jacobi relaxation to relative accuracy 1e-12. */
hs_status hdm_step_adjoint(hs_ctx* ctx, const double* q_out, const double* lam_in, double* lam_out,
                           hs_step_info* info /* host, may be NULL */);
/* lam_out = (d gamma_k / d gamma_{k-1})^T lam_in for a hybrid step replayed
 * into tape (HS_TAPE_REPLAY) with basis Phi (m columns, FP64 only).  Reverse order of the
 * forward: transposed filter passes, Phi^T on the unsampled rows, then per
 * subiteration (last first) Phi^T on the ring, the pseudo-inverse transpose,
 * a transposed restricted Newton-matrix solve and the coupling to the ring. */
hs_status rom_hybrid_step_adjoint(hs_ctx* ctx, const double* Phi, int32_t m, const hs_htape* tape,
                                  const double* lam_in, double* lam_out, hs_step_info* info /* host */);
/* The same adjoint, and with lam_psi (device, N; nullptr: not formed) also
 * (d gamma_k / d psi_k)^T lam_in, the adjoint with respect to the step's
 * reference state (eq. mean): the step is linear in psi, which enters the
 * ring values psi + Phi y of every subiteration, the fit
 * (P^T Phi)^+ P^T (v - psi) (eq. red_coord) and the reconstruction psi + Phi y
 * off the sampled cells (eq. rom_approx).  lam_psi must not alias lam_in or
 * lam_out. */
hs_status rom_hybrid_step_adjoint_psi(hs_ctx* ctx, const double* Phi, int32_t m, const hs_htape* tape,
                                      const double* lam_in, double* lam_out, double* lam_psi,
                                      hs_step_info* info /* host */);

/* -------------------------------------------- trajectory and its adjoint */
/* A whole run of Algorithm 1 and the frozen-decision adjoint of its map
 * gamma_0 -> gamma_T (Alg. 1; eq. hdm for full steps, eq. hybrid with the
 * subiterations of Sec. 2.3.2 and the gated filters of Sec. 2.3.4 for hybrid
 * steps).  Schedule: full steps for k + 1 <= w, k mod z == 0 and wherever no
 * sampled set or basis exists; a hybrid step that fails with
 * HS_ERR_NOT_CONVERGED or HS_ERR_RANK is redone as a full step.  After step
 * k (k >= w - 1, step k + 1 not full, k < steps) the indicator of gamma_k
 * selects the sampled set of step k + 1 (sample_select with `sample`) and the
 * basis and reference state are rebuilt from the last w + 1 snapshots
 * (basis_update with m, tau_pod). */
typedef struct hs_traj_params {
  int32_t steps;              /* N_t >= 1 */
  int32_t checkpoint_every;   /* K >= 1: a checkpoint of gamma every K steps */
  int32_t w, m, z;            /* window length, POD rank, full-step period */
  double  tau_pod;            /* POD cut (1e-8) */
  hs_sample_params sample;    /* selection rule, fraction / delta, halo */
  hs_hybrid_params hybrid;    /* hybrid step parameters; precision must be HS_FP64 */
  int32_t psi_adjoint;        /* hs_traj_backward: 0: psi_k frozen like the bases; 1: also through
                                 psi_k, the mean of the w snapshots its basis update averages (eq. mean) */
} hs_traj_params;
/* Library-owned record of one forward run: per step its kind, the basis it
 * used and its hybrid-step tape; every basis; the checkpoints.  Its device
 * memory grows with the run: one N x m basis per update, a tape per hybrid
 * step, a state per checkpoint (freed by the next hs_traj_forward on the
 * same tape or by hs_tape_destroy). */
typedef struct hs_tape hs_tape;
hs_status hs_tape_create(hs_ctx* ctx, hs_tape** out /* host */);
hs_status hs_tape_destroy(hs_tape* tape);
/* Run Alg. 1 from q0 (device, N) for params->steps steps, recording into
 * tape; qT (device, N) = gamma_T.  Synchronous.  Errors: those of the calls
 * it makes (a failed full step ends the run with its error). */
hs_status hs_traj_forward(hs_ctx* ctx, const double* q0, const hs_traj_params* params /* host */,
                          hs_tape* tape, double* qT);
/* lam_0 = (d gamma_T / d gamma_0)^T lam_T with every decision of the
 * recorded run frozen (device, N each; may alias).  Segments of K steps, last
 * first: replayed from their checkpoints (full steps re-solved, hybrid steps
 * in HS_TAPE_REPLAY mode), the replayed end state checked against the next
 * checkpoint bit for bit (HS_ERR_INVALID_ARG if it differs: the inputs or a
 * basis changed), then hdm_step_adjoint / rom_hybrid_step_adjoint in reverse.
 * Synchronous. */
hs_status hs_traj_backward(hs_ctx* ctx, hs_tape* tape, const double* lam_T, double* lam_0);
/* The recorded run, step k (1..steps): kind (0 full, 1 hybrid), the index
 * of the basis a hybrid step used (-1 otherwise) and its hybrid-step tape
 * (borrowed, NULL for a full step); any pointer may be NULL. */
hs_status hs_tape_step(const hs_tape* tape, int32_t k, int32_t* kind /* host */, int32_t* basis /* host */,
                       hs_htape** htape /* host */);
/* Copy basis `basis` out: Phi (device, N x m, column-major), psi (device, N),
 * m (host); any of them may be NULL. */
hs_status hs_tape_basis(hs_ctx* ctx, const hs_tape* tape, int32_t basis, double* Phi_out, double* psi_out,
                        int32_t* m);
/* Copy the checkpoint of step k (0 and every multiple of K, and steps) out. */
hs_status hs_tape_checkpoint(hs_ctx* ctx, const hs_tape* tape, int32_t k, double* q_out);

/* ----------------------------------------------------------- options */
/* HS_OPT_TILED_SWEEPS: how the relaxation sweeps run.  0: one sweep per
 * launch over the compact cell list; 1 (default): LDS tiles, several sweeps
 * per launch, for scalar problems where the tiles are dense enough to pay,
 * else the list (Euler's 4x4 blocks always use the list); 2: tiles wherever
 * the tile list fits the statistics capacity.  All give the same iterates bit
 * for bit (a switch for measurement and testing). */
#define HS_OPT_TILED_SWEEPS 1
/* HS_OPT_SMALL_PINV: the fit's truncated pseudo-inverse (eq. red_coord) for
 * m <= 8 basis columns.  1 (default): one wavefront with the matrix in
 * registers; 0: the general LDS routine used for every m.  Both take the same
 * Jacobi rotations in the same order and give the same result bit for bit (a
 * switch for measurement and testing). */
#define HS_OPT_SMALL_PINV 2
/* HS_OPT_FIT_CHOLESKY: for m > 8 the fit's pseudo-inverse is the inverse
 * from a Cholesky factorisation of the gathered Gram whenever a bound on its
 * condition (||G||_F ||G^-1||_F < 1e6) shows that no direction is cut
 * (1, default); 0: always the Jacobi eigendecomposition. */
#define HS_OPT_FIT_CHOLESKY 3
/* Returns HS_ERR_INVALID_ARG for an unknown option or a value out of range. */
hs_status hs_set_option(hs_ctx* ctx, int32_t option, int64_t value);

/* ------------------------------------------------------- measurement */
/* Kernel classes that can be timed with HIP events on the context's stream. */
#define HS_PROF_NONE        0
#define HS_PROF_BASIS_GRAM  1   /* window pass of basis_update: means + Gram on MFMA */
#define HS_PROF_BASIS_FORM  2   /* formation pass of basis_update: Phi = X T on MFMA */
#define HS_PROF_RECON       3   /* reconstruction psi + Phi y (hybrid step) */
#define HS_PROF_RESJAC      4   /* residual + Jacobian relaxation data (Newton) */
#define HS_PROF_SWEEP       5   /* Jacobi relaxation sweeps */
#define HS_PROF_CELLRES     6   /* cell residual norms (filter) */
#define HS_PROF_FILTER      7   /* fused filter pass: S_y S_x, gate, merged residual norms */
#define HS_PROF_RESIDUAL    8   /* hs_residual: R(q; q_prev) on the full mesh */
#define HS_PROF_BASIS_PGRAM 9   /* second window pass of basis_update: Gram of the preconditioned window */
#define HS_PROF_STREAM      10  /* hs_stream_add: the plain streaming reference */
/* Start timing every launch of one kernel class (HS_PROF_NONE stops).  Each
 * launch is bracketed by two HIP events recorded on the context's stream, and
 * the algorithmic bytes of that launch (the minimum reads and writes the
 * operation needs) are accumulated. */
hs_status hs_prof_enable(hs_ctx* ctx, int32_t kernel_class);
/* Synchronise, return the summed event time (ms), launch count and
 * algorithmic bytes since enable or the last read, and reset the counters. */
hs_status hs_prof_read(hs_ctx* ctx, double* total_ms /* host */, int32_t* launches /* host */,
                       double* bytes /* host */);

/* A plain streaming kernel, c = a + b over n doubles (device; reads 16 n
 * bytes, writes 8 n, one element per thread): what a launch with the full-mesh
 * residual's traffic reaches on this device at all, the reference beside which
 * the residual kernels' HBM rates are read.  Not part of the method.  c may
 * alias neither input; n <= 2^38.  Errors: HS_ERR_INVALID_ARG. */
hs_status hs_stream_add(hs_ctx* ctx, const double* a, const double* b, double* c, int64_t n);

#ifdef __cplusplus
}
#endif
#endif /* HSROM_H */
