/*
 * pmx.h -- C ABI of the MI355X parametrix surface-PDE library.
 *
 * Solves div_G(a grad_G u) = f on a smooth closed surface G (the c = 0, b = 0
 * case of the surface PDE in the paper's introduction, eq:surf_PDE) through
 * the second-kind integral equation of the parametrix method (eq:IE):
 *
 *     sigma(x) + int_G R(x, x') sigma(x') da(x') + int_G sigma = f(x),
 *     u(x) = int_G K(x, x') sigma(x') da(x')  - its mean,
 *
 * with K(x, x') = log|x - x'| / (2 pi a(x')) (Section 4.1, eq:diff_param) and
 * the remainder R of eq:explicit_remainder; the rank-one term int_G sigma
 * removes the one-dimensional null space (Section 3).  The system is
 * discretized by the Nystrom method on quad patches with tensor
 * Gauss-Legendre nodes (Section 6.1), with singular (Section 6.1.1),
 * nearly singular (Section 6.1.2) and smooth (Section 6.1.3) quadrature.
 *
 * Conventions
 *  - Every function returns a pmx_status (0 = OK, < 0 = error) and never
 *    throws; pmx_last_error() returns a message for the calling thread.
 *  - Ownership: the caller owns every array it passes.  The library copies
 *    inputs during *_create, so they may be freed on return.  Handles are
 *    owned by the library and released by *_destroy (NULL-safe).
 *  - mem_kind says where caller arrays live: PMX_MEM_HOST (pageable or pinned
 *    host memory) or PMX_MEM_DEVICE (device memory of the context's GPU).
 *  - stream: a hipStream_t (may be NULL = the null stream).  All device work
 *    of a call is enqueued on it; calls with host outputs return after the
 *    results are copied out.
 *  - Threads: calls on one operator (or one server) must not overlap; calls on
 *    different operators may run at once from different threads, on their own
 *    streams.  Contexts and surfaces may be shared by such threads.
 *  - Node order: node i = P*q*q + iu*q + iv sits at the Gauss-Legendre pair
 *    (t_iu, t_iv) of patch P on [-1,1]^2.  Arrays of 3-vectors are row-major
 *    N x 3.  Multi-RHS arrays are n_rhs contiguous vectors of length N
 *    (element r*N + i).
 */
#ifndef PMX_H
#define PMX_H

#include <stdint.h>

#if defined(__GNUC__)
#define PMX_API __attribute__((visibility("default")))
#else
#define PMX_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pmx_status;
typedef struct pmx_ctx pmx_ctx;
typedef struct pmx_surface pmx_surface;
typedef struct pmx_operator pmx_operator;
typedef struct pmx_server pmx_server;
typedef struct pmx_edge pmx_edge;

enum {
  PMX_OK = 0,
  PMX_PENDING = 1,
  PMX_ERR_INVALID = -1,        /* bad argument: shape, q < 2, a <= 0, non-finite data */
  PMX_ERR_OOM = -2,            /* device allocation failed */
  PMX_ERR_TOO_LARGE = -3,      /* footprint over the context's HBM budget */
  PMX_ERR_NOT_CONVERGED = -4,  /* iteration limit reached; best iterate written */
  PMX_ERR_ORIENTATION = -5,    /* surface normals point inward (sum w n.x <= 0) */
  PMX_ERR_DEVICE = -6,         /* HIP runtime error */
  PMX_ERR_CANCELLED = -7
};

enum { PMX_MEM_HOST = 0, PMX_MEM_DEVICE = 1 };

/* Far-field evaluation of the apply. */
enum {
  PMX_PREC_FP64_DIRECT = 0,  /* FP64 direct sum over all pairs (the reference operator A64) */
  PMX_PREC_MIXED_FMM = 1,    /* FP32 interpolation FMM far field, FP64 near field (A32) */
  PMX_PREC_FP32_DIRECT = 2   /* FP32 direct sum, FP64 near field */
};

typedef struct pmx_options {
  double eta_near;     /* near criterion: within eta patch radii of the centroid (Section 6.1.2: 1.5) */
  int n_gl;            /* Gauss-Legendre order of the local rules (Section 6.1.1: 16) */
  int fmm_order;       /* Chebyshev points per box edge of the FMM: 4, 5 or 6 (default 6) */
  int fmm_leaf;        /* mean points per FMM leaf box: the leaf level is the first with at most this (default 256) */
  double gmres_tol;    /* relative residual target of GMRES (FP64 path) */
  int gmres_restart;   /* Krylov space size before restart */
  int max_iter;        /* total GMRES iteration limit */
  double ir_tol;       /* mixed path: final relative residual (FP64 operator) */
  double inner_tol;    /* mixed path: relative residual of each inner GMRES */
  int max_ir;          /* mixed path: outer refinement step limit */
  int precision;       /* PMX_PREC_* used by pmx_solve */
  int overlap;         /* mixed applies: 1 = run the near correction and the P2P sums on a second
                          stream of the operator, overlapping the FMM's M2L chain (default);
                          0 = every kernel on the caller's stream */
} pmx_options;

typedef struct pmx_info {
  int iters_total;       /* GMRES iterations (all inner solves) */
  int ir_steps;          /* outer refinement steps (mixed path), 0 otherwise */
  int applies_fp64;      /* FP64 operator applies */
  int applies_low;       /* FP32-far-field operator applies */
  double rel_residual;   /* ||f - A64 sigma|| / ||f|| (2-norm of the Nystrom system) */
  double removed_mean;   /* weighted mean removed from f (c = 0 needs mean-zero data) */
  double t_setup;        /* seconds spent in operator setup */
  double t_solve;        /* seconds spent in the solve */
} pmx_info;

typedef struct pmx_operator_stats {
  int64_t n_nodes;
  int64_t n_patches;
  int32_t q;
  int32_t fmm_levels;     /* 0 until the FMM tree is built */
  int64_t near_pairs;     /* (target, patch) pairs with local-rule correction blocks */
  int64_t fmm_boxes;
  int64_t fmm_m2l_pairs;
  int64_t fmm_p2p_pairs;  /* source-target point pairs handled directly by the FMM */
  uint64_t device_bytes;  /* device memory held by the operator */
} pmx_operator_stats;

/* Context on one GPU.  hbm_budget_bytes bounds what the context's operators and
 * server may hold (0 = no bound).  Errors: INVALID (no such device), DEVICE.
 * Handle lifetimes: a surface holds a reference on its context, an operator on its surface
 * and a server on its context, so the destroy calls may come in any order (a garbage
 * collector's, say): a context or surface is freed once it has been destroyed and the last
 * handle made from it is gone.  Each handle is destroyed once; destroy calls are NULL-safe. */
PMX_API pmx_status pmx_ctx_create(int device, uint64_t hbm_budget_bytes, pmx_ctx** out);
PMX_API void pmx_ctx_destroy(pmx_ctx* ctx);
/* Message of the last error on the calling thread ("" if none). */
PMX_API const char* pmx_last_error(void);
/* Defaults: eta 1.5, n_gl 16, fmm_order 6, fmm_leaf 256, gmres_tol 1e-10, restart 60,
 * max_iter 400, ir_tol 1e-8, inner_tol 1e-4, max_ir 20, precision FP64_DIRECT. */
PMX_API void pmx_default_options(pmx_options* opts);

/* Surface from node data (Section 6.1: patches y_P(u, v) on [-1,1]^2): position x and
 * the parameter derivatives x_u, x_v, x_uu, x_uv, x_vv at the N = n_patches*q*q nodes.
 * Computes normals, area elements, weights, mean curvature (Section 2.2), patch
 * centroids and radii (Section 6.1.2).  Errors: INVALID (q < 2 or q > 16, n_patches < 1,
 * non-finite data, degenerate metric), ORIENTATION (inward normals), OOM, DEVICE. */
PMX_API pmx_status pmx_surface_create(pmx_ctx* ctx, int n_patches, int q, const double* x, const double* xu,
                              const double* xv, const double* xuu, const double* xuv, const double* xvv,
                              int mem_kind, void* stream, pmx_surface** out);
PMX_API void pmx_surface_destroy(pmx_surface* s);

/* Operator for the coefficient a > 0 at the nodes (N) with its ambient or surface
 * gradient (N x 3; the tangential part is used, Section 4.1).  Builds near lists and
 * the FP64 correction blocks of the self and near rules (Sections 6.1.1, 6.1.2).
 * opts may be NULL (defaults).  The operator holds a reference on the surface.
 * Errors: INVALID (a <= 0 or non-finite), TOO_LARGE (budget), OOM, DEVICE. */
PMX_API pmx_status pmx_operator_create(pmx_surface* s, const double* a, const double* grad_a, const pmx_options* opts,
                               int mem_kind, void* stream, pmx_operator** out);
/* Operator of the general surface PDE div_G(a grad_G u) + b . grad_G u + c u = f (eq:surf_PDE) for a
 * coefficient c of one sign at every node (N values): c < 0, the modified Helmholtz-Beltrami type, or
 * c > 0, the Helmholtz-Beltrami type (Section 4.1, Section 7.3), and an optional advection field b
 * (3N values, node i's vector at b[3i..3i+2] as for grad_a, ambient components; its tangential part
 * is used; NULL: b = 0).  The parametrix is G(r; a, c) = -(i / 4a) H0(sqrt(c/a) r) with the
 * coefficients at the source (eq:diff_param; the printed Hankel form read with the sign for which
 * (a Delta + c) G = delta): for c < 0 the real -K0(sqrt(-c/a) r) / (2 pi a), for c > 0 complex
 * (H0 = J0 + i Y0, the Hankel function of the first kind).  The remainder is eq:explicit_remainder
 * with its c-term, plus b . grad_G K with b (eq:adv_remainder; the system is then eq:IE_adv).  b is
 * taken with c != 0 only: with c = 0 the solvability condition on f is not a zero mean once b != 0.
 * With c != 0 the problem has no null space: the system is sigma + R sigma = f (Theorem
 * thm:second_kind, no rank-one term), f is used as given (info.removed_mean = 0) and u = K sigma is
 * not shifted.
 * With c > 0 the operator is complex (pmx_operator_is_complex): every vector that pmx_apply, pmx_solve
 * and pmx_represent take or return holds 2N doubles per right-hand side, the real parts of the N node
 * values followed by their imaginary parts (n_rhs counts complex vectors; right-hand side r starts
 * at offset 2 r N); GMRES runs in complex arithmetic, and info has n_rhs entries.
 * Only the FP64 direct far field is available (PMX_PREC_FP64_DIRECT for pmx_apply, pmx_solve and
 * the allocation-free apply; other precisions give INVALID): the FMM's translation operators need a
 * kernel of x - y alone up to a per-source factor, while here the wavenumber sqrt(|c|/a) changes from
 * source to source.  Arguments as for pmx_operator_create, plus c (N) and b (3N or NULL), both in
 * mem_kind memory and read during the call only.
 * Errors: INVALID (c null, c zero or non-finite at some node, c of both signs, b non-finite, and as
 * pmx_operator_create), TOO_LARGE, OOM, DEVICE. */
PMX_API pmx_status pmx_operator_create_c(pmx_surface* s, const double* a, const double* grad_a, const double* c,
                                 const double* b, const pmx_options* opts, int mem_kind, void* stream,
                                 pmx_operator** out);
PMX_API void pmx_operator_destroy(pmx_operator* op);
PMX_API pmx_status pmx_operator_get_stats(pmx_operator* op, pmx_operator_stats* out);

/* y = A sigma for n_rhs densities (eq:IE discretized, with the rank-one term):
 * y_i = sigma_i + sum_{j != i} w_j R(x_i, x_j) sigma_j + sum_{P near i} C_{i,P,:} sigma_P
 *       + sum_j w_j sigma_j.  precision selects the far-field evaluation (PMX_PREC_*).
 * sigma and y: n_rhs rows of N doubles (row r at offset r N).  The first mixed apply of an
 * operator builds its FMM tree, and the first with a larger n_rhs sizes its multi-rhs buffers
 * (with n_rhs >= 8 also a by-patch view of the near lists, built on the host); these first
 * calls allocate device memory and synchronize the stream, later ones with the same or a smaller
 * n_rhs only enqueue work.  Mixed applies use the operator's second stream (pmx_options.overlap).
 * Errors: INVALID, OOM, DEVICE. */
PMX_API pmx_status pmx_apply(pmx_operator* op, int precision, int n_rhs, const double* sigma, double* y, int mem_kind,
                     void* stream);

/* Allocation-free y = A sigma with the FP64 direct far field: the same result, bit for bit,
 * as pmx_apply(op, PMX_PREC_FP64_DIRECT, n_rhs, sigma, y, PMX_MEM_DEVICE, stream).
 * For callers that cannot allocate device memory: code under HIP graph capture, serving loops
 * and harnesses that forbid hipMalloc.  It calls no hipMalloc, hipFree or allocating library
 * routine and does not synchronize; its scratch (source strengths, packed source rows, partial
 * sums) lives in one static device array of PMX_NOALLOC_SCRATCH_BYTES per GPU, which the
 * library holds until the process ends.  Every buffer of that scratch is written before it is
 * read, so nothing needs clearing between calls, and results do not depend on earlier calls.
 * Calls that overlap on one GPU (from two threads, or on two streams) share the array and race:
 * the caller must order them.  sigma and y: device arrays of the operator's GPU, n_rhs rows of
 * N doubles; the operator must be a fully built one (pmx_operator_create returned OK).
 * Scratch needed: about 8 (n_rhs (N (1 + c) + N / 256) + N (3 + g + 1)) bytes, with c the
 * direct sum's source chunks (between 1 and 64: 7 for 153,600 nodes, 1 from 1,048,576) and g the
 * largest right-hand-side group (1, 2, 4, 8 or 16); for example up to 4 densities at 153,600 nodes.
 * A complex operator (c > 0) takes n_rhs complex densities, 2N doubles each (real parts, then
 * imaginary parts, as for pmx_apply), and needs the scratch of 2 n_rhs real columns.
 * Errors: INVALID (null or host arrays, n_rhs out of range), TOO_LARGE (scratch above the maximum),
 * DEVICE. */
#define PMX_NOALLOC_SCRATCH_BYTES (64ull << 20)
PMX_API pmx_status pmx_apply_noalloc(pmx_operator* op, int n_rhs, const double* sigma, double* y, void* stream);

/* Solve A sigma = f - mean_w(f) for n_rhs right-hand sides.  opts->precision (or the
 * operator's options when opts is NULL) selects GMRES on A64 (FP64 path) or iterative
 * refinement with residuals on A64 and inner GMRES on A32 (mixed path).  sigma: in =
 * warm start (pass sigma_in_is_guess = 1) or ignored, out = solution.  u (nullable):
 * the mean-zero representation K[sigma] (eq:representation).  info (nullable): n_rhs
 * entries.  Errors: INVALID, NOT_CONVERGED (best iterate written, info filled), OOM, DEVICE. */
PMX_API pmx_status pmx_solve(pmx_operator* op, const pmx_options* opts, int n_rhs, const double* f, double* sigma,
                     int sigma_in_is_guess, double* u, int mem_kind, void* stream, pmx_info* info);

/* u = K[sigma] - mean_w(K[sigma]) (eq:representation), FP64.  Builds the parametrix
 * correction blocks on first use.  Errors: INVALID, OOM, DEVICE. */
PMX_API pmx_status pmx_represent(pmx_operator* op, int n_rhs, const double* sigma, double* u, int mem_kind, void* stream);

/* ---- Continuous-batching solve server (many independent problems of eq:IE) ----
 * Requests queue in arrival order; pmx_server_step admits them while fewer than
 * max_active run and their device footprints fit the context's HBM budget: a request counts
 * with its footprint estimated at submit until it has built its operator, then with its
 * measured footprint if that is larger.  The budget acts at admission only; a running request
 * allocates from its own accounting and is never failed because others are larger than
 * estimated.
 * Each admitted request gets its own stream and worker thread, builds its surface and
 * operator on the device, solves with opts->precision (NULL opts: defaults with the
 * mixed path), and releases its device memory; active requests run concurrently.
 * The operator applies of all solving requests are batched: every kernel of the apply
 * path is launched once for all requests that have an apply pending (one argument
 * record per request), on the server's own stream.  A request that finishes setup
 * joins the next batch.  No call blocks on another request's work.  All input arrays
 * are host memory and are copied by submit. */
PMX_API pmx_status pmx_server_create(pmx_ctx* ctx, const pmx_options* opts, int max_active, pmx_server** out);
/* Queue one problem (same node layout as pmx_surface_create; a, grad_a, f as in
 * pmx_operator_create and pmx_solve with n_rhs = 1).  want_u: also compute u.
 * Errors: INVALID, TOO_LARGE (estimated footprint above the budget even when idle). */
PMX_API pmx_status pmx_server_submit(pmx_server* sv, int n_patches, int q, const double* x, const double* xu,
                                     const double* xv, const double* xuu, const double* xuv, const double* xvv,
                                     const double* a, const double* grad_a, const double* f, int want_u,
                                     uint64_t* ticket);
/* Retire finished requests and admit queued ones; reports active and queued counts. */
PMX_API pmx_status pmx_server_step(pmx_server* sv, int* n_active, int* n_queued);
/* PMX_PENDING while queued or running.  When finished: copies sigma (N) and u (N, if
 * requested; either pointer may be NULL), info, and times[3] = seconds queued, in service,
 * and submit-to-done; returns the request's status (OK, NOT_CONVERGED with the best
 * iterate, CANCELLED, ...) and forgets the ticket.  Unknown ticket: INVALID. */
PMX_API pmx_status pmx_server_poll(pmx_server* sv, uint64_t ticket, double* sigma, double* u, pmx_info* info,
                                   double* times);
/* Cancel a queued or running request (its poll then returns CANCELLED). */
PMX_API pmx_status pmx_server_cancel(pmx_server* sv, uint64_t ticket);
/* Cancels running requests, waits for their workers, frees the server (NULL-safe). */
PMX_API void pmx_server_destroy(pmx_server* sv);
/* Counters since creation: number of shared launches of the apply path (batches), applies
 * they carried, the largest batch, requests that stayed queued for memory while a slot was free
 * (admission by the HBM budget), and the largest estimated footprint admitted at once.  Any
 * pointer may be NULL. */
PMX_API pmx_status pmx_server_get_stats(pmx_server* sv, uint64_t* n_batches, uint64_t* n_applies,
                                        uint64_t* max_batch, uint64_t* n_held_for_memory,
                                        uint64_t* peak_reserved_bytes);

/* Per-phase device timing of the apply (HIP events recorded on the call's stream around
 * each phase while enabled).  Phases: PMX_PHASE_*.  pmx_profile_read synchronizes the
 * recorded events and returns, per phase, the summed milliseconds and the number of
 * timed launches; reading resets the accumulators.  Errors: INVALID, DEVICE. */
enum {
  PMX_PHASE_PREP = 0,        /* qt = w sigma / a and sum w sigma */
  PMX_PHASE_DIRECT64 = 1,    /* FP64 direct far-field kernel */
  PMX_PHASE_DIRECT32 = 2,    /* FP32 direct far-field kernel */
  PMX_PHASE_NEAR = 3,        /* near correction + combine */
  PMX_PHASE_FMM_P2M = 4,
  PMX_PHASE_FMM_M2M = 5,
  PMX_PHASE_FMM_M2L = 6,     /* M2L translations (MFMA), one output slot per pair */
  PMX_PHASE_FMM_L2L = 7,
  PMX_PHASE_FMM_L2P = 8,
  PMX_PHASE_FMM_P2P = 9,
  PMX_PHASE_LOG = 10,        /* representation far field */
  PMX_PHASE_FMM_M2L_SUM = 11,  /* sum of each box's M2L output slots */
  PMX_PHASE_EDGE = 12,       /* edge-operator pair sums (pmx_edge_apply) */
  PMX_N_PHASES = 13
};
PMX_API pmx_status pmx_profile_enable(pmx_operator* op, int enable);
PMX_API pmx_status pmx_profile_read(pmx_operator* op, double* ms /* PMX_N_PHASES */, int64_t* count /* PMX_N_PHASES */);

/* Copy-out of operator internals to host arrays (any pointer may be NULL):
 * node normal n (N x 3), mean curvature H (N), weight w (N), surface gradient of a (N x 3). */
PMX_API pmx_status pmx_operator_export_geometry(pmx_operator* op, double* n, double* H, double* w, double* grad_s_a);
/* Near lists in CSR form by target (ptr: N + 1, patch: near_pairs, sorted per target) and
 * the FP64 correction blocks C (near_pairs x q*q; D for the parametrix, NULL to skip). */
PMX_API pmx_status pmx_operator_export_near(pmx_operator* op, int64_t* ptr, int32_t* patch, double* C, double* D);
/* Complex operators (c > 0): the imaginary parts of the correction blocks C and D, in the layout of
 * pmx_operator_export_near (which returns the real parts).  Either pointer may be NULL.
 * Errors: INVALID (null handle, a real operator), DEVICE. */
PMX_API pmx_status pmx_operator_export_near_imag(pmx_operator* op, double* Ci, double* Di);
/* *out = 1 for a complex operator (built with c > 0: vectors of 2N doubles), 0 otherwise.
 * Errors: INVALID (null argument). */
PMX_API pmx_status pmx_operator_is_complex(pmx_operator* op, int* out);

/* ---------------------------------------------------------------- open surfaces: edge operators
 * Section 5 solves the problem on an open surface Gamma with Neumann or Dirichlet data on its
 * boundary gamma through a second density mu on gamma.  Four operators map mu to the surface nodes:
 *   PMX_EDGE_K: K_gamma[mu](x) = int_gamma K(x, x') mu ds          (eq:BC_rep, the Neumann u)
 *   PMX_EDGE_N: N_gamma[mu](x) = int_gamma nu . grad'_G K mu ds     (eq:DirichletRep, the Dirichlet u)
 *   PMX_EDGE_R: R_gamma[mu](x) = int_gamma R(x, x') mu ds          (eq:NeuBVPsystem, Lemma lem:surf_term)
 *   PMX_EDGE_T: T_gamma[mu](x) = int_gamma nu . grad'_G R mu ds     (eq:DirBVPsystem, Lemma lem:Dirichlet_surf_term)
 * nu is the unit conormal at x' (tangent to Gamma, normal to gamma, out of Gamma); the primed gradient
 * acts on the source point x', through r = x - x' and through a(x') in K(x, x') = log r / (2 pi a(x')).
 * Discretization (Section 6.1.4): every quantity sampled on a curve is replaced by its trigonometric
 * interpolant at m times as many equispaced points, and the trapezoid rule runs there.  Only the
 * c = 0 operators (variable a, no advection) are provided. */
enum { PMX_EDGE_K = 0, PMX_EDGE_N = 1, PMX_EDGE_R = 2, PMX_EDGE_T = 3 };

/* Boundary curves for the edge operators.  n_curves (1..64) closed curves, curve k sampled at
 * n_samples[k] (>= 3) equispaced values t_j = 2 pi j / n_k of a smooth periodic parameter t; the M
 * samples are stored curve after curve.  Per sample (row-major M x 3 arrays, M arrays for a): the
 * position x, its derivative xt = dx/dt, a direction d tangent to the surface, pointing out of it
 * and not along the curve (e.g. the surface map's derivative across the curve; its part normal to
 * the curve is normalized into nu), the coefficient a > 0 and its gradient grad_a (ambient; only
 * nu . grad_a is used).  oversample: m in [1, 1024], with m * M < 2^31.  The arrays are in mem_kind
 * memory and read during the call only.
 * Errors: INVALID (bad sizes, a <= 0, a zero xt, d along the curve or non-finite data, at a sample
 * or at an interpolated point), TOO_LARGE, OOM, DEVICE. */
PMX_API pmx_status pmx_edge_create(pmx_ctx* ctx, int n_curves, const int64_t* n_samples, const double* x,
                                   const double* xt, const double* d, const double* a, const double* grad_a,
                                   int oversample, int mem_kind, void* stream, pmx_edge** out);
PMX_API void pmx_edge_destroy(pmx_edge* e);
/* *m_samples = M, *n_fine = m M (either pointer may be NULL).  Errors: INVALID (null handle). */
PMX_API pmx_status pmx_edge_size(pmx_edge* e, int64_t* m_samples, int64_t* n_fine);
/* The fine quadrature points to host arrays (any pointer may be NULL): position y (n_fine x 3),
 * conormal nu (n_fine x 3), trapezoid weight w, coefficient a and nu . grad a (n_fine each).
 * Errors: INVALID (null handle), DEVICE. */
PMX_API pmx_status pmx_edge_export_points(pmx_edge* e, double* y, double* nu, double* w, double* a,
                                          double* nu_grad_a);
/* y = op_kind[mu] at the N nodes of the operator's surface (the targets; their n, H, a and
 * grad_G a come from op): mu holds n_rhs rows of M doubles (row r at offset r M), y n_rhs rows of N,
 * both in mem_kind memory.  The operator's surface may be open (a set of patches that does not
 * close); the targets must lie off the curves.  Calls on one edge object must not overlap (it holds
 * the apply's scratch); different edge objects may run concurrently.
 * Errors: INVALID (null argument, unknown kind, n_rhs outside [1, 1024], op and e on different
 * devices, an operator with c != 0 or an advection field), OOM, DEVICE. */
PMX_API pmx_status pmx_edge_apply(pmx_operator* op, pmx_edge* e, int kind, int n_rhs, const double* mu, double* y,
                                  int mem_kind, void* stream);
/* y = K'_gamma[mu] at the M samples of the curves: the conormal derivative at a target on gamma of the
 * potential of K, K'_gamma[mu](x) = int_gamma nu(x) . grad_G K(x, x') mu(x') ds(x') (Theorem
 * thm:NeumannBCsrep, eq:neumann; the mu-term of the boundary rows of eq:NeuBVPsystem and
 * eq:DirBVPsystem, whose -mu / (2a) the caller adds).  The kernel nu(x) . (x - x') / (2 pi a(x') r^2)
 * is smooth (Theorem thm:kern_smth): the trapezoid rule on the samples (no oversampling), with the
 * kernel's limit -(nu . gamma'') / (4 pi a |gamma'|^2) at x' = x, gamma'' the derivative of the
 * trigonometric interpolant of the sampled dgamma/dt.  mu and y: n_rhs rows of M doubles, mem_kind
 * memory.  Errors: INVALID (null argument, n_rhs outside [1, 1024]), OOM, DEVICE. */
PMX_API pmx_status pmx_edge_apply_kprime(pmx_edge* e, int n_rhs, const double* mu, double* y, int mem_kind,
                                         void* stream);
/* y = D_gamma[mu] at the M samples: the double layer on the curves, D_gamma[mu](x) = int_gamma nu(x') .
 * grad' K(x, x') mu(x') ds(x') for x on gamma, i.e. N_gamma[mu] on gamma less its jump (eq:DirichletRep;
 * the mu-term of the boundary row of eq:DirBVPsystem: from the surface side N_gamma[mu] tends to
 * +mu / (2a) + D_gamma[mu] with the outward conormal).  Taken when nu . grad a = 0 at every sample, where
 * the kernel nu(x') . (x' - x) / (2 pi a(x') r^2) is smooth: the trapezoid rule on the samples, with the
 * limit -(nu . gamma'') / (4 pi a |gamma'|^2) at x' = x.  mu and y as for pmx_edge_apply_kprime.
 * Errors: INVALID (null argument, n_rhs outside [1, 1024], nu . grad a != 0 at some sample: the kernel
 * then has a log|x - x'| term), OOM, DEVICE. */
PMX_API pmx_status pmx_edge_apply_dlayer(pmx_edge* e, int n_rhs, const double* mu, double* y, int mem_kind,
                                         void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PMX_H */
