/*
 * ibim.h - C ABI of the CTR-IBIM linearised Poisson-Boltzmann solver for
 * AMD MI355X (gfx950).
 *
 * The library discretises Juffer's second-kind boundary integral equations
 * (eq. PB-BIE-1/2 of Izzo, Zhong, Runborg, Tsai, arXiv:2210.03699) with the
 * implicit boundary integral method (Section 2.1) and the second-order
 * corrected trapezoidal rule CTR2 (Sections 2.2-2.4), and solves the resulting
 * system  Lambda p + h^3 K W p + h^2 Omega W p = g  (eq. linear-system,
 * Section 2.5) with GMRES on the GPU.  The dense part K is evaluated on the
 * fly by tiled all-pairs HIP kernels; Omega (the correction weights) is built
 * once per problem.
 *
 * Conventions for every call:
 *  - Host pointers ("host") are read during the call only; the caller keeps
 *    ownership.  Device pointers ("device") are caller-allocated HIP device
 *    memory (for example torch tensors); the library never frees them.
 *  - Vectors of unknowns are stacked p = [psi(0..M-1); psi_n(0..M-1)] (length
 *    2M, float64) in the library's node order, which is the C-order scan of
 *    the grid (ibim_node_grid_index gives the grid index of every node).
 *    psi_n is the interior normal derivative; the outward normal is used.
 *  - "stream" is a hipStream_t (NULL = the legacy default stream); all device
 *    work of a call is enqueued on it.  Calls that return a host value
 *    (ibim_energy, ibim_solve) synchronise that stream.
 *  - Return codes: 0 success; 1 = GMRES did not reach the tolerance (the
 *    iterate is still written); negative = error, with a message from
 *    ibim_last_error():
 *      IBIM_EINVAL (-1) bad argument, IBIM_EGEOM (-2) geometry (empty tube,
 *      tube touching the grid edge, NaN in the signed distance, a node whose
 *      own normal line misses it), IBIM_ENOMEM (-3) device allocation failed,
 *      IBIM_EHIP (-4) HIP runtime error, IBIM_ENAN (-5) NaN produced,
 *      IBIM_ENODEV (-6) call needs a device but the context is host-only.
 *  - No exception crosses the ABI.  A context may be used from one host
 *    thread at a time; distinct contexts are independent.
 */
#ifndef IBIM_H
#define IBIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IBIM_OK 0
#define IBIM_NOT_CONVERGED 1
#define IBIM_EINVAL (-1)
#define IBIM_EGEOM (-2)
#define IBIM_ENOMEM (-3)
#define IBIM_EHIP (-4)
#define IBIM_ENAN (-5)
#define IBIM_ENODEV (-6)

#define IBIM_FP64 0  /* every pair evaluated and summed in float64 */
#define IBIM_MIXED 1 /* pairs evaluated in float32, sums and corrections in float64 */

typedef struct ibim_ctx ibim_ctx;

typedef struct {
  int precision;       /* IBIM_FP64 (default) or IBIM_MIXED */
  int restart;         /* GMRES Krylov dimension before a restart (default 60) */
  int max_iter;        /* total GMRES iterations allowed (default 300) */
  int check_residual;  /* 1: ibim_solve recomputes b - A x explicitly (default 1) */
  int device;          /* HIP device ordinal; -1 = host-only context (setup
                          and inspection only, no device memory) */
  double r_near;       /* IBIM_MIXED: pairs closer than r_near (Angstrom) are
                          evaluated in float64 (direct sum: re-evaluated in
                          the finishing kernel; treecode: in its direct
                          part) (default 0 = 2 h) */
  int hybrid;          /* IBIM_CTR2 (default), IBIM_HYB or IBIM_KREG, below */
  int precond;         /* IBIM_PRECOND_DIAG (default) or IBIM_PRECOND_NONE, below */
  int summation;       /* IBIM_SUM_DIRECT (default) or IBIM_SUM_TREE, below */
  int tree_order;      /* IBIM_SUM_TREE: Chebyshev points per dimension, 2..12 (default 8) */
  double tree_theta;   /* IBIM_SUM_TREE: separation parameter, (0, 1] (default 0.7) */
  int64_t tree_min_nodes; /* IBIM_SUM_TREE: problems with fewer tube nodes use the
                             direct sum instead (default 0: every problem) */
  int64_t pair_scratch_max; /* direct sum: device bytes the symmetric pair kernel may
                               use for its partial sums (default 0: 32 GiB); a problem
                               needing more uses the one-directional kernels */
} ibim_options;

/*
 * Evaluation of the dense pair sum h^3 K W p (Section 2.5):
 *  IBIM_SUM_DIRECT  every (target, source) pair, exactly as written (the path
 *                   the parity bars of this header refer to).
 *  IBIM_SUM_TREE    a treecode, the far-field acceleration that the paper
 *                   obtains with a black-box fast multipole method: sources of
 *                   a cluster far from a batch of 256 targets are replaced by
 *                   charges at tree_order^3 tensor Chebyshev points of the
 *                   cluster's box (Lagrange interpolation of the kernels in the
 *                   source variable, normal derivatives through the derivative
 *                   of the interpolant); nearer clusters are summed directly,
 *                   with the pairs of N_k skipped by index as in the direct
 *                   path.  A cluster is far when (r_batch + r_cluster) <
 *                   tree_theta * distance of the box centres, it holds more
 *                   than c tree_order^3 nodes and the box gap exceeds the
 *                   largest corrected-pair distance; c is the cost of a
 *                   target-proxy evaluation in direct pairs: 0.44 with
 *                   IBIM_FP64, 0.26 with IBIM_MIXED.  An approximation: its error falls
 *                   geometrically with tree_order and with smaller tree_theta.
 *                   With IBIM_FP64 all of it is float64; with IBIM_MIXED the
 *                   target-proxy evaluations run in float32 (on float64-formed
 *                   differences, summed in float32 over n proxies, then in
 *                   float64), and so do the direct pairs at distance r_near
 *                   or more (float64-formed differences, float64 sums); direct
 *                   pairs nearer than r_near and the proxy charges stay
 *                   float64.  A problem with fewer than tree_min_nodes tube
 *                   nodes is summed directly instead, in the same precision;
 *                   the solve server applies this rule per request.  The
 *                   corrections, GMRES and energy are those of the direct path.
 */
#define IBIM_SUM_DIRECT 0
#define IBIM_SUM_TREE 1

/*
 * System handed to GMRES (Section 2.5):
 *  IBIM_PRECOND_DIAG  Lambda^-1 A p = Lambda^-1 g: each block row divided by its
 *                     free-term coefficient (lambda1 = (1 + eps_E/eps_I)/2 on the
 *                     psi rows, lambda2 = (1 + eps_I/eps_E)/2 on the psi_n rows).
 *                     Same solution; the stopping test and the reported residuals
 *                     refer to the scaled system.
 *  IBIM_PRECOND_NONE  A p = g as written in eq. (linear-system).
 */
#define IBIM_PRECOND_NONE 0
#define IBIM_PRECOND_DIAG 1

/*
 * Quadrature of the rows (Section 3.2, eq. linear-system-hyb):
 *  IBIM_CTR2  corrected trapezoidal rule CTR2 in every row.
 *  IBIM_HYB   HYB-IBIM: rows of "bad" nodes, whose finite-difference geometry
 *             is unreliable (| |grad_h d| - 1 | > 0.05, or |g.H g| > 0.1/h for
 *             the normalised gradient g and Hessian H, or a corrected plane with
 *             1 - |eta| max|kappa| < 0.2), use the kernel regularisation K-reg
 *             of eq. (regularized-kernel) with tau = 2h, and bad nodes carry
 *             J = 1 (eq. Jacobian-hybrid); other rows use CTR2.
 *  IBIM_KREG  every node bad (K-reg rows and J = 1 everywhere).
 * K-reg replaces the kernels by their tangent-disc means for the tube nodes y
 * with |(I - n n^T)(y - P(y_k))| < tau and |n.(y - P(y_k))| <= eps + h: 0 for
 * K11, K21, K22 and (e^{-k tau} - 1 + k tau) / (2 pi k tau^2) for K12.
 */
#define IBIM_CTR2 0
#define IBIM_HYB 1
#define IBIM_KREG 2

typedef struct {
  int iters;                 /* GMRES iterations */
  int applies;               /* operator applications, including restarts and the
                                explicit residual */
  int converged;             /* 1 if |g_{j+1}| <= tol ||b|| was reached */
  double rel_resid;          /* GMRES residual estimate |g_{j+1}| / ||b|| */
  double explicit_rel_resid; /* ||b - A x|| / ||b|| (-1 if not computed) */
  double seconds;            /* wall time of the solve */
} ibim_solve_info;

/* Fill *opt with the defaults listed above. */
void ibim_default_options(ibim_options* opt);

/*
 * Build a problem from a signed-distance grid.
 *   sdf        host, float64, nx*ny*nz, C order (z fastest); node (i,j,k) at
 *              origin + h*(i,j,k); positive inside the molecule (eq.
 *              signed-distance).
 *   eps_tube   tube half-width epsilon: nodes with |d| < epsilon are the
 *              quadrature nodes (Section 2.2); every such node needs two
 *              grid nodes on each side for the curvature stencil.
 *   eps_in, eps_out, kappa  dielectric constants inside/outside and the
 *              Debye parameter of eq. linearized-Poisson-Boltzmann (> 0, > 0,
 *              >= 0).
 *   charge_xyz host, 3*n_charges (x,y,z interleaved); charge_q host,
 *              n_charges.  Charges define the right-hand side (eq.
 *              PB-lambda-g) and the energy (eq. pol-energy).
 *   opt        NULL for defaults.
 * Geometry and correction sets are computed on the host; the correction
 * weights (eq. single_correction_weight, Theorem 2.1) and all per-problem
 * arrays are then built on the device on "stream".  *out receives the new
 * context (NULL on error).
 * Device memory held by the context: O(M) geometry and corrections; for the
 * direct pair sum, row and column partial sums of about (M/256)^2/8 x 4 KiB
 * (0.3 GB at M = 1.2e5, 21 GB at M = 1.5e6; above 32 GiB, or if that
 * allocation fails, a kernel with O(M) partial sums is used instead); the
 * GMRES basis, (restart + 1) x 2M doubles, allocated at the first solve.
 */
int ibim_setup(const double* sdf, int nx, int ny, int nz, const double origin[3], double h,
               double eps_tube, double eps_in, double eps_out, double kappa,
               const double* charge_xyz, const double* charge_q, int n_charges,
               const ibim_options* opt, void* stream, ibim_ctx** out);

/* Release every resource of the context (safe on NULL). */
void ibim_destroy(ibim_ctx* ctx);

/* Thread-local message describing the last error (never NULL). */
const char* ibim_last_error(void);

/*
 * The options this context runs with (host, one struct): those given to
 * ibim_setup, with IBIM_SUM_TREE resolved for the problem's size (summation
 * IBIM_SUM_DIRECT below tree_min_nodes).
 */
int ibim_context_options(const ibim_ctx* ctx, ibim_options* opt);

/* Number of tube nodes M (unknowns are 2M). */
int ibim_num_nodes(const ibim_ctx* ctx, int64_t* M);

/* idx host, M: linear grid index (i*ny + j)*nz + k of every node. */
int ibim_node_grid_index(const ibim_ctx* ctx, int64_t* idx);

/*
 * Host copies of the node geometry (Section 2.1): P (3M, projection
 * y - d grad d / |grad d|), n (3M, outward unit normal), w (M, Jacobian times
 * delta_eps(d), eq. phi-averaging-kernel / eq. jacobian).  Any pointer may
 * be NULL.
 */
int ibim_node_geometry(const ibim_ctx* ctx, double* P, double* n, double* w);

/* bad (host, M): 1 for the nodes of M_B (K-reg row, J = 1), else 0.  All zero
 * with IBIM_CTR2.  *n_bad (may be NULL) receives their number. */
int ibim_node_flags(const ibim_ctx* ctx, uint8_t* bad, int64_t* n_bad);

/* Number of correction entries (sum over rows of |N_h(y_k)|). */
int ibim_num_corrections(const ibim_ctx* ctx, int64_t* nnz);

/*
 * Host copies of the correction sets N_h(y_k) (Section 2.4): rowptr (M+1),
 * col (nnz, sorted ascending in each row), axis (nnz, dominant axis 0..2),
 * alpha, beta (nnz, shifts of the nearest node in [-1/2, 1/2)), eta (nnz,
 * signed distance of the normal-line point in that plane).  In K-reg rows
 * the entries are the regularised nodes: axis -1, alpha = beta = 0, eta the
 * normal offset n.(y - P(y_k)).  Any pointer may be NULL.
 */
int ibim_corrections(const ibim_ctx* ctx, int64_t* rowptr, int64_t* col, int32_t* axis,
                     double* alpha, double* beta, double* eta);

/*
 * Correction weights computed on the device, copied to host: om11, om21
 * (nnz each) are omega[s0^(11)] and omega[s0^(21)] of eq. corr-trapz-rule-sys1/2
 * (omega^(22) = -(eps_in/eps_out) omega^(11), omega^(12) = kappa/(4 pi)).
 * Synchronises "stream".
 */
int ibim_correction_weights(const ibim_ctx* ctx, double* om11, double* om21, void* stream);

/*
 * Right-hand side g = [g1; g2] of eq. PB-lambda-g at the projected nodes.
 * g: device, 2M float64.
 */
int ibim_rhs(ibim_ctx* ctx, double* g, void* stream);

/*
 * out = A u with A = Lambda + h^3 K W + h^2 Omega W (eq. linear-system).
 * u, out: device, 2M float64, must not overlap.  Pure: no state changes.
 */
int ibim_apply(ibim_ctx* ctx, const double* u, double* out, void* stream);

/*
 * Allocation-free variant of ibim_apply, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, layout and result as ibim_apply.
 * The partial sums of the dense pair sum go to a static device array of
 * IBIM_NOALLOC_SCRATCH_BYTES owned by the library (one per GPU, held until
 * the process ends) instead of context memory:
 *   - symmetric kernels when the context's plan fits there (result
 *     bit-identical to ibim_apply);
 *   - otherwise the one-directional kernels when their nsplit x 2M partial
 *     sums fit (result equal to ibim_apply within float64 rounding).
 * Larger problems and treecode contexts fail with IBIM_EINVAL (message in
 * ibim_last_error).  The call makes no device allocation or free.  Every call
 * on one GPU shares that GPU's array and overwrites it: calls that overlap in
 * time on the same GPU (other streams or threads) race and must be serialised
 * by the caller.  Pair-kernel timing (ibim_pair_timing) skips these calls.
 */
#define IBIM_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int ibim_apply_noalloc(ibim_ctx* ctx, const double* u, double* out, void* stream);

/*
 * Solve A x = rhs by GMRES(restart) from x0 = 0 until |g_{j+1}| <= tol ||b||
 * (Section 2.5), where b = rhs, or Lambda^-1 rhs for the row-scaled system of
 * IBIM_PRECOND_DIAG (the residuals in info refer to that system).  rhs, x:
 * device, 2M float64, distinct.  info may be NULL.  Returns 0 when converged,
 * 1 when max_iter was reached (x holds the last iterate).  Workspace
 * ((restart+4) vectors of 2M float64) is allocated on first use and kept with
 * the context.
 */
int ibim_solve(ibim_ctx* ctx, const double* rhs, double tol, double* x, ibim_solve_info* info,
               void* stream);

/* As ibim_solve, but GMRES starts from the x given on entry (a warm start,
 * for example the solution of a nearby geometry mapped onto this one's nodes
 * through ibim_node_grid_index). */
int ibim_solve_guess(ibim_ctx* ctx, const double* rhs, double tol, double* x,
                     ibim_solve_info* info, void* stream);

/*
 * Polarisation energy G_pol = 1/2 sum_k q_k psi_rxn(z_k) (eq. pol-energy,
 * eq. psi-rxn with the plain trapezoidal IBIM sum) from a solution x
 * (device, 2M).  *g_pol is written on the host.
 */
int ibim_energy(ibim_ctx* ctx, const double* x, double* g_pol, void* stream);

/*
 * Pair-kernel timing: while enabled, every dense pair-kernel launch made by
 * ibim_apply / ibim_solve on this context is bracketed by HIP events on its
 * launch stream.  ibim_pair_timing(ctx, 1) starts a new collection (and
 * clears the previous one), ibim_pair_timing(ctx, 0) stops collecting.
 * ibim_pair_timing_read waits for the last recorded launch and returns the
 * number of launches and the sum of their durations in milliseconds.
 */
int ibim_pair_timing(ibim_ctx* ctx, int enable);
int ibim_pair_timing_read(ibim_ctx* ctx, int64_t* launches, double* total_ms);

/*
 * Work of one dense pair-sum launch as this context performs it (device
 * contexts only): *pairs = M^2 ordered (target, source) pairs; *flops = the
 * floating-point operations of the pair formulas (FMA counted as 2, exp and
 * rsqrt not counted): 60 per ordered pair when each pair is evaluated on its
 * own, 68 per unordered pair when both directions share one evaluation (the
 * symmetric kernels; 66 when they evaluate pairs in units of the Debye
 * length and so need no kappa factors: float64 with kappa > 1e-30, the
 * mixed form with kappa h >= 1e-6; tile pairs holding corrected pairs and
 * the diagonal tiles are still evaluated one direction at a time).  In the mixed form
 * these are float32 operations.  For IBIM_SUM_TREE, *pairs is still M^2 (the
 * pairs the sum stands for) and *flops counts what the treecode performs: 60
 * per direct pair, 36 per target-proxy evaluation, 15 per source-proxy term
 * and 12 tree_order^4 per child-to-parent transfer of proxy charges.
 */
int ibim_pair_work(const ibim_ctx* ctx, double* pairs, double* flops);

/*
 * Work of one treecode pair sum (IBIM_SUM_TREE contexts; IBIM_EINVAL for
 * others).  out (host, 6 doubles): [0] target-proxy evaluations, [1] direct
 * pair evaluations, [2] source-proxy terms of the proxy charges, [3] batches
 * of targets, [4] proxy clusters, [5] child-to-parent charge transfers.  Each
 * application performs exactly these.
 */
int ibim_tree_counts(const ibim_ctx* ctx, double* out);

/*
 * Two-way pairs of the treecode plan (IBIM_SUM_TREE contexts, host-only ones
 * too; IBIM_EINVAL for others).  Two leaves (batches of targets, which are
 * also the finest source clusters) that are near each other both ways and
 * hold no pair of N_k either way are taken out of both batches' direct
 * ranges (ibim_tree_plan's nlo, nhi) and evaluated once for both
 * directions.  *n (host) receives their
 * number; lower, upper (host, n int32 each, or NULL) the batches b < b' of
 * each pair, in order of b, then b'.
 */
int ibim_tree_pairs(const ibim_ctx* ctx, int64_t* n, int32_t* lower, int32_t* upper);

/*
 * The treecode plan of an IBIM_SUM_TREE context (host-only contexts too: the
 * plan is built on the host with the geometry), for inspection.  Call once
 * with counts (host, 8 int64) to learn the sizes: [0] M, [1] batches B,
 * [2] proxy clusters C, [3] far entries F, [4] direct ranges R, [5] work
 * items, [6] tree_order, [7] 0.  Every non-NULL host array is then filled:
 *   perm (M)            node at each tree position (all ranges below are in
 *                       tree positions);
 *   bstart (B+1)        batch b holds bstart[b] .. bstart[b+1]-1;
 *   cstart, cend (C)    range of proxy cluster c; cbox (6C) its box (lo x, y,
 *                       z, hi x, y, z; flat sides padded to width h);
 *   kid (2C)            children of c that carry proxies (-1: none);
 *   dstart, dend (C)    the sources whose charges c takes directly;
 *   frow (B+1), fcol (F) proxy clusters summed for batch b;
 *   nrow (B+1), nlo, nhi (R) source ranges summed directly for batch b;
 *   gap (1)             the largest distance |x_k - P_m| over m in N_k.
 * IBIM_EINVAL for other contexts.
 */
int ibim_tree_plan(const ibim_ctx* ctx, int64_t* counts, int32_t* perm, int32_t* bstart,
                   int32_t* cstart, int32_t* cend, double* cbox, int32_t* kid, int32_t* dstart,
                   int32_t* dend, int32_t* frow, int32_t* fcol, int32_t* nrow, int32_t* nlo,
                   int32_t* nhi, double* gap);

/* ------------------------------------------------------------------------ */
/*
 * Solve server: continuous batching of many independent problems on one GPU.
 *
 * Requests (a signed-distance grid and charges, as for ibim_setup, plus a
 * GMRES tolerance) are queued by ibim_server_submit, which copies the inputs
 * and starts the host part of their setup on a background thread.  Each
 * ibim_server_step is one round of the direct-sum solves:
 *   1. admission: prepared requests get a solve slot, in submission order,
 *      while one is free and the estimated device footprint (geometry,
 *      corrections, partial sums, Krylov basis) fits in the HBM budget (a
 *      request that does not fit lets later smaller ones pass; memory of
 *      finished requests counts until a background thread has freed it).
 *      Their device setup runs on one of two background threads, each with a
 *      stream of its own, while rounds continue, and they join the first
 *      round after it (with no solve running, the step sets them up itself);
 *   2. ONE persistent batched pair-kernel launch covers a work list of
 *      (request, target tile, source chunk) items of every active solve; each
 *      item is computed exactly as in the single-problem kernel.  Requests
 *      that the options send to the treecode (IBIM_SUM_TREE, at least
 *      tree_min_nodes nodes) run rounds of their own instead (their treecode
 *      launches, then steps 3 and 4) on a second stream: a step starts the
 *      next such round once the previous one has completed, and waits for
 *      it only when no direct-sum solve is active;
 *   3. per request: sparse correction, one GMRES (Arnoldi + Givens) step or a
 *      residual step, all on the device, then a single status read-back;
 *   4. finished solves compute G_pol (eq. pol-energy), keep their solution on
 *      the host and release their device memory.
 * Every request runs the same arithmetic as ibim_solve followed by ibim_energy
 * with the server's options, so its results do not depend on which other
 * requests share the rounds.  All server calls must come from one host thread.
 */
typedef struct ibim_server ibim_server;

typedef struct {
  int64_t submitted, admitted, finished, failed;
  int64_t rounds;           /* rounds of the direct-sum solves */
  int64_t batched_items;    /* pair-kernel work items over all rounds */
  size_t bytes_in_use;      /* device bytes charged to the budget: active solves (a
                               request's setup allocates one block of its footprint
                               estimate, held whole until the request is released, plus
                               what did not fit in it), and requests being set up at
                               their estimate.  Admission also counts the bytes of
                               released requests whose memory is not yet freed */
  size_t bytes_peak;
  size_t budget_bytes;
  int active, waiting, max_active_seen;
  /* admission passes (one per request and round) that held a set-up request
   * back: for want of a free slot, or because its footprint estimate did not
   * fit the budget left */
  int64_t held_for_slot, held_for_budget;
  /* largest amount by which an admitted request's device bytes (at the peak
   * of its setup, or after it) exceeded the footprint estimate it was
   * admitted on; 0 while every estimate was an upper bound */
  size_t estimate_shortfall;
} ibim_server_stats;

#define IBIM_REQ_WAITING 0 /* preparing on the host or queued for admission */
#define IBIM_REQ_ACTIVE 1
#define IBIM_REQ_DONE 2
#define IBIM_REQ_FAILED (-1)

/* opt: solver options of every request (precision, restart, max_iter,
 * check_residual, device, r_near, hybrid, precond, summation and the
 * treecode fields, resolved per request by its size as in ibim_setup;
 * validated as there); hbm_budget_bytes > 0; max_slots >= 1
 * concurrent solves; host_threads >= 1 background setup threads; stream:
 * the hipStream_t the direct-sum solves' rounds run on (NULL: the null
 * stream); the treecode solves' rounds and the device setups use streams the
 * server creates. */
int ibim_server_create(const ibim_options* opt, size_t hbm_budget_bytes, int max_slots,
                       int host_threads, void* stream, ibim_server** out);
/* Inputs as in ibim_setup (host, copied); tol > 0.  *ticket identifies the
 * request.  Never blocks on the device. */
int ibim_server_submit(ibim_server* srv, const double* sdf, int nx, int ny, int nz,
                       const double origin[3], double h, double eps_tube, double eps_in,
                       double eps_out, double kappa, const double* charge_xyz,
                       const double* charge_q, int n_charges, double tol, int64_t* ticket);
/* One round (see above); *active, *waiting may be NULL.  With no solve
 * active it first waits for a background setup to finish.  A request that
 * fails (setup error, footprint above the whole budget, NaN) is marked
 * IBIM_REQ_FAILED and the others go on.  A nonzero return is a device error
 * (launch or copy failure); the server should then be destroyed. */
int ibim_server_step(ibim_server* srv, int* active, int* waiting);
/* State of a request (IBIM_REQ_*); for a finished request also G_pol and the
 * solve information; for a failed one the error code is returned. */
int ibim_server_poll(ibim_server* srv, int64_t ticket, int* state, double* g_pol,
                     ibim_solve_info* info);
/* Solution of a finished request: *M nodes; x (host, 2M) may be NULL to query M. */
int ibim_server_solution(ibim_server* srv, int64_t ticket, double* x, int64_t* M);
/* Forget a finished or failed request (frees its stored solution). */
int ibim_server_release(ibim_server* srv, int64_t ticket);
/* Counters of the server (host values, no device synchronisation). */
int ibim_server_get_stats(ibim_server* srv, ibim_server_stats* st);
/* Waits for background setup threads, frees everything (safe on NULL). */
void ibim_server_destroy(ibim_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* IBIM_H */
