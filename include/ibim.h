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
                          re-evaluated in float64 (default 0 = 4 h) */
} ibim_options;

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
 */
int ibim_setup(const double* sdf, int nx, int ny, int nz, const double origin[3], double h,
               double eps_tube, double eps_in, double eps_out, double kappa,
               const double* charge_xyz, const double* charge_q, int n_charges,
               const ibim_options* opt, void* stream, ibim_ctx** out);

/* Release every resource of the context (safe on NULL). */
void ibim_destroy(ibim_ctx* ctx);

/* Thread-local message describing the last error (never NULL). */
const char* ibim_last_error(void);

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

/* Number of correction entries (sum over rows of |N_h(y_k)|). */
int ibim_num_corrections(const ibim_ctx* ctx, int64_t* nnz);

/*
 * Host copies of the correction sets N_h(y_k) (Section 2.4): rowptr (M+1),
 * col (nnz, sorted ascending in each row), axis (nnz, dominant axis 0..2),
 * alpha, beta (nnz, shifts of the nearest node in [-1/2, 1/2)), eta (nnz,
 * signed distance of the normal-line point in that plane).  Any pointer may
 * be NULL.
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
 * Solve A x = rhs by GMRES(restart) from x0 = 0 until |g_{j+1}| <= tol ||rhs||
 * (Section 2.5).  rhs, x: device, 2M float64.  info may be NULL.  Returns 0
 * when converged, 1 when max_iter was reached (x holds the last iterate).
 * Workspace ((restart+1) vectors of 2M float64) is allocated on first use and
 * kept with the context.
 */
int ibim_solve(ibim_ctx* ctx, const double* rhs, double tol, double* x, ibim_solve_info* info,
               void* stream);

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

#ifdef __cplusplus
}
#endif

#endif /* IBIM_H */
