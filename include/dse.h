/*
 * dse.h -- C ABI of the MI355X (gfx950) ghost-gluon Dyson-Schwinger solver.
 *
 * Method: Hopfer, Alkofer, Haase, "Solving the Ghost-Gluon System of
 * Yang-Mills Theory on GPUs" (arXiv:1206.1779).  The Landau-gauge ghost and
 * gluon dressing functions G(p^2), Z(p^2) are expanded as
 *     ln Z(x) = a_0/2 + sum_{j>=1} a_j T_j(s(x)),  ln G(x) = b_0/2 + ...
 * with the mapping s(x) = log10(x/(Lambda eps)) / log10(Lambda/eps) (Sec. 3),
 * and the renormalised DSEs (Sec. 3, MOM subtraction at x_Z = Lambda^2 for the
 * gluon and x_G = 0 for the ghost)
 *     z(x_i) = Z(x_i)^{-1} - Z(x_Z)^{-1} - Pi_Z(x_i) + Pi_Z(x_Z) = 0
 *     g(x_i) = G(x_i)^{-1} - G(x_G)^{-1} - Pi_G(x_i) + Pi_G(x_G) = 0
 * are collocated at the mapped Chebyshev roots and solved by Newton-Raphson
 * with under-relaxation (Sec. 3).  Pi_Z and Pi_G are the radial x angular
 * integrals of Sec. 2 (ghost loop with the (1-xi^2)^{3/2} angular weight,
 * gluon loop with the kernels M, Q and the vertex dressing
 * (G(y)G(z))^{-2-6 delta} (Z(y)Z(z))^{-3 delta}).
 *
 * Layouts (all FP64, row-major, device memory):
 *   c  [n]      unknowns [a_0..a_{n_z-1}, b_0..b_{n_g-1}],  n = n_z + n_g
 *   F  [n]      residual [z(x^Z_0..x^Z_{n_z-1}), g(x^G_0..x^G_{n_g-1})]
 *   J  [n x n]  J[r*n + k] = dF_r / dc_k  (the Newton matrix of Sec. 3)
 *
 * Ownership: the caller allocates every device buffer, including one
 * workspace of dse_workspace_bytes() bytes that stays alive (and untouched by
 * the caller) until dse_destroy().  The library allocates no device memory.
 * A context belongs to one HIP stream and one device and is not thread-safe.
 *
 * Synchrony: dse_residual, dse_jacobian and dse_start_guess enqueue work on
 * the context's stream and return without synchronising.  dse_newton_solve
 * synchronises (it reads the residual norm every iteration) and returns when
 * the solve is finished.
 *
 * Errors: every call returns a dse_status and never throws.  Invalid
 * arguments are reported before any launch (DSE_E_INVALID, message in
 * dse_last_error).  HIP runtime failures give DSE_E_DEVICE.
 */
#ifndef DSE_H
#define DSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DSE_ABI_VERSION 2
/* largest Chebyshev order per function */
#define DSE_MAX_N 128

typedef enum {
  DSE_OK = 0,
  DSE_E_INVALID = 1,   /* bad argument or parameter; nothing was launched      */
  DSE_E_DEVICE = 2,    /* HIP runtime error                                    */
  DSE_E_NOMEM = 3,     /* workspace smaller than dse_workspace_bytes()        */
  DSE_E_SINGULAR = 4,  /* a pivot of the Newton LU is zero, not finite, or at
                          most n eps times the largest entry of its row         */
  DSE_E_NOCONV = 5,    /* Newton did not converge within max_iter             */
  DSE_E_NONFINITE = 6  /* residual or Jacobian not finite                      */
} dse_status;

/* DSE_MIXED: the Newton matrix's derivative sums and its B.T contraction in
 * FP32 (F, its scale, norms and the LU stay FP64).  dse_newton_solve uses
 * FP32 matrices while a step at least halves the 2-norm merit and the scaled
 * residual is above 1e-6, FP64 ones afterwards; the root is that of the FP64
 * residual either way. */
typedef enum { DSE_FP64 = 0, DSE_MIXED = 1 } dse_precision;

/* Quadrature rules of the paper (dse_params.quad, bits):
 * DSE_QUAD_TANH_SINH: the angular integral by the tanh-sinh rule in
 *   xi = cos(theta) (Sec. 2): xi_k = tanh((pi/2) sinh(k h)), k = -K .. K,
 *   n_ang = 2K + 1 (odd, >= 3), h = 3/K;
 * DSE_QUAD_SPLIT: the radial integral split at each row's external momentum,
 *   [0, eps2] + [eps2, x] + [x, lambda2] (Sec. 3), n_rad log-GL nodes on each
 *   interval above eps2 and the IR panel below (rows at x = 0 and
 *   x = lambda2: the one interval [eps2, lambda2]).  Every row then has its
 *   own grid, and the q-side derivative sums are accumulated per row in the
 *   point kernels (no B.T product).  FP64 only: with DSE_MIXED, in a batched
 *   family, or for dse_vjp it is rejected (DSE_E_INVALID). */
enum { DSE_QUAD_TANH_SINH = 1, DSE_QUAD_SPLIT = 2 };

typedef struct dse_ctx dse_ctx; /* opaque */

/* Problem definition (Sec. 2-3).  dse_params_default() fills the paper's
 * physics: alpha(mu^2) = 1, N_c = 3, kappa = (93 - sqrt(1201))/98,
 * delta = -9/44, gamma = -13/22. */
typedef struct {
  int32_t abi_version;   /* DSE_ABI_VERSION                                      */
  int32_t n_z, n_g;      /* Chebyshev coefficients of ln Z (a) and ln G (b),
                            1 .. DSE_MAX_N each                                  */
  int32_t n_rad;         /* Gauss-Legendre nodes in ln y on [eps2, lambda2]     */
  int32_t n_ir;          /* Gauss-Legendre nodes in ln y on the IR panel
                            [eps2 exp(-ir_efolds), eps2] (stands for the
                            integral from 0 to eps2 of the radial split, Sec. 3) */
  int32_t n_ang;         /* angular nodes                                        */
  int32_t precision;     /* dse_precision                                        */
  int32_t quad;          /* quadrature rules (dse_quadrature bits); 0: one
                            radial grid shared by all rows (Gauss-Legendre in
                            ln y on [eps2, lambda2] with n_rad nodes, plus the
                            IR panel) and Gauss-Legendre in theta               */
  double eps2, lambda2;  /* interval [epsilon^2, Lambda^2] of the expansion      */
  double ir_efolds;      /* length of the IR panel in ln y                       */
  double alpha_mu;       /* alpha(mu^2) = g^2/(4 pi)                              */
  double n_c;            /* number of colours                                    */
  double g0_inv;         /* G(x_G = 0)^{-1}; 0 selects the scaling solution      */
  double z_lambda_inv;   /* Z(x_Z = Lambda^2)^{-1}                               */
  double kappa;          /* IR exponent (Z ~ x^{2 kappa}, G ~ x^{-kappa})        */
  double delta, gamma;   /* ghost and gluon anomalous dimensions                 */
} dse_params;

/* Newton options (Sec. 3 under-relaxed Newton-Raphson).  The relaxation rho
 * starts at 1 and is halved, at most max_halvings times, while the Euclidean
 * norm of the scaled residual, (sum_r (F_r / S_r)^2)^{1/2}, at the trial point
 * is not below the current one.  Convergence: scaled residual
 * max_r |F_r| / S_r < tol, where S_r is the magnitude of the terms that
 * cancel in F_r (direct term, parameter, and the sums of |integrand| at x_r
 * and at the subtraction point).  Then extra_iters full steps follow,
 * stopping early once rho ||Delta||_inf < step_tol. */
typedef struct {
  double tol;
  int32_t max_iter;
  int32_t extra_iters;
  int32_t max_halvings;
  int32_t reserved_;
  double step_tol;
} dse_newton_opts;

typedef struct {
  int32_t iters;           /* Newton iterations taken                             */
  int32_t status;          /* dse_status of the solve                             */
  double fnorm;            /* final scaled residual                               */
  double fnorm2;           /* final ||F||_2                                       */
  double fnorm_hist[128];  /* scaled residual before iteration i (i <= iters)     */
  double relax_hist[128];  /* rho used in iteration i                             */
  int32_t n_jacobians;     /* assemblies of J and F                               */
  int32_t n_residuals;     /* residual-only evaluations (line search)             */
  double t_total_ms;       /* wall time of the call                               */
  int32_t n_jacobians_mixed; /* of n_jacobians, those with FP32 derivative sums   */
  int32_t reserved2_;
  double t_assembly_ms;    /* device time of the Newton-matrix assemblies (the
                              first one: wall time including its norms)          */
  double t_lu_ms;          /* device time of the LU solves                        */
} dse_newton_report;

/* Fills *p with the physics defaults above and the small grid
 * n_z = n_g = 16, n_rad = 64, n_ir = 16, n_ang = 16, eps2 = 1e-6,
 * lambda2 = 1e6, ir_efolds = 40, g0_inv = 0, z_lambda_inv = 1. */
dse_status dse_params_default(dse_params* p);

/* Device workspace bytes a context with these parameters needs (0 if the
 * parameters are invalid). */
size_t dse_workspace_bytes(const dse_params* p);

/* Validates p, builds the quadrature grid, collocation points and Chebyshev
 * tables on the host (Sec. 3 expansion and mapping; Sec. 2 radial and angular
 * integrals) and uploads them into the workspace on `hip_stream` (a
 * hipStream_t; NULL = default stream) of the current device.  d_workspace must
 * be 256-byte aligned.  *out receives a host-allocated context. */
dse_status dse_init(const dse_params* p, void* d_workspace, size_t ws_bytes,
                    void* hip_stream, dse_ctx** out);

/* Releases the host context (not the workspace).  NULL is allowed. */
dse_status dse_destroy(dse_ctx* ctx);

/* Writes the start guess to d_c[n]: the asymptotic forms of Sec. 2 (IR power
 * laws joined to the one-loop UV logarithms, scale fixed by Z(Lambda^2))
 * interpolated at the collocation points. */
dse_status dse_start_guess(dse_ctx* ctx, double* d_c);

/* Residual F(c) (Sec. 3, the collocated equations z(x_i), g(x_i)).
 * d_S (nullable) receives the per-row scale S_r defined at dse_newton_opts. */
dse_status dse_residual(dse_ctx* ctx, const double* d_c, double* d_F, double* d_S);

/* Newton matrix J = dF/dc (Sec. 3 matrix layout, analytic derivatives of the
 * integrands) and, if d_F != NULL, F at the same c. */
dse_status dse_jacobian(dse_ctx* ctx, const double* d_c, double* d_J, double* d_F);

/* Newton matrix by central differences of the residual, the paper's own
 * method (Sec. 4.2, finite-difference Jacobian with a step relative to each
 * coefficient): column j = (F(c + h_j e_j) - F(c - h_j e_j)) / (2 h_j) with
 * h_j = h_rel max(1, |c_j|).  2n full residual evaluations, enqueued on the
 * context's stream; for comparison with dse_jacobian (same layout: d_J is
 * [n][n] row-major on the device, d_c [n] on the device).  h_rel in (0, 1),
 * else DSE_E_INVALID.  Uses the context's scratch vectors, so it must not
 * overlap other calls on the same context. */
dse_status dse_jacobian_fd(dse_ctx* ctx, const double* d_c, double* d_J, double h_rel);

/* The dressings and the running coupling at m arbitrary momenta u > 0
 * (Sec. 2 running coupling alpha(x) = alpha(mu^2) G^2(x) Z(x); Sec. 3
 * expansion with the IR power laws below eps2 and the UV logarithms above
 * lambda2, the same extension the equations use): d_alpha[i] = alpha(u_i),
 * d_lnZ[i] = ln Z(u_i), d_lnG[i] = ln G(u_i).  d_c [n], d_u [m] and the
 * outputs (each nullable) on the device; enqueued on the context's stream.
 * m < 0 or a NULL d_c / d_u with m > 0: DSE_E_INVALID. */
dse_status dse_running_coupling(dse_ctx* ctx, const double* d_c, const double* d_u, int32_t m, double* d_alpha,
                                double* d_lnZ, double* d_lnG);

/* Vector-Jacobian product of the dressings at m momenta u > 0 with respect to
 * the coefficients (Sec. 3 expansion in Chebyshev polynomials of the mapped
 * momentum; the IR power laws and UV logarithms used outside [eps2, lambda2]
 * are matched at the interval ends and do not depend on the coefficients, so
 * d ln Z(u)/d a_j = d ln G(u)/d b_j = Tilde-T_j(s(u)), s clamped to [-1, 1]):
 *   d_grad[j]       = sum_i d_wZ[i] d ln Z(u_i) / d a_j    (j < n_z)
 *   d_grad[n_z + j] = sum_i d_wG[i] d ln G(u_i) / d b_j    (j < n_g)
 * For a loss L(ln Z(u_i), ln G(u_i)) the weights are dL/d ln Z(u_i) and
 * dL/d ln G(u_i), and d_grad is dL/dc.  d_u [m], d_wZ [m], d_wG [m] (either
 * weight vector nullable: that half of d_grad is zero) and d_grad [n] on the
 * device; enqueued on the context's stream.  m < 0, d_grad NULL, or d_u NULL
 * with m > 0: DSE_E_INVALID. */
dse_status dse_dressing_vjp(dse_ctx* ctx, const double* d_u, int32_t m, const double* d_wZ, const double* d_wG,
                            double* d_grad);

/* Renormalisation scale (Sec. 2.1 footnote: mu is fixed by the condition
 * G^2(mu^2) Z(mu^2) = 1 for the given alpha(mu^2)): d_mu2[0] receives the
 * largest root mu^2 in [eps2, lambda2] of 2 ln G(x) + ln Z(x) = 0 (where the
 * running coupling alpha(x) = alpha(mu^2) G^2 Z passes alpha(mu^2) on its
 * perturbative side; a decoupling solution's coupling also rises through it
 * in the infrared), or NaN if there is none.  Found in the mapped variable s
 * (Sec. 3) by a scan of 4096 equal intervals from s = 1 down and multisection
 * to adjacent doubles.  d_c [n] and d_mu2 [1] on the device; enqueued on the
 * context's stream. */
dse_status dse_renorm_scale(dse_ctx* ctx, const double* d_c, double* d_mu2);

/* Gauss-Legendre rule of n nodes on [-1, 1] (1 <= n <= 2^24) computed on the
 * device: Newton's method on P_n with the three-term recurrence from
 * Tricomi's estimate of each root, the weight 2 / ((1 - x^2) P_n'(x)^2) at the
 * converged node (the node generation the paper parallelises for the
 * Schwinger function, Sec. 5).  d_x [n] (ascending) and d_w [n] on the device;
 * d_ws: device workspace of dse_gauss_legendre_workspace_bytes(n) bytes,
 * 256-byte aligned (the recurrence coefficients).  Enqueued on hip_stream
 * without synchronising.  Errors: DSE_E_INVALID (message in
 * dse_last_error(NULL)), DSE_E_NOMEM for a short workspace. */
size_t dse_gauss_legendre_workspace_bytes(int32_t n);
dse_status dse_gauss_legendre(int32_t n, double* d_x, double* d_w, void* d_ws, size_t ws_bytes, void* hip_stream);

/* Schwinger function of the gluon propagator (Sec. 2.2):
 *   d_delta[j] = Delta(t_j) = (1/pi) int_0^p_max dp cos(t_j p) Z(p^2)/p^2,
 * j < m, for the dressing Z of the coefficients d_c (expansion with its IR and
 * UV extension), by the n-node Gauss-Legendre rule generated on the device
 * (as dse_gauss_legendre) and mapped by p = p_max ((1 + x)/2)^2 (Sec. 5: a
 * mapped Gauss-Legendre rule; the paper uses 2^17 nodes).  The oscillating
 * tail beyond p_max is left out (of order Z(p_max^2) / (t p_max^2)).
 * d_c [n_z + n_g], d_t [m] (GeV^-1 when momenta are in GeV), d_delta [m] on
 * the device; d_ws: workspace of dse_schwinger_workspace_bytes(n, m) bytes,
 * 256-byte aligned.  Enqueued on the context's stream. */
size_t dse_schwinger_workspace_bytes(int32_t n, int32_t m);
dse_status dse_schwinger(dse_ctx* ctx, const double* d_c, int32_t n, double p_max, const double* d_t, int32_t m,
                         double* d_delta, void* d_ws, size_t ws_bytes);

/* Solves F(c) = 0 by the under-relaxed Newton iteration of Sec. 3 starting
 * from d_c (overwritten by the last iterate).  opts may be NULL (tol 1e-10,
 * max_iter 60, extra_iters 0, max_halvings 30, step_tol 1e-14); h_report
 * (host memory) may be NULL.  Each step solves J Delta = F with an FP64 LU
 * with partial pivoting on the device.  Returns DSE_E_NOCONV with the last
 * iterate in d_c if max_iter is reached. */
dse_status dse_newton_solve(dse_ctx* ctx, double* d_c, const dse_newton_opts* opts,
                            dse_newton_report* h_report);

/* One Newton iteration (Sec. 3) in one call: J and F at d_c (kept in the
 * workspace), the LU solve J Delta = F, d_c_new = d_c - rho Delta, and the
 * residual at d_c_new into d_F_new (and its scale into d_S_new, nullable).
 * Enqueued on the context's stream; returns without synchronising unless
 * check != 0, which synchronises and reports a singular J (DSE_E_SINGULAR: a
 * pivot zero, not finite, or at most n eps times the largest |J_rk| of its
 * row; d_c_new is then undefined).  d_c and d_c_new must differ.  By default
 * the kernels are launched one by one; with graphs on (dse_set_graphs) the
 * launch sequence is recorded into a HIP graph on the first call for a given
 * set of pointers and rho and replayed afterwards (the arrays must stay
 * allocated while the context uses them).  Kernel by kernel is the default
 * because it measured faster on MI355X (0.140 against 0.145 ms per step at
 * N = 64 on a non-default stream: a graph launch adds a gap before its first
 * kernel).  Stage timings (dse_set_timing) are recorded only with graphs off. */
dse_status dse_newton_step(dse_ctx* ctx, const double* d_c, double rho, double* d_c_new, double* d_F_new,
                           double* d_S_new, int32_t check);
/* Switches the recorded-graph replay of dse_newton_step on or off (default). */
dse_status dse_set_graphs(dse_ctx* ctx, int32_t on);

/* Solves J x = b (trans = 0) or J^T x = b (trans != 0) for a row-major
 * n x n d_J with the device LU (partial pivoting).  d_J is not modified; the
 * factors go to the workspace.  d_x may equal d_b.  DSE_E_SINGULAR (d_x then
 * undefined) when a pivot is zero, not finite, or at most n eps times the
 * largest |entry| of its row of d_J: the test is relative to each row, so
 * scaling a row of the system changes neither the solution nor the verdict. */
dse_status dse_lu_solve(dse_ctx* ctx, const double* d_J, const double* d_b, double* d_x,
                        int32_t trans);

/* For callers that cannot allocate device memory (code under stream capture,
 * serving loops, harnesses that forbid hipMalloc): the solve of dse_lu_solve
 * without a context or workspace.  Solves J x = b (trans = 0) or J^T x = b
 * (trans != 0) for a row-major n x n d_J, 1 <= n <= 2 * DSE_MAX_N, with the
 * same device LU (partial pivoting; results identical to dse_lu_solve).  d_J,
 * d_b (length n) are not modified; d_x (length n) may equal d_b.  d_info
 * (device int32, nullable) receives 0 or DSE_E_SINGULAR (a pivot zero, not
 * finite, or at most n eps times the largest |entry| of its row of d_J; d_x is
 * then undefined).  Enqueued on hip_stream (a hipStream_t; NULL = default
 * stream) of the current device without synchronising; allocates nothing.
 * Scratch: one static device array of 517.25 KiB per GPU (the padded factors
 * when they do not fit in LDS, the pivot rows, the status word when d_info is
 * NULL, the largest entry of each row), taken by the first call on that GPU
 * and kept until the process ends.  Every call on a GPU shares that array: calls that overlap on
 * one GPU (several streams or threads at once) race.  Invalid n or NULL
 * d_J / d_b / d_x: DSE_E_INVALID before any launch, message in
 * dse_last_error(NULL). */
dse_status dse_lu_solve_noalloc(int32_t n, const double* d_J, const double* d_b, double* d_x, int32_t trans,
                                int32_t* d_info, void* hip_stream);

/* Vector-Jacobian products at c for a weight vector u (length n):
 *   d_uJ[k]     = sum_r u_r dF_r/dc_k                     (n entries; nullable)
 *   d_utheta[0] = sum_r u_r dF_r/d alpha_mu                (3 entries; nullable)
 *   d_utheta[1] = sum_r u_r dF_r/d g0_inv,  d_utheta[2] = sum_r u_r dF_r/d z_lambda_inv
 * alpha_mu enters F through the prefactor g^2 N_c/(2 pi)^3 of both
 * self-energies and through omega = 11 N_c alpha/(12 pi) in the UV
 * extrapolation of the dressings (Sec. 2); G(x_G)^{-1} and Z(x_Z)^{-1} enter
 * the MOM-subtracted equations linearly (Sec. 3).  One weighted pass of the
 * point kernels; with d_uJ == NULL the k- and q-side derivative sums are
 * skipped (the cost of one residual).  Enqueued on the context's stream. */
dse_status dse_vjp(dse_ctx* ctx, const double* d_c, const double* d_u, double* d_uJ, double* d_utheta);

/* Changes alpha(mu^2), G(x_G)^{-1} and Z(x_Z)^{-1} of an existing context (the
 * grid and tables do not depend on them).  Validated like dse_init. */
dse_status dse_set_physics(dse_ctx* ctx, double alpha_mu, double g0_inv, double z_lambda_inv);

const char* dse_status_string(dse_status s);
/* Message of the last failed call on ctx (or of the last failed dse_init when
 * ctx is NULL). */
const char* dse_last_error(const dse_ctx* ctx);

/* Numbers that size the problem: n = n_z + n_g, radial nodes, angular nodes. */
dse_status dse_sizes(const dse_ctx* ctx, int32_t* n, int32_t* n_radial, int32_t* n_angular);

/* Device-time instrumentation of dse_jacobian, for benchmarks.  While on,
 * every dse_jacobian call records HIP events on the context's stream around
 * its stages (no synchronisation at record time).  dse_read_timings()
 * synchronises, and returns the average milliseconds per call since timing
 * was switched on: [0] dressing, [1] gluon point kernel, [2] ghost point
 * kernel, [3] B.T contraction, [4] assembly; *count = calls averaged.
 * dse_set_timing() resets the averages. */
dse_status dse_set_timing(dse_ctx* ctx, int32_t on);
dse_status dse_read_timings(dse_ctx* ctx, double* ms5, int32_t* count);

/* ------------------------------------------------------------------------
 * Batched family.  `count` independent problems, each with its own
 * dse_params (orders, grids and physics may differ: e.g. the family of
 * decoupling solutions labelled by G(0), Sec. 2), assembled and solved
 * together: every stage is one launch for the whole family, and the
 * point work is one queue of (problem, row, radial tile, angular slice)
 * items, largest first.
 *
 * Packed layouts: the unknowns of problem b occupy c[off_c[b] .. off_c[b+1])
 * of one vector (same order as a single problem), and its Newton matrix
 * J[off_J[b] .. off_J[b+1]) (n_b x n_b, row-major); dse_batch_offsets gives
 * both (count + 1 entries each, off[0] = 0).
 * Ownership, stream and error rules are those of the single-problem calls;
 * the workspace of dse_batch_workspace_bytes() holds every problem's tables
 * and buffers and the work queue.
 * ------------------------------------------------------------------------ */
typedef struct dse_batch dse_batch; /* opaque */

/* Result of dse_batch_autotune: the launch chosen and every candidate timed
 * (device ms of one Newton-matrix assembly of the whole family). */
typedef struct {
  int32_t slices;             /* angular slices per (row, radial tile)                */
  int32_t persistent_blocks;  /* 0: one workgroup per queue item; > 0: that many
                                 persistent workgroups taking items from the queue    */
  int32_t order;              /* 1: queue ordered largest item first; 0: problem order */
  int32_t n_candidates;
  double best_ms;
  int32_t cand_slices[32];
  int32_t cand_blocks[32];
  int32_t cand_order[32];
  double cand_ms[32];
  int32_t tiles_per_item;     /* partial tiles (64 radial nodes x one angular slice)
                                 of one row per queue item                            */
  int32_t fused;              /* 1: dressings, points, contraction and assembly rows
                                 in one cooperative launch of persistent_blocks
                                 resident workgroups, stages separated by grid-wide
                                 barriers; 0: one launch per stage                    */
  int32_t cand_tiles[32];
  int32_t cand_fused[32];
} dse_batch_tuning;

size_t dse_batch_workspace_bytes(const dse_params* p, int32_t count);
/* p[count]: validated like dse_init (DSE_E_INVALID names the problem). */
dse_status dse_batch_init(const dse_params* p, int32_t count, void* d_workspace, size_t ws_bytes,
                          void* hip_stream, dse_batch** out);
dse_status dse_batch_destroy(dse_batch* b);
const char* dse_batch_last_error(const dse_batch* b);
/* h_off_c, h_off_J: host arrays of count + 1 entries (either may be NULL). */
dse_status dse_batch_offsets(const dse_batch* b, int64_t* h_off_c, int64_t* h_off_J);
/* Start guesses (as dse_start_guess) of every problem into the packed d_c. */
dse_status dse_batch_start_guess(dse_batch* b, double* d_c);
/* Newton matrices and residuals of every problem at the packed d_c, into the
 * packed d_J and d_F (nullable).  Synchronises. */
dse_status dse_batch_jacobian(dse_batch* b, const double* d_c, double* d_J, double* d_F);
/* Every problem solved by the iteration of dse_newton_solve, step for step,
 * from the packed d_c (overwritten by the last iterates).  h_reports: host
 * array of count reports (nullable).  Returns DSE_OK when every problem
 * converged, else the status of the first problem that did not (its report
 * says which). */
dse_status dse_batch_newton_solve(dse_batch* b, double* d_c, const dse_newton_opts* opts,
                                  dse_newton_report* h_reports);
/* Times every launch candidate on the family's Newton-matrix assembly at d_c
 * (Sec. 5 studies the GPU block size by hand; this searches the launch
 * instead): angular slices 1, 2, 4 as the angular grid allows x one workgroup
 * per queue item, persistent workgroups filling the device, or the fused
 * cooperative launch (when the device offers cooperative launches) x 1, 2 or
 * 4 partial tiles per queue item, queue largest first; then problem order for
 * the best of them.  Keeps the fastest.  h_out nullable. */
dse_status dse_batch_autotune(dse_batch* b, const double* d_c, dse_batch_tuning* h_out);
/* Sets (or reads back) the launch explicitly: slices a power of two within
 * what the angular grid allows; tiles_per_item in [1, 64]; fused = 1 needs a
 * device with cooperative launches and 1 <= persistent_blocks <= the number of
 * workgroups that can be resident at once (else DSE_E_INVALID, message names
 * the limit).  The fused form changes the Newton-matrix assembly only; the
 * residual passes run staged with the same persistent workgroups.  Results
 * are bit-identical across launch forms with the same slices. */
dse_status dse_batch_set_launch_ex(dse_batch* b, int32_t slices, int32_t persistent_blocks, int32_t order,
                                   int32_t tiles_per_item, int32_t fused);
dse_status dse_batch_get_launch_ex(const dse_batch* b, int32_t* slices, int32_t* persistent_blocks,
                                   int32_t* order, int32_t* tiles_per_item, int32_t* fused);
/* The same with tiles_per_item = 1 and fused = 0. */
dse_status dse_batch_set_launch(dse_batch* b, int32_t slices, int32_t persistent_blocks, int32_t order);
dse_status dse_batch_get_launch(const dse_batch* b, int32_t* slices, int32_t* persistent_blocks,
                                int32_t* order);

#ifdef __cplusplus
}
#endif
#endif
