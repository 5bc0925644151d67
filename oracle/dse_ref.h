/*
 * dse_ref.h -- FP64 CPU oracle for the Landau-gauge ghost-gluon Dyson-Schwinger
 * system (Hopfer, Alkofer, Haase, "Solving the Ghost-Gluon System of Yang-Mills
 * Theory on GPUs", CPC / arXiv:1206.1779).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain reference that the
 * HIP implementation is checked against.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * Every function computes in double precision with straightforward loops.
 * Sums over quadrature points are taken in a fixed order (radial node outer,
 * angle inner) with Neumaier-compensated accumulation.
 *
 * Discrete problem (readings of the paper, each cited where implemented):
 *   unknowns  c = [a_0..a_{NZ-1}, b_0..b_{NG-1}]   (ln Z and ln G Chebyshev
 *             coefficients, Sec. 3 "vector notation for the Chebyshev
 *             coefficients")
 *   residual  F = [z(x^Z_0..x^Z_{NZ-1}); g(x^G_0..x^G_{NG-1})]  (Sec. 3, the
 *             collocation equations g(x_i;a,b)=0, z(x_i;a,b)=0)
 *   Jacobian  J[r][c] = dF_r/dc_c, row-major (Sec. 3 Newton matrix layout).
 */
#ifndef DSE_REF_H
#define DSE_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Physical and discretisation parameters (Sec. 2-3 of the paper). */
typedef struct {
  int32_t n_z;          /* Chebyshev coefficients of ln Z (vector a)            */
  int32_t n_g;          /* Chebyshev coefficients of ln G (vector b)            */
  int32_t n_rad;        /* Gauss-Legendre nodes in ln y on [eps2, lambda2]      */
  int32_t n_ir;         /* Gauss-Legendre nodes in ln y on the IR panel         */
  int32_t n_ang;        /* angular nodes                                        */
  int32_t quad;         /* quadrature rules, bits: 1 = tanh-sinh rule in
                           xi = cos(theta) for the angle (Sec. 2), 2 = radial
                           integral split at the external momentum x (Sec. 3);
                           0 = Gauss-Legendre in theta and one log-GL radial
                           grid shared by all rows                            */
  double eps2;          /* IR matching point epsilon^2 (lower end of mapping)  */
  double lambda2;       /* UV cutoff Lambda^2 (upper end of mapping)           */
  double ir_efolds;     /* IR panel covers [eps2*exp(-ir_efolds), eps2]        */
  double alpha_mu;      /* alpha(mu^2) = g^2/(4 pi)                             */
  double n_c;           /* number of colours                                   */
  double g0_inv;        /* G(x_G = 0)^{-1}; 0 selects the scaling solution     */
  double z_lambda_inv;  /* Z(x_Z = Lambda^2)^{-1}                              */
  double kappa;         /* IR exponent of the power laws                       */
  double delta;         /* ghost anomalous dimension                           */
  double gamma;         /* gluon anomalous dimension                           */
} dse_ref_params;

/* Newton options and report (Sec. 3 Newton-Raphson with under-relaxation). */
typedef struct {
  double tol;           /* stop once max_r |F_r| / S_r < tol                    */
  int32_t max_iter;     /* Newton iterations allowed                           */
  int32_t extra_iters;  /* full steps taken after convergence                  */
  int32_t max_halvings; /* backtracking halvings of the relaxation factor      */
  int32_t pad_;
  double step_tol;      /* after convergence, stop once rho*||Delta||_inf < it  */
} dse_ref_newton_opts;

typedef struct {
  int32_t iters;
  int32_t status;       /* 0 ok, 5 no convergence, 4 singular, 6 non-finite    */
  double fnorm;          /* final scaled residual max_r |F_r| / S_r             */
  double fnorm2;         /* final ||F||_2                                        */
  double fnorm_hist[128]; /* scaled residual before each iteration               */
  double relax_hist[128];
} dse_ref_newton_report;

/* -------- building blocks (exported so tests can pin each of them) -------- */

/* n-point Gauss-Legendre rule on [-1,1]: nodes ascending. */
int dse_ref_gauss_legendre(int n, double* nodes, double* weights);
/* Node i (ascending) of the same rule and its weight, computed alone. */
int dse_ref_gl_node(int n, int i, double* node, double* weight);

/* Tilde-T_j(s), j<n, with the c0/2 convention of Sec. 3 (Tilde-T_0 = 1/2). */
void dse_ref_cheb(double s, int n, double* out);

/* Mapping s(u) of Sec. 3, clamped to [-1,1]. */
double dse_ref_map(const dse_ref_params* p, double u);

/* ln Z(u), ln G(u): Chebyshev series inside [eps2, lambda2]; IR power laws
 * (Sec. 2, Z = A x^{2 kappa}, G = B x^{-kappa}) below eps2 and UV logs (Sec. 2,
 * G_UV [omega ln(x/x_UV)+1]^delta, likewise Z with gamma) above lambda2, both
 * matched to the series at the interval ends (Sec. 3, extrapolation by region). */
double dse_ref_lnZ(const dse_ref_params* p, const double* a, double u);
double dse_ref_lnG(const dse_ref_params* p, const double* b, double u);

/* Integral kernels of the gluon DSE (Sec. 2).  theta is the angle between p and q,
 * z = x + y - 2 sqrt(xy) cos(theta). */
double dse_ref_kernel_Q_printed(double x, double y, double z);
double dse_ref_kernel_Q(double x, double y, double theta);
double dse_ref_kernel_M_printed(double x, double y, double z);
double dse_ref_kernel_M(double x, double y, double theta);
double dse_ref_momentum_z(double x, double y, double theta);

/* Quadrature grid of the discretised problem: the shared radial grid (IR
 * panel, then n_rad log-GL nodes on [eps2, lambda2]), the angular rule as
 * theta nodes with d-theta weights v, and the external points. */
int dse_ref_grid_sizes(const dse_ref_params* p, int32_t* nq, int32_t* nk);
int dse_ref_grid(const dse_ref_params* p, double* y, double* W, double* theta, double* v,
                 double* x_z, double* x_g);
/* Radial grid of the row at external momentum x with the split of Sec. 3
 * (quad bit 2): the IR panel, then n_rad log-GL nodes on [eps2, x] and n_rad
 * on [x, lambda2]; for x outside (eps2, lambda2) the one interval
 * [eps2, lambda2].  y and W hold n_ir + 2 n_rad entries; returns the number
 * of nodes, or -1 for invalid parameters. */
int dse_ref_row_grid(const dse_ref_params* p, double x, double* y, double* W);

/* Self-energies Pi_Z(x), Pi_G(x) (Sec. 2) on an arbitrary radial grid
 * (y[q], W[q]: integral over y = sum_q W[q] f(y[q])) and angular grid
 * (theta[k], v[k]: integral over theta = sum_k v[k] f(theta[k])). */
double dse_ref_pi_gluon(const dse_ref_params* p, const double* c, double x,
                        int nq, const double* y, const double* W,
                        int nk, const double* theta, const double* v);
double dse_ref_pi_ghost(const dse_ref_params* p, const double* c, double x,
                        int nq, const double* y, const double* W,
                        int nk, const double* theta, const double* v);

/* ------------------------------ the method ------------------------------- */

/* F (length n_z+n_g). */
int dse_ref_residual(const dse_ref_params* p, const double* c, double* F);
/* Per-row magnitude scale: |direct| + |parameter| + sum |integrand| at the row
 * and at its subtraction point.  Bounds the rounding error of F. */
int dse_ref_residual_scale(const dse_ref_params* p, const double* c, double* S);
/* Analytic Jacobian (row-major n x n) and F (F may be NULL).  If rows != NULL
 * only the nrows listed rows of J are written (others untouched). */
int dse_ref_jacobian(const dse_ref_params* p, const double* c, double* J, double* F,
                     int nrows, const int32_t* rows);
/* Central finite-difference Jacobian, Sec. 4.2: column j uses c +- h_j e_j,
 * h_j = h_rel * max(1, |c_j|). */
int dse_ref_jacobian_fd(const dse_ref_params* p, const double* c, double h_rel, double* J);
/* Partial derivatives of F with respect to theta = (alpha_mu, g0_inv,
 * z_lambda_inv): out is n x 3 row-major. */
int dse_ref_dF_dtheta(const dse_ref_params* p, const double* c, double* out);

/* LU with partial pivoting, solves A x = b (A n x n row-major, overwritten by
 * its factors; x may alias b).  trans != 0 solves A^T x = b.  Returns 0 or 4
 * (singular). */
int dse_ref_lu_solve(int n, double* A, double* b, double* x, int trans);

/* Start guess built from the IR power laws and UV logarithms of Sec. 2,
 * interpolated at the collocation points. */
int dse_ref_start_guess(const dse_ref_params* p, double* c);
/* Newton iteration c <- c - rho J^{-1} F from the given c (Sec. 3). */
int dse_ref_newton(const dse_ref_params* p, double* c, const dse_ref_newton_opts* o,
                   dse_ref_newton_report* rep);

/* Renormalisation scale of Sec. 2.1 (footnote): the largest root mu2 in
 * [eps2, lambda2] of G^2(x) Z(x) = 1, found by a scan of `scan` equal
 * intervals in the mapped variable s (from s = 1 down) and bisection.
 * Returns 0, or 1 when there is no root (*mu2 = NaN). */
int dse_ref_renorm_scale(const dse_ref_params* p, const double* c, int scan, double* mu2);

/* Schwinger function of the gluon propagator (Sec. 2.2),
 * Delta(t) = (1/pi) int dp cos(t p) Z(p^2)/p^2, by the mapped Gauss-Legendre
 * rule p = p_max ((1 + x)/2)^2 on n nodes (Sec. 5): out[j] = Delta(t[j]).
 * dse_ref_schwinger_nodes gives the rule itself (p[n], weights W[n]). */
int dse_ref_schwinger_nodes(int n, double p_max, double* p, double* W);
int dse_ref_schwinger(const dse_ref_params* p, const double* c, int n, double p_max, const double* t, int m,
                      double* out);

/* Summation order of all quadrature sums: 0 forward, 1 reversed (used to
 * measure the oracle's own rounding floor). */
void dse_ref_set_order(int reversed);
/* Multiplies every quadrature weight by 1 +- rel (fixed sign pattern) to probe
 * how far the solution moves under rounding-level changes of the discrete
 * problem; 0 (default) switches it off. */
void dse_ref_set_jitter(double rel);
/* Number of OpenMP threads used (0 = library default). */
void dse_ref_set_threads(int n);
int dse_ref_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
