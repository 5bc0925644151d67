/*
 * dse_ref.c -- FP64 CPU oracle for the ghost-gluon Dyson-Schwinger system of
 * Hopfer, Alkofer, Haase (arXiv:1206.1779).
 *
 * TEST INFRASTRUCTURE ONLY: the plain reference the HIP library is checked
 * against.  Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg load it.  Nothing here is shared with the GPU library.
 *
 * Readings of the paper taken here (every one is listed with its reason in the
 * design notes of the repository):
 *  - ghost angular weight (1 - xi^2)^{3/2}: the printed (1 - xi)^{3/2} is a
 *    typesetting slip (the ghost loop carries p.P(k).q ~ (1 - xi^2) times the
 *    sqrt(1 - xi^2) measure of Sec. 2);
 *  - Newton step: solve J Delta = F and set c <- c - rho Delta (Sec. 3 update
 *    rule; the matrix equation of Sec. 3 has F on the right-hand side);
 *  - radial rule: Gauss-Legendre in t = ln y on [eps2, lambda2] plus an IR
 *    panel [eps2 e^{-ir_efolds}, eps2] standing for the integral from 0 to
 *    eps2 of the radial split in Sec. 3; one grid shared by all rows;
 *  - angular rule: Gauss-Legendre in theta on (0, pi) with the sin^2 (gluon)
 *    and sin^4 (ghost) measure factors written out;
 *  - external points: mapped roots of T_{n_z} for the gluon rows and of
 *    T_{n_g} for the ghost rows (Sec. 3 footnote), ascending;
 *  - the IR power laws extrapolate below eps2 for every boundary condition;
 *  - under-relaxation: rho starts at 1 and is halved while ||F|| does not
 *    decrease (Sec. 3 leaves the schedule open); no backtracking once
 *    ||F|| < tol.
 */
#include "dse_ref.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define REF_PI 3.14159265358979323846264338327950288
/* largest Gauss-Legendre rule the grid builder takes (nodes per panel) */
#define GL_MAX 4096

static int g_reversed = 0;
static int g_threads = 0;
static double g_jitter = 0.0;

void dse_ref_set_order(int reversed) { g_reversed = reversed ? 1 : 0; }
void dse_ref_set_jitter(double rel) { g_jitter = rel; }
void dse_ref_set_threads(int n) { g_threads = n > 0 ? n : 0; }
int dse_ref_get_threads(void) {
#ifdef _OPENMP
  return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Neumaier-compensated sum.                                                 */
typedef struct { double s, c; } ksum;
static void kadd(ksum* k, double v) {
  double t = k->s + v;
  if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
  else k->c += (v - t) + k->s;
  k->s = t;
}
static double kval(const ksum* k) { return k->s + k->c; }

/* ------------------------------------------------------------------------ */
/* Gauss-Legendre rule: Newton iteration on P_n from the three-term
 * recurrence (n+1) P_{n+1} = (2n+1) s P_n - n P_{n-1}.  One node at a time:
 * node i (ascending order) and its weight.                                 */
int dse_ref_gl_node(int n, int i, double* node, double* weight) {
  if (n < 1 || i < 0 || i >= n) return 1;
  /* root counted from +1 downwards */
  const int r = n - 1 - i;
  double s = cos(REF_PI * (r + 0.75) / (n + 0.5));
  double dp = 1.0;
  for (int it = 0; it < 100; ++it) {
    double p0 = 1.0, p1 = s;
    for (int k = 1; k < n; ++k) {
      double p2 = ((2.0 * k + 1.0) * s * p1 - k * p0) / (k + 1.0);
      p0 = p1;
      p1 = p2;
    }
    if (n == 1) { p1 = s; p0 = 1.0; }
    /* P_n'(s) = n (s P_n - P_{n-1}) / (s^2 - 1) */
    dp = n * (s * p1 - p0) / (s * s - 1.0);
    double ds = p1 / dp;
    s -= ds;
    if (fabs(ds) < 1e-16) {
      /* one more pass to settle the derivative at the final node */
      p0 = 1.0; p1 = s;
      for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * s * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = s; p0 = 1.0; }
      dp = n * (s * p1 - p0) / (s * s - 1.0);
      break;
    }
  }
  *node = s;
  *weight = 2.0 / ((1.0 - s * s) * dp * dp);
  return 0;
}

/* All n nodes, ascending (each node independently, so the threads change
 * nothing in the result). */
int dse_ref_gauss_legendre(int n, double* nodes, double* weights) {
  if (n < 1) return 1;
#pragma omp parallel for schedule(dynamic, 16) num_threads(dse_ref_get_threads()) if (n >= 2048)
  for (int i = 0; i < n; ++i) dse_ref_gl_node(n, i, &nodes[i], &weights[i]);
  return 0;
}

/* Tilde-T_j(s): T_0 carries the factor 1/2 of the expansion in Sec. 3. */
void dse_ref_cheb(double s, int n, double* out) {
  if (n <= 0) return;
  double tm1 = 1.0, t = s;
  out[0] = 0.5;
  if (n > 1) out[1] = s;
  for (int j = 2; j < n; ++j) {
    double tn = 2.0 * s * t - tm1;
    out[j] = tn;
    tm1 = t;
    t = tn;
  }
}

/* ------------------------------------------------------------------------ */
/* Derived constants (Sec. 2).                                               */
typedef struct {
  double C;      /* g^2 N_c / (2 pi)^3 = alpha N_c / (2 pi^2)                    */
  double omega;  /* 11 N_c alpha(mu^2) / (12 pi)                                 */
  double e1;     /* exponent of G(y)G(z) in the gluon loop: -2 - 6 delta         */
  double e2;     /* exponent of Z(y)Z(z) in the gluon loop: -3 delta             */
  double L0, L1; /* ln u = L0 + L1 s                                             */
} consts;

static consts make_consts(const dse_ref_params* p) {
  consts k;
  k.C = p->alpha_mu * p->n_c / (2.0 * REF_PI * REF_PI);
  k.omega = 11.0 * p->n_c * p->alpha_mu / (12.0 * REF_PI);
  k.e1 = -2.0 - 6.0 * p->delta;
  k.e2 = -3.0 * p->delta;
  k.L0 = 0.5 * (log(p->eps2) + log(p->lambda2));
  k.L1 = 0.5 * (log(p->lambda2) - log(p->eps2));
  return k;
}

/* Sec. 3: s(x) = log10(x / (Lambda eps)) / log10(Lambda / eps). */
double dse_ref_map(const dse_ref_params* p, double u) {
  double lam_eps = sqrt(p->lambda2 * p->eps2);
  double s = log10(u / lam_eps) / log10(sqrt(p->lambda2 / p->eps2));
  if (s < -1.0) s = -1.0;
  if (s > 1.0) s = 1.0;
  return s;
}

/* Extrapolation terms added to the Chebyshev series outside [eps2, lambda2]. */
static double ext_Z(const dse_ref_params* p, const consts* k, double u) {
  if (u < p->eps2) return 2.0 * p->kappa * log(u / p->eps2);
  if (u > p->lambda2) return p->gamma * log(k->omega * log(u / p->lambda2) + 1.0);
  return 0.0;
}
static double ext_G(const dse_ref_params* p, const consts* k, double u) {
  if (u < p->eps2) return -p->kappa * log(u / p->eps2);
  if (u > p->lambda2) return p->delta * log(k->omega * log(u / p->lambda2) + 1.0);
  return 0.0;
}
/* d(ext)/d(alpha) through omega (UV branch only). */
static double dext_dalpha(const dse_ref_params* p, const consts* k, double u, double expo) {
  if (u > p->lambda2) {
    double l = log(u / p->lambda2);
    return expo * (k->omega / p->alpha_mu) * l / (k->omega * l + 1.0);
  }
  return 0.0;
}

static double series(const double* coef, int n, const double* T) {
  double s = 0.0;
  for (int j = 0; j < n; ++j) s += coef[j] * T[j];
  return s;
}

double dse_ref_lnZ(const dse_ref_params* p, const double* a, double u) {
  consts k = make_consts(p);
  double T[1024];
  int n = p->n_z;
  dse_ref_cheb(dse_ref_map(p, u), n, T);
  return series(a, n, T) + ext_Z(p, &k, u);
}
double dse_ref_lnG(const dse_ref_params* p, const double* b, double u) {
  consts k = make_consts(p);
  double T[1024];
  int n = p->n_g;
  dse_ref_cheb(dse_ref_map(p, u), n, T);
  return series(b, n, T) + ext_G(p, &k, u);
}

/* ------------------------------------------------------------------------ */
/* Kernels of the gluon DSE (Sec. 2).                                        */
double dse_ref_kernel_M_printed(double x, double y, double z) {
  return (1.0 / z) * (-0.25 * x + 0.5 * y - 0.25 * y * y / x) + 0.5 + 0.5 * y / x - 0.25 * z / x;
}
double dse_ref_kernel_Q_printed(double x, double y, double z) {
  return (1.0 / (z * z)) * (x * x * x / (8.0 * y) + x * x - 2.25 * x * y + y * y + y * y * y / (8.0 * x))
       + (1.0 / z) * (x * x / y - 4.0 * (x + y) + y * y / x)
       - (2.25 * x / y + 4.0 + 2.25 * y / x)
       + z * (1.0 / x + 1.0 / y) + z * z / (8.0 * x * y) + 3.75;
}

/* z = x + y - 2 sqrt(xy) cos(theta), written as
 * max(x,y) [ (1-t)^2 + 4 t sin^2(theta/2) ],  t = sqrt(min/max),
 * which is the same number without the cancellation at y ~ x, theta ~ 0. */
double dse_ref_momentum_z(double x, double y, double theta) {
  double mx = x > y ? x : y, mn = x > y ? y : x;
  double t = sqrt(mn / mx);
  double sh = sin(0.5 * theta);
  return mx * ((1.0 - t) * (1.0 - t) + 4.0 * t * sh * sh);
}

/* Q(x,y,z) multiplied out over the common denominator z^2 and expressed in
 * t = sqrt(min/max), xi = cos(theta), w = z / max: algebraically identical to
 * the printed kernel (symmetric in x <-> y), free of the cancellation the
 * printed form suffers when y/x is far from 1. */
double dse_ref_kernel_Q(double x, double y, double theta) {
  double mx = x > y ? x : y, mn = x > y ? y : x;
  double t = sqrt(mn / mx);
  double xi = cos(theta);
  double sh = sin(0.5 * theta);
  double w = (1.0 - t) * (1.0 - t) + 4.0 * t * sh * sh;
  double t2 = t * t, t4 = t2 * t2;
  double num = -2.25 * (1.0 + t4) - 8.5 * t2
             + 2.0 * t2 * xi * xi * xi * xi
             - 12.0 * t * (1.0 + t2) * xi * xi * xi
             + (6.0 * (1.0 + t4) + 29.0 * t2) * xi * xi
             - 3.0 * t * (1.0 + t2) * xi;
  return num / (w * w);
}

/* M = y (1 - xi^2) / z, the printed kernel simplified (Sec. 2). */
double dse_ref_kernel_M(double x, double y, double theta) {
  double st = sin(theta);
  return y * st * st / dse_ref_momentum_z(x, y, theta);
}

/* ------------------------------------------------------------------------ */
/* Grid.                                                                     */
int dse_ref_grid_sizes(const dse_ref_params* p, int32_t* nq, int32_t* nk) {
  *nq = p->n_rad + p->n_ir;
  *nk = p->n_ang;
  return 0;
}

static int check_params(const dse_ref_params* p) {
  if (p->n_z < 1 || p->n_g < 1 || p->n_z > 1024 || p->n_g > 1024) return 1;
  if (p->quad & ~3) return 1;
  /* the tanh-sinh rule is symmetric about xi = 0: 2K + 1 nodes, K >= 1 */
  if ((p->quad & 1) && (p->n_ang < 3 || p->n_ang % 2 == 0)) return 1;
  /* the grid builder's Gauss-Legendre scratch holds GL_MAX nodes per rule */
  if (p->n_rad < 1 || p->n_ir < 0 || p->n_ang < 1) return 1;
  if (p->n_rad > GL_MAX || p->n_ir > GL_MAX || p->n_ang > GL_MAX) return 1;
  if (!(p->eps2 > 0.0) || !(p->lambda2 > p->eps2)) return 1;
  if (!(p->alpha_mu > 0.0) || !(p->n_c > 0.0)) return 1;
  if (p->n_ir > 0 && !(p->ir_efolds > 0.0)) return 1;
  return 0;
}

/* Tanh-sinh (double exponential) rule of Takahasi and Mori in xi = cos(theta)
 * on (-1, 1), the angular rule of Sec. 2: xi_k = tanh(u_k), u_k = (pi/2)
 * sinh(k h), weight h (pi/2) cosh(k h) / cosh(u_k)^2, k = -K .. K, n_ang =
 * 2K + 1, truncated at |k h| = 3 (there 1 - |xi| = 4e-14 and the weight is
 * 1e-12 of the central one): h = 3/K.  The
 * nodes go to the caller as angles, theta = 2 atan(sqrt((1 - xi)/(1 + xi)))
 * with 1 - xi = 2/(1 + e^{2u}) and 1 + xi = 2/(1 + e^{-2u}) (no cancellation
 * next to the ends), and d-theta weights v = w_xi / sin(theta): then
 * sum_k v_k sin^2(theta_k) f = sum_k w_k sqrt(1 - xi_k^2) f, the measure of
 * Sec. 2, and sum_k v_k sin^4(theta_k) f is the ghost's (1 - xi^2)^{3/2}.
 * Otherwise: Gauss-Legendre in theta on (0, pi). */
#define TS_TMAX 3.0
static void angular_rule(const dse_ref_params* p, double* theta, double* v) {
  if (p->quad & 1) {
    const int K = (p->n_ang - 1) / 2;
    const double h = TS_TMAX / K;
    for (int k = -K; k <= K; ++k) {
      double uk = 0.5 * REF_PI * sinh(k * h);
      double om = 2.0 / (1.0 + exp(2.0 * uk));   /* 1 - xi */
      double op = 2.0 / (1.0 + exp(-2.0 * uk));  /* 1 + xi */
      double ch = cosh(uk);
      double w = h * 0.5 * REF_PI * cosh(k * h) / (ch * ch);
      double th = 2.0 * atan(sqrt(om / op));
      theta[k + K] = th;
      v[k + K] = w / sqrt(om * op);
    }
    return;
  }
  double* u = (double*)malloc(sizeof(double) * p->n_ang);
  double* wu = (double*)malloc(sizeof(double) * p->n_ang);
  dse_ref_gauss_legendre(p->n_ang, u, wu);
  for (int k = 0; k < p->n_ang; ++k) {
    theta[k] = 0.5 * REF_PI * (1.0 + u[k]);
    v[k] = 0.5 * REF_PI * wu[k];
  }
  free(u);
  free(wu);
}

/* Gauss-Legendre in ln y on [ln a, ln b] (n nodes, starting at y[0]): the
 * integral over y of f is the integral over t = ln y of y f(y). */
static void log_gl(int n, double a, double b, const double* u, const double* wu, double* y, double* W) {
  for (int i = 0; i < n; ++i) {
    double t = 0.5 * (a + b) + 0.5 * (b - a) * u[i];
    y[i] = exp(t);
    W[i] = 0.5 * (b - a) * wu[i] * y[i];
  }
}

int dse_ref_row_grid(const dse_ref_params* p, double x, double* y, double* W) {
  if (check_params(p)) return -1;
  double lo = log(p->eps2), hi = log(p->lambda2);
  double* u = (double*)malloc(sizeof(double) * GL_MAX);
  double* wu = (double*)malloc(sizeof(double) * GL_MAX);
  int q = 0;
  if (p->n_ir > 0) {
    dse_ref_gauss_legendre(p->n_ir, u, wu);
    log_gl(p->n_ir, lo - p->ir_efolds, lo, u, wu, y, W);
    q = p->n_ir;
  }
  dse_ref_gauss_legendre(p->n_rad, u, wu);
  if (x > p->eps2 && x < p->lambda2) {
    log_gl(p->n_rad, lo, log(x), u, wu, y + q, W + q);
    q += p->n_rad;
    log_gl(p->n_rad, log(x), hi, u, wu, y + q, W + q);
    q += p->n_rad;
  } else {
    log_gl(p->n_rad, lo, hi, u, wu, y + q, W + q);
    q += p->n_rad;
  }
  if (g_jitter != 0.0)
    for (int i = 0; i < q; ++i) W[i] *= 1.0 + ((i * 7919 % 13) % 2 ? g_jitter : -g_jitter);
  free(u);
  free(wu);
  return q;
}

/* Radial: Gauss-Legendre in t = ln y on [ln eps2, ln lambda2] (n_rad nodes)
 * and on [ln eps2 - ir_efolds, ln eps2] (n_ir nodes); the integral over y of
 * f is the integral over t of y f(y), so W = w_t * y.  Angular: Gauss-Legendre
 * in theta on (0, pi).  External points: x_i = s^{-1}(-cos(pi (i+1/2)/N)). */
int dse_ref_grid(const dse_ref_params* p, double* y, double* W, double* theta, double* v,
                 double* x_z, double* x_g) {
  if (check_params(p)) return 1;
  double lo = log(p->eps2), hi = log(p->lambda2);
  double* u = (double*)malloc(sizeof(double) * GL_MAX);
  double* wu = (double*)malloc(sizeof(double) * GL_MAX);
  int q = 0;
  if (p->n_ir > 0) {
    dse_ref_gauss_legendre(p->n_ir, u, wu);
    double a = lo - p->ir_efolds, b = lo;
    for (int i = 0; i < p->n_ir; ++i, ++q) {
      double t = 0.5 * (a + b) + 0.5 * (b - a) * u[i];
      y[q] = exp(t);
      W[q] = 0.5 * (b - a) * wu[i] * y[q];
    }
  }
  dse_ref_gauss_legendre(p->n_rad, u, wu);
  for (int i = 0; i < p->n_rad; ++i, ++q) {
    double t = 0.5 * (lo + hi) + 0.5 * (hi - lo) * u[i];
    y[q] = exp(t);
    W[q] = 0.5 * (hi - lo) * wu[i] * y[q];
  }
  angular_rule(p, theta, v);
  /* rounding-floor probe: scale every weight by 1 +- g_jitter (0 by default) */
  if (g_jitter != 0.0) {
    for (int i = 0; i < p->n_ir + p->n_rad; ++i) W[i] *= 1.0 + ((i * 7919 % 13) % 2 ? g_jitter : -g_jitter);
    for (int k = 0; k < p->n_ang; ++k) v[k] *= 1.0 + ((k * 104729 % 11) % 2 ? g_jitter : -g_jitter);
  }
  consts kc = make_consts(p);
  for (int i = 0; i < p->n_z; ++i)
    x_z[i] = exp(kc.L0 + kc.L1 * (-cos(REF_PI * (i + 0.5) / p->n_z)));
  for (int i = 0; i < p->n_g; ++i)
    x_g[i] = exp(kc.L0 + kc.L1 * (-cos(REF_PI * (i + 0.5) / p->n_g)));
  free(u);
  free(wu);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* One row of the self-energies with its derivatives.                        */
typedef struct {
  double pi;      /* Pi(x)                                                     */
  double abssum;  /* sum of |integrand|                                        */
  double dalpha;  /* dPi/d alpha                                               */
  double* da;     /* dPi/da_j (n_z) or NULL                                    */
  double* db;     /* dPi/db_j (n_g) or NULL                                    */
} rowres;

/* kind 0: gluon self-energy Pi_Z(x); kind 1: ghost self-energy Pi_G(x).
 * Sec. 2 (after the MOM-free form):
 *   Pi_G(x) = -C int dy y G(y) int dxi (1-xi^2)^{3/2} Z(z)/z^2
 *   Pi_Z(x) =  C/(3x) int dy int dxi (1-xi^2)^{1/2}
 *                [Q (G(y)G(z))^{-2-6 delta} (Z(y)Z(z))^{-3 delta} + M G(y)G(z)]
 * with int dxi (1-xi^2)^{1/2} f = int dtheta sin^2 theta f,
 *      int dxi (1-xi^2)^{3/2} f = int dtheta sin^4 theta f. */
static void row_eval(const dse_ref_params* p, const double* c, double x,
                     int nq, const double* y, const double* W,
                     int nk, const double* th, const double* v,
                     int kind, rowres* out) {
  consts k = make_consts(p);
  const double* a = c;
  const double* b = c + p->n_z;
  int nz = p->n_z, ng = p->n_g;
  int nmax = nz > ng ? nz : ng;
  double* Ty = (double*)malloc(sizeof(double) * nmax);
  double* Tz = (double*)malloc(sizeof(double) * nmax);
  ksum pi = {0, 0}, abss = {0, 0}, dal = {0, 0};
  ksum* da = out->da ? (ksum*)calloc(nz, sizeof(ksum)) : NULL;
  ksum* db = out->db ? (ksum*)calloc(ng, sizeof(ksum)) : NULL;

  for (int qq = 0; qq < nq; ++qq) {
    int q = g_reversed ? nq - 1 - qq : qq;
    double yq = y[q];
    dse_ref_cheb(dse_ref_map(p, yq), nmax, Ty);
    double lnGy = series(b, ng, Ty) + ext_G(p, &k, yq);
    double lnZy = series(a, nz, Ty) + ext_Z(p, &k, yq);
    for (int kk = 0; kk < nk; ++kk) {
      int kq = g_reversed ? nk - 1 - kk : kk;
      double theta = th[kq];
      double st = sin(theta);
      double z = dse_ref_momentum_z(x, yq, theta);
      dse_ref_cheb(dse_ref_map(p, z), nmax, Tz);
      double lnZz = series(a, nz, Tz) + ext_Z(p, &k, z);
      if (kind == 0) {
        double lnGz = series(b, ng, Tz) + ext_G(p, &k, z);
        double Fgl = exp(k.e1 * (lnGy + lnGz) + k.e2 * (lnZy + lnZz));
        double Fgh = exp(lnGy + lnGz);
        double Qk = dse_ref_kernel_Q(x, yq, theta);
        double Mk = dse_ref_kernel_M(x, yq, theta);
        double omg = k.C / (3.0 * x) * W[q] * v[kq] * st * st;
        double val = omg * (Qk * Fgl + Mk * Fgh);
        kadd(&pi, val);
        kadd(&abss, fabs(omg * Qk * Fgl) + fabs(omg * Mk * Fgh));
        double Pa = omg * Qk * Fgl * k.e2;            /* d val / d lnZ(y or z) */
        double Pb = omg * (Qk * Fgl * k.e1 + Mk * Fgh); /* d val / d lnG(y or z) */
        /* alpha: linear through C, and through omega in the UV extension */
        double dz = dext_dalpha(p, &k, z, p->gamma), dg = dext_dalpha(p, &k, z, p->delta);
        kadd(&dal, val / p->alpha_mu + Pa * dz + Pb * dg);
        if (da) for (int j = 0; j < nz; ++j) kadd(&da[j], Pa * (Ty[j] + Tz[j]));
        if (db) for (int j = 0; j < ng; ++j) kadd(&db[j], Pb * (Ty[j] + Tz[j]));
      } else {
        double Gy = exp(lnGy), Zz = exp(lnZz);
        double rho = -k.C * W[q] * yq * v[kq] * st * st * st * st;
        double val = rho * Gy * Zz / (z * z);
        kadd(&pi, val);
        kadd(&abss, fabs(val));
        kadd(&dal, val / p->alpha_mu + val * dext_dalpha(p, &k, z, p->gamma));
        if (da) for (int j = 0; j < nz; ++j) kadd(&da[j], val * Tz[j]);
        if (db) for (int j = 0; j < ng; ++j) kadd(&db[j], val * Ty[j]);
      }
    }
  }
  out->pi = kval(&pi);
  out->abssum = kval(&abss);
  out->dalpha = kval(&dal);
  if (da) for (int j = 0; j < nz; ++j) out->da[j] = kval(&da[j]);
  if (db) for (int j = 0; j < ng; ++j) out->db[j] = kval(&db[j]);
  free(Ty); free(Tz); free(da); free(db);
}

double dse_ref_pi_gluon(const dse_ref_params* p, const double* c, double x,
                        int nq, const double* y, const double* W,
                        int nk, const double* theta, const double* v) {
  rowres r = {0, 0, 0, NULL, NULL};
  row_eval(p, c, x, nq, y, W, nk, theta, v, 0, &r);
  return r.pi;
}
double dse_ref_pi_ghost(const dse_ref_params* p, const double* c, double x,
                        int nq, const double* y, const double* W,
                        int nk, const double* theta, const double* v) {
  rowres r = {0, 0, 0, NULL, NULL};
  row_eval(p, c, x, nq, y, W, nk, theta, v, 1, &r);
  return r.pi;
}

/* ------------------------------------------------------------------------ */
/* The discretised system of Sec. 3.                                         */
typedef struct {
  int nq, nk;
  double *y, *W, *th, *v, *xz, *xg;
} grid_t;

static int grid_make(const dse_ref_params* p, grid_t* g) {
  if (check_params(p)) return 1;
  g->nq = p->n_rad + p->n_ir;
  g->nk = p->n_ang;
  g->y = (double*)malloc(sizeof(double) * g->nq);
  g->W = (double*)malloc(sizeof(double) * g->nq);
  g->th = (double*)malloc(sizeof(double) * g->nk);
  g->v = (double*)malloc(sizeof(double) * g->nk);
  g->xz = (double*)malloc(sizeof(double) * p->n_z);
  g->xg = (double*)malloc(sizeof(double) * p->n_g);
  return dse_ref_grid(p, g->y, g->W, g->th, g->v, g->xz, g->xg);
}
static void grid_free(grid_t* g) {
  free(g->y); free(g->W); free(g->th); free(g->v); free(g->xz); free(g->xg);
}

static int all_finite(const double* v, int n) {
  for (int i = 0; i < n; ++i) if (!isfinite(v[i])) return 0;
  return 1;
}

/* Row index r of F: r < n_z is the gluon equation at x^Z_r, otherwise the
 * ghost equation at x^G_{r-n_z}.  The two subtraction rows (x_Z = lambda2
 * for the gluon, x_G = 0 for the ghost, Sec. 2 MOM scheme) are rows
 * n and n+1 of the internal row list. */
static void row_point(const dse_ref_params* p, const grid_t* g, int r, double* x, int* kind) {
  int n = p->n_z + p->n_g;
  if (r < p->n_z) { *x = g->xz[r]; *kind = 0; }
  else if (r < n) { *x = g->xg[r - p->n_z]; *kind = 1; }
  else if (r == n) { *x = p->lambda2; *kind = 0; }
  else { *x = 0.0; *kind = 1; }
}

/* Evaluates every requested internal row and always the two subtraction
 * rows; rows run in parallel, each row's sums stay sequential. */
static void eval_rows(const dse_ref_params* p, const double* c, const grid_t* g,
                      const unsigned char* need, rowres* rr) {
  int n = p->n_z + p->n_g;
  int nthreads = dse_ref_get_threads();
  (void)nthreads;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
  for (int r = 0; r < n + 2; ++r) {
    if (r < n && need && !need[r]) continue;
    double x; int kind;
    row_point(p, g, r, &x, &kind);
    if (p->quad & 2) {
      /* the row's own radial grid, split at x (Sec. 3) */
      double* y = (double*)malloc(sizeof(double) * (p->n_ir + 2 * p->n_rad));
      double* W = (double*)malloc(sizeof(double) * (p->n_ir + 2 * p->n_rad));
      int nq = dse_ref_row_grid(p, x, y, W);
      row_eval(p, c, x, nq, y, W, g->nk, g->th, g->v, kind, &rr[r]);
      free(y);
      free(W);
    } else {
      row_eval(p, c, x, g->nq, g->y, g->W, g->nk, g->th, g->v, kind, &rr[r]);
    }
  }
}

static rowres* rows_alloc(const dse_ref_params* p, int want_d) {
  int n = p->n_z + p->n_g;
  rowres* rr = (rowres*)calloc(n + 2, sizeof(rowres));
  for (int r = 0; r < n + 2; ++r) {
    if (want_d) {
      rr[r].da = (double*)calloc(p->n_z, sizeof(double));
      rr[r].db = (double*)calloc(p->n_g, sizeof(double));
    }
  }
  return rr;
}
static void rows_free(const dse_ref_params* p, rowres* rr) {
  int n = p->n_z + p->n_g;
  for (int r = 0; r < n + 2; ++r) { free(rr[r].da); free(rr[r].db); }
  free(rr);
}

/* Direct term G(x)^{-1} or Z(x)^{-1} at a row's external point. */
static double direct_term(const dse_ref_params* p, const double* c, double x, int kind) {
  if (kind == 0) return exp(-dse_ref_lnZ(p, c, x));
  return exp(-dse_ref_lnG(p, c + p->n_z, x));
}

/* Sec. 3:
 *   z(x_i) = Z(x_i)^{-1} - Z(x_Z)^{-1} - Pi_Z(x_i) + Pi_Z(x_Z)
 *   g(x_i) = G(x_i)^{-1} - G(x_G)^{-1} - Pi_G(x_i) + Pi_G(x_G)          */
static void assemble_F(const dse_ref_params* p, const double* c, const grid_t* g,
                       const rowres* rr, double* F) {
  int n = p->n_z + p->n_g;
  for (int r = 0; r < n; ++r) {
    double x; int kind;
    row_point(p, g, r, &x, &kind);
    double sub = kind == 0 ? rr[n].pi : rr[n + 1].pi;
    double par = kind == 0 ? p->z_lambda_inv : p->g0_inv;
    F[r] = direct_term(p, c, x, kind) - par - rr[r].pi + sub;
  }
}

/* F and, if S != NULL, the per-row scale S_r = |direct| + |parameter| +
 * sum|integrand| at x_r + sum|integrand| at the subtraction point: the size of
 * the terms that cancel in F_r, which bounds its rounding error. */
static int resid_scale(const dse_ref_params* p, const double* c, double* F, double* S) {
  grid_t g;
  if (grid_make(p, &g)) return 1;
  int n = p->n_z + p->n_g;
  rowres* rr = rows_alloc(p, 0);
  eval_rows(p, c, &g, NULL, rr);
  assemble_F(p, c, &g, rr, F);
  if (S)
    for (int r = 0; r < n; ++r) {
      double x; int kind;
      row_point(p, &g, r, &x, &kind);
      double sub = kind == 0 ? rr[n].abssum : rr[n + 1].abssum;
      double par = kind == 0 ? p->z_lambda_inv : p->g0_inv;
      S[r] = fabs(direct_term(p, c, x, kind)) + fabs(par) + rr[r].abssum + sub;
    }
  rows_free(p, rr);
  grid_free(&g);
  return all_finite(F, n) ? 0 : 6;
}

int dse_ref_residual(const dse_ref_params* p, const double* c, double* F) {
  return resid_scale(p, c, F, NULL);
}

int dse_ref_residual_scale(const dse_ref_params* p, const double* c, double* S) {
  int n = p->n_z + p->n_g;
  double* F = (double*)malloc(sizeof(double) * n);
  int st = resid_scale(p, c, F, S);
  free(F);
  return st == 1 ? 1 : 0;
}

/* Analytic Jacobian: differentiate F term by term.  d lnZ(u)/d a_j =
 * d lnG(u)/d b_j = Tilde-T_j(s(u)) for every u (the extrapolations are
 * matched at the interval ends and carry the coefficients along).
 *   dz(x_i)/da_j = -Z(x_i)^{-1} T_j(s_i) - dPi_Z(x_i)/da_j + dPi_Z(x_Z)/da_j
 *   dz(x_i)/db_j =                      - dPi_Z(x_i)/db_j + dPi_Z(x_Z)/db_j
 *   dg(x_i)/da_j =                      - dPi_G(x_i)/da_j + dPi_G(x_G)/da_j
 *   dg(x_i)/db_j = -G(x_i)^{-1} T_j(s_i) - dPi_G(x_i)/db_j + dPi_G(x_G)/db_j */
int dse_ref_jacobian(const dse_ref_params* p, const double* c, double* J, double* F,
                     int nrows, const int32_t* rows) {
  grid_t g;
  if (grid_make(p, &g)) return 1;
  int n = p->n_z + p->n_g;
  unsigned char* need = NULL;
  if (rows) {
    need = (unsigned char*)calloc(n, 1);
    for (int i = 0; i < nrows; ++i)
      if (rows[i] >= 0 && rows[i] < n) need[rows[i]] = 1;
  }
  /* F needs every row */
  if (F) { free(need); need = NULL; }
  rowres* rr = rows_alloc(p, 1);
  eval_rows(p, c, &g, need, rr);
  double* T = (double*)malloc(sizeof(double) * (n + 1));
  for (int r = 0; r < n; ++r) {
    if (need && !need[r]) continue;
    double x; int kind;
    row_point(p, &g, r, &x, &kind);
    const rowres* sub = kind == 0 ? &rr[n] : &rr[n + 1];
    double* Jr = J + (size_t)r * n;
    for (int j = 0; j < p->n_z; ++j) Jr[j] = -rr[r].da[j] + sub->da[j];
    for (int j = 0; j < p->n_g; ++j) Jr[p->n_z + j] = -rr[r].db[j] + sub->db[j];
    int nn = kind == 0 ? p->n_z : p->n_g;
    dse_ref_cheb(dse_ref_map(p, x), nn, T);
    double d = direct_term(p, c, x, kind);
    int off = kind == 0 ? 0 : p->n_z;
    for (int j = 0; j < nn; ++j) Jr[off + j] += -d * T[j];
  }
  if (F) assemble_F(p, c, &g, rr, F);
  int ok = 1;
  for (int r = 0; r < n; ++r) {
    if (need && !need[r]) continue;
    if (!all_finite(J + (size_t)r * n, n)) ok = 0;
  }
  free(T);
  free(need);
  rows_free(p, rr);
  grid_free(&g);
  if (F && !all_finite(F, n)) ok = 0;
  return ok ? 0 : 6;
}

int dse_ref_jacobian_fd(const dse_ref_params* p, const double* c, double h_rel, double* J) {
  int n = p->n_z + p->n_g;
  double* cp = (double*)malloc(sizeof(double) * n);
  double* Fp = (double*)malloc(sizeof(double) * n);
  double* Fm = (double*)malloc(sizeof(double) * n);
  int st = 0;
  for (int j = 0; j < n && !st; ++j) {
    double h = h_rel * (fabs(c[j]) > 1.0 ? fabs(c[j]) : 1.0);
    memcpy(cp, c, sizeof(double) * n);
    cp[j] = c[j] + h;
    st |= dse_ref_residual(p, cp, Fp);
    cp[j] = c[j] - h;
    st |= dse_ref_residual(p, cp, Fm);
    for (int r = 0; r < n; ++r) J[(size_t)r * n + j] = (Fp[r] - Fm[r]) / (2.0 * h);
  }
  free(cp); free(Fp); free(Fm);
  return st;
}

/* dF/dtheta, theta = (alpha_mu, g0_inv, z_lambda_inv). */
int dse_ref_dF_dtheta(const dse_ref_params* p, const double* c, double* out) {
  grid_t g;
  if (grid_make(p, &g)) return 1;
  int n = p->n_z + p->n_g;
  rowres* rr = rows_alloc(p, 0);
  eval_rows(p, c, &g, NULL, rr);
  for (int r = 0; r < n; ++r) {
    int kind = r < p->n_z ? 0 : 1;
    double sub = kind == 0 ? rr[n].dalpha : rr[n + 1].dalpha;
    out[3 * r + 0] = -rr[r].dalpha + sub;
    out[3 * r + 1] = kind == 1 ? -1.0 : 0.0;
    out[3 * r + 2] = kind == 0 ? -1.0 : 0.0;
  }
  rows_free(p, rr);
  grid_free(&g);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Dense LU with partial pivoting (Doolittle, row interchanges).  The matrix */
/* counts as singular (status 4) when a pivot is zero, not finite, or at    */
/* most n eps times the largest |entry| of its row of the input: singular   */
/* to working precision, whatever the scale of each row.                    */
int dse_ref_lu_solve(int n, double* A, double* b, double* x, int trans) {
  int* piv = (int*)malloc(sizeof(int) * n);
  double* rm = (double*)malloc(sizeof(double) * n);
  int st = 0;
  for (int i = 0; i < n; ++i) {
    rm[i] = 0.0;
    for (int j = 0; j < n; ++j) rm[i] = fmax(rm[i], fabs(A[(size_t)i * n + j]));
  }
  for (int k = 0; k < n; ++k) {
    int pr = k;
    double best = fabs(A[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      double a = fabs(A[(size_t)i * n + k]);
      if (a > best) { best = a; pr = i; }
    }
    piv[k] = pr;
    if (!(best > 0.0) || !isfinite(best)) { st = 4; break; }
    if (pr != k) {
      for (int j = 0; j < n; ++j) {
        double t = A[(size_t)k * n + j];
        A[(size_t)k * n + j] = A[(size_t)pr * n + j];
        A[(size_t)pr * n + j] = t;
      }
      double t = rm[k]; rm[k] = rm[pr]; rm[pr] = t;
    }
    double d = A[(size_t)k * n + k];
    if (!(fabs(d) > n * DBL_EPSILON * rm[k])) { st = 4; break; }
    for (int i = k + 1; i < n; ++i) {
      double l = A[(size_t)i * n + k] / d;
      A[(size_t)i * n + k] = l;
      for (int j = k + 1; j < n; ++j) A[(size_t)i * n + j] -= l * A[(size_t)k * n + j];
    }
  }
  free(rm);
  if (st) { free(piv); return st; }
  double* w = (double*)malloc(sizeof(double) * n);
  memcpy(w, b, sizeof(double) * n);
  if (!trans) {
    /* P A = L U: apply P, then L y = P b, then U x = y */
    for (int k = 0; k < n; ++k) { double t = w[k]; w[k] = w[piv[k]]; w[piv[k]] = t; }
    for (int i = 0; i < n; ++i) {
      double s = w[i];
      for (int j = 0; j < i; ++j) s -= A[(size_t)i * n + j] * w[j];
      w[i] = s;
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = w[i];
      for (int j = i + 1; j < n; ++j) s -= A[(size_t)i * n + j] * w[j];
      w[i] = s / A[(size_t)i * n + i];
    }
  } else {
    /* A^T = U^T L^T P: U^T y = b, L^T z = y, x = P^T z */
    for (int i = 0; i < n; ++i) {
      double s = w[i];
      for (int j = 0; j < i; ++j) s -= A[(size_t)j * n + i] * w[j];
      w[i] = s / A[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = w[i];
      for (int j = i + 1; j < n; ++j) s -= A[(size_t)j * n + i] * w[j];
      w[i] = s;
    }
    for (int k = n - 1; k >= 0; --k) { double t = w[k]; w[k] = w[piv[k]]; w[piv[k]] = t; }
  }
  memcpy(x, w, sizeof(double) * n);
  free(w);
  free(piv);
  return 0;
}

static double norm2(const double* v, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += v[i] * v[i];
  return sqrt(s);
}
static double norminf(const double* v, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) if (fabs(v[i]) > s) s = fabs(v[i]);
  return s;
}
/* Scaled residual max_r |F_r| / S_r: F relative to the size of its terms
 * (the convergence test). */
static double merit(const double* F, const double* S, int n) {
  double m = 0.0;
  for (int i = 0; i < n; ++i) {
    double v = S[i] > 0.0 ? fabs(F[i]) / S[i] : fabs(F[i]);
    if (!(v <= m)) m = v; /* propagates NaN */
  }
  return m;
}
/* Euclidean norm of the scaled residual, (sum_r (F_r / S_r)^2)^{1/2}: the
 * function the relaxation must decrease (smooth, unlike the maximum, whose
 * plateaus stall the halving rule far from the root). */
static double merit2(const double* F, const double* S, int n) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) {
    double v = S[i] > 0.0 ? F[i] / S[i] : F[i];
    s += v * v;
  }
  return sqrt(s);
}

/* Sec. 3: c^{n+1} = c^n - rho Delta^{n+1} with J Delta = F.  rho starts at 1
 * and is halved (at most max_halvings times) while the scaled residual of the
 * trial point does not drop below the current one.  Convergence: scaled
 * residual < tol; then extra_iters full steps are taken (no backtracking),
 * stopping early once rho ||Delta||_inf < step_tol. */
int dse_ref_newton(const dse_ref_params* p, double* c, const dse_ref_newton_opts* o,
                   dse_ref_newton_report* rep) {
  int n = p->n_z + p->n_g;
  double* F = (double*)malloc(sizeof(double) * n);
  double* S = (double*)malloc(sizeof(double) * n);
  double* J = (double*)malloc(sizeof(double) * n * n);
  double* d = (double*)malloc(sizeof(double) * n);
  double* ct = (double*)malloc(sizeof(double) * n);
  double* Ft = (double*)malloc(sizeof(double) * n);
  double* St = (double*)malloc(sizeof(double) * n);
  memset(rep, 0, sizeof(*rep));
  int st = resid_scale(p, c, F, S);
  double f = st ? INFINITY : merit(F, S, n);
  double f2 = st ? INFINITY : merit2(F, S, n);
  rep->fnorm_hist[0] = f;
  int it = 0, extra = 0;
  if (st) goto done;
  for (;;) {
    if (f < o->tol) {
      if (extra >= o->extra_iters) { st = 0; break; }
      ++extra;
    }
    if (it >= o->max_iter) { st = 5; break; }
    st = dse_ref_jacobian(p, c, J, NULL, 0, NULL);
    if (st) break;
    st = dse_ref_lu_solve(n, J, F, d, 0);
    if (st) break;
    double rho = 1.0, ft = INFINITY, ft2 = INFINITY;
    int converged = f < o->tol;
    for (int h = 0;; ++h) {
      for (int i = 0; i < n; ++i) ct[i] = c[i] - rho * d[i];
      int s2 = resid_scale(p, ct, Ft, St);
      ft = s2 ? INFINITY : merit(Ft, St, n);
      ft2 = s2 ? INFINITY : merit2(Ft, St, n);
      if (!isfinite(ft)) ft2 = INFINITY;
      if (converged || ft2 < f2 || h >= o->max_halvings) break;
      rho *= 0.5;
    }
    if (!isfinite(ft)) { st = 6; break; }
    memcpy(c, ct, sizeof(double) * n);
    memcpy(F, Ft, sizeof(double) * n);
    memcpy(S, St, sizeof(double) * n);
    f = ft;
    f2 = ft2;
    ++it;
    if (it < 128) { rep->fnorm_hist[it] = f; rep->relax_hist[it - 1] = rho; }
    if (converged && rho * norminf(d, n) < o->step_tol) { st = 0; break; }
  }
done:
  rep->iters = it;
  rep->status = st;
  rep->fnorm = f;
  rep->fnorm2 = norm2(F, n);
  free(F); free(S); free(J); free(d); free(ct); free(Ft); free(St);
  return st;
}

/* Start guess from the asymptotic forms of Sec. 2: IR power laws
 * (G ~ x^{-kappa}, Z ~ x^{2 kappa}) joined to the one-loop UV logarithms
 * (G ~ [omega ln x + 1]^delta, Z ~ [...]^gamma) at a scale mu2 chosen so that
 * Z(lambda2) equals the subtraction value:
 *   L(x)   = ln(1 + omega ln(1 + x/mu2))
 *   ln G0  = -kappa ln((x + m2)/(x + mu2)) + delta L(x)
 *   ln Z0  = 2 kappa ln(x/(x + mu2)) + gamma L(x)        (g0_inv = 0)
 *   ln Z0  = ln(x/(x + mu2)) + gamma L(x)                (g0_inv > 0)
 * with m2 = 0 for the scaling case and m2 = mu2 g0_inv^{1/kappa} otherwise
 * (so that G0(0) = 1/g0_inv).  The coefficients interpolate ln G0, ln Z0 at
 * the collocation points (discrete Chebyshev transform at the roots). */
int dse_ref_start_guess(const dse_ref_params* p, double* c) {
  if (check_params(p)) return 1;
  consts k = make_consts(p);
  double zl = 1.0 / p->z_lambda_inv;
  double r = pow(zl, 1.0 / p->gamma);
  double mu2 = r > 1.0 + 1e-9 ? p->lambda2 / (exp((r - 1.0) / k.omega) - 1.0) : 1e6 * p->lambda2;
  double m2 = p->g0_inv > 0.0 ? mu2 * pow(p->g0_inv, 1.0 / p->kappa) : 0.0;
  for (int f = 0; f < 2; ++f) {
    int N = f == 0 ? p->n_z : p->n_g;
    double* out = f == 0 ? c : c + p->n_z;
    double* T = (double*)malloc(sizeof(double) * N);
    for (int j = 0; j < N; ++j) out[j] = 0.0;
    for (int i = 0; i < N; ++i) {
      double s = -cos(REF_PI * (i + 0.5) / N);
      double x = exp(k.L0 + k.L1 * s);
      double L = log(1.0 + k.omega * log(1.0 + x / mu2));
      double val;
      if (f == 0)
        val = (p->g0_inv > 0.0 ? log(x / (x + mu2)) : 2.0 * p->kappa * log(x / (x + mu2)))
            + p->gamma * L;
      else
        val = -p->kappa * log((x + m2) / (x + mu2)) + p->delta * L;
      dse_ref_cheb(s, N, T);
      T[0] = 1.0; /* the transform uses T_0 itself; the series halves c_0 */
      for (int j = 0; j < N; ++j) out[j] += 2.0 / N * val * T[j];
    }
    free(T);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Renormalisation scale (Sec. 2.1 footnote): mu^2 is where the running
 * coupling alpha(x) = alpha(mu^2) G^2(x) Z(x) equals alpha(mu^2), i.e. the
 * root of h(x) = 2 ln G(x) + ln Z(x).  Of several roots in [eps2, lambda2]
 * the largest is taken (the perturbative side: a decoupling solution's
 * alpha(x) also rises through alpha(mu^2) in the infrared).  The search runs
 * in the mapped variable s: a scan of `scan` equal intervals from s = 1
 * downwards finds the first sign change, bisection narrows it to adjacent
 * doubles.  Returns 0 and *mu2, or 1 (no root; *mu2 = NaN). */
static double renorm_h(const dse_ref_params* p, const double* c, double s) {
  double u = exp(make_consts(p).L0 + make_consts(p).L1 * s);
  if (s <= -1.0) u = p->eps2;
  if (s >= 1.0) u = p->lambda2;
  return 2.0 * dse_ref_lnG(p, c + p->n_z, u) + dse_ref_lnZ(p, c, u);
}
int dse_ref_renorm_scale(const dse_ref_params* p, const double* c, int scan, double* mu2) {
  *mu2 = NAN;
  if (check_params(p) || scan < 1) return 1;
  double hi = 1.0, hhi = renorm_h(p, c, hi);
  for (int k = scan - 1; k >= 0; --k) {
    double lo = -1.0 + 2.0 * k / scan;
    double hlo = renorm_h(p, c, lo);
    if (hhi == 0.0) { *mu2 = exp(make_consts(p).L0 + make_consts(p).L1 * hi); return 0; }
    if ((hlo < 0.0) != (hhi < 0.0) || hlo == 0.0) {
      /* bisection on [lo, hi], h(lo) and h(hi) of opposite sign (or h(lo) = 0) */
      for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        double hm = renorm_h(p, c, mid);
        if ((hm < 0.0) == (hhi < 0.0) && hm != 0.0) { hi = mid; hhi = hm; }
        else { lo = mid; hlo = hm; }
      }
      double s = fabs(hlo) <= fabs(hhi) ? lo : hi;
      *mu2 = exp(make_consts(p).L0 + make_consts(p).L1 * s);
      return 0;
    }
    hi = lo;
    hhi = hlo;
  }
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Schwinger function of the gluon propagator (Sec. 2.2):
 *   Delta(t) = (1/pi) int_0^inf dp cos(t p) sigma(p^2),  sigma = Z(p^2)/p^2,
 * with a mapped Gauss-Legendre rule (Sec. 5): p = p_max ((1 + x)/2)^2 over the
 * n nodes x_i of [-1, 1], dp = p_max (1 + x)/2 dx, so the rule covers
 * [0, p_max] (the oscillating tail beyond p_max is left out; it is of order
 * Z(p_max^2) / (t p_max^2)).  The square clusters the nodes towards p = 0,
 * where sigma carries the infrared power law.                              */
int dse_ref_schwinger_nodes(int n, double p_max, double* pn, double* Wn) {
  if (n < 1 || !(p_max > 0.0)) return 1;
  double* x = (double*)malloc(sizeof(double) * n);
  double* w = (double*)malloc(sizeof(double) * n);
  dse_ref_gauss_legendre(n, x, w);
  for (int i = 0; i < n; ++i) {
    double h = 0.5 * (1.0 + x[i]);
    pn[i] = p_max * h * h;
    Wn[i] = w[i] * p_max * h;
  }
  free(x); free(w);
  return 0;
}

int dse_ref_schwinger(const dse_ref_params* p, const double* c, int n, double p_max, const double* t, int m,
                      double* out) {
  if (check_params(p) || n < 1 || m < 0 || !(p_max > 0.0)) return 1;
  double* pn = (double*)malloc(sizeof(double) * n);
  double* Wn = (double*)malloc(sizeof(double) * n);
  double* g = (double*)malloc(sizeof(double) * n);
  dse_ref_schwinger_nodes(n, p_max, pn, Wn);
  /* per node: W_i sigma(p_i^2) / pi, the dressing from the expansion and its
   * IR / UV extension */
  for (int i = 0; i < n; ++i) {
    double u = pn[i] * pn[i];
    g[i] = Wn[i] * exp(dse_ref_lnZ(p, c, u)) / u / REF_PI;
  }
#pragma omp parallel for schedule(static) num_threads(dse_ref_get_threads()) if (m >= 4)
  for (int j = 0; j < m; ++j) {
    ksum acc = {0.0, 0.0};
    for (int i = 0; i < n; ++i) kadd(&acc, g[i] * cos(t[j] * pn[i]));
    out[j] = kval(&acc);
  }
  free(pn); free(Wn); free(g);
  return 0;
}
