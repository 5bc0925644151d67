// dse_host.hip -- host side of the C ABI: parameter checks, quadrature grid
// and Chebyshev tables, workspace layout, the Newton driver.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <new>
#include <vector>

#include "dse_impl.h"


static char g_init_err[512];

namespace dse {

void set_err(char* buf, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, 512, fmt, ap);
  va_end(ap);
}

char* global_err() { return g_init_err; }

}  // namespace dse

namespace {

using dse::kPi;
using dse::set_err;

#define HIP_TRY(ctx, expr)                                                          \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) {                                                         \
      set_err((ctx)->err, "%s: %s", #expr, hipGetErrorString(e_));                  \
      return DSE_E_DEVICE;                                                          \
    }                                                                               \
  } while (0)

}  // namespace

namespace dse {

// Gauss-Legendre nodes (ascending) and weights on [-1, 1]: Newton's method on
// the Legendre polynomial evaluated by Bonnet's recursion, started from the
// Tricomi estimate of the k-th root.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int k = 1; k <= (n + 1) / 2; ++k) {
    const double th = kPi * (4.0 * k - 1.0) / (4.0 * n + 2.0);
    double r = (1.0 - (n - 1.0) / (8.0 * n * n * n)) * cos(th);
    double dP = 1.0;
    for (int it = 0; it < 64; ++it) {
      double P0 = 1.0, P1 = r;
      for (int m = 2; m <= n; ++m) {
        const double P2 = ((2.0 * m - 1.0) * r * P1 - (m - 1.0) * P0) / m;
        P0 = P1;
        P1 = P2;
      }
      if (n == 1) { P1 = r; P0 = 1.0; }
      dP = n * (P0 - r * P1) / (1.0 - r * r);
      const double step = P1 / dP;
      r -= step;
      if (fabs(step) <= 1e-16 * fabs(r) + 1e-300) {
        P0 = 1.0; P1 = r;
        for (int m = 2; m <= n; ++m) {
          const double P2 = ((2.0 * m - 1.0) * r * P1 - (m - 1.0) * P0) / m;
          P0 = P1;
          P1 = P2;
        }
        if (n == 1) { P1 = r; P0 = 1.0; }
        dP = n * (P0 - r * P1) / (1.0 - r * r);
        break;
      }
    }
    const double wt = 2.0 / ((1.0 - r * r) * dP * dP);
    x[n - k] = r;
    w[n - k] = wt;
    x[k - 1] = -r;
    w[k - 1] = wt;
  }
  if (n % 2 == 1) x[n / 2] = 0.0;
}

// Tilde-T_j(s) for j < m with Tilde-T_0 = 1/2 (the c_0/2 convention, Sec. 3).
void cheb_row(double s, int m, double* out) {
  double a = 1.0, b = s;
  for (int j = 0; j < m; ++j) {
    out[j] = j == 0 ? 0.5 : (j == 1 ? s : 0.0);
    if (j >= 2) {
      const double c = 2.0 * s * b - a;
      out[j] = c;
      a = b;
      b = c;
    }
  }
}

dse_status validate(const dse_params* p, char* err) {
  if (!p) { set_err(err, "params is NULL"); return DSE_E_INVALID; }
  if (p->abi_version != DSE_ABI_VERSION) {
    set_err(err, "abi_version %d, library has %d", p->abi_version, DSE_ABI_VERSION);
    return DSE_E_INVALID;
  }
  if (p->n_z < 1 || p->n_z > DSE_MAX_N || p->n_g < 1 || p->n_g > DSE_MAX_N) {
    set_err(err, "n_z = %d, n_g = %d: each must be in [1, %d]", p->n_z, p->n_g, DSE_MAX_N);
    return DSE_E_INVALID;
  }
  if (p->n_rad < 1 || p->n_rad > 65536 || p->n_ir < 0 || p->n_ir > 65536 || p->n_ang < 1 ||
      p->n_ang > 65536) {
    set_err(err, "quadrature sizes n_rad = %d, n_ir = %d, n_ang = %d out of range", p->n_rad, p->n_ir,
            p->n_ang);
    return DSE_E_INVALID;
  }
  const double vals[] = {p->eps2, p->lambda2, p->ir_efolds, p->alpha_mu, p->n_c, p->g0_inv,
                         p->z_lambda_inv, p->kappa, p->delta, p->gamma};
  for (double d : vals)
    if (!isfinite(d)) { set_err(err, "non-finite parameter"); return DSE_E_INVALID; }
  if (!(p->eps2 > 0.0) || !(p->lambda2 > p->eps2)) {
    set_err(err, "need 0 < eps2 < lambda2 (got %g, %g)", p->eps2, p->lambda2);
    return DSE_E_INVALID;
  }
  if (!(p->alpha_mu > 0.0) || !(p->n_c > 0.0)) {
    set_err(err, "alpha_mu and n_c must be positive");
    return DSE_E_INVALID;
  }
  if (p->n_ir > 0 && !(p->ir_efolds > 0.0)) {
    set_err(err, "ir_efolds must be positive when n_ir > 0");
    return DSE_E_INVALID;
  }
  if (p->g0_inv < 0.0 || !(p->z_lambda_inv > 0.0)) {
    set_err(err, "need g0_inv >= 0 and z_lambda_inv > 0");
    return DSE_E_INVALID;
  }
  if (p->precision != DSE_FP64 && p->precision != DSE_MIXED) {
    set_err(err, "precision %d unknown", p->precision);
    return DSE_E_INVALID;
  }
  if (p->quad & ~(DSE_QUAD_TANH_SINH | DSE_QUAD_SPLIT)) {
    set_err(err, "quad = %d: unknown quadrature bits", p->quad);
    return DSE_E_INVALID;
  }
  if ((p->quad & DSE_QUAD_TANH_SINH) && (p->n_ang < 3 || p->n_ang % 2 == 0)) {
    set_err(err, "the tanh-sinh rule needs an odd n_ang >= 3 (got %d)", p->n_ang);
    return DSE_E_INVALID;
  }
  if ((p->quad & DSE_QUAD_SPLIT) && p->precision != DSE_FP64) {
    set_err(err, "the split radial grid runs in FP64 only");
    return DSE_E_INVALID;
  }
  return DSE_OK;
}

Phys make_phys(const dse_params& p) {
  Phys ph;
  ph.C = p.alpha_mu * p.n_c / (2.0 * kPi * kPi);
  ph.omega = 11.0 * p.n_c * p.alpha_mu / (12.0 * kPi);
  ph.e1 = -2.0 - 6.0 * p.delta;
  ph.e2 = -3.0 * p.delta;
  ph.ln_eps2 = log(p.eps2);
  ph.ln_lam2 = log(p.lambda2);
  ph.L0 = 0.5 * (ph.ln_eps2 + ph.ln_lam2);
  ph.invL1 = 1.0 / (0.5 * (ph.ln_lam2 - ph.ln_eps2));
  ph.kappa = p.kappa;
  ph.delta = p.delta;
  ph.gamma = p.gamma;
  ph.g0_inv = p.g0_inv;
  ph.z_lambda_inv = p.z_lambda_inv;
  ph.inv_alpha = 1.0 / p.alpha_mu;
  ph.omega_per_alpha = 11.0 * p.n_c / (12.0 * kPi);
  return ph;
}

// Carves the workspace; with base == nullptr only sizes it.  ks > 0 fixes the
// number of angular slices (the buffers are sized for it); 0 picks it from the
// problem size.
size_t layout(const dse_params& p, Views* v, char* base, int ks) {
  Views t{};
  t.n_z = p.n_z;
  t.n_g = p.n_g;
  t.n = p.n_z + p.n_g;
  t.NJ = padded_order(p.n_z > p.n_g ? p.n_z : p.n_g);
  t.split = (p.quad & DSE_QUAD_SPLIT) ? 1 : 0;
  t.Q = (t.split ? 2 * p.n_rad : p.n_rad) + p.n_ir;  // nodes per row
  t.Qp = pad_up(t.Q, kQPad);
  t.K = p.n_ang;
  t.Kp = pad_up(t.K, kKPad);
  t.RZ = p.n_z + 1;
  t.RG = p.n_g + 1;
  t.nqt = t.Qp / 64;
  // angular slices: the block count of the larger row kind closest to 1024
  // (about four blocks per CU), at most eight slices and at least two angles
  // per wave.  Fewer, longer blocks win over a power of two that overshoots:
  // each wave's set-up and reductions are paid once per block.
  {
    const int per_slice = (t.RZ > t.RG ? t.RZ : t.RG) * t.nqt;
    const int kmax = std::max(1, std::min(8, t.Kp / 8));
    t.KS = 1;
    for (int k = 2; k <= kmax; ++k)
      if (std::abs(per_slice * k - 1024) < std::abs(per_slice * t.KS - 1024)) t.KS = k;
  }
  if (ks > 0) t.KS = ks;
  t.Rb = 2 * t.RZ + t.RG;
  t.Rbp = pad_up(t.Rb, 16);
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* ptr = base ? base + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return ptr;
  };
  const size_t d = sizeof(double);
  t.coef = (double*)take(2 * t.NJ * d);
  t.y = (double*)take(t.Qp * d);
  t.W = (double*)take(t.Qp * d);
  t.lnZy = (double*)take(t.Qp * d);
  t.lnGy = (double*)take(t.Qp * d);
  t.Ttab = (double*)take((size_t)t.Qp * t.NJ * d);
  t.Ttab32 = (float*)take((size_t)t.Qp * t.NJ * sizeof(float));
  t.Text = (double*)take((size_t)t.n * t.NJ * d);
  t.TtabT = (double*)take((size_t)t.Qp * t.NJ * d);
  t.TextT = (double*)take((size_t)t.n * t.NJ * d);
  t.xrow = (double*)take((t.RZ + t.RG) * d);
  t.lnX = (double*)take(t.n * d);
  t.ang = (double*)take(5 * t.Kp * d);
  const size_t nr = t.split ? (size_t)(t.RZ + t.RG) * t.Qp : 0;
  t.yr = t.split ? (double*)take(nr * d) : nullptr;
  t.Wr = t.split ? (double*)take(nr * d) : nullptr;
  t.syr = t.split ? (double*)take(nr * d) : nullptr;
  t.lnZyr = t.split ? (double*)take(nr * d) : nullptr;
  t.lnGyr = t.split ? (double*)take(nr * d) : nullptr;
  t.Bm = (double*)take((size_t)t.KS * t.Rbp * t.Qp * d);
  t.Dp = (double*)take((size_t)(2 * t.RZ + t.RG + (t.split ? t.RG : 0)) * t.nqt * t.KS * t.NJ * d);
  t.Pip = (double*)take((size_t)2 * (t.RZ + t.RG) * t.nqt * t.KS * d);
  t.Absp = (double*)take((size_t)(t.RZ + t.RG) * t.nqt * t.KS * d);
  t.Eq = (double*)take((size_t)dse::kCS * t.Rbp * t.NJ * d);
  t.Dgh = (double*)take((size_t)dse::kCS * t.RG * t.NJ * d);
  t.rw = (double*)take((size_t)(t.RZ + t.RG) * d);
  const size_t np16 = (size_t)(t.n + 15) / 16 * 16;
  t.LU = (double*)take(np16 * (np16 + 1) * d);  // padded [A | b] when it does not fit LDS
  t.piv = (int32_t*)take(t.n * sizeof(int32_t));
  t.flag = (int32_t*)take(4 * sizeof(int32_t));
  t.rowmax = (double*)take(t.n * d);
  t.rowmax_u = (double*)take(t.n * d);
  t.F = (double*)take(t.n * d);
  t.S = (double*)take(t.n * d);
  t.Ft = (double*)take(t.n * d);
  t.St = (double*)take(t.n * d);
  t.dlt = (double*)take(t.n * d);
  t.ct = (double*)take(t.n * d);
  t.J = (double*)take((size_t)t.n * t.n * d);
  t.scal = (double*)take(8 * d);
  if (v) *v = t;
  return off;
}

// Host tables of one problem, uploaded once (synchronises the stream).
dse_status upload_tables(const dse_params& p, const Views& v, const Phys& ph, hipStream_t st, char* err) {
  const int NJ = v.NJ;
  std::vector<double> y(v.Qp, 1.0), W(v.Qp, 0.0), sq(v.Qp, 0.0);
  std::vector<double> u, wu;
  int q = 0;
  if (p.n_ir > 0) {
    gauss_legendre(p.n_ir, u, wu);
    const double a = ph.ln_eps2 - p.ir_efolds, b = ph.ln_eps2;
    for (int i = 0; i < p.n_ir; ++i, ++q) {
      const double tq = 0.5 * (a + b) + 0.5 * (b - a) * u[i];
      y[q] = exp(tq);
      W[q] = 0.5 * (b - a) * wu[i] * y[q];
      sq[q] = -1.0;  // below eps2 the series is frozen at s = -1
    }
  }
  gauss_legendre(p.n_rad, u, wu);
  const double L1 = 0.5 * (ph.ln_lam2 - ph.ln_eps2);
  for (int i = 0; i < p.n_rad; ++i, ++q) {
    const double tq = ph.L0 + L1 * u[i];
    y[q] = exp(tq);
    W[q] = L1 * wu[i] * y[q];
    sq[q] = u[i];  // the mapped coordinate of a main-panel node is the GL node
  }
  std::vector<double> Ttab((size_t)v.Qp * NJ);
  for (int i = 0; i < v.Qp; ++i) cheb_row(sq[i], NJ, &Ttab[(size_t)i * NJ]);
  std::vector<float> Ttab32(Ttab.size());
  for (size_t i = 0; i < Ttab.size(); ++i) Ttab32[i] = (float)Ttab[i];

  std::vector<double> Text((size_t)v.n * NJ), xrow(v.RZ + v.RG);
  for (int r = 0; r < v.n; ++r) {
    const bool gl = r < p.n_z;
    const int N = gl ? p.n_z : p.n_g;
    const int i = gl ? r : r - p.n_z;
    const double s = -cos(kPi * (i + 0.5) / N);
    cheb_row(s, NJ, &Text[(size_t)r * NJ]);
    const double x = exp(ph.L0 + L1 * s);
    xrow[gl ? i : v.RZ + i] = x;
  }
  std::vector<double> TtabT(Ttab.size()), TextT(Text.size());
  for (int i = 0; i < v.Qp; ++i)
    for (int j = 0; j < NJ; ++j) TtabT[(size_t)j * v.Qp + i] = Ttab[(size_t)i * NJ + j];
  for (int r = 0; r < v.n; ++r)
    for (int j = 0; j < NJ; ++j) TextT[(size_t)j * v.n + r] = Text[(size_t)r * NJ + j];
  xrow[v.RZ - 1] = p.lambda2;         // gluon subtraction point x_Z = Lambda^2
  xrow[v.RZ + v.RG - 1] = 0.0;        // ghost subtraction point x_G = 0

  std::vector<double> ang(5 * (size_t)v.Kp, 0.0);
  for (int k = p.n_ang; k < v.Kp; ++k) ang[v.Kp + k] = 0.5;  // padding angles: zero weight
  if (p.quad & DSE_QUAD_TANH_SINH) {
    // tanh-sinh in xi = cos(theta) (Sec. 2): int dtheta sin^2 f = int dxi
    // sqrt(1 - xi^2) f; xi_k = tanh(u_k), u_k = (pi/2) sinh(k h), weight
    // h (pi/2) cosh(k h) / cosh^2(u_k), k = -K .. K, h = 3 / K.  1 - xi and
    // 1 + xi come from e^{+-2u} (no cancellation next to the ends), so
    // sin^2(theta/2) = (1 - xi)/2 and sin^2(theta) = (1 - xi)(1 + xi).
    const int K = (p.n_ang - 1) / 2;
    const double h = 3.0 / K;
    for (int k = -K; k <= K; ++k) {
      const int i = k + K;
      const double uk = 0.5 * kPi * sinh(k * h);
      const double om = 2.0 / (1.0 + exp(2.0 * uk));
      const double op = 2.0 / (1.0 + exp(-2.0 * uk));
      const double ch = cosh(uk);
      const double w = h * 0.5 * kPi * cosh(k * h) / (ch * ch);
      const double s2 = om * op, sn = sqrt(s2);
      ang[i] = tanh(uk);
      ang[v.Kp + i] = 0.5 * om;
      ang[2 * v.Kp + i] = w * sn;
      ang[3 * v.Kp + i] = w * s2 * sn;
      ang[4 * v.Kp + i] = s2;
    }
  } else {
    gauss_legendre(p.n_ang, u, wu);
    for (int k = 0; k < p.n_ang; ++k) {
      const double th = 0.5 * kPi * (1.0 + u[k]);
      const double vk = 0.5 * kPi * wu[k];
      const double sn = sin(th), sh = sin(0.5 * th);
      ang[k] = cos(th);
      ang[v.Kp + k] = sh * sh;
      ang[2 * v.Kp + k] = vk * sn * sn;
      ang[3 * v.Kp + k] = vk * sn * sn * sn * sn;
      ang[4 * v.Kp + k] = sn * sn;
    }
  }
  // split radial grids (Sec. 3): per row the IR panel, then n_rad log-GL
  // nodes on [eps2, x] and on [x, lambda2] (rows at x = 0 or lambda2: n_rad on
  // [eps2, lambda2]); s(y) from ln y directly
  const size_t nr = v.split ? (size_t)(v.RZ + v.RG) * v.Qp : 0;
  std::vector<double> yr(nr, 1.0), Wr(nr, 0.0), syr(nr, 0.0);
  if (v.split) {
    std::vector<double> gi, gwi, gr, gwr;
    if (p.n_ir > 0) gauss_legendre(p.n_ir, gi, gwi);
    gauss_legendre(p.n_rad, gr, gwr);
    auto panel = [&](const std::vector<double>& g, const std::vector<double>& gw, double a, double b,
                     double* yo, double* Wo, double* so) {
      for (size_t i = 0; i < g.size(); ++i) {
        const double tq = 0.5 * (a + b) + 0.5 * (b - a) * g[i];
        yo[i] = exp(tq);
        Wo[i] = 0.5 * (b - a) * gw[i] * yo[i];
        so[i] = std::min(1.0, std::max(-1.0, (tq - ph.L0) * ph.invL1));
      }
    };
    for (int r = 0; r < v.RZ + v.RG; ++r) {
      double* yo = &yr[(size_t)r * v.Qp];
      double* Wo = &Wr[(size_t)r * v.Qp];
      double* so = &syr[(size_t)r * v.Qp];
      int off = 0;
      if (p.n_ir > 0) {
        panel(gi, gwi, ph.ln_eps2 - p.ir_efolds, ph.ln_eps2, yo, Wo, so);
        off = p.n_ir;
      }
      const double xr = xrow[r];
      if (xr > p.eps2 && xr < p.lambda2) {
        const double lx = log(xr);
        panel(gr, gwr, ph.ln_eps2, lx, yo + off, Wo + off, so + off);
        panel(gr, gwr, lx, ph.ln_lam2, yo + off + p.n_rad, Wo + off + p.n_rad, so + off + p.n_rad);
      } else {
        panel(gr, gwr, ph.ln_eps2, ph.ln_lam2, yo + off, Wo + off, so + off);
      }
    }
  }
  std::vector<double> zeros((size_t)v.KS * v.Rbp * v.Qp, 0.0);
  struct { void* dst; const void* src; size_t bytes; } up[] = {
      {v.y, y.data(), v.Qp * 8u},
      {v.W, W.data(), v.Qp * 8u},
      {v.Ttab, Ttab.data(), Ttab.size() * 8},
      {v.Ttab32, Ttab32.data(), Ttab32.size() * 4},
      {v.Text, Text.data(), Text.size() * 8},
      {v.TtabT, TtabT.data(), TtabT.size() * 8},
      {v.TextT, TextT.data(), TextT.size() * 8},
      {v.xrow, xrow.data(), xrow.size() * 8},
      {v.ang, ang.data(), ang.size() * 8},
      {v.yr, yr.data(), nr * 8},
      {v.Wr, Wr.data(), nr * 8},
      {v.syr, syr.data(), nr * 8},
      // the padding rows of B must be finite (they only feed padding rows of Eq)
      {v.Bm, zeros.data(), zeros.size() * 8},
  };
  for (auto& u_ : up) {
    if (u_.bytes == 0) continue;
    const hipError_t e = hipMemcpyAsync(u_.dst, u_.src, u_.bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) { set_err(err, "table upload: %s", hipGetErrorString(e)); return DSE_E_DEVICE; }
  }
  const hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) { set_err(err, "table upload: %s", hipGetErrorString(e)); return DSE_E_DEVICE; }
  return DSE_OK;
}

// Start guess (see dse_start_guess) of one problem into c[n] (host).
void start_guess_host(const dse_params& p, const Phys& ph, double* c_out) {
  const double L1 = 0.5 * (ph.ln_lam2 - ph.ln_eps2);
  const double zl = 1.0 / p.z_lambda_inv;
  const double r = pow(zl, 1.0 / p.gamma);  // = 1 + omega ln(1 + Lambda^2/mu2)
  const double mu2 = r > 1.0 + 1e-9 ? p.lambda2 / expm1((r - 1.0) / ph.omega) : 1e6 * p.lambda2;
  const double m2 = p.g0_inv > 0.0 ? mu2 * pow(p.g0_inv, 1.0 / p.kappa) : 0.0;
  for (int i = 0; i < p.n_z + p.n_g; ++i) c_out[i] = 0.0;
  for (int f = 0; f < 2; ++f) {
    const int N = f == 0 ? p.n_z : p.n_g;
    double* o = c_out + (f == 0 ? 0 : p.n_z);
    for (int i = 0; i < N; ++i) {
      const double phi = kPi * (i + 0.5) / N;
      const double s = -cos(phi);
      const double x = exp(ph.L0 + L1 * s);
      const double L = log1p(ph.omega * log1p(x / mu2));
      double val;
      if (f == 0)
        val = (p.g0_inv > 0.0 ? 1.0 : 2.0 * p.kappa) * log(x / (x + mu2)) + p.gamma * L;
      else
        val = -p.kappa * log((x + m2) / (x + mu2)) + p.delta * L;
      // T_j(-cos phi) = cos(j (pi - phi)) = (-1)^j cos(j phi)
      for (int j = 0; j < N; ++j) o[j] += (2.0 / N) * val * ((j & 1) ? -1.0 : 1.0) * cos(j * phi);
    }
  }
}

}  // namespace dse

namespace {

using dse::validate;
using dse::make_phys;

dse_status build_tables(dse_ctx* ctx) { return dse::upload_tables(ctx->p, ctx->v, ctx->ph, ctx->st, ctx->err); }

dse_status check_ctx(const dse_ctx* ctx) { return ctx ? DSE_OK : DSE_E_INVALID; }

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

dse_status eval_residual(dse_ctx* ctx, const double* c, double* F, double* S) {
  const dse::Views& v = ctx->v;
  HIP_TRY(ctx, dse::launch_dressing(v, ctx->ph, c, ctx->st));
  HIP_TRY(ctx, dse::launch_points(v, ctx->ph, 0, false, ctx->st, nullptr));
  HIP_TRY(ctx, dse::launch_residual_rows(v, ctx->ph, F, S, ctx->st));
  return DSE_OK;
}

dse_status flush_timings(dse_ctx* ctx);

// mix < 0: the context's precision; 0: FP64; 1: FP32 derivative sums
dse_status eval_jacobian(dse_ctx* ctx, const double* c, double* J, double* F, double* S, int mix_override = -1,
                         double* F2 = nullptr, double* S2 = nullptr) {
  const dse::Views& v = ctx->v;
  hipEvent_t* ev = nullptr;
  if (ctx->timing) {
    if (ctx->ring_count == dse_ctx::kRing) {
      dse_status s = flush_timings(ctx);
      if (s != DSE_OK) return s;
    }
    ev = ctx->ev[ctx->ring_count++];
  }
  if (ev) HIP_TRY(ctx, hipEventRecord(ev[0], ctx->st));
  HIP_TRY(ctx, dse::launch_dressing(v, ctx->ph, c, ctx->st));
  const bool mix = mix_override < 0 ? ctx->p.precision == DSE_MIXED : mix_override != 0;
  HIP_TRY(ctx, dse::launch_points(v, ctx->ph, 1, mix, ctx->st, ev ? ev + 1 : nullptr));
  HIP_TRY(ctx, dse::launch_contract(v, mix, ctx->st));
  if (ev) HIP_TRY(ctx, hipEventRecord(ev[4], ctx->st));
  HIP_TRY(ctx, dse::launch_assemble(v, ctx->ph, J, F, S, mix, ctx->st, F2, S2));
  if (ev) HIP_TRY(ctx, hipEventRecord(ev[5], ctx->st));
  return DSE_OK;
}

// Folds the recorded event pairs into the running sums (synchronises).
dse_status flush_timings(dse_ctx* ctx) {
  for (int i = 0; i < ctx->ring_count; ++i) {
    hipEvent_t* e = ctx->ev[i];
    HIP_TRY(ctx, hipEventSynchronize(e[5]));
    float ms[5];
    for (int k = 0; k < 5; ++k) HIP_TRY(ctx, hipEventElapsedTime(&ms[k], e[k], e[k + 1]));
    for (int k = 0; k < 5; ++k) ctx->acc_ms[k] += ms[k];
    ++ctx->acc_n;
  }
  ctx->ring_count = 0;
  return DSE_OK;
}

// Reads max_r |F_r|/S_r, ||F||_2, ||d||_inf and ||F/S||_2 (synchronises the stream).
dse_status read_norms(dse_ctx* ctx, const double* F, const double* S, const double* d, double out[4]) {
  HIP_TRY(ctx, dse::launch_norms(ctx->v, F, S, d, ctx->v.scal, ctx->st));
  HIP_TRY(ctx, hipMemcpyAsync(ctx->hpin, ctx->v.scal, 4 * sizeof(double), hipMemcpyDeviceToHost, ctx->st));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->st));
  for (int i = 0; i < 4; ++i) out[i] = ctx->hpin[i];
  return DSE_OK;
}

}  // namespace

extern "C" {

const char* dse_status_string(dse_status s) {
  switch (s) {
    case DSE_OK: return "ok";
    case DSE_E_INVALID: return "invalid argument";
    case DSE_E_DEVICE: return "HIP device error";
    case DSE_E_NOMEM: return "workspace too small";
    case DSE_E_SINGULAR: return "singular Newton matrix";
    case DSE_E_NOCONV: return "Newton iteration did not converge";
    case DSE_E_NONFINITE: return "non-finite residual or Jacobian";
  }
  return "unknown status";
}

const char* dse_last_error(const dse_ctx* ctx) { return ctx ? ctx->err : g_init_err; }

dse_status dse_params_default(dse_params* p) {
  if (!p) return DSE_E_INVALID;
  memset(p, 0, sizeof(*p));
  p->abi_version = DSE_ABI_VERSION;
  p->n_z = p->n_g = 16;
  p->n_rad = 64;
  p->n_ir = 16;
  p->n_ang = 16;
  p->precision = DSE_FP64;
  p->eps2 = 1e-6;
  p->lambda2 = 1e6;
  p->ir_efolds = 40.0;
  p->alpha_mu = 1.0;
  p->n_c = 3.0;
  p->g0_inv = 0.0;
  p->z_lambda_inv = 1.0;
  p->kappa = (93.0 - sqrt(1201.0)) / 98.0;
  p->delta = -9.0 / 44.0;
  p->gamma = -13.0 / 22.0;
  return DSE_OK;
}

size_t dse_workspace_bytes(const dse_params* p) {
  char tmp[512];
  if (validate(p, tmp) != DSE_OK) return 0;
  return dse::layout(*p, nullptr, nullptr, 0);
}

dse_status dse_init(const dse_params* p, void* d_workspace, size_t ws_bytes, void* hip_stream,
                    dse_ctx** out) {
  if (!out) { set_err(g_init_err, "out is NULL"); return DSE_E_INVALID; }
  *out = nullptr;
  dse_status s = validate(p, g_init_err);
  if (s != DSE_OK) return s;
  if (!d_workspace || ((uintptr_t)d_workspace & 255u)) {
    set_err(g_init_err, "workspace must be a non-NULL, 256-byte aligned device pointer");
    return DSE_E_INVALID;
  }
  const size_t need = dse::layout(*p, nullptr, nullptr, 0);
  if (ws_bytes < need) {
    set_err(g_init_err, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    return DSE_E_NOMEM;
  }
  dse_ctx* ctx = new (std::nothrow) dse_ctx();
  if (!ctx) { set_err(g_init_err, "host allocation failed"); return DSE_E_INVALID; }
  ctx->p = *p;
  ctx->ph = make_phys(*p);
  ctx->st = (hipStream_t)hip_stream;
  ctx->ws = (char*)d_workspace;
  ctx->ws_bytes = ws_bytes;
  dse::layout(*p, &ctx->v, ctx->ws, 0);
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    set_err(g_init_err, "hipGetDevice failed");
    delete ctx;
    return DSE_E_DEVICE;
  }
  for (auto& row : ctx->ev)
    for (auto& e : row) {
      if (hipEventCreate(&e) != hipSuccess) {
        set_err(g_init_err, "hipEventCreate failed");
        delete ctx;
        return DSE_E_DEVICE;
      }
    }
  if (hipHostMalloc((void**)&ctx->hpin, 8 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    set_err(g_init_err, "hipHostMalloc failed");
    for (auto& row : ctx->ev)
      for (auto& e : row) (void)hipEventDestroy(e);
    delete ctx;
    return DSE_E_DEVICE;
  }
  dse::lu_setup();
  s = build_tables(ctx);
  if (s != DSE_OK) {
    set_err(g_init_err, "%s", ctx->err);
    for (auto& row : ctx->ev)
      for (auto& e : row) (void)hipEventDestroy(e);
    (void)hipHostFree(ctx->hpin);
    delete ctx;
    return s;
  }
  *out = ctx;
  return DSE_OK;
}

dse_status dse_destroy(dse_ctx* ctx) {
  if (!ctx) return DSE_OK;
  for (auto& row : ctx->ev)
    for (auto& e : row) (void)hipEventDestroy(e);
  for (auto& g : ctx->steps)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  for (auto& e : ctx->nev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->cap_st) (void)hipStreamDestroy(ctx->cap_st);
  if (ctx->hpin) (void)hipHostFree(ctx->hpin);
  delete ctx;
  return DSE_OK;
}

dse_status dse_sizes(const dse_ctx* ctx, int32_t* n, int32_t* nr, int32_t* na) {
  if (!ctx) return DSE_E_INVALID;
  if (n) *n = ctx->v.n;
  if (nr) *nr = ctx->v.Q;
  if (na) *na = ctx->v.K;
  return DSE_OK;
}

// Start guess of Sec. 2's asymptotic forms, as interpolation coefficients at
// the collocation points:  L(x) = ln(1 + omega ln(1 + x / mu2)),
//   ln G0 = -kappa ln((x + m2) / (x + mu2)) + delta L,
//   ln Z0 = 2 kappa ln(x / (x + mu2)) + gamma L   (scaling, g0_inv = 0),
//   ln Z0 = ln(x / (x + mu2)) + gamma L           (decoupling),
// mu2 from Z0(Lambda^2) = 1/z_lambda_inv, m2 = mu2 g0_inv^{1/kappa}.
dse_status dse_start_guess(dse_ctx* ctx, double* d_c) {
  if (!ctx || !d_c) return DSE_E_INVALID;
  DeviceGuard dg(ctx->device);
  std::vector<double> c(ctx->v.n, 0.0);
  dse::start_guess_host(ctx->p, ctx->ph, c.data());
  HIP_TRY(ctx, hipMemcpyAsync(d_c, c.data(), c.size() * 8, hipMemcpyHostToDevice, ctx->st));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->st));
  return DSE_OK;
}

dse_status dse_residual(dse_ctx* ctx, const double* d_c, double* d_F, double* d_S) {
  if (!ctx) return DSE_E_INVALID;
  if (!d_c || !d_F) { set_err(ctx->err, "d_c and d_F must not be NULL"); return DSE_E_INVALID; }
  DeviceGuard dg(ctx->device);
  return eval_residual(ctx, d_c, d_F, d_S);
}

dse_status dse_jacobian(dse_ctx* ctx, const double* d_c, double* d_J, double* d_F) {
  if (!ctx) return DSE_E_INVALID;
  if (!d_c || !d_J) { set_err(ctx->err, "d_c and d_J must not be NULL"); return DSE_E_INVALID; }
  DeviceGuard dg(ctx->device);
  return eval_jacobian(ctx, d_c, d_J, d_F, d_F ? ctx->v.St : nullptr);
}

dse_status dse_running_coupling(dse_ctx* ctx, const double* d_c, const double* d_u, int32_t m, double* d_alpha,
                                double* d_lnZ, double* d_lnG) {
  if (!ctx) return DSE_E_INVALID;
  if (m < 0 || (m > 0 && (!d_c || !d_u))) {
    set_err(ctx->err, "m must be >= 0, d_c and d_u non-NULL");
    return DSE_E_INVALID;
  }
  DeviceGuard dg(ctx->device);
  HIP_TRY(ctx, dse::launch_coupling(ctx->v, ctx->ph, ctx->p.alpha_mu, d_c, d_u, m, d_alpha, d_lnZ, d_lnG, ctx->st));
  return DSE_OK;
}

dse_status dse_dressing_vjp(dse_ctx* ctx, const double* d_u, int32_t m, const double* d_wZ, const double* d_wG,
                            double* d_grad) {
  if (!ctx) return DSE_E_INVALID;
  if (m < 0 || !d_grad || (m > 0 && !d_u)) {
    set_err(ctx->err, "m must be >= 0, d_grad non-NULL and d_u non-NULL when m > 0");
    return DSE_E_INVALID;
  }
  DeviceGuard dg(ctx->device);
  HIP_TRY(ctx, dse::launch_dressing_vjp(ctx->v, ctx->ph, d_u, m, m > 0 ? d_wZ : nullptr, m > 0 ? d_wG : nullptr,
                                        d_grad, ctx->st));
  return DSE_OK;
}

dse_status dse_jacobian_fd(dse_ctx* ctx, const double* d_c, double* d_J, double h_rel) {
  if (!ctx) return DSE_E_INVALID;
  if (!d_c || !d_J) { set_err(ctx->err, "d_c and d_J must not be NULL"); return DSE_E_INVALID; }
  if (!(h_rel > 0.0) || !(h_rel < 1.0)) { set_err(ctx->err, "h_rel must lie in (0, 1)"); return DSE_E_INVALID; }
  DeviceGuard dg(ctx->device);
  const dse::Views& v = ctx->v;
  double* hbuf = v.scal + 4;
  ctx->jac_at = nullptr;  // the residuals below overwrite the held F and S
  for (int j = 0; j < v.n; ++j) {
    HIP_TRY(ctx, dse::launch_fd_shift(v.n, d_c, j, h_rel, 1.0, v.ct, hbuf, ctx->st));
    dse_status s = eval_residual(ctx, v.ct, v.Ft, v.St);
    if (s != DSE_OK) return s;
    HIP_TRY(ctx, dse::launch_fd_shift(v.n, d_c, j, h_rel, -1.0, v.ct, hbuf, ctx->st));
    if ((s = eval_residual(ctx, v.ct, v.F, v.S)) != DSE_OK) return s;
    HIP_TRY(ctx, dse::launch_fd_column(v.n, v.Ft, v.F, hbuf, j, d_J, ctx->st));
  }
  return DSE_OK;
}

dse_status dse_set_timing(dse_ctx* ctx, int32_t on) {
  if (!ctx) return DSE_E_INVALID;
  DeviceGuard dg(ctx->device);
  dse_status s = flush_timings(ctx);
  ctx->timing = on != 0;
  for (double& a : ctx->acc_ms) a = 0.0;
  ctx->acc_n = 0;
  return s;
}

dse_status dse_read_timings(dse_ctx* ctx, double* ms5, int32_t* count) {
  if (!ctx || !ms5) return DSE_E_INVALID;
  DeviceGuard dg(ctx->device);
  dse_status s = flush_timings(ctx);
  if (s != DSE_OK) return s;
  for (int i = 0; i < 5; ++i) ms5[i] = ctx->acc_n ? ctx->acc_ms[i] / ctx->acc_n : 0.0;
  if (count) *count = ctx->acc_n;
  return DSE_OK;
}

dse_status dse_lu_solve(dse_ctx* ctx, const double* d_J, const double* d_b, double* d_x, int32_t trans) {
  if (!ctx) return DSE_E_INVALID;
  if (!d_J || !d_b || !d_x) { set_err(ctx->err, "NULL argument"); return DSE_E_INVALID; }
  DeviceGuard dg(ctx->device);
  HIP_TRY(ctx, dse::launch_row_absmax(ctx->v.n, d_J, ctx->v.rowmax_u, ctx->st));
  HIP_TRY(ctx, dse::launch_lu_solve(ctx->v, d_J, d_b, d_x, trans, ctx->st, nullptr, 0.0, nullptr, ctx->v.rowmax_u));
  HIP_TRY(ctx, hipMemcpyAsync(ctx->hflag(), ctx->v.flag, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->st));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->st));
  const int32_t flag = *ctx->hflag();
  if (flag == DSE_E_SINGULAR) {
    set_err(ctx->err, "singular matrix: a pivot is zero, not finite, or below n eps times its row's largest entry");
    return DSE_E_SINGULAR;
  }
  return DSE_OK;
}

dse_status dse_vjp(dse_ctx* ctx, const double* d_c, const double* d_u, double* d_uJ, double* d_utheta) {
  if (!ctx) return DSE_E_INVALID;
  if (!d_c || !d_u || (!d_uJ && !d_utheta)) {
    set_err(ctx->err, "d_c, d_u and one of d_uJ, d_utheta are required");
    return DSE_E_INVALID;
  }
  if (ctx->v.split) {
    set_err(ctx->err, "dse_vjp: not available on split radial grids (DSE_QUAD_SPLIT)");
    return DSE_E_INVALID;
  }
  DeviceGuard dg(ctx->device);
  const dse::Views& v = ctx->v;
  HIP_TRY(ctx, dse::launch_row_weights(v, d_u, ctx->st));
  HIP_TRY(ctx, dse::launch_dressing(v, ctx->ph, d_c, ctx->st));
  HIP_TRY(ctx, dse::launch_points(v, ctx->ph, d_uJ ? 2 : 3, false, ctx->st, nullptr));
  if (d_uJ) HIP_TRY(ctx, dse::launch_contract(v, false, ctx->st));
  HIP_TRY(ctx, dse::launch_vjp_reduce(v, d_u, d_uJ, d_utheta, ctx->st));
  return DSE_OK;
}

dse_status dse_set_physics(dse_ctx* ctx, double alpha_mu, double g0_inv, double z_lambda_inv) {
  if (!ctx) return DSE_E_INVALID;
  dse_params p = ctx->p;
  p.alpha_mu = alpha_mu;
  p.g0_inv = g0_inv;
  p.z_lambda_inv = z_lambda_inv;
  dse_status s = validate(&p, ctx->err);
  if (s != DSE_OK) return s;
  ctx->p = p;
  ctx->ph = make_phys(p);
  // the recorded Newton steps carry the physics constants as kernel
  // arguments: record them again; the held Newton matrix is the old problem's
  DeviceGuard dg(ctx->device);
  for (auto& g : ctx->steps)
    if (g.exec) {
      (void)hipGraphExecDestroy(g.exec);
      g = dse_ctx::StepGraph();
    }
  ctx->jac_at = nullptr;
  return DSE_OK;
}

namespace {

// The kernels of one Newton step: [J, F, S at c into the workspace, unless
// they are held there already (reuse)]; LU solve J Delta = F with the update
// c_new = c - rho Delta; J, F, S at c_new into the workspace (the matrix the
// next step starts from), F and S also into the caller's vectors.
dse_status enqueue_step(dse_ctx* ctx, const double* c, double rho, double* c_new, double* F_new, double* S_new,
                        bool reuse, bool capturing) {
  const dse::Views& v = ctx->v;
  const bool timing = ctx->timing;
  if (capturing) ctx->timing = false;  // no stage events inside a recorded graph
  dse_status s = DSE_OK;
  if (!reuse) s = eval_jacobian(ctx, c, v.J, v.F, v.S);
  if (s == DSE_OK) {
    const hipError_t e = dse::launch_lu_solve(v, v.J, v.F, v.dlt, 0, ctx->st, c, rho, c_new, v.rowmax);
    if (e != hipSuccess) {
      set_err(ctx->err, "LU launch: %s", hipGetErrorString(e));
      s = DSE_E_DEVICE;
    }
  }
  // the assembly at c_new also writes F and S to the caller's vectors
  if (s == DSE_OK) s = eval_jacobian(ctx, c_new, v.J, v.F, v.S, -1, F_new, S_new);
  ctx->timing = timing;
  return s;
}

}  // namespace

dse_status dse_set_graphs(dse_ctx* ctx, int32_t on) {
  if (!ctx) return DSE_E_INVALID;
  ctx->graphs = on != 0;
  return DSE_OK;
}

dse_status dse_newton_step(dse_ctx* ctx, const double* d_c, double rho, double* d_c_new, double* d_F_new,
                           double* d_S_new, int32_t check) {
  if (!ctx) return DSE_E_INVALID;
  if (!d_c || !d_c_new || !d_F_new || d_c == d_c_new || !isfinite(rho)) {
    set_err(ctx->err, "d_c, d_c_new (distinct) and d_F_new are required, rho finite");
    return DSE_E_INVALID;
  }
  DeviceGuard dg(ctx->device);
  const bool reuse = ctx->jac_at == d_c;
  ctx->jac_at = nullptr;  // until this step is enqueued
  if (!ctx->graphs) {
    dse_status s = enqueue_step(ctx, d_c, rho, d_c_new, d_F_new, d_S_new, reuse, false);
    if (s != DSE_OK) return s;
  } else {
    const void* key[4] = {d_c, d_c_new, d_F_new, d_S_new};
    dse_ctx::StepGraph* hit = nullptr;
    for (auto& g : ctx->steps)
      if (g.exec && g.rho == rho && g.reuse == reuse && memcmp(key, g.key, sizeof key) == 0) hit = &g;
    if (!hit) {
      // record into the least recently used slot
      dse_ctx::StepGraph* slot = &ctx->steps[0];
      for (auto& g : ctx->steps)
        if (!g.exec || (slot->exec && g.used < slot->used)) slot = &g;
      if (slot->exec) (void)hipGraphExecDestroy(slot->exec);
      *slot = dse_ctx::StepGraph();
      if (!ctx->cap_st) HIP_TRY(ctx, hipStreamCreateWithFlags(&ctx->cap_st, hipStreamNonBlocking));
      HIP_TRY(ctx, hipStreamBeginCapture(ctx->cap_st, hipStreamCaptureModeThreadLocal));
      const hipStream_t user_st = ctx->st;
      ctx->st = ctx->cap_st;
      dse_status s = enqueue_step(ctx, d_c, rho, d_c_new, d_F_new, d_S_new, reuse, true);
      ctx->st = user_st;
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(ctx->cap_st, &g);
      if (s != DSE_OK || ec != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        if (s == DSE_OK) set_err(ctx->err, "stream capture failed: %s", hipGetErrorString(ec));
        return s != DSE_OK ? s : DSE_E_DEVICE;
      }
      const hipError_t ei = hipGraphInstantiate(&slot->exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ei != hipSuccess) {
        slot->exec = nullptr;
        set_err(ctx->err, "graph instantiation failed: %s", hipGetErrorString(ei));
        return DSE_E_DEVICE;
      }
      memcpy(slot->key, key, sizeof key);
      slot->rho = rho;
      slot->reuse = reuse;
      hit = slot;
    }
    hit->used = ++ctx->step_clock;
    HIP_TRY(ctx, hipGraphLaunch(hit->exec, ctx->st));
  }
  ctx->jac_at = d_c_new;
  if (check) {
    HIP_TRY(ctx, hipMemcpyAsync(ctx->hflag(), ctx->v.flag, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->st));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->st));
    if (*ctx->hflag() == DSE_E_SINGULAR) {
      ctx->jac_at = nullptr;
      set_err(ctx->err, "zero pivot");
      return DSE_E_SINGULAR;
    }
  }
  return DSE_OK;
}

dse_status dse_newton_solve(dse_ctx* ctx, double* d_c, const dse_newton_opts* opts, dse_newton_report* rep) {
  if (!ctx) return DSE_E_INVALID;
  if (!d_c) { set_err(ctx->err, "d_c is NULL"); return DSE_E_INVALID; }
  DeviceGuard dg(ctx->device);
  const auto t0 = std::chrono::steady_clock::now();
  dse_newton_opts o;
  if (opts) {
    o = *opts;
  } else {
    o.tol = 1e-10; o.max_iter = 60; o.extra_iters = 0; o.max_halvings = 30; o.reserved_ = 0; o.step_tol = 1e-14;
  }
  if (!(o.tol > 0.0) || o.max_iter < 0 || o.extra_iters < 0 || o.max_halvings < 0) {
    set_err(ctx->err, "invalid Newton options");
    return DSE_E_INVALID;
  }
  dse_newton_report r;
  memset(&r, 0, sizeof(r));
  const dse::Views& v = ctx->v;
  const int n = v.n;
  hipStream_t st = ctx->st;
  ctx->jac_at = nullptr;  // the workspace's J, F, S now belong to this solve
  // mixed precision: FP32 Newton matrices while they make progress, FP64 ones
  // once a step reduces the merit by less than half or it is below 1e-6 (the
  // FP32 matrix then limits the linear convergence rate)
  bool use_mix = ctx->p.precision == DSE_MIXED;
  // J, F, S at the start: every evaluation of an accepted point is an
  // assembly, so the next step's matrix comes with the residual that accepts it
  double nrm[4];
  const auto ta = std::chrono::steady_clock::now();
  dse_status s = eval_jacobian(ctx, d_c, v.J, v.F, v.S, use_mix ? 1 : 0);
  if (s == DSE_OK) s = read_norms(ctx, v.F, v.S, nullptr, nrm);
  r.t_assembly_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - ta).count();
  ++r.n_jacobians;
  if (use_mix) ++r.n_jacobians_mixed;
  bool have_J = true;      // v.J belongs to d_c
  bool j_mix = use_mix;    // ... in this precision
  double f = nrm[0];       // convergence test: max_r |F_r| / S_r
  double f2 = nrm[3];      // line-search merit: ||F / S||_2
  r.fnorm_hist[0] = f;
  r.fnorm2 = nrm[1];
  int it = 0, extra = 0;
  dse_status status = s;
  if (s == DSE_OK && !isfinite(f)) status = DSE_E_NONFINITE;
  while (status == DSE_OK) {
    if (f < o.tol) {
      if (extra >= o.extra_iters) break;
      ++extra;
    }
    if (it >= o.max_iter) { status = DSE_E_NOCONV; break; }
    if (!have_J || j_mix != use_mix) {
      // after a relaxed step, or when the precision of the matrix changes
      if (!ctx->nev[0])
        for (auto& e : ctx->nev) HIP_TRY(ctx, hipEventCreate(&e));
      HIP_TRY(ctx, hipEventRecord(ctx->nev[0], st));
      if ((s = eval_jacobian(ctx, d_c, v.J, v.F, v.S, use_mix ? 1 : 0)) != DSE_OK) { status = s; break; }
      HIP_TRY(ctx, hipEventRecord(ctx->nev[1], st));
      HIP_TRY(ctx, hipEventSynchronize(ctx->nev[1]));
      float ma = 0.f;
      HIP_TRY(ctx, hipEventElapsedTime(&ma, ctx->nev[0], ctx->nev[1]));
      r.t_assembly_ms += ma;
      ++r.n_jacobians;
      if (use_mix) ++r.n_jacobians_mixed;
      j_mix = use_mix;
    }
    if (hipGetLastError() != hipSuccess) { status = DSE_E_DEVICE; break; }
    // the solve also writes the full step c - Delta (the update kernel's FMA)
    if (!ctx->nev[0])
      for (auto& e : ctx->nev) HIP_TRY(ctx, hipEventCreate(&e));
    HIP_TRY(ctx, hipEventRecord(ctx->nev[2], st));
    HIP_TRY(ctx, dse::launch_lu_solve(v, v.J, v.F, v.dlt, 0, st, d_c, 1.0, v.ct, v.rowmax));
    HIP_TRY(ctx, hipEventRecord(ctx->nev[3], st));
    const bool conv = f < o.tol;
    double rho = 1.0, ft = INFINITY, ft2 = INFINITY, dinf = 0.0;
    int32_t flag = 0;
    for (int h = 0;; ++h) {
      if (h == 0) {
        // the full step in Jacobian mode: accepted, its matrix is the next one
        HIP_TRY(ctx, hipEventRecord(ctx->nev[0], st));
        if ((s = eval_jacobian(ctx, v.ct, v.J, v.F, v.S, use_mix ? 1 : 0)) != DSE_OK) { status = s; break; }
        HIP_TRY(ctx, hipEventRecord(ctx->nev[1], st));
        ++r.n_jacobians;
        if (use_mix) ++r.n_jacobians_mixed;
        have_J = true;
        j_mix = use_mix;
        // the pivot flag arrives with the norms (one synchronisation)
        HIP_TRY(ctx, hipMemcpyAsync(ctx->hflag(), v.flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      } else {
        // relaxed steps in residual mode
        HIP_TRY(ctx, dse::launch_axpy(n, d_c, rho, v.dlt, v.ct, st));
        if ((s = eval_residual(ctx, v.ct, v.F, v.S)) != DSE_OK) { status = s; break; }
        ++r.n_residuals;
        have_J = false;
      }
      if ((s = read_norms(ctx, v.F, v.S, v.dlt, nrm)) != DSE_OK) { status = s; break; }
      if (h == 0) flag = *ctx->hflag();  // copied before the norms, complete after their wait
      if (h == 0) {
        // read_norms synchronised the stream: the phase events are complete
        float ma = 0.f, ml = 0.f;
        HIP_TRY(ctx, hipEventElapsedTime(&ma, ctx->nev[0], ctx->nev[1]));
        HIP_TRY(ctx, hipEventElapsedTime(&ml, ctx->nev[2], ctx->nev[3]));
        r.t_assembly_ms += ma;
        r.t_lu_ms += ml;
      }
      if (h == 0 && flag == DSE_E_SINGULAR) {
        status = DSE_E_SINGULAR;
        set_err(ctx->err, "singular Newton matrix: a pivot is zero, not finite, or below n eps times its row's largest entry");
        break;
      }
      ft = isfinite(nrm[0]) ? nrm[0] : INFINITY;
      ft2 = isfinite(nrm[0]) && isfinite(nrm[3]) ? nrm[3] : INFINITY;
      dinf = nrm[2];
      if (conv || ft2 < f2 || h >= o.max_halvings) break;
      rho *= 0.5;
    }
    if (status != DSE_OK) break;
    if (!isfinite(ft)) { status = DSE_E_NONFINITE; break; }
    HIP_TRY(ctx, hipMemcpyAsync(d_c, v.ct, n * 8, hipMemcpyDeviceToDevice, st));
    if (use_mix && (ft2 > 0.5 * f2 || ft < 1e-6)) use_mix = false;
    f = ft;
    f2 = ft2;
    ++it;
    if (it < 128) { r.fnorm_hist[it] = f; r.relax_hist[it - 1] = rho; }
    r.fnorm2 = nrm[1];
    if (conv && rho * dinf < o.step_tol) break;
  }
  HIP_TRY(ctx, hipStreamSynchronize(st));
  r.iters = it;
  r.status = status;
  r.fnorm = f;
  r.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (rep) *rep = r;
  if (status == DSE_E_NOCONV) set_err(ctx->err, "no convergence after %d iterations (scaled residual %g)", it, f);
  return status;
}

}  // extern "C"
