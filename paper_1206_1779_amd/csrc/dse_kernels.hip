// dse_kernels.hip -- gfx950 kernels of the ghost-gluon DSE solver.
//
// One Newton matrix assembly (Sec. 3) is four launches on one stream:
//   dressing  : ln Z, ln G at the radial nodes and collocation points
//               (Chebyshev series of Sec. 3 plus the IR/UV extrapolations of
//               Sec. 2), and the coefficient vector with c_0 halved;
//   points    : the fused per-point kernel: for every row momentum x, radial
//               node y_q and angle theta_k it evaluates z, s(z), the Chebyshev
//               recurrence, ln Z(z), ln G(z), the kernels M and Q (Sec. 2) and
//               the integrand of Pi_Z or Pi_G, accumulating
//                 Pi and sum|integrand|                  (residual),
//                 B[row][q] = sum_k dI/d ln(dressing at y) (q-side, LDS reduce),
//                 D[row][j] = sum_qk dI/d ln(dressing at z) T_j(s(z)) (k-side);
//   contract  : Eq = B . T on v_mfma_f64_16x16x4f64 (the q-side derivative
//               needs T_j(s(y_q)), the same for every row: a dense product);
//   assemble  : J = direct term - (Eq + D)(x_i) + (Eq + D)(subtraction row),
//               F and its scale S (MOM-subtracted equations of Sec. 3).
// The Newton step adds an FP64 LU with partial pivoting (one workgroup) and
// a relaxation update.
//
// Determinism: every sum runs in a fixed order; no floating-point atomics.

#include <hip/hip_runtime.h>
#include <math.h>

#include "dse_impl.h"

namespace dse {

enum { GLUON = 0, GHOST = 1 };

// Lane-group width G of the k-side accumulation for each (row kind, padded
// order): G lanes share G points and each accumulates NJ/G coefficients.
template <int KIND, int NJ>
struct Tile {
  static constexpr int G = KIND == GLUON ? (NJ <= 16 ? 1 : (NJ <= 32 ? 2 : (NJ <= 64 ? 4 : 8)))
                                         : (NJ <= 32 ? 1 : (NJ <= 64 ? 2 : 4));
  static constexpr int JT = NJ / G;
  static_assert(JT * G == NJ, "order must split evenly");
};

// Compensated accumulation (Neumaier): the residual's self-energy sums keep
// their rounding error in a second word so that F does not depend on the
// summation order beyond the last bits.
__device__ __forceinline__ void two_sum_add(double& s, double& c, double v) {
  const double t = s + v;
  const double bp = t - s;
  c += (s - (t - bp)) + (v - bp);
  s = t;
}
__device__ __forceinline__ void wave_sum2(double& s, double& c) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const double s2 = __shfl_xor(s, o, 64);
    const double c2 = __shfl_xor(c, o, 64);
    two_sum_add(s, c, s2);
    c += c2;
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// --------------------------------------------------------------------------
// dressing: coef (c_0 halved, zero padded), ln Z / ln G at radial nodes and at
// the collocation points.
__global__ __launch_bounds__(256) void dressing_kernel(Views v, Phys ph, const double* __restrict__ c) {
  __shared__ double sa[DSE_MAX_N], sb[DSE_MAX_N];
  const int t = threadIdx.x;
  const int NJ = v.NJ;
  for (int j = t; j < NJ; j += blockDim.x) {
    double a = j < v.n_z ? c[j] : 0.0;
    double b = j < v.n_g ? c[v.n_z + j] : 0.0;
    if (j == 0) { a *= 0.5; b *= 0.5; }
    // the table holds Tilde-T_0 = 1/2: keep the unhalved value for the GEMV
    sa[j] = j < v.n_z ? c[j] : 0.0;
    sb[j] = j < v.n_g ? c[v.n_z + j] : 0.0;
    v.coef[j] = a;
    v.coef[NJ + j] = b;
  }
  __syncthreads();
  const int nout = v.Qp + v.n;
  for (int o = t; o < nout; o += blockDim.x) {
    if (o < v.Qp) {
      const double* T = v.Ttab + (size_t)o * NJ;
      double z = 0.0, g = 0.0;
      for (int j = 0; j < NJ; ++j) { z = fma(sa[j], T[j], z); g = fma(sb[j], T[j], g); }
      double ly = log(v.y[o]);
      if (ly < ph.ln_eps2) {
        z += 2.0 * ph.kappa * (ly - ph.ln_eps2);
        g += -ph.kappa * (ly - ph.ln_eps2);
      } else if (ly > ph.ln_lam2) {
        double L = log(fma(ph.omega, ly - ph.ln_lam2, 1.0));
        z += ph.gamma * L;
        g += ph.delta * L;
      }
      v.lnZy[o] = z;
      v.lnGy[o] = g;
    } else {
      int r = o - v.Qp;
      const double* T = v.Text + (size_t)r * NJ;
      const double* cc = r < v.n_z ? sa : sb;
      double s = 0.0;
      for (int j = 0; j < NJ; ++j) s = fma(cc[j], T[j], s);
      v.lnX[r] = s;  // collocation points lie in [eps2, lambda2]: no extension
    }
  }
}

// --------------------------------------------------------------------------
// The fused point kernel.  Block = one row x 64 radial nodes; wave w takes the
// angles k = w, w+4, ...; lane = radial node.  Pass 1 (every lane, own point):
// recurrence + series with wave-uniform coefficients.  Pass 2 (Jacobian only):
// a group of G lanes shares its G points; member m accumulates
// j in [m JT, (m+1) JT) for all G points, starting the recurrence from
// (T_{m JT - 1}, T_{m JT}) saved in pass 1.
template <int KIND, int NJ, bool JAC>
__global__ __launch_bounds__(256) void point_kernel(Views v, Phys ph) {
  using TL = Tile<KIND, NJ>;
  constexpr int G = TL::G;
  constexpr int JT = TL::JT;
  constexpr int NT = KIND == GLUON ? 2 : 1;  // k-side targets

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int row = blockIdx.x / v.nqt;
  const int qt = blockIdx.x - row * v.nqt;
  const int q = qt * 64 + lane;
  const int growrow = KIND == GLUON ? row : v.RZ + row;  // index into xrow / Pip

  const double x = v.xrow[growrow];
  const double y = v.y[q];
  const double W = v.W[q];
  const double lGy = v.lnGy[q];
  const double lZy = v.lnZy[q];

  // per (row, node) constants: z = mx [(1-t)^2 + 4 t sin^2(theta/2)]
  const double mx = fmax(x, y), mn = fmin(x, y);
  const double tt = sqrt(mn / mx);
  const double Aw = (1.0 - tt) * (1.0 - tt);
  const double Bw = 4.0 * tt;
  const double lnmx = log(mx);
  double pref, ymx = 0.0, qc0 = 0.0, qc1 = 0.0, qc2 = 0.0, qc3 = 0.0, qc4 = 0.0;
  if (KIND == GLUON) {
    pref = ph.C / (3.0 * x) * W;
    ymx = y / mx;
    // Q w^2 as a polynomial in xi = cos(theta) with t-dependent coefficients
    const double t2 = tt * tt, t4 = t2 * t2;
    qc0 = -2.25 * (1.0 + t4) - 8.5 * t2;
    qc1 = -3.0 * tt * (1.0 + t2);
    qc2 = 6.0 * (1.0 + t4) + 29.0 * t2;
    qc3 = -12.0 * tt * (1.0 + t2);
    qc4 = 2.0 * t2;
  } else {
    pref = -ph.C * W * y;
  }

  const double* __restrict__ ca = v.coef;
  const double* __restrict__ cb = v.coef + NJ;
  const double* __restrict__ ang = v.ang;
  const int Kp = v.Kp;

  double pi_s = 0.0, pi_c = 0.0, abs_acc = 0.0, Ba = 0.0, Bb = 0.0;
  double Da[JAC ? JT : 1], Db[JAC && NT == 2 ? JT : 1];
  if (JAC) {
#pragma unroll
    for (int jj = 0; jj < JT; ++jj) { Da[jj] = 0.0; if (NT == 2) Db[jj] = 0.0; }
  }
  const int member = lane & (G - 1);

  for (int k = wave; k < Kp; k += 4) {
    const double ck = ang[k];
    const double s2h = ang[Kp + k];
    const double wk = KIND == GLUON ? ang[2 * Kp + k] : ang[3 * Kp + k];
    const double st2 = ang[4 * Kp + k];

    const double w = fma(Bw, s2h, Aw);
    const double lz = lnmx + log(w);
    double s = (lz - ph.L0) * ph.invL1;
    s = fmin(fmax(s, -1.0), 1.0);
    const double s2 = s + s;

    // ---- pass 1: recurrence and series (coefficients are wave-uniform)
    double sa = ca[0], sb = KIND == GLUON ? cb[0] : 0.0;
    double Tp = 1.0, Tc = s;
    double stp[G > 1 ? G : 1], stc[G > 1 ? G : 1];
    stp[0] = s; stc[0] = 1.0;  // (T_{-1}, T_0)
#pragma unroll
    for (int j = 1; j < NJ; ++j) {
      if (G > 1 && (j % JT) == 0) { stp[j / JT] = Tp; stc[j / JT] = Tc; }
      sa = fma(ca[j], Tc, sa);
      if (KIND == GLUON) sb = fma(cb[j], Tc, sb);
      const double Tn = fma(s2, Tc, -Tp);
      Tp = Tc;
      Tc = Tn;
    }
    double XZ = 0.0, XG = 0.0;
    if (lz < ph.ln_eps2) {
      XZ = 2.0 * ph.kappa * (lz - ph.ln_eps2);
      XG = -ph.kappa * (lz - ph.ln_eps2);
    } else if (lz > ph.ln_lam2) {
      const double L = log(fma(ph.omega, lz - ph.ln_lam2, 1.0));
      XZ = ph.gamma * L;
      XG = ph.delta * L;
    }
    const double lZz = sa + XZ;

    double Pa, Pb;
    if (KIND == GLUON) {
      const double lGz = sb + XG;
      const double iw = 1.0 / w;
      const double Qn = fma(fma(fma(fma(qc4, ck, qc3), ck, qc2), ck, qc1), ck, qc0);
      const double Qk = Qn * iw * iw;
      const double Mk = ymx * st2 * iw;
      const double lg = lGy + lGz;
      const double Fgl = exp(ph.e1 * lg + ph.e2 * (lZy + lZz));
      const double Fgh = exp(lg);
      const double om = pref * wk;
      const double tq = om * Qk * Fgl;
      const double tm = om * Mk * Fgh;
      two_sum_add(pi_s, pi_c, tq + tm);
      abs_acc += fabs(tq) + fabs(tm);
      Pa = tq * ph.e2;           // d integrand / d ln Z (at y or at z)
      Pb = fma(tq, ph.e1, tm);   // d integrand / d ln G (at y or at z)
      if (JAC) { Ba += Pa; Bb += Pb; }
    } else {
      const double val = pref * wk * exp(lGy + lZz - 2.0 * lz);  // rho G(y) Z(z) / z^2
      two_sum_add(pi_s, pi_c, val);
      abs_acc += fabs(val);
      Pa = val;                  // k-side: d / d ln Z(z)
      Pb = val;
      if (JAC) Bb += val;        // q-side: d / d ln G(y)
    }

    if (JAC) {
      // ---- pass 2: k-side accumulation over the G points of the lane group
#pragma unroll
      for (int r = 0; r < G; ++r) {
        double tp, tc, pa, pb;
        if (r == 0) {
          tp = stp[0]; tc = stc[0];
#pragma unroll
          for (int m = 1; m < G; ++m) if (member == m) { tp = stp[m]; tc = stc[m]; }
          pa = Pa; pb = Pb;
        } else {
          // send the start pair the reading lane (member ^ r) needs
          const int want = member ^ r;
          double sp = stp[0], sc = stc[0];
#pragma unroll
          for (int m = 1; m < G; ++m) if (want == m) { sp = stp[m]; sc = stc[m]; }
          tp = __shfl_xor(sp, r, 64);
          tc = __shfl_xor(sc, r, 64);
          pa = __shfl_xor(Pa, r, 64);
          pb = NT == 2 ? __shfl_xor(Pb, r, 64) : 0.0;
        }
        // the owner's mapped momentum drives its recurrence
        const double sr = r == 0 ? s : __shfl_xor(s, r, 64);
        const double sr2 = sr + sr;
#pragma unroll
        for (int jj = 0; jj < JT; ++jj) {
          Da[jj] = fma(pa, tc, Da[jj]);
          if (NT == 2) Db[jj] = fma(pb, tc, Db[jj]);
          const double tn = fma(sr2, tc, -tp);
          tp = tc;
          tc = tn;
        }
      }
    }
  }

  // ---- epilogue: residual partials (compensated, as pairs)
  __shared__ double red[3][4];
  {
    wave_sum2(pi_s, pi_c);
    const double a = wave_sum(abs_acc);
    if (lane == 0) { red[0][wave] = pi_s; red[1][wave] = pi_c; red[2][wave] = a; }
  }
  __syncthreads();
  if (t == 0) {
    double ps = red[0][0], pc = red[1][0];
    for (int w = 1; w < 4; ++w) { two_sum_add(ps, pc, red[0][w]); pc += red[1][w]; }
    const double a = ((red[2][0] + red[2][1]) + red[2][2]) + red[2][3];
    const size_t idx = (size_t)growrow * v.nqt + qt;
    v.Pip[2 * idx] = ps;
    v.Pip[2 * idx + 1] = pc;
    v.Absp[idx] = a;
  }
  if (!JAC) return;

  // ---- q-side: angular sums staged in LDS, reduced over the four waves
  __shared__ double bs[2][4][64];
  bs[0][wave][lane] = Ba;
  bs[1][wave][lane] = Bb;
  // ---- k-side: reduce each coefficient over the lanes of the wave that hold
  // the same slice, then over the waves through LDS
  __shared__ double ds[4][NT][NJ];
#pragma unroll
  for (int jj = 0; jj < JT; ++jj) {
    double a = Da[jj];
    double b = NT == 2 ? Db[jj] : 0.0;
#pragma unroll
    for (int o = 32; o >= G; o >>= 1) {
      a += __shfl_xor(a, o, 64);
      if (NT == 2) b += __shfl_xor(b, o, 64);
    }
    if (lane < G) {
      ds[wave][0][lane * JT + jj] = a;
      if (NT == 2) ds[wave][NT - 1][lane * JT + jj] = b;
    }
  }
  __syncthreads();
  if (t < 64) {
    const double sa_ = ((bs[0][0][t] + bs[0][1][t]) + bs[0][2][t]) + bs[0][3][t];
    const double sb_ = ((bs[1][0][t] + bs[1][1][t]) + bs[1][2][t]) + bs[1][3][t];
    if (KIND == GLUON) {
      v.Bm[(size_t)row * v.Qp + qt * 64 + t] = sa_;
      v.Bm[(size_t)(v.RZ + row) * v.Qp + qt * 64 + t] = sb_;
    } else {
      v.Bm[(size_t)(2 * v.RZ + row) * v.Qp + qt * 64 + t] = sb_;
    }
  }
  for (int o = t; o < NT * NJ; o += 256) {
    const int tg = o / NJ, j = o - tg * NJ;
    double s = ((ds[0][tg][j] + ds[1][tg][j]) + ds[2][tg][j]) + ds[3][tg][j];
    if (j == 0) s *= 0.5;  // Tilde-T_0 = 1/2
    int grp = KIND == GLUON ? tg : 2;
    size_t base = (size_t)grp * v.RZ * v.nqt * NJ;
    v.Dp[base + ((size_t)row * v.nqt + qt) * NJ + j] = s;
  }
}

// --------------------------------------------------------------------------
// Eq = B . T on the FP64 matrix cores.  Block = one 16 x 16 tile of Eq; the
// four waves split the radial sum and meet in LDS.
__global__ __launch_bounds__(256) void contract_kernel(Views v) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int r0 = blockIdx.x * 16, j0 = blockIdx.y * 16;
  const int Qp = v.Qp, NJ = v.NJ;
  const int qper = Qp / 4;
  const int qbeg = wave * qper;
  const int i = lane & 15, kk = lane >> 4;
  typedef double d4 __attribute__((ext_vector_type(4)));
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  const double* A = v.Bm + (size_t)(r0 + i) * Qp + kk;
  const double* B = v.Ttab + (size_t)kk * NJ + j0 + i;
  for (int q = qbeg; q < qbeg + qper; q += 4) {
    const double a = A[q];
    const double b = B[(size_t)q * NJ];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  __shared__ double part[4][4][64];
#pragma unroll
  for (int r = 0; r < 4; ++r) part[wave][r][lane] = acc[r];
  __syncthreads();
  if (t < 64) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double s = ((part[0][r][t] + part[1][r][t]) + part[2][r][t]) + part[3][r][t];
      // v_mfma_f64_16x16x4f64: lane l, register r holds D[l/16 + 4 r][l % 16]
      const int row = r0 + (t >> 4) + 4 * r;
      const int col = j0 + (t & 15);
      v.Eq[(size_t)row * NJ + col] = s;
    }
  }
}

// --------------------------------------------------------------------------
// helpers for assembly: partial sums over the radial tiles, in tile order
__device__ __forceinline__ double sum_tiles(const double* p, int nqt) {
  double s = 0.0;
  for (int i = 0; i < nqt; ++i) s += p[i];
  return s;
}
__device__ __forceinline__ double sum_tiles_strided(const double* p, int nqt, int stride) {
  double s = 0.0;
  for (int i = 0; i < nqt; ++i) s += p[(size_t)i * stride];
  return s;
}

// Self-energy of one row from its (sum, error) tile pairs.
__device__ __forceinline__ double pi_row(const double* p, int nqt) {
  double s = 0.0, c = 0.0;
  for (int i = 0; i < nqt; ++i) { two_sum_add(s, c, p[2 * i]); c += p[2 * i + 1]; }
  return s + c;
}

// F_r and S_r for one row (Sec. 3: z(x_i) and g(x_i) with MOM subtraction).
__device__ __forceinline__ void row_residual(const Views& v, const Phys& ph, int r, double* F,
                                             double* S) {
  const bool gl = r < v.n_z;
  const int rr = gl ? r : v.RZ + (r - v.n_z);          // row in xrow / Pip
  const int sub = gl ? v.RZ - 1 : v.RZ + v.RG - 1;      // subtraction row
  const double pix = pi_row(v.Pip + (size_t)2 * rr * v.nqt, v.nqt);
  const double pis = pi_row(v.Pip + (size_t)2 * sub * v.nqt, v.nqt);
  const double abx = sum_tiles(v.Absp + (size_t)rr * v.nqt, v.nqt);
  const double abs_ = sum_tiles(v.Absp + (size_t)sub * v.nqt, v.nqt);
  const double d = exp(-v.lnX[r]);
  const double par = gl ? ph.z_lambda_inv : ph.g0_inv;
  F[r] = d - par - pix + pis;
  if (S) S[r] = fabs(d) + fabs(par) + abx + abs_;
}

__global__ __launch_bounds__(256) void residual_rows_kernel(Views v, Phys ph, double* F, double* S) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < v.n) row_residual(v, ph, r, F, S);
}

// J row r = one block.
__global__ __launch_bounds__(256) void assemble_kernel(Views v, Phys ph, double* __restrict__ J,
                                                       double* F, double* S) {
  const int r = blockIdx.x;
  const int t = threadIdx.x;
  const int NJ = v.NJ, nqt = v.nqt, n = v.n;
  const bool gl = r < v.n_z;
  const int i = gl ? r : r - v.n_z;
  const double d = exp(-v.lnX[r]);
  const double* Tx = v.Text + (size_t)r * NJ;
  double* Jr = J + (size_t)r * n;
  const size_t dstride = (size_t)nqt * NJ;
  if (gl) {
    const int sub = v.RZ - 1;
    const double* Dga = v.Dp;
    const double* Dgb = v.Dp + (size_t)v.RZ * dstride;
    for (int c = t; c < n; c += blockDim.x) {
      double val;
      if (c < v.n_z) {
        const int j = c;
        double ex = v.Eq[(size_t)i * NJ + j] + sum_tiles_strided(Dga + (size_t)i * dstride + j, nqt, NJ);
        double es = v.Eq[(size_t)sub * NJ + j] + sum_tiles_strided(Dga + (size_t)sub * dstride + j, nqt, NJ);
        val = -d * Tx[j] - ex + es;
      } else {
        const int j = c - v.n_z;
        double ex = v.Eq[(size_t)(v.RZ + i) * NJ + j] + sum_tiles_strided(Dgb + (size_t)i * dstride + j, nqt, NJ);
        double es = v.Eq[(size_t)(v.RZ + sub) * NJ + j] + sum_tiles_strided(Dgb + (size_t)sub * dstride + j, nqt, NJ);
        val = -ex + es;
      }
      Jr[c] = val;
    }
  } else {
    const int sub = v.RG - 1;
    const double* Dha = v.Dp + (size_t)2 * v.RZ * dstride;
    for (int c = t; c < n; c += blockDim.x) {
      double val;
      if (c < v.n_z) {
        const int j = c;
        val = -sum_tiles_strided(Dha + (size_t)i * dstride + j, nqt, NJ)
              + sum_tiles_strided(Dha + (size_t)sub * dstride + j, nqt, NJ);
      } else {
        const int j = c - v.n_z;
        val = -d * Tx[j] - v.Eq[(size_t)(2 * v.RZ + i) * NJ + j] + v.Eq[(size_t)(2 * v.RZ + sub) * NJ + j];
      }
      Jr[c] = val;
    }
  }
  if (t == 0 && F) row_residual(v, ph, r, F, S);
}

// --------------------------------------------------------------------------
// merit max_r |F_r| / S_r, ||F||_2 and ||d||_inf (one block).
__global__ __launch_bounds__(256) void norms_kernel(int n, const double* F, const double* S,
                                                   const double* d, double* out) {
  const int t = threadIdx.x;
  double m = 0.0, s2 = 0.0, dm = 0.0;
  bool bad = false;
  for (int r = t; r < n; r += 256) {
    const double f = F[r];
    const double sc = S ? S[r] : 0.0;
    const double q = sc > 0.0 ? fabs(f) / sc : fabs(f);
    if (!(q == q) || isinf(q)) bad = true;
    m = fmax(m, q);
    s2 = fma(f, f, s2);
    if (d) dm = fmax(dm, fabs(d[r]));
  }
  __shared__ double sm[256], ss[256], sd[256];
  __shared__ int sbad;
  if (t == 0) sbad = 0;
  __syncthreads();
  if (bad) sbad = 1;
  sm[t] = m; ss[t] = s2; sd[t] = dm;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) { sm[t] = fmax(sm[t], sm[t + o]); ss[t] += ss[t + o]; sd[t] = fmax(sd[t], sd[t + o]); }
    __syncthreads();
  }
  if (t == 0) {
    out[0] = sbad ? __longlong_as_double(0x7ff8000000000000LL) : sm[0];
    out[1] = sqrt(ss[0]);
    out[2] = sd[0];
  }
}

__global__ void axpy_kernel(int n, const double* c, double rho, const double* d, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = c[i] - rho * d[i];
}

// --------------------------------------------------------------------------
// FP64 LU with partial pivoting and the triangular solves, one workgroup.
// Right-looking: per column k the pivot is the first row of largest |A[i][k]|,
// rows are interchanged whole, multipliers A[i][k] / A[k][k] are stored in
// place and the trailing block is updated.  M is the matrix storage (LDS or
// global), row stride ld.
template <bool IN_LDS>
__global__ __launch_bounds__(1024) void lu_solve_kernel(int n, const double* __restrict__ Ain,
                                                        const double* __restrict__ b, double* x,
                                                        double* __restrict__ Aglob, int* piv,
                                                        int trans, int* flag) {
  extern __shared__ double lds[];
  const int t = threadIdx.x, nt = blockDim.x;
  const int ld = IN_LDS ? n + 1 : n;
  double* M = IN_LDS ? lds : Aglob;
  double* w = IN_LDS ? lds + (size_t)n * ld : lds;  // [n] right-hand side
  __shared__ int sp;
  __shared__ int sing;
  for (int e = t; e < n * n; e += nt) {
    const int i = e / n, j = e - i * n;
    M[(size_t)i * ld + j] = Ain[e];
  }
  for (int i = t; i < n; i += nt) w[i] = b[i];
  if (t == 0) sing = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (t < 64) {
      double best = -1.0;
      int bi = n;
      for (int i = k + t; i < n; i += 64) {
        const double a = fabs(M[(size_t)i * ld + k]);
        if (a > best) { best = a; bi = i; }
      }
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (t == 0) {
        sp = bi;
        piv[k] = bi;
        if (!(best > 0.0) || isinf(best)) sing = 1;
      }
    }
    __syncthreads();
    if (sing) break;
    const int p = sp;
    if (p != k)
      for (int j = t; j < n; j += nt) {
        const double tmp = M[(size_t)k * ld + j];
        M[(size_t)k * ld + j] = M[(size_t)p * ld + j];
        M[(size_t)p * ld + j] = tmp;
      }
    __syncthreads();
    const double dk = M[(size_t)k * ld + k];
    for (int i = k + 1 + t; i < n; i += nt) M[(size_t)i * ld + k] = M[(size_t)i * ld + k] / dk;
    __syncthreads();
    const int m = n - k - 1;
    for (int e = t; e < m * m; e += nt) {
      const int i = k + 1 + e / m, j = k + 1 + e % m;
      M[(size_t)i * ld + j] -= M[(size_t)i * ld + k] * M[(size_t)k * ld + j];
    }
    __syncthreads();
  }
  if (sing) {
    if (t == 0) flag[0] = 4;
    return;
  }
  if (!trans) {
    if (t == 0)
      for (int k = 0; k < n; ++k) {
        const int pk = piv[k];
        const double tmp = w[k]; w[k] = w[pk]; w[pk] = tmp;
      }
    __syncthreads();
    for (int i = 0; i < n; ++i) {  // L y = P b (unit lower)
      const double wi = w[i];
      for (int r = i + 1 + t; r < n; r += nt) w[r] -= M[(size_t)r * ld + i] * wi;
      __syncthreads();
    }
    for (int i = n - 1; i >= 0; --i) {  // U x = y
      if (t == 0) w[i] = w[i] / M[(size_t)i * ld + i];
      __syncthreads();
      const double wi = w[i];
      for (int r = t; r < i; r += nt) w[r] -= M[(size_t)r * ld + i] * wi;
      __syncthreads();
    }
  } else {
    for (int i = 0; i < n; ++i) {  // U^T y = b
      if (t == 0) w[i] = w[i] / M[(size_t)i * ld + i];
      __syncthreads();
      const double wi = w[i];
      for (int r = i + 1 + t; r < n; r += nt) w[r] -= M[(size_t)i * ld + r] * wi;
      __syncthreads();
    }
    for (int i = n - 1; i >= 0; --i) {  // L^T z = y
      const double wi = w[i];
      for (int r = t; r < i; r += nt) w[r] -= M[(size_t)i * ld + r] * wi;
      __syncthreads();
    }
    if (t == 0)
      for (int k = n - 1; k >= 0; --k) {
        const int pk = piv[k];
        const double tmp = w[k]; w[k] = w[pk]; w[pk] = tmp;
      }
    __syncthreads();
  }
  for (int i = t; i < n; i += nt) x[i] = w[i];
  if (t == 0) flag[0] = 0;
}

// --------------------------------------------------------------------------
// launchers

hipError_t launch_dressing(const Views& v, const Phys& ph, const double* c, hipStream_t st) {
  hipLaunchKernelGGL(dressing_kernel, dim3(1), dim3(256), 0, st, v, ph, c);
  return hipGetLastError();
}

template <int NJ, bool JAC>
static hipError_t points_nj(const Views& v, const Phys& ph, hipStream_t st, hipEvent_t* ev) {
  if (ev) (void)hipEventRecord(ev[0], st);
  hipLaunchKernelGGL((point_kernel<GLUON, NJ, JAC>), dim3(v.RZ * v.nqt), dim3(256), 0, st, v, ph);
  if (ev) (void)hipEventRecord(ev[1], st);
  hipLaunchKernelGGL((point_kernel<GHOST, NJ, JAC>), dim3(v.RG * v.nqt), dim3(256), 0, st, v, ph);
  if (ev) (void)hipEventRecord(ev[2], st);
  return hipGetLastError();
}

template <bool JAC>
static hipError_t points_dispatch(const Views& v, const Phys& ph, hipStream_t st, hipEvent_t* ev) {
  switch (v.NJ) {
    case 16: return points_nj<16, JAC>(v, ph, st, ev);
    case 32: return points_nj<32, JAC>(v, ph, st, ev);
    case 48: return points_nj<48, JAC>(v, ph, st, ev);
    case 64: return points_nj<64, JAC>(v, ph, st, ev);
    case 96: return points_nj<96, JAC>(v, ph, st, ev);
    case 128: return points_nj<128, JAC>(v, ph, st, ev);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_points(const Views& v, const Phys& ph, bool jacobian, hipStream_t st, hipEvent_t* ev) {
  return jacobian ? points_dispatch<true>(v, ph, st, ev) : points_dispatch<false>(v, ph, st, ev);
}

hipError_t launch_contract(const Views& v, hipStream_t st) {
  hipLaunchKernelGGL(contract_kernel, dim3(v.Rbp / 16, v.NJ / 16), dim3(256), 0, st, v);
  return hipGetLastError();
}

hipError_t launch_assemble(const Views& v, const Phys& ph, double* J, double* F, double* S, hipStream_t st) {
  hipLaunchKernelGGL(assemble_kernel, dim3(v.n), dim3(256), 0, st, v, ph, J, F, S);
  return hipGetLastError();
}

hipError_t launch_residual_rows(const Views& v, const Phys& ph, double* F, double* S, hipStream_t st) {
  hipLaunchKernelGGL(residual_rows_kernel, dim3((v.n + 255) / 256), dim3(256), 0, st, v, ph, F, S);
  return hipGetLastError();
}

hipError_t launch_norms(const Views& v, const double* F, const double* S, const double* d, double* out,
                        hipStream_t st) {
  hipLaunchKernelGGL(norms_kernel, dim3(1), dim3(256), 0, st, v.n, F, S, d, out);
  return hipGetLastError();
}

hipError_t launch_axpy(int n, const double* c, double rho, const double* d, double* out, hipStream_t st) {
  hipLaunchKernelGGL(axpy_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, c, rho, d, out);
  return hipGetLastError();
}

hipError_t launch_lu_solve(const Views& v, const double* A, const double* b, double* x, int trans,
                           hipStream_t st) {
  const int n = v.n;
  const size_t lds_bytes = ((size_t)n * (n + 1) + n) * sizeof(double);
  // largest dynamic LDS a workgroup may use on this device (160 KiB on gfx950)
  static int max_lds = -1;
  if (max_lds < 0) {
    int dev = 0, val = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&val, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      val = 64 * 1024;
    max_lds = val;
    if (max_lds > 64 * 1024 &&
        hipFuncSetAttribute((const void*)lu_solve_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            max_lds - 1024) != hipSuccess)
      max_lds = 64 * 1024;
  }
  if (lds_bytes + 1024 <= (size_t)max_lds) {
    hipLaunchKernelGGL(lu_solve_kernel<true>, dim3(1), dim3(1024), lds_bytes, st, n, A, b, x, v.LU, v.piv,
                       trans, v.flag);
  } else {
    hipLaunchKernelGGL(lu_solve_kernel<false>, dim3(1), dim3(1024), (size_t)n * sizeof(double), st, n, A, b,
                       x, v.LU, v.piv, trans, v.flag);
  }
  return hipGetLastError();
}

}  // namespace dse
