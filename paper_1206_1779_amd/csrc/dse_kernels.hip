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

#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>
#include <utility>

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

// 1 / x for a finite nonzero x away from the exponent extremes: the hardware
// reciprocal estimate and two Newton steps r <- r + r (1 - x r), within 1 ulp
// (the correctly rounded division is a longer dependent sequence).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  return fma(fma(-x, r, 1.0), r, r);
}

// Natural logarithm of a positive normal x, from the classical series
//   ln m = 2 atanh f = 2 (f + f^3/3 + f^5/5 + ...),  f = (m - 1) / (m + 1),
// with x = m 2^e and the significand m in [1/sqrt 2, sqrt 2), so |f| < 0.172
// and f^2 < 0.0295: the terms up to f^19/19 leave a relative truncation
// error below f^20/21 < 2.3e-17 (a fifth of the rounding unit); ln 2 is split
// into a part with 32 significant bits (e ln2_hi exact) and the rest.
// Within 2.5 ulp of the exact value (measured against a long-double log over
// 2e7 arguments in [e^-40, e^40], the same with three more terms), against
// about 80 dependent instructions of the library's double-double log.
__device__ __forceinline__ double log_series(double x) {
  int e;
  double m = frexp(x, &e);  // [1/2, 1)
  const bool lo = m < 0.70710678118654752440;
  m = lo ? m + m : m;
  e = lo ? e - 1 : e;
  const double f = (m - 1.0) * recip(m + 1.0);
  const double f2 = f * f;
  double q = 1.0 / 19;
  q = fma(q, f2, 1.0 / 17);
  q = fma(q, f2, 1.0 / 15);
  q = fma(q, f2, 1.0 / 13);
  q = fma(q, f2, 1.0 / 11);
  q = fma(q, f2, 1.0 / 9);
  q = fma(q, f2, 1.0 / 7);
  q = fma(q, f2, 1.0 / 5);
  q = fma(q, f2, 1.0 / 3);
  const double ln2_hi = 0.6931471806019545, ln2_lo = -4.2009150726810846e-11;
  const double ed = (double)e;
  const double t = fma(f * f2, q, f);  // atanh f
  return fma(ed, ln2_hi, fma(2.0, t, ed * ln2_lo));
}

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

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// v of lane (lane ^ r) for a constant r (the switch folds once r is known):
// partners inside a quad of lanes by a DPP quad permutation (vector moves,
// no LDS round trip and no address operand), others by ds_bpermute.
template <int CTRL>
__device__ __forceinline__ int quad_perm_i(int v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ double quad_perm_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = quad_perm_i<CTRL>((int)(b & 0xffffffffLL)), hi = quad_perm_i<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_xor(double v, int r) {
  switch (r) {
    case 1: return quad_perm_d<0xB1>(v);  // quad_perm [1,0,3,2]
    case 2: return quad_perm_d<0x4E>(v);  // [2,3,0,1]
    case 3: return quad_perm_d<0x1B>(v);  // [3,2,1,0]
    default: return __shfl_xor(v, r, 64);
  }
}
__device__ __forceinline__ float lane_xor(float v, int r) {
  switch (r) {
    case 1: return __int_as_float(quad_perm_i<0xB1>(__float_as_int(v)));
    case 2: return __int_as_float(quad_perm_i<0x4E>(__float_as_int(v)));
    case 3: return __int_as_float(quad_perm_i<0x1B>(__float_as_int(v)));
    default: return __shfl_xor(v, r, 64);
  }
}

// --------------------------------------------------------------------------
// dressing: coef (c_0 halved, zero padded), ln Z / ln G at radial nodes and at
// the collocation points.
// Outputs o0 + t, o0 + t + ostep, ... of [radial nodes | collocation points];
// the block with write_coef also stores the coefficient vector.  Tables are
// read transposed (j-major), so consecutive threads read consecutive words.
__device__ __forceinline__ void dressing_body(const Views& v, const Phys& ph, const double* __restrict__ c,
                                              int o0, int ostep, bool write_coef) {
  __shared__ double sa[DSE_MAX_N], sb[DSE_MAX_N];
  const int t = threadIdx.x;
  const int NJ = v.NJ;
  for (int j = t; j < NJ; j += 256) {
    double a = j < v.n_z ? c[j] : 0.0;
    double b = j < v.n_g ? c[v.n_z + j] : 0.0;
    if (j == 0) { a *= 0.5; b *= 0.5; }
    // the table holds Tilde-T_0 = 1/2: keep the unhalved value for the GEMV
    sa[j] = j < v.n_z ? c[j] : 0.0;
    sb[j] = j < v.n_g ? c[v.n_z + j] : 0.0;
    if (write_coef) {
      v.coef[j] = a;
      v.coef[NJ + j] = b;
    }
  }
  __syncthreads();
  const int nout = v.Qp + v.n;
  for (int o = o0 + t; o < nout; o += ostep) {
    if (o < v.Qp) {
      const double* T = v.TtabT + o;
      double z = 0.0, g = 0.0;
      // the table entries of a chunk of 16 are all requested before the sums
      // use them (NJ is a multiple of 16): a few memory round trips per
      // output instead of one per unrolled group of eight
      for (int j0 = 0; j0 < NJ; j0 += 16) {
        double tj[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) tj[u] = T[(size_t)(j0 + u) * v.Qp];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          z = fma(sa[j0 + u], tj[u], z);
          g = fma(sb[j0 + u], tj[u], g);
        }
      }
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
      const double* T = v.TextT + r;
      const double* cc = r < v.n_z ? sa : sb;
      double s = 0.0;
      for (int j0 = 0; j0 < NJ; j0 += 16) {
        double tj[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) tj[u] = T[(size_t)(j0 + u) * v.n];
#pragma unroll
        for (int u = 0; u < 16; ++u) s = fma(cc[j0 + u], tj[u], s);
      }
      v.lnX[r] = s;  // collocation points lie in [eps2, lambda2]: no extension
    }
  }
}

__global__ __launch_bounds__(256) void dressing_kernel(Views v, Phys ph, const double* __restrict__ c) {
  dressing_body(v, ph, c, blockIdx.x * 256, gridDim.x * 256, blockIdx.x == 0);
}

// ln Z and ln G at the nodes of every row's own radial grid (the split at x,
// Sec. 3): one thread per (row, node), the Chebyshev recurrence at the node's
// mapped coordinate (a table) plus the IR power laws below eps2 (the grids end
// at lambda2, so no UV extension).
__global__ __launch_bounds__(256) void dressing_split_kernel(Views v, Phys ph, const double* __restrict__ c) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= (v.RZ + v.RG) * v.Qp) return;
  const double s = v.syr[i];
  const double s2 = s + s;
  double z = 0.5 * c[0], g = 0.5 * c[v.n_z];
  double Tp = 1.0, Tc = s;
  const int nmax = v.n_z > v.n_g ? v.n_z : v.n_g;
  for (int j = 1; j < nmax; ++j) {
    if (j < v.n_z) z = fma(c[j], Tc, z);
    if (j < v.n_g) g = fma(c[v.n_z + j], Tc, g);
    const double Tn = fma(s2, Tc, -Tp);
    Tp = Tc;
    Tc = Tn;
  }
  const double ly = log(v.yr[i]);
  if (ly < ph.ln_eps2) {
    z += 2.0 * ph.kappa * (ly - ph.ln_eps2);
    g += -ph.kappa * (ly - ph.ln_eps2);
  }
  v.lnZyr[i] = z;
  v.lnGyr[i] = g;
}

// --------------------------------------------------------------------------
// Reduce-scatter of NV values per lane over the lanes that share a slice
// (lane bits log2(G) .. 5).  While the count is even a stage halves it: the
// lane keeps one half and sends the other to its partner; an odd count falls
// back to a butterfly all-reduce (then only the lane with the bit clear
// writes).  On return vals[0 .. slice_count) hold complete sums for indices
// base .. base + slice_count - 1.
template <int NV, int G>
__host__ __device__ constexpr int slice_count() {
  int c = NV;
  for (int o = G; o < 64; o <<= 1)
    if (c % 2 == 0) c /= 2;
  return c;
}

template <int CNT, int O, typename T>
__device__ __forceinline__ void slice_stage(T* vals, int lane, int& base, bool& writer) {
  if constexpr (O < 64) {
    if constexpr (CNT % 2 == 0) {
      constexpr int H = CNT / 2;
      const bool hi = (lane & O) != 0;
#pragma unroll
      for (int i = 0; i < H; ++i) {
        const T send = hi ? vals[i] : vals[i + H];
        const T keep = hi ? vals[i + H] : vals[i];
        vals[i] = keep + __shfl_xor(send, O, 64);
      }
      if (hi) base += H;
      slice_stage<H, O * 2, T>(vals, lane, base, writer);
    } else {
#pragma unroll
      for (int i = 0; i < CNT; ++i) vals[i] += __shfl_xor(vals[i], O, 64);
      if (lane & O) writer = false;
      slice_stage<CNT, O * 2, T>(vals, lane, base, writer);
    }
  }
}

template <int NV, int G, typename T>
__device__ __forceinline__ void slice_reduce(T* vals, int lane, int& base, bool& writer) {
  slice_stage<NV, G, T>(vals, lane, base, writer);
}

// --------------------------------------------------------------------------
// The fused point kernel.  Block = one row x 64 radial nodes; wave w takes the
// angles k = w, w+4, ...; lane = radial node.  Pass 1 (every lane, own point):
// recurrence + series with wave-uniform coefficients.  Pass 2 (Jacobian only):
// a group of G lanes shares its G points; member m accumulates
// j in [m JT, (m+1) JT) for all G points, starting the recurrence from
// (T_{m JT - 1}, T_{m JT}) saved in pass 1.
//
// MODE: 0 residual (Pi and sum|.| per tile); 1 Jacobian (also B and D);
// 2 vector-Jacobian product (every integrand and its derivatives weighted by
// the row weight rw[row]: B and D then sum to u^T dF/dc; the pair slots of
// Pip carry d Pi / d alpha, weighted); 3 parameter VJP only (weighted
// d Pi / d alpha, no B, no D).
// MIX (Jacobian mode): the derivative sums B and D, and the k-side
// recurrence, in FP32; every quantity that enters F stays FP64.
enum { MODE_RES = 0, MODE_JAC = 1, MODE_VJP = 2, MODE_VTH = 3 };

// LDS of one point-kernel block (doubles): red[3][4] at 0, bs[2][4][64] at 16,
// ds[4][NT*NJ] at 528; in the batch kernel the coefficients a | b at 528 + 8 NJ.
template <int NJ, bool BATCH>
__host__ __device__ constexpr int point_smem() { return 528 + (BATCH ? 10 : 8) * NJ; }

// BATCH: a body of the batch kernel, which holds one body per order and row
// kind and so has few registers to spare: the coefficients are staged in LDS
// and ln z comes from the library's log (the series below needs more
// registers and cost the batch kernel half its occupancy).
// SPLIT: every row has its own radial grid (the split at x of Sec. 3); the
// q-side derivative, d integrand / d ln(dressing at y) times Tilde-T_j(s(y)),
// then depends on the row as well and is accumulated here with the k-side
// sums (each lane adds its angular sums B at its node y as one more point of
// the k-side pass), so no B . T contraction follows.  FP64 only.
template <int KIND, int NJ, int MODE, bool MIX = false, bool BATCH = false, bool SPLIT = false>
__device__ __forceinline__ void point_body(const Views& v, const Phys& ph, int row, int tile,
                                           double* __restrict__ smem) {
  using TL = Tile<KIND, NJ>;
  using acc_t = typename std::conditional<MIX, float, double>::type;
  constexpr int G = TL::G;
  constexpr int JT = TL::JT;
  constexpr bool JAC = MODE == MODE_JAC || MODE == MODE_VJP;  // B and D wanted
  constexpr int NTA = KIND == GLUON ? 2 : 1;                   // k-side targets of the angle loop
  constexpr int NT = KIND == GLUON || (SPLIT && JAC) ? 2 : 1;  // targets of D (ghost: b from the q-side)
  constexpr bool WEIGHTED = MODE == MODE_VJP || MODE == MODE_VTH;
  static_assert(!SPLIT || (!MIX && !BATCH && !WEIGHTED), "the split radial grid is FP64 residual/Jacobian only");

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);  // uniform: angle data through scalar loads
  const int KS = v.KS;
  const int ntile = v.nqt * KS;                   // partial tiles per row; tile = qt * KS + ks
  const int qt = tile / KS, ks = tile - qt * KS;
  const int q = qt * 64 + lane;
  const int growrow = KIND == GLUON ? row : v.RZ + row;  // index into xrow / Pip

  const double x = v.xrow[growrow];
  const size_t qi = SPLIT ? (size_t)growrow * v.Qp + q : (size_t)q;
  const double y = SPLIT ? v.yr[qi] : v.y[q];
  const double W = SPLIT ? v.Wr[qi] : v.W[q];
  const double lGy = SPLIT ? v.lnGyr[qi] : v.lnGy[q];
  const double lZy = SPLIT ? v.lnZyr[qi] : v.lnZy[q];

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

  // Chebyshev coefficients a | b: wave-uniform, read a chunk at a time inside
  // the recurrence; the chunk loop stays a loop, so they are neither held in
  // registers across it nor gathered at its top.  Read through the scalar
  // cache into scalar registers (no LDS traffic), or, in the batch kernel
  // (no scalar registers to spare), staged in LDS and read with broadcast
  // loads.
  const double* __restrict__ coef = v.coef;
  if constexpr (BATCH) {
    double* __restrict__ cl = smem + 528 + 8 * NJ;
    for (int j = t; j < 2 * NJ; j += 256) cl[j] = v.coef[j];
    __syncthreads();
    coef = cl;
  }
  const double* __restrict__ ang = v.ang;
  const int Kp = v.Kp;
  const double rw = WEIGHTED ? v.rw[growrow] : 1.0;

  double pi_s = 0.0, pi_c = 0.0, abs_acc = 0.0;
  acc_t Ba = 0, Bb = 0;
  acc_t Da[JAC ? JT : 1], Db[JAC && NT == 2 ? JT : 1];
  if (JAC) {
#pragma unroll
    for (int jj = 0; jj < JT; ++jj) { Da[jj] = 0; if (NT == 2) Db[jj] = 0; }
  }
  const int member = lane & (G - 1);

  for (int k = ks * 4 + wave; k < Kp; k += 4 * KS) {
    const double ck = ang[k];
    const double s2h = ang[Kp + k];
    const double wk = KIND == GLUON ? ang[2 * Kp + k] : ang[3 * Kp + k];
    const double st2 = ang[4 * Kp + k];

    const double w = fma(Bw, s2h, Aw);
    const double lz = lnmx + (BATCH ? log(w) : log_series(w));
    double s = (lz - ph.L0) * ph.invL1;
    s = fmin(fmax(s, -1.0), 1.0);
    const double s2 = s + s;

    // ---- pass 1: recurrence and series
    double sa = 0.0, sb = 0.0;
    double Tp = s, Tc = 1.0;  // (T_{-1}, T_0)
    double stp[G > 1 ? G : 1], stc[G > 1 ? G : 1];
    // chunk width: a divisor of the pass-2 slice width JT
    constexpr int CH = JT % 8 == 0 ? 8 : 4;
    static_assert(JT % CH == 0, "chunks must tile the slices");
    auto chunk = [&](int j0) {
      double c8a[CH], c8b[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        c8a[u] = coef[j0 + u];
        c8b[u] = KIND == GLUON ? coef[NJ + j0 + u] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        sa = fma(c8a[u], Tc, sa);
        if (KIND == GLUON) sb = fma(c8b[u], Tc, sb);
        const double Tn = fma(s2, Tc, -Tp);
        Tp = Tc;
        Tc = Tn;
      }
    };
    // start pairs (T_{m JT - 1}, T_{m JT}) of pass 2.  Up to two slices: a
    // uniform branch in the one chunk loop saves the second.  More: one chunk
    // loop per slice, each pair saved into its fixed registers before it (a
    // branch over several targets would become selects run on every chunk).
    stp[0] = Tp;
    stc[0] = Tc;
    if constexpr (G > 2) {
#pragma unroll
      for (int m = 0; m < G; ++m) {
        if (m > 0) { stp[m] = Tp; stc[m] = Tc; }
#pragma clang loop unroll(disable)
        for (int j0 = m * JT; j0 < (m + 1) * JT; j0 += CH) chunk(j0);
      }
    } else {
#pragma clang loop unroll(disable)
      for (int j0 = 0; j0 < NJ; j0 += CH) {
        if (G == 2 && j0 == JT) { stp[G - 1] = Tp; stc[G - 1] = Tc; }
        chunk(j0);
      }
    }
    double XZ = 0.0, XG = 0.0, dXa = 0.0;  // dXa: d ln(1 + omega l) / d alpha (UV)
    if (lz < ph.ln_eps2) {
      XZ = 2.0 * ph.kappa * (lz - ph.ln_eps2);
      XG = -ph.kappa * (lz - ph.ln_eps2);
    } else if (lz > ph.ln_lam2) {
      const double l = lz - ph.ln_lam2;
      const double arg = fma(ph.omega, l, 1.0);
      const double L = BATCH ? log(arg) : log_series(arg);
      XZ = ph.gamma * L;
      XG = ph.delta * L;
      if (WEIGHTED) dXa = ph.omega_per_alpha * l / arg;
    }
    const double lZz = sa + XZ;

    double Pa, Pb;
    if (KIND == GLUON) {
      const double lGz = sb + XG;
      const double iw = BATCH ? 1.0 / w : recip(w);
      const double Qn = fma(fma(fma(fma(qc4, ck, qc3), ck, qc2), ck, qc1), ck, qc0);
      const double Qk = Qn * iw * iw;
      const double Mk = ymx * st2 * iw;
      const double lg = lGy + lGz;
      const double Fgl = exp(ph.e1 * lg + ph.e2 * (lZy + lZz));
      const double Fgh = exp(lg);
      const double om = pref * wk;
      const double tq = om * Qk * Fgl;
      const double tm = om * Mk * Fgh;
      Pa = tq * ph.e2;           // d integrand / d ln Z (at y or at z)
      Pb = fma(tq, ph.e1, tm);   // d integrand / d ln G (at y or at z)
      if (WEIGHTED) {
        // d integrand / d alpha: linear through C, and through omega in the
        // UV extrapolation of ln Z(z), ln G(z)
        const double da = (tq + tm) * ph.inv_alpha + (Pa * ph.gamma + Pb * ph.delta) * dXa;
        two_sum_add(pi_s, pi_c, rw * da);
        Pa *= rw;
        Pb *= rw;
      } else {
        two_sum_add(pi_s, pi_c, tq + tm);
        abs_acc += fabs(tq) + fabs(tm);
      }
      if (JAC) { Ba += (acc_t)Pa; Bb += (acc_t)Pb; }
    } else {
      double val = pref * wk * exp(lGy + lZz - 2.0 * lz);  // rho G(y) Z(z) / z^2
      if (WEIGHTED) {
        const double da = val * ph.inv_alpha + val * ph.gamma * dXa;
        two_sum_add(pi_s, pi_c, rw * da);
        val *= rw;
      } else {
        two_sum_add(pi_s, pi_c, val);
        abs_acc += fabs(val);
      }
      Pa = val;                  // k-side: d / d ln Z(z)
      Pb = val;
      if (JAC) Bb += (acc_t)val; // q-side: d / d ln G(y)
    }

    if (JAC) {
      // ---- pass 2: k-side accumulation over the G points of the lane group
      const acc_t sA = (acc_t)s, PaA = (acc_t)Pa, PbA = (acc_t)Pb;
#pragma unroll
      for (int r = 0; r < G; ++r) {
        acc_t tp, tc, pa, pb;
        if (r == 0) {
          double tp_ = stp[0], tc_ = stc[0];
#pragma unroll
          for (int m = 1; m < G; ++m) if (member == m) { tp_ = stp[m]; tc_ = stc[m]; }
          tp = (acc_t)tp_; tc = (acc_t)tc_;
          pa = PaA; pb = PbA;
        } else {
          // send the start pair the reading lane (member ^ r) needs
          const int want = member ^ r;
          double sp = stp[0], sc = stc[0];
#pragma unroll
          for (int m = 1; m < G; ++m) if (want == m) { sp = stp[m]; sc = stc[m]; }
          tp = lane_xor((acc_t)sp, r);
          tc = lane_xor((acc_t)sc, r);
          pa = lane_xor(PaA, r);
          pb = NT == 2 ? lane_xor(PbA, r) : (acc_t)0;
        }
        // the owner's mapped momentum drives its recurrence
        const acc_t sr = r == 0 ? sA : lane_xor(sA, r);
        const acc_t sr2 = sr + sr;
#pragma unroll
        for (int jj = 0; jj < JT; ++jj) {
          Da[jj] = fma(pa, tc, Da[jj]);
          if (NTA == 2) Db[jj] = fma(pb, tc, Db[jj]);
          const acc_t tn = fma(sr2, tc, -tp);
          tp = tc;
          tc = tn;
        }
      }
    }
  }

  if constexpr (SPLIT && JAC) {
    // ---- q-side on the row's own grid: this wave's angular sums Ba, Bb at
    // the lane's node y enter like one more point of the k-side pass, with the
    // Chebyshev recurrence at s(y) (gluon rows: both targets; ghost rows: the
    // b target only, d / d ln G(y))
    const double sy = v.syr[qi];
    const double sy2 = sy + sy;
    double qtp[G], qtc[G];
    {
      double Tp = sy, Tc = 1.0;  // (T_{-1}, T_0)
#pragma unroll
      for (int m = 0; m < G; ++m) {
        qtp[m] = Tp;
        qtc[m] = Tc;
#pragma clang loop unroll(disable)
        for (int j = 0; j < JT; ++j) {
          const double Tn = fma(sy2, Tc, -Tp);
          Tp = Tc;
          Tc = Tn;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < G; ++r) {
      double tp, tc, pa, pb;
      if (r == 0) {
        tp = qtp[0]; tc = qtc[0];
#pragma unroll
        for (int m = 1; m < G; ++m) if (member == m) { tp = qtp[m]; tc = qtc[m]; }
        pa = Ba; pb = Bb;
      } else {
        const int want = member ^ r;
        double sp = qtp[0], sc = qtc[0];
#pragma unroll
        for (int m = 1; m < G; ++m) if (want == m) { sp = qtp[m]; sc = qtc[m]; }
        tp = lane_xor(sp, r);
        tc = lane_xor(sc, r);
        pa = KIND == GLUON ? lane_xor((double)Ba, r) : 0.0;
        pb = lane_xor((double)Bb, r);
      }
      const double sr = r == 0 ? sy : lane_xor(sy, r);
      const double sr2 = sr + sr;
#pragma unroll
      for (int jj = 0; jj < JT; ++jj) {
        if (KIND == GLUON) Da[jj] = fma(pa, tc, Da[jj]);
        Db[jj] = fma(pb, tc, Db[jj]);
        const double tn = fma(sr2, tc, -tp);
        tp = tc;
        tc = tn;
      }
    }
  }

  // ---- epilogue: residual partials (compensated, as pairs)
  double (*red)[4] = reinterpret_cast<double (*)[4]>(smem);
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
    const size_t idx = (size_t)growrow * ntile + tile;
    v.Pip[2 * idx] = ps;
    v.Pip[2 * idx + 1] = pc;
    v.Absp[idx] = a;
  }
  if (!JAC) return;

  // ---- q-side: angular sums staged in LDS, reduced over the four waves
  acc_t (*bs)[4][64] = reinterpret_cast<acc_t (*)[4][64]>(smem + 16);
  if (!SPLIT) {
    bs[0][wave][lane] = Ba;
    bs[1][wave][lane] = Bb;
  }
  // ---- k-side: reduce-scatter over the lanes that hold the same slice, then
  // over the waves through LDS
  acc_t (*ds)[NT * NJ] = reinterpret_cast<acc_t (*)[NT * NJ]>(smem + 528);
  {
    acc_t vals[NT * JT];
#pragma unroll
    for (int jj = 0; jj < JT; ++jj) {
      vals[jj] = Da[jj];
      if (NT == 2) vals[JT + jj] = Db[jj];
    }
    int base = 0;        // index (within this lane's NT*JT values) of vals[0]
    bool writer = true;  // one lane of each group of equal partial sums writes
    slice_reduce<NT * JT, G, acc_t>(vals, lane, base, writer);
    constexpr int CNT = slice_count<NT * JT, G>();
    if (writer) {
#pragma unroll
      for (int i = 0; i < CNT; ++i) {
        const int idx = base + i;           // 0 .. NT*JT-1
        const int tg = idx / JT, jj = idx - tg * JT;
        ds[wave][tg * NJ + member * JT + jj] = vals[i];
      }
    }
  }
  __syncthreads();
  if (!SPLIT && t < 64) {
    const acc_t sa_ = ((bs[0][0][t] + bs[0][1][t]) + bs[0][2][t]) + bs[0][3][t];
    const acc_t sb_ = ((bs[1][0][t] + bs[1][1][t]) + bs[1][2][t]) + bs[1][3][t];
    acc_t* Bk = reinterpret_cast<acc_t*>(v.Bm) + (size_t)ks * v.Rbp * v.Qp;
    if (KIND == GLUON) {
      Bk[(size_t)row * v.Qp + qt * 64 + t] = sa_;
      Bk[(size_t)(v.RZ + row) * v.Qp + qt * 64 + t] = sb_;
    } else {
      Bk[(size_t)(2 * v.RZ + row) * v.Qp + qt * 64 + t] = sb_;
    }
  }
  for (int o = t; o < NT * NJ; o += 256) {
    const int tg = o / NJ, j = o - tg * NJ;
    acc_t sum = ((ds[0][o] + ds[1][o]) + ds[2][o]) + ds[3][o];
    if (j == 0) sum *= (acc_t)0.5;  // Tilde-T_0 = 1/2
    // groups: gluon-a, gluon-b (RZ rows each), ghost-a, ghost-b (RG rows each)
    const int grp_row0 = KIND == GLUON ? tg * v.RZ : 2 * v.RZ + tg * v.RG;
    const size_t base = (size_t)grp_row0 * ntile * NJ;
    reinterpret_cast<acc_t*>(v.Dp)[base + ((size_t)row * ntile + tile) * NJ + j] = sum;
  }
}

// One block per (row, tile): blockIdx.x = row * (nqt KS) + tile.  The gluon
// rows' FP64 Jacobian kernel up to order 64 is held to three waves per SIMD
// (168 VGPRs, no spills) instead of the two its free allocation gives.
template <int KIND, int NJ, int MODE, bool MIX>
constexpr int point_waves() { return KIND == GLUON && MODE == MODE_JAC && !MIX && NJ <= 64 ? 3 : 1; }

template <int KIND, int NJ, int MODE, bool MIX, bool SPLIT = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(point_waves<KIND, NJ, MODE, MIX>())))
void point_kernel(Views v, Phys ph) {
  __shared__ double smem[point_smem<NJ, false>()];
  const int ntile = v.nqt * v.KS;
  const int row = blockIdx.x / ntile;
  point_body<KIND, NJ, MODE, MIX, false, SPLIT>(v, ph, row, blockIdx.x - row * ntile, smem);
}

// --------------------------------------------------------------------------
// Eq = B . T on the FP64 matrix cores, plus the k-side sums, in kCS parts:
// part p takes the radial nodes [p Qp/kCS, (p+1) Qp/kCS) and the partial
// tiles [p ntile/kCS, (p+1) ntile/kCS) and writes Eq[p] (the assembly adds the
// parts in a fixed order).  Splitting the sum keeps few dependent loads per
// wave: the operands were written by other XCDs and come from beyond the L2.
// Blocks with bx < Rbp/16 compute one 16 x 16 tile (the four waves split the
// part's radial range and meet in LDS) and add, for gluon rows, the k-side
// partial sums of the same target; the remaining blocks reduce the ghost
// rows' k-side partials into Dgh[p].
// SPLIT (each row on its own radial grid): the q-side sums are already in the
// k-side partials, so there is no product: Eq = the partial sums of the
// gluon rows' targets and of the ghost rows' b target.
template <bool MIX, bool SPLIT = false>
__device__ __forceinline__ void contract_body(const Views& v, int bx, int by, int part) {
  using acc_t = typename std::conditional<MIX, float, double>::type;
  const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int Qp = v.Qp, NJ = v.NJ;
  const int ntile = v.nqt * v.KS;
  const int tlo = part * ntile / kCS, thi = (part + 1) * ntile / kCS;
  const size_t dstride = (size_t)ntile * NJ;
  const int ntiles_r = v.Rbp / 16;
  const acc_t* __restrict__ Dp = reinterpret_cast<const acc_t*>(v.Dp);
  if (bx >= ntiles_r) {
    // ghost rows, k-side (target a): Dgh[part][row][j] = sum over the part's tiles
    const int row0 = (bx - ntiles_r) * 16;
    const acc_t* D = Dp + (size_t)2 * v.RZ * dstride;
    acc_t* out = reinterpret_cast<acc_t*>(v.Dgh) + (size_t)part * v.RG * NJ;
    for (int e = t; e < 16 * 16; e += 256) {
      const int r = row0 + (e >> 4), j = by * 16 + (e & 15);
      if (r < v.RG) {
        const acc_t* src = D + (size_t)r * dstride + j;
        acc_t sum = 0;
#pragma unroll 4
        for (int k = tlo; k < thi; ++k) sum += src[(size_t)k * NJ];
        out[(size_t)r * NJ + j] = sum;
      }
    }
    return;
  }
  const int r0 = bx * 16, j0 = by * 16;
  if constexpr (SPLIT) {
    for (int e = t; e < 16 * 16; e += 256) {
      const int row = r0 + (e >> 4), col = j0 + (e & 15);
      double sum = 0.0;
      if (row < 2 * v.RZ + v.RG) {
        // groups gluon-a, gluon-b, ghost-a, ghost-b: ghost-b rows follow ghost-a
        const int grow = row < 2 * v.RZ ? row : row + v.RG;
        const double* src = reinterpret_cast<const double*>(Dp) + (size_t)grow * dstride + col;
#pragma unroll 4
        for (int k = tlo; k < thi; ++k) sum += src[(size_t)k * NJ];
      }
      reinterpret_cast<double*>(v.Eq)[((size_t)part * v.Rbp + row) * NJ + col] = sum;
    }
    return;
  }
  // this thread's output element (ri, cj) of the tile, and for gluon rows
  // the k-side partial sums of the same target, requested before the product
  // so that their loads overlap the operand loads
  const int ri = t >> 4, cj = t & 15;
  const int orow = r0 + ri, ocol = j0 + cj;
  acc_t ds_ = 0;
  if (orow < 2 * v.RZ) {  // groups a, b are contiguous
    const acc_t* src = Dp + (size_t)orow * dstride + ocol;
#pragma unroll 4
    for (int k = tlo; k < thi; ++k) ds_ += src[(size_t)k * NJ];
  }
  // this wave's MFMA steps (4 radial nodes each): the Qp / 4 steps split
  // evenly over the kCS parts x 4 waves
  const int nsteps = Qp / 4, wpart = part * 4 + wave;
  const int sbeg = wpart * nsteps / (4 * kCS), send = (wpart + 1) * nsteps / (4 * kCS);
  const int qbeg = 4 * sbeg, qper = 4 * (send - sbeg);
  const int i = lane & 15, kk = lane >> 4;
  const acc_t* A = reinterpret_cast<const acc_t*>(v.Bm) + (size_t)(r0 + i) * Qp + kk;
  const size_t kstride = (size_t)v.Rbp * Qp;  // angular slices of B
  __shared__ acc_t part_[4][4][64];
  if constexpr (MIX) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    const float* B = v.Ttab32 + (size_t)kk * NJ + j0 + i;
#pragma unroll 8
    for (int q = qbeg; q < qbeg + qper; q += 4) {
      float a = A[q];
      for (int k = 1; k < v.KS; ++k) a += A[k * kstride + q];
      const float b = B[(size_t)q * NJ];
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) part_[wave][r][lane] = acc[r];
  } else {
    typedef double d4 __attribute__((ext_vector_type(4)));
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    const double* B = v.Ttab + (size_t)kk * NJ + j0 + i;
#pragma unroll 8
    for (int q = qbeg; q < qbeg + qper; q += 4) {
      double a = A[q];
      for (int k = 1; k < v.KS; ++k) a += A[k * kstride + q];
      const double b = B[(size_t)q * NJ];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) part_[wave][r][lane] = acc[r];
  }
  __syncthreads();
  {
    // one output element per thread.  Result layouts:
    // v_mfma_f64_16x16x4f64, lane l, register r: D[l/16 + 4 r][l % 16];
    // v_mfma_f32_16x16x4f32, lane l, register r: D[4 (l/16) + r][l % 16]
    const int l = MIX ? (ri >> 2) * 16 + cj : (ri & 3) * 16 + cj;
    const int rg = MIX ? (ri & 3) : (ri >> 2);
    acc_t sum = ((part_[0][rg][l] + part_[1][rg][l]) + part_[2][rg][l]) + part_[3][rg][l];
    if (orow < 2 * v.RZ) sum += ds_;  // gluon rows: the k-side sums of the same target
    reinterpret_cast<acc_t*>(v.Eq)[((size_t)part * v.Rbp + orow) * NJ + ocol] = sum;
  }
}

template <bool MIX, bool SPLIT = false>
__global__ __launch_bounds__(256) void contract_kernel(Views v) {
  contract_body<MIX, SPLIT>(v, blockIdx.x, blockIdx.y, blockIdx.z);
}


// --------------------------------------------------------------------------
// F_r and S_r for one row (Sec. 3: z(x_i) and g(x_i) with MOM subtraction),
// by one wave: lane k takes the partial tiles k, k + 64, ... of the row and of
// its subtraction row (compensated sums of the (sum, error) pairs), then a
// fixed-order wave reduction.
__device__ __forceinline__ void row_residual_wave(const Views& v, const Phys& ph, int r, double* F,
                                                  double* S, int lane, double* F2 = nullptr,
                                                  double* S2 = nullptr) {
  const bool gl = r < v.n_z;
  const int rr = gl ? r : v.RZ + (r - v.n_z);          // row in xrow / Pip
  const int sub = gl ? v.RZ - 1 : v.RZ + v.RG - 1;      // subtraction row
  const int nt = v.nqt * v.KS;
  const double* __restrict__ px = v.Pip + (size_t)2 * rr * nt;
  const double* __restrict__ ps = v.Pip + (size_t)2 * sub * nt;
  const double* __restrict__ ax_ = v.Absp + (size_t)rr * nt;
  const double* __restrict__ as_ = v.Absp + (size_t)sub * nt;
  double xs = 0.0, xc = 0.0, ss = 0.0, sc = 0.0, ax = 0.0, as = 0.0;
  for (int k = lane; k < nt; k += 64) {
    two_sum_add(xs, xc, px[2 * k]);
    xc += px[2 * k + 1];
    two_sum_add(ss, sc, ps[2 * k]);
    sc += ps[2 * k + 1];
    ax += ax_[k];
    as += as_[k];
  }
  wave_sum2(xs, xc);
  wave_sum2(ss, sc);
  ax = wave_sum(ax);
  as = wave_sum(as);
  if (lane == 0) {
    const double d = exp(-v.lnX[r]);
    const double par = gl ? ph.z_lambda_inv : ph.g0_inv;
    const double f = d - par - (xs + xc) + (ss + sc);
    const double sc_ = fabs(d) + fabs(par) + ax + as;
    F[r] = f;
    if (S) S[r] = sc_;
    if (F2) F2[r] = f;   // second copies for a caller's vectors
    if (S2) S2[r] = sc_;
  }
}

// one wave per row
__global__ __launch_bounds__(256) void residual_rows_kernel(Views v, Phys ph, double* F, double* S) {
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r < v.n) row_residual_wave(v, ph, r, F, S, threadIdx.x & 63);
}

// J row r = one block.  MIX: Eq and Dgh hold FP32 sums.
template <typename T>
__device__ __forceinline__ double sum_parts(const T* p, size_t stride) {
  double s_ = (double)p[0];
#pragma unroll
  for (int q = 1; q < kCS; ++q) s_ += (double)p[q * stride];
  return s_;
}

template <bool MIX>
__device__ __forceinline__ void assemble_body(const Views& v, const Phys& ph, int r, double* __restrict__ J,
                                              double* F, double* S, double* F2 = nullptr, double* S2 = nullptr) {
  using acc_t = typename std::conditional<MIX, float, double>::type;
  const acc_t* __restrict__ Eq = reinterpret_cast<const acc_t*>(v.Eq);
  const acc_t* __restrict__ Dgh = reinterpret_cast<const acc_t*>(v.Dgh);
  const size_t es = (size_t)v.Rbp * v.NJ, gs = (size_t)v.RG * v.NJ;  // part strides
  const int t = threadIdx.x;
  const int NJ = v.NJ, n = v.n;
  // the row's residual by the last wave, before its matrix entries (for
  // n <= 192 it has none): its loads then overlap those of the entries
  if (F && t >= 192) row_residual_wave(v, ph, r, F, S, t - 192, F2, S2);
  const bool gl = r < v.n_z;
  const int i = gl ? r : r - v.n_z;
  const double d = exp(-v.lnX[r]);
  const double* Tx = v.Text + (size_t)r * NJ;
  double* Jr = J + (size_t)r * n;
  double amax = 0.0;
  if (gl) {
    const int sub = v.RZ - 1;
    const acc_t* Ea = Eq;
    const acc_t* Eb = Eq + (size_t)v.RZ * NJ;
    for (int c = t; c < n; c += 256) {
      double val;
      if (c < v.n_z) {
        val = -d * Tx[c] - sum_parts(Ea + (size_t)i * NJ + c, es) + sum_parts(Ea + (size_t)sub * NJ + c, es);
      } else {
        const int j = c - v.n_z;
        val = -sum_parts(Eb + (size_t)i * NJ + j, es) + sum_parts(Eb + (size_t)sub * NJ + j, es);
      }
      Jr[c] = val;
      amax = fmax(amax, fabs(val));
    }
  } else {
    const int sub = v.RG - 1;
    const acc_t* Eb = Eq + (size_t)2 * v.RZ * NJ;
    for (int c = t; c < n; c += 256) {
      double val;
      if (c < v.n_z) {
        val = -sum_parts(Dgh + (size_t)i * NJ + c, gs) + sum_parts(Dgh + (size_t)sub * NJ + c, gs);
      } else {
        const int j = c - v.n_z;
        val = -d * Tx[j] - sum_parts(Eb + (size_t)i * NJ + j, es) + sum_parts(Eb + (size_t)sub * NJ + j, es);
      }
      Jr[c] = val;
      amax = fmax(amax, fabs(val));
    }
  }
  if (v.rowmax) {
    // the row's largest |entry|: the scale of the LU's relative pivot test
    __shared__ double red[4];
    amax = wave_max(amax);
    if ((t & 63) == 0) red[t >> 6] = amax;
    __syncthreads();
    if (t == 0) v.rowmax[r] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  }
}

template <bool MIX>
__global__ __launch_bounds__(256) void assemble_kernel(Views v, Phys ph, double* __restrict__ J,
                                                       double* F, double* S, double* F2, double* S2) {
  assemble_body<MIX>(v, ph, blockIdx.x, J, F, S, F2, S2);
}

// --------------------------------------------------------------------------
// max_r |F_r| / S_r, ||F||_2, ||d||_inf and ||F / S||_2 (one block).
__device__ __forceinline__ void norms_body(int n, const double* F, const double* S, const double* d,
                                           double* out) {
  const int t = threadIdx.x;
  double m = 0.0, s2 = 0.0, dm = 0.0, q2 = 0.0;
  bool bad = false;
  for (int r = t; r < n; r += 256) {
    const double f = F[r];
    const double sc = S ? S[r] : 0.0;
    const double qs = sc > 0.0 ? f / sc : f;
    const double q = fabs(qs);
    if (!(q == q) || isinf(q)) bad = true;
    m = fmax(m, q);
    s2 = fma(f, f, s2);
    q2 = fma(qs, qs, q2);
    if (d) dm = fmax(dm, fabs(d[r]));
  }
  __shared__ double sm[256], ss[256], sd[256], sq[256];
  __shared__ int sbad;
  if (t == 0) sbad = 0;
  __syncthreads();
  if (bad) sbad = 1;
  sm[t] = m; ss[t] = s2; sd[t] = dm; sq[t] = q2;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) {
      sm[t] = fmax(sm[t], sm[t + o]);
      ss[t] += ss[t + o];
      sd[t] = fmax(sd[t], sd[t + o]);
      sq[t] += sq[t + o];
    }
    __syncthreads();
  }
  if (t == 0) {
    const double nan = __longlong_as_double(0x7ff8000000000000LL);
    out[0] = sbad ? nan : sm[0];  // max_r |F_r| / S_r (convergence test)
    out[1] = sqrt(ss[0]);         // ||F||_2
    out[2] = sd[0];               // ||d||_inf
    out[3] = sbad ? nan : sqrt(sq[0]);  // ||F / S||_2 (line-search merit)
  }
}

__global__ __launch_bounds__(256) void norms_kernel(int n, const double* F, const double* S,
                                                   const double* d, double* out) {
  norms_body(n, F, S, d, out);
}

// The dressings and the running coupling at arbitrary momenta u (Sec. 2):
// ln Z(u), ln G(u) from the Chebyshev series (Sec. 3, c_0/2 convention) plus
// the IR power laws below eps2 and the UV logarithms above lambda2, and
// alpha(u) = alpha(mu^2) G(u)^2 Z(u).  One thread per point; outputs nullable.
__global__ __launch_bounds__(256) void coupling_kernel(Views v, Phys ph, double alpha_mu,
                                                       const double* __restrict__ c,
                                                       const double* __restrict__ u, int m,
                                                       double* __restrict__ alpha, double* __restrict__ lnZo,
                                                       double* __restrict__ lnGo) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double lu = log(u[i]);
  const double s = fmin(fmax((lu - ph.L0) * ph.invL1, -1.0), 1.0);
  const double s2 = s + s;
  double z = 0.5 * c[0], g = 0.5 * c[v.n_z];
  double Tp = 1.0, Tc = s;
  const int nmax = v.n_z > v.n_g ? v.n_z : v.n_g;
  for (int j = 1; j < nmax; ++j) {
    if (j < v.n_z) z = fma(c[j], Tc, z);
    if (j < v.n_g) g = fma(c[v.n_z + j], Tc, g);
    const double Tn = fma(s2, Tc, -Tp);
    Tp = Tc;
    Tc = Tn;
  }
  if (lu < ph.ln_eps2) {
    z += 2.0 * ph.kappa * (lu - ph.ln_eps2);
    g += -ph.kappa * (lu - ph.ln_eps2);
  } else if (lu > ph.ln_lam2) {
    const double L = log(fma(ph.omega, lu - ph.ln_lam2, 1.0));
    z += ph.gamma * L;
    g += ph.delta * L;
  }
  if (alpha) alpha[i] = alpha_mu * exp(2.0 * g + z);
  if (lnZo) lnZo[i] = z;
  if (lnGo) lnGo[i] = g;
}

// Vector-Jacobian product of the dressings at arbitrary momenta u > 0 with
// respect to the coefficients (Sec. 3 expansion; the IR power laws and UV
// logarithms outside [eps2, lambda2] do not depend on them, so
// d ln Z(u)/d a_j = d ln G(u)/d b_j = Tilde-T_j(s(u)) with s clamped to
// [-1, 1]):  grad[j] = sum_i wZ_i Tilde-T_j(s(u_i)) for j < n_z and
// grad[n_z + j] = sum_i wG_i Tilde-T_j(s(u_i)) for j < n_g.  One block per
// output entry; each thread sums its points in order, then a fixed tree over
// the block.
__global__ __launch_bounds__(256) void dressing_vjp_kernel(Views v, Phys ph, const double* __restrict__ u, int m,
                                                           const double* __restrict__ wZ,
                                                           const double* __restrict__ wG,
                                                           double* __restrict__ grad) {
  __shared__ double red[256];
  const int k = blockIdx.x;
  const bool isz = k < v.n_z;
  const int j = isz ? k : k - v.n_z;
  const double* __restrict__ w = isz ? wZ : wG;
  double acc = 0.0;
  if (w) {
    for (int i = threadIdx.x; i < m; i += 256) {
      const double s = fmin(fmax((log(u[i]) - ph.L0) * ph.invL1, -1.0), 1.0);
      const double s2 = s + s;
      double Tp = 1.0, Tc = s;  // T_0, T_1
      for (int q = 1; q < j; ++q) {
        const double Tn = fma(s2, Tc, -Tp);
        Tp = Tc;
        Tc = Tn;
      }
      const double T = j == 0 ? 0.5 : Tc;
      acc = fma(w[i], T, acc);
    }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) grad[k] = red[0];
}

// Central differences of the residual (the paper's own Jacobian, Sec. 4.2):
// the shifted coefficients c + sgn h e_j with h = h_rel max(1, |c_j|), h kept
// in hbuf[0] for the column kernel; then column j of J from the two residuals.
__global__ void fd_shift_kernel(int n, const double* __restrict__ c, int j, double h_rel, double sgn,
                                double* __restrict__ cs, double* __restrict__ hbuf) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double cj = c[j];
  const double h = h_rel * fmax(1.0, fabs(cj));
  cs[i] = i == j ? cj + sgn * h : c[i];
  if (i == 0) hbuf[0] = h;
}

__global__ void fd_column_kernel(int n, const double* __restrict__ Fp, const double* __restrict__ Fm,
                                 const double* __restrict__ hbuf, int j, double* __restrict__ J) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) J[(size_t)i * n + j] = (Fp[i] - Fm[i]) / (2.0 * hbuf[0]);
}

__global__ void axpy_kernel(int n, const double* c, double rho, const double* d, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = fma(-rho, d[i], c[i]);
}

// --------------------------------------------------------------------------
// FP64 LU with partial pivoting and the triangular solves, one workgroup of
// four waves; the padded matrix [A | b] lives in LDS (or in global memory
// when it does not fit).  The matrix is padded to np = 16 ceil(n/16) with an
// identity block (padded rows have zeros in the real columns, so they are
// never chosen as a pivot and the real factors are unchanged) and the
// right-hand side is column np.  Rows never move: a map from row position to
// physical row (rmap) carries the interchanges, and every access to a row
// position goes through it.  Blocked right-looking elimination, panel width 16:
//   panel    wave 0 holds the rows of the panel (MR per lane) in registers
//            and factors it column by column: pivot = largest |a| (wave
//            maximum by DPP; among equal maxima the first register row), the
//            pivot row's entries read across lanes, multipliers
//            a * (1 / pivot), rank-1 update.  Interchanges only change the
//            logical positions of the register rows; at the end the panel's
//            columns go back to their physical rows and rmap is updated;
//   U12      U12 = L11^{-1} A12, one column per thread;
//   update   A22 -= L21 U12 on v_mfma_f64_16x16x4f64 (16 x 16 tiles, two at
//            a time per wave); the right-hand-side column on the vector ALUs.
// The right-hand-side column ends as L^{-1} P b; wave 0 back-substitutes by
// blocks of 16 rows with the reciprocal pivots kept from the panels.  The
// transposed solve (A^T x = b) runs U^T, L^T and P^T with wave 0.
constexpr int LU_NB = 16;

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo0 = (int)(b & 0xffffffffLL), hi0 = (int)(b >> 32);
  // lanes of rows outside ROW_MASK keep their own value
  const int lo = __builtin_amdgcn_update_dpp(lo0, lo0, CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(hi0, hi0, CTRL, ROW_MASK, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Maximum of v over the wave, returned uniformly (v >= 0, or -1 for none):
// rotations within rows of 16 lanes, then row broadcasts; lane 63 ends with
// the maximum of all four rows.
__device__ __forceinline__ double wave_max_nonneg(double v) {
  v = fmax(v, dpp_d<0x121, 0xf>(v));  // row_ror:1
  v = fmax(v, dpp_d<0x122, 0xf>(v));  // row_ror:2
  v = fmax(v, dpp_d<0x124, 0xf>(v));  // row_ror:4
  v = fmax(v, dpp_d<0x128, 0xf>(v));  // row_ror:8
  v = fmax(v, dpp_d<0x142, 0xa>(v));  // row_bcast:15 into rows 1 and 3
  v = fmax(v, dpp_d<0x143, 0xc>(v));  // row_bcast:31 into rows 2 and 3
  return readlane_d(v, 63);
}

// Lanes of one wave exchanging values through memory: the stores before this
// point are visible to every lane's loads after it (release + acquire at
// wavefront scope; also a compiler barrier, so no load is hoisted above a
// store made by another lane).
__device__ __forceinline__ void wave_memory_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Shared state of one factorisation.
struct LUShared {
  int spiv[256];     // spiv[k]: position interchanged with k at step k
  int rmap[256];     // row position -> physical row
  double dinv[256];  // 1 / U[k][k]
  double wsv[256];   // staging of the transposed solve
  int sing;
};

// The panel's columns run as a pipeline.  Column O has three stages:
//   A(O)  pivot: wave maximum of |P[.][O]| over the rows not yet used, the
//         first register row holding it, its reciprocal;
//   B(O)  interchange (logical positions only), multipliers of column O and
//         the update of column O + 1;
//   C(O)  the update of columns O + 2 .. 15.
// Order: A(O), C(O - 1), B(O).  A(O) needs column O only (final after B(O-1)
// and C(O-2)), so its DPP reduction and C(O - 1)'s lane reads and FMAs are
// independent and interleave; the serial chain per column is A and B.  Every
// element receives the same FMAs in the same order as in a column-by-column
// elimination.  The code is branch-free: a singular column only raises sing
// (the caller then abandons the factorisation).  lpos[m] is the logical
// position of register row m (-1: no row); lane O of the wave collects
// column O's interchange and reciprocal pivot.
struct LUPivot {
  int lp;      // lane holding the pivot row
  int mp;      // its register row
  int p;       // its logical position
  double inv;  // 1 / pivot
};

// Maximum of an unsigned key over the wave, returned uniformly (the same
// rotations and row broadcasts as wave_max_nonneg, on 32-bit lanes).  Lanes
// outside ROW_MASK read 0, the identity of the maximum, so the DPP move
// folds into the maximum (one instruction per step).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ unsigned dpp_u(unsigned v) {
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xf, false);
}

__device__ __forceinline__ unsigned umax_(unsigned a, unsigned b) { return a > b ? a : b; }

__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  v = umax_(v, dpp_u<0x121, 0xf>(v));  // row_ror:1
  v = umax_(v, dpp_u<0x122, 0xf>(v));  // row_ror:2
  v = umax_(v, dpp_u<0x124, 0xf>(v));  // row_ror:4
  v = umax_(v, dpp_u<0x128, 0xf>(v));  // row_ror:8
  v = umax_(v, dpp_u<0x142, 0xa>(v));  // row_bcast:15 into rows 1 and 3
  v = umax_(v, dpp_u<0x143, 0xc>(v));  // row_bcast:31 into rows 2 and 3
  return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// 1 / x for any x: the significand's reciprocal (x = m 2^e, |m| in [1/2, 1),
// where the refined hardware estimate is within 1 ulp) scaled by 2^-e
// exactly; zero, infinite or NaN x give a non-finite result.  No branch.
__device__ __forceinline__ double recip_any(double x) {
  const double m = __builtin_amdgcn_frexp_mant(x);
  const int e = __builtin_amdgcn_frexp_exp(x);
  return __builtin_amdgcn_ldexp(recip(m), -e);
}

// Pivot of column O: the largest |P[m][O]| over the rows not yet used; among
// equal maxima the first register row (lowest m), then the lowest lane.  The
// wave reduction runs on the leading 32 bits of each lane's largest |value|
// (for non-negative doubles their order is the order of the values, up to
// ties): when one lane holds the largest key it holds the maximum; when
// several do, the exact maximum among them is reduced in FP64 and the first
// register row holding it found by ballots (that lane's own first row holding
// its maximum is the same row).  Every lane forms the reciprocal of its own
// candidate while the reduction runs; the pivot lane's is read afterwards.
template <int MR, int O>
__device__ __forceinline__ LUPivot lu_pivot(const double (&P)[MR][LU_NB], const int (&lpos)[MR], int kc,
                                            int& sing) {
  double cand[MR];
  double lmax = -1.0, pl = P[0][O];
  int lm = 0, ll = lpos[0];
  if constexpr (MR <= 2) {
#pragma unroll
    for (int m = 0; m < MR; ++m) {
      cand[m] = lpos[m] >= kc ? fabs(P[m][O]) : -1.0;  // rows not yet used as pivots
      if (cand[m] > lmax) {
        lmax = cand[m];
        lm = m;
      }
    }
#pragma unroll
    for (int m = 1; m < MR; ++m)
      if (lm == m) {
        pl = P[m][O];
        ll = lpos[m];
      }
  } else {
    // more register rows: the row's value and position are picked up in the
    // same scan (an index into P taken after it makes the compiler move P to
    // scratch memory)
#pragma unroll
    for (int m = 0; m < MR; ++m) {
      cand[m] = lpos[m] >= kc ? fabs(P[m][O]) : -1.0;
      const bool gt = cand[m] > lmax;
      lmax = gt ? cand[m] : lmax;
      lm = gt ? m : lm;
      pl = gt ? P[m][O] : pl;
      ll = gt ? lpos[m] : ll;
    }
  }
  const double il = recip_any(pl);
  const unsigned key = lmax >= 0.0 ? (unsigned)((unsigned long long)__double_as_longlong(lmax) >> 32) : 0u;
  const unsigned kmax = wave_max_u32(key);
  // the reciprocal is materialised after the reduction and before the branch
  // below (not sunk past it), so that its latency overlaps the reduction
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("" ::"v"(il));
  const unsigned long long tied = __ballot(key == kmax);
  int lp = (int)__builtin_ctzll(tied);
  if (__popcll(tied) != 1) {
    const double gmax = wave_max_nonneg(key == kmax ? lmax : -1.0);
    int f = -1;
#pragma unroll
    for (int m = 0; m < MR; ++m) {
      const unsigned long long mk = __ballot(cand[m] == gmax);
      if (f < 0 && mk) f = (int)__builtin_ctzll(mk);
    }
    lp = f & 63;  // no maximum only when singular: any lane
  }
  LUPivot r;
  r.lp = lp;
  r.mp = MR == 1 ? 0 : __builtin_amdgcn_readlane(lm, lp);
  r.p = __builtin_amdgcn_readlane(ll, lp);
  r.inv = readlane_d(il, lp);
  // a zero, infinite or NaN pivot leaves a non-finite or zero reciprocal
  sing |= (!(fabs(r.inv) < __builtin_huge_val()) || r.inv == 0.0) ? 1 : 0;
  return r;
}

// Entries FROM .. LU_NB - 1 of the pivot row, read across lanes from the lane
// that holds it.  The register row mp is uniform, so the choice is one scalar
// branch around lane reads of one row (readlane cannot be speculated, so the
// branch stays), not a select per entry.
template <int MR, int FROM>
__device__ __forceinline__ void lu_prow(const double (&P)[MR][LU_NB], const LUPivot& pv, double (&rp)[LU_NB]) {
  if constexpr (MR == 1) {
#pragma unroll
    for (int cc = FROM; cc < LU_NB; ++cc) rp[cc] = readlane_d(P[0][cc], pv.lp);
  } else {
#pragma unroll
    for (int m = 0; m < MR; ++m) {
      if (pv.mp == m) {
#pragma unroll
        for (int cc = FROM; cc < LU_NB; ++cc) rp[cc] = readlane_d(P[m][cc], pv.lp);
      }
    }
  }
}

// B(O): interchange, multipliers of column O, update of column O + 1; the
// pivot row's entries O + 1 .. 15 are read here (rp) for C(O) as well.
template <int MR, int O>
__device__ __forceinline__ void lu_stage_b(double (&P)[MR][LU_NB], int (&lpos)[MR], const LUPivot& pv, int kc,
                                           int lane, int& mypiv, double& myinv, double (&rp)[LU_NB]) {
  mypiv = lane == O ? pv.p : mypiv;
  myinv = lane == O ? pv.inv : myinv;
#pragma unroll
  for (int m = 0; m < MR; ++m) {
    const int q = lpos[m];
    lpos[m] = q == kc ? pv.p : (q == pv.p ? kc : q);
  }
  if constexpr (O + 1 < LU_NB) lu_prow<MR, O + 1>(P, pv, rp);
#pragma unroll
  for (int m = 0; m < MR; ++m) {
    const bool below = lpos[m] > kc;
    const double l = below ? P[m][O] * pv.inv : 0.0;
    if (below) P[m][O] = l;
    if constexpr (O + 1 < LU_NB) P[m][O + 1] = fma(-l, rp[O + 1], P[m][O + 1]);
  }
}

// C(O): the update of columns O + 2 .. 15 with the multipliers B(O) stored
// and the pivot row's entries rp that B(O) read.
template <int MR, int O>
__device__ __forceinline__ void lu_stage_c(double (&P)[MR][LU_NB], const int (&lpos)[MR],
                                           const double (&rp)[LU_NB], int kc) {
  if constexpr (O + 2 < LU_NB) {
#pragma unroll
    for (int m = 0; m < MR; ++m) {
      const double l = lpos[m] > kc ? P[m][O] : 0.0;
#pragma unroll
      for (int cc = O + 2; cc < LU_NB; ++cc) P[m][cc] = fma(-l, rp[cc], P[m][cc]);
    }
  }
}

// rp: the pivot-row entries of column O - 1, read by B(O - 1).
template <int MR, int O>
__device__ __forceinline__ void lu_pipe(double (&P)[MR][LU_NB], int (&lpos)[MR], int k0, int lane, int& sing,
                                        int& mypiv, double& myinv, const double (&rp)[LU_NB]) {
  const LUPivot pv = lu_pivot<MR, O>(P, lpos, k0 + O, sing);
  if constexpr (O > 0) lu_stage_c<MR, O - 1>(P, lpos, rp, k0 + O - 1);
  double rp_next[LU_NB];
  lu_stage_b<MR, O>(P, lpos, pv, k0 + O, lane, mypiv, myinv, rp_next);
  if constexpr (O + 1 < LU_NB) lu_pipe<MR, O + 1>(P, lpos, k0, lane, sing, mypiv, myinv, rp_next);
}

// Loads the rows of the panel at k0 (positions k0 ..) into wave 0's registers
// and factors it; lpos/phys return each register row's new position and its
// physical row (the caller publishes them to the row map).  FIRST: the panel
// at 0, read straight from the n x n input (identity padding, identity row
// map) instead of from M.  R <= MR register rows per lane hold the np - k0
// rows left (R 64 >= np - k0); register rows R .. MR-1 return no row.
template <int MR, bool FIRST, int R = MR>
__device__ __forceinline__ void lu_factor_panel(double* M, int ld, int np, const int* rmap, int k0, int lane,
                                                LUShared& sh, int (&lpos)[MR], int (&phys)[MR], int& sg,
                                                const double* __restrict__ Ain = nullptr, int n = 0) {
  static_assert(R >= 1 && R <= MR, "register rows");
  double P[R][LU_NB];
  int lp_[R];
#pragma unroll
  for (int m = 0; m < R; ++m) {
    const int pos = k0 + lane + 64 * m;
    lp_[m] = pos < np ? pos : -1;  // -1: no row (never a candidate, never updated)
    // loads from clamped (in-bounds) addresses, then selects: no load waits
    // inside a divergent branch
    if (FIRST) {
      phys[m] = pos < np ? pos : 0;
      const int pc = pos < n ? pos : n - 1;
#pragma unroll
      for (int c = 0; c < LU_NB; ++c) {
        const double a = Ain[(size_t)pc * n + (c < n ? c : n - 1)];
        P[m][c] = pos < n && c < n ? a : (pos == c ? 1.0 : 0.0);
      }
    } else {
      const int ph = rmap[pos < np ? pos : np - 1];
      phys[m] = pos < np ? ph : 0;
#pragma unroll
      for (int c = 0; c < LU_NB; ++c) {
        const double a = M[(size_t)ph * ld + k0 + c];
        P[m][c] = pos < np ? a : 0.0;
      }
    }
  }
#pragma unroll
  for (int m = R; m < MR; ++m) {
    lpos[m] = -1;
    phys[m] = 0;
  }
  sg = 0;
  int mypiv = 0;
  double myinv = 0.0;
  const double none[LU_NB] = {};  // no column before the first
  lu_pipe<R, 0>(P, lp_, k0, lane, sg, mypiv, myinv, none);
  // the factored panel back to its physical rows; interchanges and
  // reciprocal pivots from lanes 0 .. 15
#pragma unroll
  for (int m = 0; m < R; ++m) {
    lpos[m] = lp_[m];
    if (lp_[m] >= 0) {
      double* Mr = M + (size_t)phys[m] * ld + k0;
#pragma unroll
      for (int cc = 0; cc < LU_NB; ++cc) Mr[cc] = P[m][cc];
    }
  }
  if (lane < LU_NB) {
    sh.spiv[k0 + lane] = mypiv;
    sh.dinv[k0 + lane] = myinv;
  }
}

// A later panel (at k0 > 0) with as many register rows per lane as its rows
// need: fewer rows, fewer selects and updates per column.
template <int MR>
__device__ __forceinline__ void lu_factor_next(double* M, int ld, int np, const int* rmap, int k0, int lane,
                                               LUShared& sh, int (&lpos)[MR], int (&phys)[MR], int& sg) {
  const int rows = np - k0;
  if constexpr (MR >= 4) {
    if (rows > 192) { lu_factor_panel<MR, false, 4>(M, ld, np, rmap, k0, lane, sh, lpos, phys, sg); return; }
  }
  if constexpr (MR >= 3) {
    if (rows > 128) { lu_factor_panel<MR, false, 3>(M, ld, np, rmap, k0, lane, sh, lpos, phys, sg); return; }
  }
  if constexpr (MR >= 2) {
    if (rows > 64) { lu_factor_panel<MR, false, 2>(M, ld, np, rmap, k0, lane, sh, lpos, phys, sg); return; }
  }
  lu_factor_panel<MR, false, 1>(M, ld, np, rmap, k0, lane, sh, lpos, phys, sg);
}

// U12 of the right-hand-side column (column col): the panel's row c in lanes
// c, c + 16, ... (lanes of equal c compute the same values; lanes 1 .. 15
// store).  Step cc reads u[cc] across lanes and the rows below it subtract
// L11[c][cc] u[cc]: the same FMAs in the same order as a column-oriented
// forward substitution, branch-free (rows not below cc keep their value).
__device__ __forceinline__ void lu_u12_rhs(double* M, int ld, int k0, const int* rmap, int col, int lane) {
  const int c = lane & 15;
  const int prow = rmap[k0 + c];
  double u = M[(size_t)prow * ld + col];
  double L[LU_NB - 1];
#pragma unroll
  for (int cc = 0; cc < LU_NB - 1; ++cc) L[cc] = M[(size_t)prow * ld + k0 + cc];
#pragma unroll
  for (int cc = 0; cc < LU_NB - 1; ++cc) {
    const double x = readlane_d(u, cc);
    const double upd = fma(-L[cc], x, u);
    u = c > cc ? upd : u;
  }
  if (lane >= 1 && lane < LU_NB) M[(size_t)prow * ld + col] = u;
}

// The same for a full 16-column block with the whole wave: quad q (lanes
// 4q .. 4q+3) takes column jc + q, lane g of the quad rows g, g+4, g+8, g+12.
// Step cc broadcasts u[cc] from its lane inside the quad (DPP quad
// permutation) and the lanes below subtract L11[c][cc] u[cc]; every element
// receives the same FMAs in the same order as in the one-lane-per-column form.
__device__ __forceinline__ double quad_bcast(double v, int o) {
  switch (o) {
    case 0: return dpp_d<0x00, 0xf>(v);  // quad_perm [0,0,0,0]
    case 1: return dpp_d<0x55, 0xf>(v);  // [1,1,1,1]
    case 2: return dpp_d<0xAA, 0xf>(v);  // [2,2,2,2]
    default: return dpp_d<0xFF, 0xf>(v);  // [3,3,3,3]
  }
}

__device__ __forceinline__ void lu_u12_block16(double* M, int ld, int k0, const int* rmap, int jc, int lane) {
  const int g = lane & 3;
  const int j = jc + (lane >> 2);
  int prow[4];
  double u[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    prow[k] = rmap[k0 + g + 4 * k];
    u[k] = M[(size_t)prow[k] * ld + j];
  }
  // branch-free: a lane whose row is not below cc computes the update and
  // keeps its value (every address is in bounds), so no load waits inside a
  // divergent branch on the chain
#pragma unroll
  for (int cc = 0; cc < LU_NB - 1; ++cc) {
    const double x = quad_bcast(u[cc >> 2], cc & 3);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (4 * k + 3 <= cc) continue;  // rows 4k .. 4k+3 all final
      const double upd = fma(-M[(size_t)prow[k] * ld + k0 + cc], x, u[k]);
      u[k] = 4 * k > cc || g + 4 * k > cc ? upd : u[k];
    }
  }
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (g + 4 * k >= 1) M[(size_t)prow[k] * ld + j] = u[k];
}

// A22[:, jc .. jc+15] -= L21 U12[:, jc .. jc+15] for tile rows below j0, by
// one wave on the matrix cores, two tile rows per step: operands
// A[i][k] = -L21 in lane i + 16 k, B[k][j] = U12 in lane j + 16 k, the tile as
// accumulator (lane l, register r: row l/16 + 4 r, column l % 16).
// Tile rows ti = t0, t0 + tstep, ... (each step takes ti and ti + 1).
__device__ __forceinline__ void lu_trail_rows(double* M, int ld, const int* rmap, int k0, int j0, int nt, int jc,
                                              const int (&brow)[4], int lane, int t0, int tstep) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  const int li = lane & 15, lk = lane >> 4;
  if (t0 >= nt) return;
  double bv[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) bv[s] = M[(size_t)brow[s] * ld + jc + li];
  // A lone last tile row (ti + 1 == nt) runs the pair with its own rows in
  // the second slot and does not store that slot: no load sits in a branch.
  for (int ti = t0; ti < nt; ti += tstep) {
    const bool two = ti + 1 < nt;
    const int i0 = j0 + 16 * ti, i1 = two ? i0 + 16 : i0;
    const int arow0 = rmap[i0 + li], arow1 = rmap[i1 + li];
    int crow0[4], crow1[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      crow0[r] = rmap[i0 + lk + 4 * r];
      crow1[r] = rmap[i1 + lk + 4 * r];
    }
    d4 acc0, acc1;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      acc0[r] = M[(size_t)crow0[r] * ld + jc + li];
      acc1[r] = M[(size_t)crow1[r] * ld + jc + li];
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const double a0 = -M[(size_t)arow0 * ld + k0 + 4 * s + lk];
      const double a1 = -M[(size_t)arow1 * ld + k0 + 4 * s + lk];
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bv[s], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bv[s], acc1, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) M[(size_t)crow0[r] * ld + jc + li] = acc0[r];
    if (two) {
#pragma unroll
      for (int r = 0; r < 4; ++r) M[(size_t)crow1[r] * ld + jc + li] = acc1[r];
    }
  }
}

// Right-hand side, rows below j0: b2 -= L21 y1 (one wave, lanes over rows).
__device__ __forceinline__ void lu_trail_rhs(double* M, int ld, const int* rmap, int k0, int j0, int np,
                                             const int (&pr)[LU_NB], int lane) {
  const int col = np;
  double y1[LU_NB];
#pragma unroll
  for (int c = 0; c < LU_NB; ++c) y1[c] = M[(size_t)pr[c] * ld + col];
  for (int i = j0 + lane; i < np; i += 64) {
    const int pi_ = rmap[i];
    const double* Li = M + (size_t)pi_ * ld + k0;
    double s_ = M[(size_t)pi_ * ld + col];
#pragma unroll
    for (int c = 0; c < LU_NB; ++c) s_ = fma(-Li[c], y1[c], s_);
    M[(size_t)pi_ * ld + col] = s_;
  }
}

// With cout != nullptr the Newton update cout = cin - rho x is written beside x.
template <bool IN_LDS, int MR>
__device__ __forceinline__ void lu_body(int n, const double* __restrict__ Ain, const double* __restrict__ b,
                                        double* x, double* __restrict__ Aglob, int* piv, int trans, int* flag,
                                        double* lds, const double* __restrict__ cin = nullptr, double rho = 0.0,
                                        double* __restrict__ cout = nullptr,
                                        const double* __restrict__ rowmax = nullptr) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  // the wave index through readfirstlane: the compiler then knows it (and
  // every branch and loop bound taken from it) to be uniform across the wave
  const int t = threadIdx.x, lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int np = (n + LU_NB - 1) / LU_NB * LU_NB;
  const int ld = np + 1;  // odd: column accesses spread over the banks
  const int ncol = np + 1;
  double* M = IN_LDS ? lds : Aglob;
  __shared__ LUShared sh;
  const int* __restrict__ rmap = sh.rmap;
  // Wave 0 factors the first panel straight from the input while waves 1-3
  // load the other columns of [A | b] (padded with an identity block): wave w
  // takes rows w - 1, w + 2, ..., lane l columns 16 + l, 80 + l, ...; sixteen
  // rows per batch.
  //
  // Panel k+1 is factored while panel k's update of the other columns runs
  // (one panel of lookahead).  Per panel: U12 of the next panel's columns
  // (and of one more block per other wave), the next panel's tile column
  // (the four waves, tile rows dealt in pairs), then wave 0 factors the next
  // panel while waves 1-3 finish U12 and update the remaining column blocks
  // and the right-hand side.  The next panel's interchanges reach the row
  // map only after the barrier, once nobody reads the old one.
  int lpos[MR], phys[MR];
  if (wave == 0) {
    for (int r = lane; r < np; r += 64) sh.rmap[r] = r;
    if (lane == 0) sh.sing = 0;
    int sg;
    lu_factor_panel<MR, true>(M, ld, np, rmap, 0, lane, sh, lpos, phys, sg, Ain, n);
    if (sg && lane == 0) sh.sing = 1;
    if (!sg) {
      wave_memory_sync();
#pragma unroll
      for (int m = 0; m < MR; ++m)
        if (lpos[m] >= 0) sh.rmap[lpos[m]] = phys[m];
    }
  } else {
    // MR column chunks of 64 right of the panel cover np - 16 < 64 MR columns;
    // RB rows per batch keep 64 values in flight per lane
    // (row r0 + 3 rr is uniform; every load reads a clamped, in-bounds
    // address and a select drops what lies outside the matrix, so that the
    // loads of a batch issue back to back).  Two register rows: 48 rows per
    // wave and batch, so that the three waves cover n <= 128 in one batch,
    // one memory round trip (96 values in flight per lane).
    constexpr int CU = MR, RB = MR == 2 ? 48 : 64 / MR;
    for (int r0 = wave - 1; r0 < np; r0 += 3 * RB) {
      double v_[RB][CU];
#pragma unroll
      for (int rr = 0; rr < RB; ++rr) {
        const int r = r0 + 3 * rr;
        const double* __restrict__ Ar = Ain + (size_t)(r < n ? r : n - 1) * n;
#pragma unroll
        for (int u = 0; u < CU; ++u) {
          const int c = LU_NB + lane + 64 * u;
          const double a = Ar[c < n ? c : n - 1];
          v_[rr][u] = r < n && c < n ? a : (r == c ? 1.0 : 0.0);
        }
      }
#pragma unroll
      for (int rr = 0; rr < RB; ++rr) {
        const int r = r0 + 3 * rr;
#pragma unroll
        for (int u = 0; u < CU; ++u) {
          const int c = LU_NB + lane + 64 * u;
          if (r < np && c < np) M[(size_t)r * ld + c] = v_[rr][u];
        }
      }
    }
    for (int r = t - 64; r < np; r += 192) M[(size_t)r * ld + np] = (r < n && !trans) ? b[r] : 0.0;
  }
  __syncthreads();
  for (int k0 = 0; k0 < np && !sh.sing; k0 += LU_NB) {
    const int j0 = k0 + LU_NB;
    int pr[LU_NB];  // physical rows of the panel's positions
#pragma unroll
    for (int c = 0; c < LU_NB; ++c) pr[c] = rmap[k0 + c];
    if (j0 >= np) {  // after the last panel only U12 of the right-hand side is left
      if (wave == 0) lu_u12_rhs(M, ld, k0, rmap, np, lane);
      __syncthreads();
      break;
    }
    const int nblk = (np - j0) / 16;
    int brow[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) brow[s] = pr[4 * s + (lane >> 4)];
    // U12 of block 0 (the next panel's columns) by wave 0; waves 1-3 take
    // the first of their blocks (column blocks bk = wave, wave + 3, ...;
    // bk == nblk is the right-hand side) here and the rest after the barrier
    if (wave == 0) {
      lu_u12_block16(M, ld, k0, rmap, j0, lane);
    } else if (wave <= nblk) {
      if (wave < nblk) lu_u12_block16(M, ld, k0, rmap, j0 + 16 * wave, lane);
      else lu_u12_rhs(M, ld, k0, rmap, np, lane);
    }
    __syncthreads();
    // block 0's tile column by all four waves (tile rows dealt in pairs)
    lu_trail_rows(M, ld, rmap, k0, j0, nblk, j0, brow, lane, 2 * wave, 8);
    __syncthreads();
    if (wave == 0) {
      int sg;
      lu_factor_next<MR>(M, ld, np, rmap, j0, lane, sh, lpos, phys, sg);
      if (sg && lane == 0) sh.sing = 1;
    } else {
      // a block's U12 rows, written by lanes 0-15, are read by every lane of
      // the same wave in its update: the fence orders them
      for (int bk = wave; bk <= nblk; bk += 3) {
        if (bk < nblk) {
          if (bk > 3) {
            lu_u12_block16(M, ld, k0, rmap, j0 + 16 * bk, lane);
            wave_memory_sync();
          }
          lu_trail_rows(M, ld, rmap, k0, j0, nblk, j0 + 16 * bk, brow, lane, 0, 2);
        } else {
          if (bk > 3) {
            lu_u12_rhs(M, ld, k0, rmap, np, lane);
            wave_memory_sync();
          }
          lu_trail_rhs(M, ld, rmap, k0, j0, np, pr, lane);
        }
      }
    }
    __syncthreads();
    if (wave == 0 && !sh.sing) {
#pragma unroll
      for (int m = 0; m < MR; ++m)
        if (lpos[m] >= 0) sh.rmap[lpos[m]] = phys[m];
    }
    __syncthreads();
  }
  if (rowmax && !sh.sing) {
    // relative test: a pivot at or below n eps times the largest entry of
    // its row in the input counts as singular (rows never move, so the
    // pivot at position k belongs to input row rmap[k])
    const double tol = n * 2.220446049250313e-16;
    for (int k = t; k < n; k += 256)
      if (!(fabs(sh.dinv[k]) * tol * rowmax[sh.rmap[k]] < 1.0)) sh.sing = 1;
    __syncthreads();
  }
  if (sh.sing) {
    if (t == 0) flag[0] = 4;
    return;
  }
  for (int i = t; i < n; i += 256) piv[i] = sh.spiv[i];
  if (wave != 0) return;
  // wave 0: w distributed as row positions lane + 64 m
  double w[MR];
  int prow[MR];  // physical row of position lane + 64 m
#pragma unroll
  for (int m = 0; m < MR; ++m) {
    const int r = lane + 64 * m;
    prow[m] = r < np ? rmap[r] : 0;
  }
  if (!trans) {
#pragma unroll
    for (int m = 0; m < MR; ++m) {
      const int r = lane + 64 * m;
      w[m] = r < np ? M[(size_t)prow[m] * ld + np] : 0.0;  // = L^{-1} P b
    }
    // U x = y by blocks of 16 rows from the bottom.  The diagonal block's 16
    // lanes (register row mi, lanes lb ..) work on one value wb: step cc reads
    // x = wb[lb + cc] / U[cc][cc] across lanes and subtracts U[:, cc] x from
    // every lane (lanes already solved keep their x in xv); then the rows
    // above subtract the block's columns times x.  Software-pipelined: a
    // block's U columns for the rows above are requested before its chain and
    // the next block's diagonal rows and reciprocal pivots during it; every
    // register row is updated branch-free (prow is a valid row for every lane,
    // rows at or below the block keep their value), so no load waits in a
    // branch.
    double ub[LU_NB], dv[LU_NB];
    auto load_diag = [&](int i0) {
      const int mi = i0 >> 6;
      int pb = prow[0];
#pragma unroll
      for (int m = 1; m < MR; ++m)
        if (mi == m) pb = prow[m];
#pragma unroll
      for (int cc = 0; cc < LU_NB; ++cc) {
        ub[cc] = M[(size_t)pb * ld + i0 + cc];
        dv[cc] = sh.dinv[i0 + cc];
      }
    };
    load_diag(np - LU_NB);
    for (int i1 = np; i1 > 0; i1 -= LU_NB) {
      const int i0 = i1 - LU_NB;
      const int mi = i0 >> 6, lb = i0 & 63;
      double ur[MR][LU_NB];
#pragma unroll
      for (int m = 0; m < MR; ++m) {
#pragma unroll
        for (int cc = 0; cc < LU_NB; ++cc) ur[m][cc] = M[(size_t)prow[m] * ld + i0 + cc];
      }
      double wb = w[0];
#pragma unroll
      for (int m = 1; m < MR; ++m)
        if (mi == m) wb = w[m];
      double xb[LU_NB];
      double xv = 0.0;
#pragma unroll
      for (int cc = LU_NB - 1; cc >= 0; --cc) {
        xb[cc] = readlane_d(wb, lb + cc) * dv[cc];
        xv = lane == lb + cc ? xb[cc] : xv;
        wb = fma(-ub[cc], xb[cc], wb);
      }
      load_diag(i0 > 0 ? i0 - LU_NB : 0);
#pragma unroll
      for (int m = 0; m < MR; ++m) {
        const int r = lane + 64 * m;
        double s_ = w[m];
#pragma unroll
        for (int cc = 0; cc < LU_NB; ++cc) s_ = fma(-ur[m][cc], xb[cc], s_);
        w[m] = r < i0 ? s_ : (r < i1 ? xv : w[m]);
      }
    }
  } else {
#pragma unroll
    for (int m = 0; m < MR; ++m) {
      const int r = lane + 64 * m;
      w[m] = r < n ? b[r] : 0.0;
    }
    for (int i = 0; i < np; ++i) {  // U^T y = b
      const int li = i & 63, mi = i >> 6;
      const double* Ui = M + (size_t)rmap[i] * ld;
      double sel = w[0];
#pragma unroll
      for (int m = 1; m < MR; ++m) if (mi == m) sel = w[m];
      const double yi = readlane_d(sel, li) * sh.dinv[i];
#pragma unroll
      for (int m = 0; m < MR; ++m) {
        const int r = lane + 64 * m;
        if (r == i) w[m] = yi;
        else if (r > i && r < np) w[m] = fma(-Ui[r], yi, w[m]);
      }
    }
    for (int i = np - 1; i >= 0; --i) {  // L^T z = y (unit diagonal)
      const int li = i & 63, mi = i >> 6;
      const double* Li = M + (size_t)rmap[i] * ld;
      double sel = w[0];
#pragma unroll
      for (int m = 1; m < MR; ++m) if (mi == m) sel = w[m];
      const double zi = readlane_d(sel, li);
#pragma unroll
      for (int m = 0; m < MR; ++m) {
        const int r = lane + 64 * m;
        if (r < i) w[m] = fma(-Li[r], zi, w[m]);
      }
    }
    // x = P^T z: undo the interchanges in reverse order (staged in LDS)
#pragma unroll
    for (int m = 0; m < MR; ++m) {
      const int r = lane + 64 * m;
      if (r < np) sh.wsv[r] = w[m];
    }
    wave_memory_sync();
    if (lane == 0)
      for (int k = np - 1; k >= 0; --k) {
        const int pk = sh.spiv[k];
        const double tmp = sh.wsv[k]; sh.wsv[k] = sh.wsv[pk]; sh.wsv[pk] = tmp;
      }
    wave_memory_sync();
#pragma unroll
    for (int m = 0; m < MR; ++m) {
      const int r = lane + 64 * m;
      if (r < np) w[m] = sh.wsv[r];
    }
  }
#pragma unroll
  for (int m = 0; m < MR; ++m) {
    const int r = lane + 64 * m;
    if (r < n) {
      x[r] = w[m];
      if (cout) cout[r] = fma(-rho, w[m], cin[r]);
    }
  }
  if (lane == 0) flag[0] = 0;
}

// Dynamic LDS of the factorisation kernels besides the matrix.
constexpr int kLUStaticBytes = (int)sizeof(LUShared) + 256;

template <bool IN_LDS, int MR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void lu_solve_kernel(
    int n, const double* __restrict__ Ain, const double* __restrict__ b, double* x, double* __restrict__ Aglob,
    int* piv, int trans, int* flag, const double* __restrict__ cin, double rho, double* __restrict__ cout,
    const double* __restrict__ rowmax) {
  extern __shared__ double lds[];
  lu_body<IN_LDS, MR>(n, Ain, b, x, Aglob, piv, trans, flag, lds, cin, rho, cout, rowmax);
}

// rowmax[r] = max_k |A[r][k]|, one wave per row.
__global__ __launch_bounds__(256) void row_absmax_kernel(int n, const double* __restrict__ A,
                                                         double* __restrict__ rowmax) {
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (r >= n) return;
  double m = 0.0;
  for (int k = lane; k < n; k += 64) m = fmax(m, fabs(A[(size_t)r * n + k]));
  m = wave_max(m);
  if (lane == 0) rowmax[r] = m;
}

// --------------------------------------------------------------------------
// Vector-Jacobian products.  With row weights rw = -u_i on the collocation
// rows and rw = sum_i u_i (over the same kind) on the subtraction rows,
//   u^T F = sum_rows rw Pi + sum_i u_i (direct_i - parameter)
// so the weighted point kernel plus the contraction give u^T dF/dc, and the
// weighted alpha sums give u^T dF/d alpha.
__global__ __launch_bounds__(256) void row_weights_kernel(Views v, const double* __restrict__ u) {
  __shared__ double red[2][256];
  const int t = threadIdx.x;
  double sz = 0.0, sg = 0.0;
  for (int i = t; i < v.n_z; i += 256) sz += u[i];
  for (int i = t; i < v.n_g; i += 256) sg += u[v.n_z + i];
  red[0][t] = sz;
  red[1][t] = sg;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) { red[0][t] += red[0][t + o]; red[1][t] += red[1][t + o]; }
    __syncthreads();
  }
  for (int i = t; i < v.n_z; i += 256) v.rw[i] = -u[i];
  for (int i = t; i < v.n_g; i += 256) v.rw[v.RZ + i] = -u[v.n_z + i];
  if (t == 0) {
    v.rw[v.RZ - 1] = red[0][0];
    v.rw[v.RZ + v.RG - 1] = red[1][0];
  }
}

// u^T dF/dc (optional) and u^T dF/dtheta, theta = (alpha_mu, g0_inv, z_lambda_inv).
__global__ __launch_bounds__(256) void vjp_reduce_kernel(Views v, const double* __restrict__ u,
                                                         double* uJ, double* uth) {
  const int t = threadIdx.x;
  const int NJ = v.NJ;
  if (uJ) {
    for (int c = t; c < v.n; c += 256) {
      double s_ = 0.0;
      if (c < v.n_z) {
        const int j = c;
        const size_t es = (size_t)v.Rbp * NJ, gs = (size_t)v.RG * NJ;
        for (int r = 0; r < v.RZ; ++r) s_ += sum_parts(v.Eq + (size_t)r * NJ + j, es);
        for (int r = 0; r < v.RG; ++r) s_ += sum_parts(v.Dgh + (size_t)r * NJ + j, gs);
        for (int i = 0; i < v.n_z; ++i) s_ -= u[i] * exp(-v.lnX[i]) * v.Text[(size_t)i * NJ + j];
      } else {
        const int j = c - v.n_z;
        const size_t es = (size_t)v.Rbp * NJ;
        for (int r = 0; r < v.RZ; ++r) s_ += sum_parts(v.Eq + (size_t)(v.RZ + r) * NJ + j, es);
        for (int r = 0; r < v.RG; ++r) s_ += sum_parts(v.Eq + (size_t)(2 * v.RZ + r) * NJ + j, es);
        for (int i = 0; i < v.n_g; ++i)
          s_ -= u[v.n_z + i] * exp(-v.lnX[v.n_z + i]) * v.Text[(size_t)(v.n_z + i) * NJ + j];
      }
      uJ[c] = s_;
    }
  }
  if (uth && t == 0) {
    const int nt = v.nqt * v.KS;
    double s_ = 0.0, c_ = 0.0;
    for (int r = 0; r < v.RZ + v.RG; ++r)
      for (int k = 0; k < nt; ++k) {
        two_sum_add(s_, c_, v.Pip[2 * ((size_t)r * nt + k)]);
        c_ += v.Pip[2 * ((size_t)r * nt + k) + 1];
      }
    double sz = 0.0, sg = 0.0;
    for (int i = 0; i < v.n_z; ++i) sz += u[i];
    for (int i = 0; i < v.n_g; ++i) sg += u[v.n_z + i];
    uth[0] = s_ + c_;   // d/d alpha: through the self-energies only
    uth[1] = -sg;       // dF^G/d g0_inv = -1
    uth[2] = -sz;       // dF^Z/d z_lambda_inv = -1
  }
}


// --------------------------------------------------------------------------
// Batched family: the same bodies, one launch per stage for every problem of
// the family.  A problem's views and constants come from its descriptor;
// problems whose mask entry is zero are skipped (converged, or not in the
// current line-search round).

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__global__ __launch_bounds__(256) void batch_dressing_kernel(const SolveDesc* __restrict__ d,
                                                             const int* __restrict__ mask,
                                                             const double* __restrict__ cpk, int which,
                                                             int* counter) {
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *counter = 0;  // queue of the next point launch
  const int b = blockIdx.y;
  if (!mask[b]) return;
  const SolveDesc& sd = d[b];
  dressing_body(sd.v, sd.ph, which ? sd.v.ct : cpk + sd.coff, blockIdx.x * 256, gridDim.x * 256, blockIdx.x == 0);
}

// One queue item: (problem, kind, row, first tile); the item takes tpi
// consecutive partial tiles of the row (each writes its own partial sums).
// The body is instantiated for every order up to NJMAX.
template <int MODE, int NJMAX>
__device__ __forceinline__ void batch_item(const SolveDesc* __restrict__ d, const int* __restrict__ mask,
                                           const int4 w, int tpi, double* smem) {
  const int b = uniform(w.x);
  if (!mask[b]) return;
  const SolveDesc& sd = d[b];
  const int kind = uniform(w.y), row = uniform(w.z), t0 = uniform(w.w);
  const int nj = uniform(sd.v.NJ);
  const int nt = sd.v.nqt * sd.v.KS;
  for (int tile = t0; tile < t0 + tpi && tile < nt; ++tile) {
    if (tile > t0) __syncthreads();  // the LDS is reused
#define DSE_BATCH_CASE(N)                                                                   \
  if constexpr (N <= NJMAX) {                                                               \
    if (nj == N) {                                                                          \
      if (kind == GLUON) point_body<GLUON, N, MODE, false, true>(sd.v, sd.ph, row, tile, smem); \
      else point_body<GHOST, N, MODE, false, true>(sd.v, sd.ph, row, tile, smem);           \
    }                                                                                       \
  }
    DSE_BATCH_CASE(16)
    DSE_BATCH_CASE(32)
    DSE_BATCH_CASE(48)
    DSE_BATCH_CASE(64)
    DSE_BATCH_CASE(96)
    DSE_BATCH_CASE(128)
#undef DSE_BATCH_CASE
  }
}

// Queue of (problem, kind, row, tile) items, largest first: one workgroup per
// item in queue order, or persistent workgroups taking items through the
// counter.
template <int MODE, int NJMAX>
__global__ __launch_bounds__(256) void batch_point_kernel(const SolveDesc* __restrict__ d,
                                                          const int* __restrict__ mask,
                                                          const int4* __restrict__ items, int n_items,
                                                          int* counter, int persistent, int tpi) {
  __shared__ double smem[point_smem<NJMAX, true>()];
  __shared__ int s_item;
  int it = blockIdx.x;
  for (;;) {
    if (persistent) {
      if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
      __syncthreads();
      it = uniform(s_item);
    }
    if (it >= n_items) break;
    batch_item<MODE, NJMAX>(d, mask, items[it], tpi, smem);
    if (!persistent) break;
    __syncthreads();  // the next item reuses s_item and the LDS
  }
}

__global__ __launch_bounds__(256) void batch_contract_kernel(const SolveDesc* __restrict__ d,
                                                             const int* __restrict__ mask, int nct) {
  const int b = blockIdx.z;
  if (!mask[b]) return;
  const Views& v = d[b].v;
  const int bx = blockIdx.x, part = blockIdx.y / nct, by = blockIdx.y - part * nct;
  if (bx >= v.Rbp / 16 + (v.RG + 15) / 16 || by >= v.NJ / 16) return;
  contract_body<false>(v, bx, by, part);
}

__global__ __launch_bounds__(256) void batch_assemble_kernel(const SolveDesc* __restrict__ d,
                                                             const int* __restrict__ mask) {
  const int b = blockIdx.y;
  if (!mask[b]) return;
  const SolveDesc& sd = d[b];
  if ((int)blockIdx.x >= sd.v.n) return;
  assemble_body<false>(sd.v, sd.ph, blockIdx.x, sd.v.J, sd.v.F, sd.v.S);
}

// The family's Newton-matrix assembly in one cooperative launch of resident
// workgroups: the dressings of every problem, the point items through the
// queue, the contraction tiles, the assembly rows.  Each stage is dealt over
// the grid and separated from the next by a grid-wide barrier (the
// cooperative launch guarantees that every workgroup is resident, so the
// barrier completes); the units of every stage are those of the staged
// launches, so the results are bit-identical to them.
template <int NJMAX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void batch_fused_kernel(
    BatchArgs a, const double* __restrict__ cpk, const int4* __restrict__ items, int n_items, int tpi,
    int* counter, int which) {
  namespace cg = cooperative_groups;
  cg::grid_group grid = cg::this_grid();
  __shared__ double smem[point_smem<NJMAX, true>()];
  __shared__ int s_item;
  const SolveDesc* __restrict__ d = a.desc;
  const int nb = gridDim.x;
  // dressings: (problem, block) units
  const int ndu = a.count * a.max_dress_blocks;
  for (int u = blockIdx.x; u < ndu; u += nb) {
    const int b = u / a.max_dress_blocks, blk = u - b * a.max_dress_blocks;
    if (a.mask[b]) {
      const SolveDesc& sd = d[b];
      dressing_body(sd.v, sd.ph, which ? sd.v.ct : cpk + sd.coff, blk * 256, a.max_dress_blocks * 256, blk == 0);
    }
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;
  grid.sync();
  // point items through the queue
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = uniform(s_item);
    if (it >= n_items) break;
    batch_item<MODE_JAC, NJMAX>(d, a.mask, items[it], tpi, smem);
    __syncthreads();
  }
  grid.sync();
  // contraction tiles: (problem, row block, part, column block) units
  const int nct = a.max_nj / 16, per = a.max_rbt * kCS * nct;
  for (int u = blockIdx.x; u < a.count * per; u += nb) {
    const int b = u / per;
    int r = u - b * per;
    const int bx = r / (kCS * nct);
    r -= bx * (kCS * nct);
    const int part = r / nct, by = r - part * nct;
    if (a.mask[b]) {
      const Views& v = d[b].v;
      if (bx < v.Rbp / 16 + (v.RG + 15) / 16 && by < v.NJ / 16) contract_body<false>(v, bx, by, part);
    }
    __syncthreads();
  }
  grid.sync();
  // assembly rows
  for (int u = blockIdx.x; u < a.count * a.max_n; u += nb) {
    const int b = u / a.max_n, row = u - b * a.max_n;
    if (a.mask[b]) {
      const SolveDesc& sd = d[b];
      if (row < sd.v.n) assemble_body<false>(sd.v, sd.ph, row, sd.v.J, sd.v.F, sd.v.S);
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void batch_residual_rows_kernel(const SolveDesc* __restrict__ d,
                                                                  const int* __restrict__ mask, int which) {
  const int b = blockIdx.y;
  if (!mask[b]) return;
  const SolveDesc& sd = d[b];
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r < sd.v.n)
    row_residual_wave(sd.v, sd.ph, r, which ? sd.v.Ft : sd.v.F, which ? sd.v.St : sd.v.S, threadIdx.x & 63);
}

// which: 0 F and S; 1 the trial's Ft and St with ||delta||_inf; 2 F and S
// with ||delta||_inf (a trial point assembled in Jacobian mode)
__global__ __launch_bounds__(256) void batch_norms_kernel(const SolveDesc* __restrict__ d,
                                                          const int* __restrict__ mask, int which,
                                                          double* out) {
  const int b = blockIdx.x;
  if (!mask[b]) return;
  const Views& v = d[b].v;
  norms_body(v.n, which == 1 ? v.Ft : v.F, which == 1 ? v.St : v.S, which ? v.dlt : nullptr, out + 4 * b);
}

// One workgroup per system: J delta = F.
template <bool IN_LDS, int MR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void batch_lu_kernel(
    const SolveDesc* __restrict__ d,
                                                       const int* __restrict__ mask, int* flags) {
  extern __shared__ double lds[];
  const int b = blockIdx.x;
  if (!mask[b]) return;
  const Views& v = d[b].v;
  lu_body<IN_LDS, MR>(v.n, v.J, v.F, v.dlt, v.LU, v.piv, 0, flags + b, lds, nullptr, 0.0, nullptr, v.rowmax);
}

__global__ __launch_bounds__(256) void batch_axpy_kernel(const SolveDesc* __restrict__ d,
                                                         const int* __restrict__ mask,
                                                         const double* __restrict__ cpk,
                                                         const double* __restrict__ rho) {
  const int b = blockIdx.y;
  if (!mask[b]) return;
  const SolveDesc& sd = d[b];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < sd.v.n) sd.v.ct[i] = cpk[sd.coff + i] - rho[b] * sd.v.dlt[i];
}

// mask 1: the trial was evaluated in residual mode (Ft, St become F, S);
// mask 2: in Jacobian mode (F and S hold it already)
__global__ __launch_bounds__(256) void batch_accept_kernel(const SolveDesc* __restrict__ d,
                                                           const int* __restrict__ mask, double* cpk) {
  const int b = blockIdx.y;
  if (!mask[b]) return;
  const SolveDesc& sd = d[b];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < sd.v.n) {
    cpk[sd.coff + i] = sd.v.ct[i];
    if (mask[b] == 1) {
      sd.v.F[i] = sd.v.Ft[i];
      sd.v.S[i] = sd.v.St[i];
    }
  }
}

__global__ __launch_bounds__(256) void batch_pack_kernel(const SolveDesc* __restrict__ d,
                                                         const int* __restrict__ mask, double* Jpk,
                                                         double* Fpk) {
  const int b = blockIdx.y;
  if (!mask[b]) return;
  const SolveDesc& sd = d[b];
  const int n = sd.v.n, r = blockIdx.x;
  if (r >= n) return;
  for (int c = threadIdx.x; c < n; c += 256) Jpk[sd.joff + (size_t)r * n + c] = sd.v.J[(size_t)r * n + c];
  if (Fpk && threadIdx.x == 0) Fpk[sd.coff + r] = sd.v.F[r];
}

// --------------------------------------------------------------------------
// launchers

hipError_t launch_dressing(const Views& v, const Phys& ph, const double* c, hipStream_t st) {
  hipLaunchKernelGGL(dressing_kernel, dim3((v.Qp + v.n + 255) / 256), dim3(256), 0, st, v, ph, c);
  if (v.split) {
    const int cnt = (v.RZ + v.RG) * v.Qp;
    hipLaunchKernelGGL(dressing_split_kernel, dim3((cnt + 255) / 256), dim3(256), 0, st, v, ph, c);
  }
  return hipGetLastError();
}

template <int NJ, int MODE, bool MIX, bool SPLIT = false>
static hipError_t points_nj(const Views& v, const Phys& ph, hipStream_t st, hipEvent_t* ev) {
  if (ev) (void)hipEventRecord(ev[0], st);
  hipLaunchKernelGGL((point_kernel<GLUON, NJ, MODE, MIX, SPLIT>), dim3(v.RZ * v.nqt * v.KS), dim3(256), 0, st, v,
                     ph);
  if (ev) (void)hipEventRecord(ev[1], st);
  hipLaunchKernelGGL((point_kernel<GHOST, NJ, MODE, MIX, SPLIT>), dim3(v.RG * v.nqt * v.KS), dim3(256), 0, st, v,
                     ph);
  if (ev) (void)hipEventRecord(ev[2], st);
  return hipGetLastError();
}

template <int MODE, bool MIX, bool SPLIT = false>
static hipError_t points_dispatch(const Views& v, const Phys& ph, hipStream_t st, hipEvent_t* ev) {
  switch (v.NJ) {
    case 16: return points_nj<16, MODE, MIX, SPLIT>(v, ph, st, ev);
    case 32: return points_nj<32, MODE, MIX, SPLIT>(v, ph, st, ev);
    case 48: return points_nj<48, MODE, MIX, SPLIT>(v, ph, st, ev);
    case 64: return points_nj<64, MODE, MIX, SPLIT>(v, ph, st, ev);
    case 96: return points_nj<96, MODE, MIX, SPLIT>(v, ph, st, ev);
    case 128: return points_nj<128, MODE, MIX, SPLIT>(v, ph, st, ev);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_points(const Views& v, const Phys& ph, int mode, bool mix, hipStream_t st, hipEvent_t* ev) {
  if (v.split) {
    // the host admits only FP64 residual and Jacobian modes on a split grid
    if (mode == MODE_RES) return points_dispatch<MODE_RES, false, true>(v, ph, st, ev);
    if (mode == MODE_JAC && !mix) return points_dispatch<MODE_JAC, false, true>(v, ph, st, ev);
    return hipErrorInvalidValue;
  }
  switch (mode) {
    case MODE_RES: return points_dispatch<MODE_RES, false>(v, ph, st, ev);
    case MODE_JAC:
      return mix ? points_dispatch<MODE_JAC, true>(v, ph, st, ev) : points_dispatch<MODE_JAC, false>(v, ph, st, ev);
    case MODE_VJP: return points_dispatch<MODE_VJP, false>(v, ph, st, ev);
    case MODE_VTH: return points_dispatch<MODE_VTH, false>(v, ph, st, ev);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_contract(const Views& v, bool mix, hipStream_t st) {
  const int gh_blocks = (v.RG + 15) / 16;
  const dim3 grid(v.Rbp / 16 + gh_blocks, v.NJ / 16, kCS);
  if (v.split) {
    if (mix) return hipErrorInvalidValue;
    hipLaunchKernelGGL((contract_kernel<false, true>), grid, dim3(256), 0, st, v);
  } else if (mix) {
    hipLaunchKernelGGL(contract_kernel<true>, grid, dim3(256), 0, st, v);
  } else {
    hipLaunchKernelGGL(contract_kernel<false>, grid, dim3(256), 0, st, v);
  }
  return hipGetLastError();
}

hipError_t launch_row_weights(const Views& v, const double* u, hipStream_t st) {
  hipLaunchKernelGGL(row_weights_kernel, dim3(1), dim3(256), 0, st, v, u);
  return hipGetLastError();
}

hipError_t launch_vjp_reduce(const Views& v, const double* u, double* uJ, double* uth, hipStream_t st) {
  hipLaunchKernelGGL(vjp_reduce_kernel, dim3(1), dim3(256), 0, st, v, u, uJ, uth);
  return hipGetLastError();
}

hipError_t launch_assemble(const Views& v, const Phys& ph, double* J, double* F, double* S, bool mix,
                           hipStream_t st, double* F2, double* S2) {
  // the row maxima belong to the workspace's Newton matrix: a Jacobian
  // written elsewhere leaves them alone
  Views w = v;
  if (J != v.J) w.rowmax = nullptr;
  if (mix)
    hipLaunchKernelGGL(assemble_kernel<true>, dim3(v.n), dim3(256), 0, st, w, ph, J, F, S, F2, S2);
  else
    hipLaunchKernelGGL(assemble_kernel<false>, dim3(v.n), dim3(256), 0, st, w, ph, J, F, S, F2, S2);
  return hipGetLastError();
}

hipError_t launch_residual_rows(const Views& v, const Phys& ph, double* F, double* S, hipStream_t st) {
  hipLaunchKernelGGL(residual_rows_kernel, dim3((v.n + 3) / 4), dim3(256), 0, st, v, ph, F, S);
  return hipGetLastError();
}

hipError_t launch_norms(const Views& v, const double* F, const double* S, const double* d, double* out,
                        hipStream_t st) {
  hipLaunchKernelGGL(norms_kernel, dim3(1), dim3(256), 0, st, v.n, F, S, d, out);
  return hipGetLastError();
}

hipError_t launch_coupling(const Views& v, const Phys& ph, double alpha_mu, const double* c, const double* u, int m,
                           double* alpha, double* lnZ, double* lnG, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(coupling_kernel, dim3((m + 255) / 256), dim3(256), 0, st, v, ph, alpha_mu, c, u, m, alpha, lnZ,
                     lnG);
  return hipGetLastError();
}

hipError_t launch_dressing_vjp(const Views& v, const Phys& ph, const double* u, int m, const double* wZ,
                               const double* wG, double* grad, hipStream_t st) {
  hipLaunchKernelGGL(dressing_vjp_kernel, dim3(v.n), dim3(256), 0, st, v, ph, u, m, wZ, wG, grad);
  return hipGetLastError();
}

hipError_t launch_fd_shift(int n, const double* c, int j, double h_rel, double sgn, double* cs, double* hbuf,
                           hipStream_t st) {
  hipLaunchKernelGGL(fd_shift_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, c, j, h_rel, sgn, cs, hbuf);
  return hipGetLastError();
}

hipError_t launch_fd_column(int n, const double* Fp, const double* Fm, const double* hbuf, int j, double* J,
                            hipStream_t st) {
  hipLaunchKernelGGL(fd_column_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, Fp, Fm, hbuf, j, J);
  return hipGetLastError();
}

hipError_t launch_axpy(int n, const double* c, double rho, const double* d, double* out, hipStream_t st) {
  hipLaunchKernelGGL(axpy_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, c, rho, d, out);
  return hipGetLastError();
}

template <bool IN_LDS, int MR>
static void set_lu_lds(int bytes) {
  (void)hipFuncSetAttribute((const void*)lu_solve_kernel<IN_LDS, MR>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

template <bool IN_LDS, int MR>
static void set_batch_lu_lds(int bytes);

// LDS limits of the factorisation kernels (once per process, before any
// launch: not inside a stream capture).
static int g_max_lds = -1;
void lu_setup() {
  if (g_max_lds >= 0) return;
  int dev = 0, val = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&val, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    val = 64 * 1024;
  const int dyn = val - kLUStaticBytes;
  set_lu_lds<true, 2>(dyn);
  set_lu_lds<true, 4>(dyn);
  set_batch_lu_lds<true, 2>(dyn);
  set_batch_lu_lds<true, 4>(dyn);
  g_max_lds = val;
}

hipError_t launch_row_absmax(int n, const double* A, double* rowmax, hipStream_t st) {
  hipLaunchKernelGGL(row_absmax_kernel, dim3((n + 3) / 4), dim3(256), 0, st, n, A, rowmax);
  return hipGetLastError();
}

hipError_t launch_lu_solve(const Views& v, const double* A, const double* b, double* x, int trans,
                           hipStream_t st, const double* cin, double rho, double* cout, const double* rowmax) {
  const int n = v.n;
  const int np = (n + LU_NB - 1) / LU_NB * LU_NB;
  // factors of [A | b], padded, in dynamic LDS when they fit
  const size_t lds_bytes = (size_t)np * (np + 1) * sizeof(double);
  const size_t static_bytes = kLUStaticBytes;
  lu_setup();
  const int max_lds = g_max_lds;
  const bool fits = lds_bytes + static_bytes <= (size_t)max_lds;
  if (np <= 128) {
    if (fits)
      hipLaunchKernelGGL((lu_solve_kernel<true, 2>), dim3(1), dim3(256), lds_bytes, st, n, A, b, x, v.LU, v.piv,
                         trans, v.flag, cin, rho, cout, rowmax);
    else
      hipLaunchKernelGGL((lu_solve_kernel<false, 2>), dim3(1), dim3(256), 0, st, n, A, b, x, v.LU, v.piv, trans,
                         v.flag, cin, rho, cout, rowmax);
  } else {
    if (fits)
      hipLaunchKernelGGL((lu_solve_kernel<true, 4>), dim3(1), dim3(256), lds_bytes, st, n, A, b, x, v.LU, v.piv,
                         trans, v.flag, cin, rho, cout, rowmax);
    else
      hipLaunchKernelGGL((lu_solve_kernel<false, 4>), dim3(1), dim3(256), 0, st, n, A, b, x, v.LU, v.piv, trans,
                         v.flag, cin, rho, cout, rowmax);
  }
  return hipGetLastError();
}


// ---- batched family

hipError_t launch_batch_dressing(const BatchArgs& a, const double* cpk, int which, int* counter,
                                 hipStream_t st) {
  hipLaunchKernelGGL(batch_dressing_kernel, dim3(a.max_dress_blocks, a.count), dim3(256), 0, st, a.desc, a.mask, cpk,
                     which, counter);
  return hipGetLastError();
}

template <int MODE, int NJMAX>
static hipError_t batch_points_nj(const BatchArgs& a, const int4* items, int n_items, int grid, int tpi,
                                  int* counter, hipStream_t st) {
  const int blocks = grid > 0 ? grid : n_items;
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL((batch_point_kernel<MODE, NJMAX>), dim3(blocks), dim3(256), 0, st, a.desc, a.mask, items,
                     n_items, counter, grid > 0 ? 1 : 0, tpi);
  return hipGetLastError();
}

template <int MODE>
static hipError_t batch_points_mode(const BatchArgs& a, const int4* items, int n_items, int grid, int tpi,
                                    int* counter, hipStream_t st) {
  switch (a.max_nj) {
    case 16: return batch_points_nj<MODE, 16>(a, items, n_items, grid, tpi, counter, st);
    case 32: return batch_points_nj<MODE, 32>(a, items, n_items, grid, tpi, counter, st);
    case 48: return batch_points_nj<MODE, 48>(a, items, n_items, grid, tpi, counter, st);
    case 64: return batch_points_nj<MODE, 64>(a, items, n_items, grid, tpi, counter, st);
    case 96: return batch_points_nj<MODE, 96>(a, items, n_items, grid, tpi, counter, st);
    case 128: return batch_points_nj<MODE, 128>(a, items, n_items, grid, tpi, counter, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_batch_points(const BatchArgs& a, const int4* items, int n_items, int mode, int grid, int tpi,
                               int* counter, hipStream_t st) {
  if (tpi < 1) return hipErrorInvalidValue;
  switch (mode) {
    case MODE_RES: return batch_points_mode<MODE_RES>(a, items, n_items, grid, tpi, counter, st);
    case MODE_JAC: return batch_points_mode<MODE_JAC>(a, items, n_items, grid, tpi, counter, st);
    default: return hipErrorInvalidValue;
  }
}

template <int NJMAX>
static const void* fused_fn() {
  return reinterpret_cast<const void*>(&batch_fused_kernel<NJMAX>);
}

static const void* fused_kernel_for(int max_nj) {
  switch (max_nj) {
    case 16: return fused_fn<16>();
    case 32: return fused_fn<32>();
    case 48: return fused_fn<48>();
    case 64: return fused_fn<64>();
    case 96: return fused_fn<96>();
    case 128: return fused_fn<128>();
    default: return nullptr;
  }
}

int batch_fused_occupancy(int max_nj) {
  const void* f = fused_kernel_for(max_nj);
  int nb = 0;
  if (!f || hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, 256, 0) != hipSuccess) return 0;
  return nb;
}

hipError_t launch_batch_fused(const BatchArgs& a, const double* cpk, const int4* items, int n_items, int tpi,
                              int grid, int* counter, hipStream_t st, int which) {
  const void* f = fused_kernel_for(a.max_nj);
  if (!f || grid < 1 || tpi < 1) return hipErrorInvalidValue;
  BatchArgs aa = a;
  void* args[] = {&aa, (void*)&cpk, (void*)&items, &n_items, &tpi, &counter, &which};
  return hipLaunchCooperativeKernel(f, dim3(grid), dim3(256), args, 0, st);
}

template <int MODE, int NJMAX>
static int occ_nj() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)batch_point_kernel<MODE, NJMAX>, 256, 0) !=
      hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

int batch_points_occupancy(int mode, int max_nj) {
  const bool jac = mode == MODE_JAC;
  switch (max_nj) {
    case 16: return jac ? occ_nj<MODE_JAC, 16>() : occ_nj<MODE_RES, 16>();
    case 32: return jac ? occ_nj<MODE_JAC, 32>() : occ_nj<MODE_RES, 32>();
    case 48: return jac ? occ_nj<MODE_JAC, 48>() : occ_nj<MODE_RES, 48>();
    case 64: return jac ? occ_nj<MODE_JAC, 64>() : occ_nj<MODE_RES, 64>();
    case 96: return jac ? occ_nj<MODE_JAC, 96>() : occ_nj<MODE_RES, 96>();
    default: return jac ? occ_nj<MODE_JAC, 128>() : occ_nj<MODE_RES, 128>();
  }
}

hipError_t launch_batch_contract(const BatchArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(batch_contract_kernel, dim3(a.max_rbt, kCS * (a.max_nj / 16), a.count), dim3(256), 0, st,
                     a.desc, a.mask, a.max_nj / 16);
  return hipGetLastError();
}

hipError_t launch_batch_assemble(const BatchArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(batch_assemble_kernel, dim3(a.max_n, a.count), dim3(256), 0, st, a.desc, a.mask);
  return hipGetLastError();
}

hipError_t launch_batch_residual_rows(const BatchArgs& a, int which, hipStream_t st) {
  hipLaunchKernelGGL(batch_residual_rows_kernel, dim3((a.max_n + 3) / 4, a.count), dim3(256), 0, st, a.desc,
                     a.mask, which);
  return hipGetLastError();
}

hipError_t launch_batch_norms(const BatchArgs& a, int which, double* out, hipStream_t st) {
  hipLaunchKernelGGL(batch_norms_kernel, dim3(a.count), dim3(256), 0, st, a.desc, a.mask, which, out);
  return hipGetLastError();
}

template <bool IN_LDS, int MR>
static void set_batch_lu_lds(int bytes) {
  (void)hipFuncSetAttribute((const void*)batch_lu_kernel<IN_LDS, MR>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            bytes);
}

hipError_t launch_batch_lu(const BatchArgs& a, int* flags, hipStream_t st) {
  const int np = a.max_np;
  const size_t lds_bytes = (size_t)np * (np + 1) * sizeof(double);
  const size_t static_bytes = kLUStaticBytes;
  lu_setup();
  const int max_lds = g_max_lds;
  const bool fits = lds_bytes + static_bytes <= (size_t)max_lds;
  if (np <= 128) {
    if (fits)
      hipLaunchKernelGGL((batch_lu_kernel<true, 2>), dim3(a.count), dim3(256), lds_bytes, st, a.desc, a.mask, flags);
    else
      hipLaunchKernelGGL((batch_lu_kernel<false, 2>), dim3(a.count), dim3(256), 0, st, a.desc, a.mask, flags);
  } else {
    if (fits)
      hipLaunchKernelGGL((batch_lu_kernel<true, 4>), dim3(a.count), dim3(256), lds_bytes, st, a.desc, a.mask, flags);
    else
      hipLaunchKernelGGL((batch_lu_kernel<false, 4>), dim3(a.count), dim3(256), 0, st, a.desc, a.mask, flags);
  }
  return hipGetLastError();
}

hipError_t launch_batch_axpy(const BatchArgs& a, const double* cpk, const double* rho, hipStream_t st) {
  hipLaunchKernelGGL(batch_axpy_kernel, dim3((a.max_n + 255) / 256, a.count), dim3(256), 0, st, a.desc, a.mask,
                     cpk, rho);
  return hipGetLastError();
}

hipError_t launch_batch_accept(const BatchArgs& a, double* cpk, hipStream_t st) {
  hipLaunchKernelGGL(batch_accept_kernel, dim3((a.max_n + 255) / 256, a.count), dim3(256), 0, st, a.desc, a.mask,
                     cpk);
  return hipGetLastError();
}

hipError_t launch_batch_pack(const BatchArgs& a, double* Jpk, double* Fpk, hipStream_t st) {
  hipLaunchKernelGGL(batch_pack_kernel, dim3(a.max_n, a.count), dim3(256), 0, st, a.desc, a.mask, Jpk, Fpk);
  return hipGetLastError();
}

}  // namespace dse
