// dse_observables.hip -- quantities computed on converged dressings and the
// large quadrature rule they need:
//   * Gauss-Legendre rules of up to 2^24 nodes generated on the device
//     (Newton's method on P_n with the three-term recurrence, Sec. 5: the
//     node generation is what the paper parallelises for the Schwinger
//     function);
//   * the Schwinger function of the gluon propagator,
//     Delta(t) = (1/pi) int dp cos(t p) Z(p^2)/p^2 (Sec. 2.2), by the mapped
//     rule p = p_max ((1 + x)/2)^2;
//   * the renormalisation scale mu^2 with G^2(mu^2) Z(mu^2) = 1 (Sec. 2.1,
//     footnote).

#include <hip/hip_runtime.h>
#include <math.h>

#include "dse_impl.h"

namespace dse {

constexpr int kGLGroup = 16;  // Gauss-Legendre recurrence steps whose coefficients are loaded together

namespace {

// ---------------------------------------------------------------------------
// Gauss-Legendre rule.
//
// P_{k+1}(s) = alpha_k s P_k(s) - beta_k P_{k-1}(s) with beta_k = k/(k+1) and
// alpha_k = 1 + beta_k.  The beta_k come from a table, read by all lanes of a
// wave at once through the scalar cache (no per-lane copies); a step is
// v = beta s + s and q = beta P_{k-1} off the dependency chain (P_{k-1} is one
// step old) and one FMA P_{k+1} = v P_k - q on it; no division in the loop.
//
// One lane per positive root (roots come in pairs +-x): root k counted from
// +1.  Start: the five roots nearest +1 at theta = j_{0,k} / (n + 1/2), the
// zeros of J_0 scaled as the Mehler-Heine limit P_n(cos(z / n)) -> J_0(z)
// puts them (exact to double precision for large n, where Tricomi's estimate
// is off by up to 5e-13 at k = 1 and the edge roots would need two more
// Newton steps); the others at Tricomi's estimate
// (1 - (n-1)/(8 n^3)) cos(pi (4k-1)/(4n+2)).
// Newton steps x <- x - h, h = P_n/P_n', P_n' = n (x P_n - P_{n-1}) / (x^2 - 1),
// until the step taken is small enough to finish on it: at a root
// P_n''/P_n' = 2x/(1 - x^2) and P_n'''/P_n' = O(n^2/(1 - x^2)) (Legendre's
// equation), so the node after the step is off by about |x| h^2/(1 - x^2)
// and the first-order value P_n' - h P_n'' at the new node by a relative
// n^2 h^2; both must stay below the rounding level (|x| h^2 <= u (1 - x^2)/4
// and n^2 h^2 <= u, u = 2^-53).  The weight w = 2 / ((1 - x^2) P_n'^2) then
// takes that first-order derivative (P_n'' from Legendre's equation, h the
// step as rounded), so the last recurrence is also the last Newton step: at
// n = 2^17 every root is final after one recurrence.  A wave keeps
// iterating while any of its lanes has not finished.


// beta[k-1] = k/(k+1) for k = 1 .. n-1, then 2 kGLGroup zeros (the read-ahead
// of the last group stays inside the table).
__global__ __launch_bounds__(256) void gl_table_kernel(int n, double* __restrict__ beta) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x + 1;
  if (k < n) beta[k - 1] = k / (k + 1.0);
  else if (k < n + 2 * kGLGroup) beta[k - 1] = 0.0;
}

__device__ __forceinline__ void gl_step(double b, double s, double& p0, double& p1) {
  const double v = fma(b, s, s);  // alpha_k s
  const double q = b * p0;        // beta_k P_{k-1}
  const double p2 = fma(v, p1, -q);
  p0 = p1;
  p1 = p2;
}

// (P_n(s), P_{n-1}(s)); every lane of the wave calls it with the same n.
// Scalar loads complete out of order, so a wait covers every load in flight:
// each group's first step (whose wait covers only that group's loads) runs
// before the next group's loads are issued, and the rest of the group hides
// their latency.
__device__ __forceinline__ void legendre_wave(int n, double s, const double* __restrict__ beta, double& pn,
                                              double& pn1) {
  const int steps = n - 1;
  double p0 = 1.0, p1 = s;
  int k = 0;
  if (steps >= 2 * kGLGroup) {
    double A[kGLGroup], B[kGLGroup];
#pragma unroll
    for (int u = 0; u < kGLGroup; ++u) A[u] = beta[u];
    for (; k + 2 * kGLGroup <= steps; k += 2 * kGLGroup) {
      gl_step(A[0], s, p0, p1);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < kGLGroup; ++u) B[u] = beta[k + kGLGroup + u];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 1; u < kGLGroup; ++u) gl_step(A[u], s, p0, p1);
      __builtin_amdgcn_sched_barrier(0);
      gl_step(B[0], s, p0, p1);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < kGLGroup; ++u) A[u] = beta[k + 2 * kGLGroup + u];  // zero padded past the end
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 1; u < kGLGroup; ++u) gl_step(B[u], s, p0, p1);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  for (; k < steps; ++k) gl_step(beta[k], s, p0, p1);
  pn = p1;
  pn1 = p0;
}

__global__ __launch_bounds__(256) void gl_node_kernel(int n, const double* __restrict__ beta, double* __restrict__ x,
                                                      double* __restrict__ w) {
  const int nh = (n + 1) / 2;
  const int k = blockIdx.x * 256 + threadIdx.x + 1;
  const bool act = k <= nh;
  const double dn = (double)n;
  // the first zeros of J_0 (Abramowitz and Stegun, Table 9.5)
  constexpr double kJ0[5] = {2.404825557695773, 5.520078110286311, 8.653727912911013, 11.79153443901428,
                             14.93091770848779};
  constexpr double kU = 1.1102230246251565e-16;  // 2^-53
  double s = 0.5;  // inactive lanes run along on a harmless point
  if (act)
    s = k <= 5 ? cos(kJ0[k - 1] / (dn + 0.5))
               : (1.0 - (dn - 1.0) / (8.0 * dn * dn * dn)) * cos(kPi * (4.0 * k - 1.0) / (4.0 * dn + 2.0));
  bool done = !act;
  double dp = 1.0;
  for (int it = 0; it < 100 && __any(done ? 0 : 1); ++it) {
    double pn, pn1;
    legendre_wave(n, s, beta, pn, pn1);
    if (!done) {
      const double d = dn * (s * pn - pn1) / (s * s - 1.0);
      const double sn = s - pn / d;
      const double h = s - sn;  // the step as taken (exact)
      const double om = 1.0 - s * s;
      if (fabs(s) * h * h <= 0.25 * kU * om && dn * dn * h * h <= kU) {
        dp = d - h * (2.0 * s * d - dn * (dn + 1.0) * pn) / om;  // P_n' at sn, to first order
        done = true;
      }
      s = sn;
    }
  }
  if (act) {
    const double wt = 2.0 / ((1.0 - s * s) * dp * dp);
    if (2 * k - 1 == n) {  // odd n: the middle node is 0
      x[k - 1] = 0.0;
      w[k - 1] = wt;
    } else {
      x[n - k] = s;
      w[n - k] = wt;
      x[k - 1] = -s;
      w[k - 1] = wt;
    }
  }
}

// ---------------------------------------------------------------------------
// Schwinger function.  Per node: p = p_max h^2 with h = (1 + x)/2 and
// g = w p_max h Z(p^2) / (pi p^2) (the rule's weight dp/dx = p_max h, and
// sigma = Z/p^2 with the dressing from the expansion and its IR / UV
// extension).  Then Delta(t_j) = sum_i g_i cos(t_j p_i): blocks of
// (256 kSchwNPT nodes) x (kSchwTT times) write partial sums, a second kernel
// adds the partial sums of each time in a fixed order.

constexpr int kSchwNPT = 4;
constexpr int kSchwTT = 16;

__device__ __forceinline__ double ln_z_at(const Views& v, const Phys& ph, const double* __restrict__ c, double lu) {
  const double s = fmin(fmax((lu - ph.L0) * ph.invL1, -1.0), 1.0);
  const double s2 = s + s;
  double z = 0.5 * c[0];
  double Tp = 1.0, Tc = s;
  for (int j = 1; j < v.n_z; ++j) {
    z = fma(c[j], Tc, z);
    const double Tn = fma(s2, Tc, -Tp);
    Tp = Tc;
    Tc = Tn;
  }
  if (lu < ph.ln_eps2) z += 2.0 * ph.kappa * (lu - ph.ln_eps2);
  else if (lu > ph.ln_lam2) z += ph.gamma * log(fma(ph.omega, lu - ph.ln_lam2, 1.0));
  return z;
}

__global__ __launch_bounds__(256) void schw_prep_kernel(Views v, Phys ph, const double* __restrict__ c, int n,
                                                        double p_max, const double* __restrict__ x,
                                                        const double* __restrict__ w, double* __restrict__ pn,
                                                        double* __restrict__ gn) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double h = 0.5 * (1.0 + x[i]);
  const double p = p_max * h * h;
  const double u = p * p;
  const double z = ln_z_at(v, ph, c, log(u));
  pn[i] = p;
  gn[i] = w[i] * p_max * h * exp(z) / u / kPi;
}

__global__ __launch_bounds__(256) void schw_sum_kernel(int n, const double* __restrict__ pn,
                                                       const double* __restrict__ gn, const double* __restrict__ t,
                                                       int m, double* __restrict__ part) {
  __shared__ double red[4][kSchwTT];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int base = blockIdx.x * 256 * kSchwNPT + threadIdx.x;
  const int t0 = blockIdx.y * kSchwTT;
  double pp[kSchwNPT], gg[kSchwNPT];
#pragma unroll
  for (int j = 0; j < kSchwNPT; ++j) {
    const int i = base + 256 * j;
    pp[j] = i < n ? pn[i] : 0.0;
    gg[j] = i < n ? gn[i] : 0.0;
  }
#pragma unroll 1
  for (int q = 0; q < kSchwTT; ++q) {
    const double tq = t0 + q < m ? t[t0 + q] : 0.0;
    double a = 0.0;
#pragma unroll
    for (int j = 0; j < kSchwNPT; ++j) a = fma(gg[j], cos(tq * pp[j]), a);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) a += __shfl_xor(a, o, 64);
    if (lane == 0) red[wave][q] = a;
  }
  __syncthreads();
  if (threadIdx.x < kSchwTT && t0 + (int)threadIdx.x < m) {
    const int q = threadIdx.x;
    part[(size_t)blockIdx.x * m + t0 + q] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
  }
}

__global__ __launch_bounds__(256) void schw_reduce_kernel(int chunks, const double* __restrict__ part, int m,
                                                          double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  double s = 0.0;
  for (int b = 0; b < chunks; ++b) s += part[(size_t)b * m + j];
  out[j] = s;
}

// ---------------------------------------------------------------------------
// Renormalisation scale: the largest root in [eps2, lambda2] of
// h(x) = 2 ln G(x) + ln Z(x) (where alpha(x) = alpha(mu^2) G^2 Z passes
// alpha(mu^2)), in the mapped variable s.  One block: a scan of `scan` equal
// intervals finds the uppermost sign change; rounds of 256-fold multisection
// narrow it to adjacent doubles; the end with the smaller |h| is the root.

__device__ __forceinline__ double renorm_h(const Views& v, const double* __restrict__ c, double s) {
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
  return 2.0 * g + z;
}

__device__ __forceinline__ bool brackets(double hlo, double hhi) { return (hlo < 0.0) != (hhi < 0.0) || hlo == 0.0; }

__global__ __launch_bounds__(256) void renorm_kernel(Views v, Phys ph, const double* __restrict__ c, int scan,
                                                     double* __restrict__ out) {
  __shared__ int kbest;
  __shared__ double hs[257];
  __shared__ double bound[4];  // lo, hi, h(lo), h(hi)
  const int t = threadIdx.x;
  if (t == 0) kbest = -1;
  __syncthreads();
  for (int k = t; k < scan; k += 256) {
    const double lo = -1.0 + 2.0 * k / scan, hi = -1.0 + 2.0 * (k + 1) / scan;
    if (brackets(renorm_h(v, c, lo), renorm_h(v, c, hi))) atomicMax(&kbest, k);
  }
  __syncthreads();
  const int kb = kbest;
  if (kb < 0) {
    if (t == 0) out[0] = __longlong_as_double(0x7ff8000000000000LL);
    return;
  }
  if (t == 0) {
    bound[0] = -1.0 + 2.0 * kb / scan;
    bound[1] = -1.0 + 2.0 * (kb + 1) / scan;
    bound[2] = renorm_h(v, c, bound[0]);
    bound[3] = renorm_h(v, c, bound[1]);
  }
  __syncthreads();
  for (int round = 0; round < 16; ++round) {
    const double lo = bound[0], hi = bound[1];
    // points lo + (hi - lo) i / 256, i = 0 .. 256 (the ends keep their values)
    const double si = t == 0 ? lo : fma((hi - lo), t / 256.0, lo);
    hs[t] = t == 0 ? bound[2] : renorm_h(v, c, si);
    if (t == 0) hs[256] = bound[3];
    __syncthreads();
    if (t == 0) {
      int ib = 0;
      for (int i = 255; i >= 0; --i)
        if (brackets(hs[i], hs[i + 1])) { ib = i; break; }
      const double nlo = ib == 0 ? lo : fma((hi - lo), ib / 256.0, lo);
      const double nhi = ib == 255 ? hi : fma((hi - lo), (ib + 1) / 256.0, lo);
      const bool progress = nlo > lo || nhi < hi;
      bound[0] = nlo;
      bound[1] = nhi;
      bound[2] = hs[ib];
      bound[3] = hs[ib + 1];
      hs[0] = progress ? 1.0 : 0.0;  // progress flag for the other threads
    }
    __syncthreads();
    const bool go_on = hs[0] != 0.0;
    __syncthreads();
    if (!go_on) break;
  }
  if (t == 0) {
    const double s = fabs(bound[2]) <= fabs(bound[3]) ? bound[0] : bound[1];
    out[0] = exp(ph.L0 + s / ph.invL1);
  }
}

}  // namespace

hipError_t launch_gl(int n, double* x, double* w, void* tab, hipStream_t st) {
  hipLaunchKernelGGL(gl_table_kernel, dim3((n - 1 + 2 * kGLGroup + 255) / 256), dim3(256), 0, st, n, (double*)tab);
  const int nh = (n + 1) / 2;
  hipLaunchKernelGGL(gl_node_kernel, dim3((nh + 255) / 256), dim3(256), 0, st, n, (const double*)tab, x, w);
  return hipGetLastError();
}

int schwinger_chunks(int n) { return (n + 256 * kSchwNPT - 1) / (256 * kSchwNPT); }

hipError_t launch_schwinger(const Views& v, const Phys& ph, const double* c, int n, double p_max, const double* x,
                            const double* w, const double* t, int m, double* out, double* pn, double* gn,
                            double* part, hipStream_t st) {
  hipLaunchKernelGGL(schw_prep_kernel, dim3((n + 255) / 256), dim3(256), 0, st, v, ph, c, n, p_max, x, w, pn, gn);
  if (m > 0) {
    const int chunks = schwinger_chunks(n);
    hipLaunchKernelGGL(schw_sum_kernel, dim3(chunks, (m + kSchwTT - 1) / kSchwTT), dim3(256), 0, st, n, pn, gn, t,
                       m, part);
    hipLaunchKernelGGL(schw_reduce_kernel, dim3((m + 255) / 256), dim3(256), 0, st, chunks, part, m, out);
  }
  return hipGetLastError();
}

hipError_t launch_renorm(const Views& v, const Phys& ph, const double* c, int scan, double* out, hipStream_t st) {
  hipLaunchKernelGGL(renorm_kernel, dim3(1), dim3(256), 0, st, v, ph, c, scan, out);
  return hipGetLastError();
}

}  // namespace dse

// ---------------------------------------------------------------------------
// C ABI

namespace {

constexpr int kGLMax = 1 << 24;
constexpr int kRenormScan = 4096;

size_t al256(size_t b) { return (b + 255) / 256 * 256; }
size_t gl_tab_bytes(int n) { return al256((size_t)(n - 1 + 2 * dse::kGLGroup) * sizeof(double)); }

struct SchwLayout {
  size_t tab, x, w, p, g, part, total;
};
SchwLayout schw_layout(int n, int m) {
  SchwLayout L;
  size_t off = 0;
  L.tab = off; off += gl_tab_bytes(n);
  L.x = off; off += al256((size_t)n * 8);
  L.w = off; off += al256((size_t)n * 8);
  L.p = off; off += al256((size_t)n * 8);
  L.g = off; off += al256((size_t)n * 8);
  L.part = off; off += al256((size_t)dse::schwinger_chunks(n) * (m > 0 ? m : 1) * 8);
  L.total = off;
  return L;
}

struct DevGuard {
  int prev = -1;
  explicit DevGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DevGuard() {
    int cur;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

extern "C" {

size_t dse_gauss_legendre_workspace_bytes(int32_t n) { return n < 1 || n > kGLMax ? 0 : gl_tab_bytes(n); }

dse_status dse_gauss_legendre(int32_t n, double* d_x, double* d_w, void* d_ws, size_t ws_bytes, void* hip_stream) {
  if (n < 1 || n > kGLMax || !d_x || !d_w) {
    dse::set_err(dse::global_err(), "dse_gauss_legendre: need 1 <= n <= %d and non-NULL d_x, d_w (n = %d)", kGLMax, n);
    return DSE_E_INVALID;
  }
  if (!d_ws || ws_bytes < gl_tab_bytes(n) || ((uintptr_t)d_ws & 255u)) {
    dse::set_err(dse::global_err(), "dse_gauss_legendre: workspace of %zu bytes (256-byte aligned) needed",
                 gl_tab_bytes(n));
    return ws_bytes < gl_tab_bytes(n) && d_ws ? DSE_E_NOMEM : DSE_E_INVALID;
  }
  const hipError_t e = dse::launch_gl(n, d_x, d_w, d_ws, (hipStream_t)hip_stream);
  if (e != hipSuccess) {
    dse::set_err(dse::global_err(), "dse_gauss_legendre: %s", hipGetErrorString(e));
    return DSE_E_DEVICE;
  }
  return DSE_OK;
}

size_t dse_schwinger_workspace_bytes(int32_t n, int32_t m) {
  if (n < 1 || n > kGLMax || m < 0) return 0;
  return schw_layout(n, m).total;
}

dse_status dse_schwinger(dse_ctx* ctx, const double* d_c, int32_t n, double p_max, const double* d_t, int32_t m,
                         double* d_delta, void* d_ws, size_t ws_bytes) {
  if (!ctx) return DSE_E_INVALID;
  if (!d_c || n < 1 || n > kGLMax || m < 0 || (m > 0 && (!d_t || !d_delta)) || !(p_max > 0.0) || !isfinite(p_max)) {
    dse::set_err(ctx->err, "dse_schwinger: need d_c, 1 <= n <= %d, m >= 0 (d_t, d_delta non-NULL when m > 0), "
                 "finite p_max > 0", kGLMax);
    return DSE_E_INVALID;
  }
  const SchwLayout L = schw_layout(n, m);
  if (!d_ws || ((uintptr_t)d_ws & 255u)) {
    dse::set_err(ctx->err, "dse_schwinger: the workspace must be a non-NULL, 256-byte aligned device pointer");
    return DSE_E_INVALID;
  }
  if (ws_bytes < L.total) {
    dse::set_err(ctx->err, "dse_schwinger: workspace has %zu bytes, needs %zu", ws_bytes, L.total);
    return DSE_E_NOMEM;
  }
  DevGuard dg(ctx->device);
  char* b = (char*)d_ws;
  double* x = (double*)(b + L.x);
  double* w = (double*)(b + L.w);
  hipError_t e = dse::launch_gl(n, x, w, b + L.tab, ctx->st);
  if (e == hipSuccess)
    e = dse::launch_schwinger(ctx->v, ctx->ph, d_c, n, p_max, x, w, d_t, m, d_delta, (double*)(b + L.p),
                              (double*)(b + L.g), (double*)(b + L.part), ctx->st);
  if (e != hipSuccess) {
    dse::set_err(ctx->err, "dse_schwinger: %s", hipGetErrorString(e));
    return DSE_E_DEVICE;
  }
  return DSE_OK;
}

dse_status dse_renorm_scale(dse_ctx* ctx, const double* d_c, double* d_mu2) {
  if (!ctx) return DSE_E_INVALID;
  if (!d_c || !d_mu2) {
    dse::set_err(ctx->err, "dse_renorm_scale: d_c and d_mu2 must not be NULL");
    return DSE_E_INVALID;
  }
  DevGuard dg(ctx->device);
  const hipError_t e = dse::launch_renorm(ctx->v, ctx->ph, d_c, kRenormScan, d_mu2, ctx->st);
  if (e != hipSuccess) {
    dse::set_err(ctx->err, "dse_renorm_scale: %s", hipGetErrorString(e));
    return DSE_E_DEVICE;
  }
  return DSE_OK;
}

}  // extern "C"
