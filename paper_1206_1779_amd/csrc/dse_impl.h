// dse_impl.h -- internal declarations of the HIP implementation (not part of
// the C ABI).  Shared by the host driver and the kernel translation unit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dse.h"

namespace dse {

// Padding of the radial grid (multiple of every q-tile), of the angular grid
// and of the Chebyshev order (the point kernels are instantiated per padded
// order).
constexpr int kQPad = 64;
constexpr int kKPad = 8;
constexpr double kPi = 3.14159265358979323846264338327950288;
// parts of the radial sum of the B . T contraction (summed by the assembly);
// eight measured faster than two, four, six, twelve or sixteen at N = 64
constexpr int kCS = 8;

inline int pad_up(int v, int m) { return (v + m - 1) / m * m; }
// Padded Chebyshev order: 16, 32, 48, 64, 96 or 128.
inline int padded_order(int n) {
  if (n <= 16) return 16;
  if (n <= 32) return 32;
  if (n <= 48) return 48;
  if (n <= 64) return 64;
  if (n <= 96) return 96;
  return 128;
}

// Derived physical constants handed to every kernel by value.
struct Phys {
  double C;          // alpha N_c / (2 pi^2)  (= g^2 N_c / (2 pi)^3)
  double omega;      // 11 N_c alpha / (12 pi)
  double e1, e2;     // -2 - 6 delta, -3 delta
  double L0, invL1;  // s = (ln u - L0) / L1
  double ln_eps2, ln_lam2;
  double kappa, delta, gamma;
  double g0_inv, z_lambda_inv;
  double inv_alpha;        // 1 / alpha(mu^2)
  double omega_per_alpha;  // d omega / d alpha = 11 N_c / (12 pi)
};

// Device views into the caller's workspace.
struct Views {
  int n_z, n_g, n;       // orders and unknowns
  int NJ;                // padded order
  int Q, Qp, K, Kp;      // radial / angular nodes and their padded counts
  int RZ, RG;            // gluon rows (n_z + subtraction at Lambda^2), ghost rows (n_g + x = 0)
  int nqt;               // radial tiles of 64 nodes per row (Qp / 64)
  int KS;                // angular slices: point-kernel blocks per (row, radial tile)
  int Rb, Rbp;           // rows of the B matrix (2 RZ + RG) and padded to 16
  int split;             // 1: every row has its own radial grid, split at its x (Sec. 3)
  // tables
  double* coef;          // [2][NJ] a then b, zero padded, j = 0 term halved
  double* y;             // [Qp] radial nodes (padding: y = 1, W = 0)
  double* W;             // [Qp] radial weights including the factor y
  double* lnZy;          // [Qp] ln Z at the radial nodes
  double* lnGy;          // [Qp]
  double* Ttab;          // [Qp][NJ] Tilde-T_j(s(y_q))
  float* Ttab32;         // [Qp][NJ] the same in FP32 (mixed-precision contraction)
  double* TtabT;         // [NJ][Qp] transposed (dressing GEMV)
  double* Text;          // [n][NJ]  Tilde-T_j(s(x_r)) at the collocation points
  double* TextT;         // [NJ][n]  transposed
  double* xrow;          // [RZ + RG] external momentum of each row
  double* lnX;           // [n] ln Z (gluon rows) / ln G (ghost rows) at x_r
  double* ang;           // [5][Kp] cos, sin^2(theta/2), v sin^2, v sin^4, sin^2
  // split radial grids (split = 1; [RZ + RG][Qp], row order as xrow, padding W = 0)
  double* yr;            // nodes
  double* Wr;            // weights including the factor y
  double* syr;           // mapped coordinate s(y), clamped to [-1, 1]
  double* lnZyr;         // ln Z, ln G at the nodes (per assembly)
  double* lnGyr;
  // per assembly
  // (in mixed precision Bm, Dp, Eq and Dgh hold FP32 values at the same indices)
  double* Bm;            // [KS][Rbp][Qp] angular sums per slice: rows gluon-a | gluon-b | ghost-b
  double* Dp;            // [3 or 4][RZ or RG][nqt*KS][NJ] k-side partials: gluon-a | gluon-b | ghost-a
                         // (| ghost-b: the q-side of the ghost rows on split grids)
  double* Pip;           // [RZ + RG][nqt*KS][2] partial self-energies (sum, rounding error)
  double* Absp;          // [RZ + RG][nqt*KS] partial sums of |integrand|
  double* Eq;            // [kCS][Rbp][NJ] B . T (+ k-side sums for the gluon rows), by part
  double* Dgh;           // [kCS][RG][NJ] k-side sums of the ghost rows (target a), by part
  double* rw;            // [RZ + RG] row weights of a vector-Jacobian product
  // Newton
  double* LU;            // [np][np+1], np = 16 ceil(n/16): padded factors of [A | b] when they do not fit LDS
  int32_t* piv;          // [n]
  int32_t* flag;         // [4] status flags written by kernels
  double* rowmax;        // [n] largest |J_rk| of each row of the Newton matrix (written by the assembly)
  double* rowmax_u;      // [n] the same for a caller's matrix (dse_lu_solve)
  double* F;             // [n]
  double* S;             // [n]
  double* Ft;            // [n]
  double* St;            // [n]
  double* dlt;           // [n]
  double* ct;            // [n]
  double* J;             // [n][n]
  double* scal;          // [8] merit, ||F||_2, ||delta||_inf
};

// One problem of a batched family as the batched kernels see it (device
// memory, one per problem).
struct SolveDesc {
  Views v;
  Phys ph;
  int coff;   // offset of the problem's unknowns in the packed coefficient vector
  int pad_;
  size_t joff;  // offset of its n x n Newton matrix in a packed matrix array
};

// Host helpers (dse_host.hip).
void set_err(char* buf, const char* fmt, ...);
// Message buffer of the calls that have no context (dse_last_error(NULL)).
char* global_err();
dse_status validate(const dse_params* p, char* err);
Phys make_phys(const dse_params& p);
size_t layout(const dse_params& p, Views* v, char* base, int ks);  // returns bytes
dse_status upload_tables(const dse_params& p, const Views& v, const Phys& ph, hipStream_t st, char* err);
void start_guess_host(const dse_params& p, const Phys& ph, double* c_out);

// Kernel launchers (dse_kernels.hip).  All enqueue on `st`.
hipError_t launch_dressing(const Views& v, const Phys& ph, const double* c, hipStream_t st);
// mode: 0 residual, 1 Jacobian, 2 vector-Jacobian product, 3 parameter VJP;
// mix (Jacobian mode only): derivative sums in FP32
hipError_t launch_points(const Views& v, const Phys& ph, int mode, bool mix, hipStream_t st,
                         hipEvent_t* ev /* nullable: [3] events before, between and after the
                                           gluon and ghost point kernels */);
hipError_t launch_contract(const Views& v, bool mix, hipStream_t st);
hipError_t launch_row_weights(const Views& v, const double* u, hipStream_t st);
hipError_t launch_vjp_reduce(const Views& v, const double* u, double* uJ, double* uth, hipStream_t st);
// F2, S2 (nullable): second copies of F and S (a caller's vectors).
hipError_t launch_assemble(const Views& v, const Phys& ph, double* J, double* F, double* S, bool mix,
                           hipStream_t st, double* F2 = nullptr, double* S2 = nullptr);
hipError_t launch_residual_rows(const Views& v, const Phys& ph, double* F, double* S,
                                hipStream_t st);
hipError_t launch_norms(const Views& v, const double* F, const double* S, const double* d,
                        double* out, hipStream_t st);
hipError_t launch_coupling(const Views& v, const Phys& ph, double alpha_mu, const double* c, const double* u, int m,
                           double* alpha, double* lnZ, double* lnG, hipStream_t st);
hipError_t launch_dressing_vjp(const Views& v, const Phys& ph, const double* u, int m, const double* wZ,
                               const double* wG, double* grad, hipStream_t st);
hipError_t launch_fd_shift(int n, const double* c, int j, double h_rel, double sgn, double* cs, double* hbuf,
                           hipStream_t st);
hipError_t launch_fd_column(int n, const double* Fp, const double* Fm, const double* hbuf, int j, double* J,
                            hipStream_t st);
hipError_t launch_axpy(int n, const double* c, double rho, const double* d, double* out,
                       hipStream_t st);
// With cout != nullptr the solve also writes the update cout = cin - rho x.
// rowmax (nullable): the largest |A_rk| of each row; a pivot at or below
// n eps rowmax of its row then counts as singular (else only zero or
// non-finite pivots do).
hipError_t launch_lu_solve(const Views& v, const double* A, const double* b, double* x,
                           int trans, hipStream_t st, const double* cin = nullptr, double rho = 0.0,
                           double* cout = nullptr, const double* rowmax = nullptr);
// rowmax[r] = max_k |A[r][k]| of a row-major n x n matrix (one wave per row).
hipError_t launch_row_absmax(int n, const double* A, double* rowmax, hipStream_t st);
void lu_setup();  // LDS attributes of the factorisation kernels (call before any capture)

// Observables (dse_observables.hip).  launch_gl: n-node Gauss-Legendre rule
// into x, w; tab holds 8 (n - 1) bytes of recurrence coefficients.
hipError_t launch_gl(int n, double* x, double* w, void* tab, hipStream_t st);
int schwinger_chunks(int n);  // partial sums per time of the Schwinger sum
hipError_t launch_schwinger(const Views& v, const Phys& ph, const double* c, int n, double p_max, const double* x,
                            const double* w, const double* t, int m, double* out, double* pn, double* gn,
                            double* part, hipStream_t st);
hipError_t launch_renorm(const Views& v, const Phys& ph, const double* c, int scan, double* out, hipStream_t st);

// Batched family (one launch per stage for all problems whose mask entry is
// set).  `which` selects the evaluation point and outputs: 0 = the packed
// coefficients cpk (outputs F, S), 1 = the trial point ct (outputs Ft, St).
struct BatchArgs {
  const SolveDesc* desc;  // [count]
  int count;
  const int* mask;        // [count] nonzero: problem takes part
  int max_n, max_np, max_nj, max_rbt;  // largest n, padded n, padded order, contraction row blocks
  int max_dress_blocks;                // dressing blocks per problem (largest Qp + n over 256)
};
hipError_t launch_batch_dressing(const BatchArgs& a, const double* cpk, int which, int* counter,
                                 hipStream_t st);
// items: (problem, kind, row, first tile), in queue order; each item takes
// tpi consecutive partial tiles of its row.  grid = 0: one block per item in
// queue order; grid > 0: that many persistent blocks take items from the
// queue through the counter (which the dressing launch resets).
hipError_t launch_batch_points(const BatchArgs& a, const int4* items, int n_items, int mode, int grid, int tpi,
                               int* counter, hipStream_t st);
int batch_points_occupancy(int mode, int max_nj);  // resident blocks per CU
// The whole Newton-matrix assembly (dressings, points, contraction, rows) in
// one cooperative launch of grid resident blocks (at most the occupancy of
// batch_fused_occupancy times the CUs).
// which 1: the dressings at each member's trial point ct instead of cpk.
hipError_t launch_batch_fused(const BatchArgs& a, const double* cpk, const int4* items, int n_items, int tpi,
                              int grid, int* counter, hipStream_t st, int which = 0);
int batch_fused_occupancy(int max_nj);  // resident blocks per CU (0: not available)
hipError_t launch_batch_contract(const BatchArgs& a, hipStream_t st);
hipError_t launch_batch_assemble(const BatchArgs& a, hipStream_t st);
hipError_t launch_batch_residual_rows(const BatchArgs& a, int which, hipStream_t st);
hipError_t launch_batch_norms(const BatchArgs& a, int which, double* out /* [count][4] */, hipStream_t st);
hipError_t launch_batch_lu(const BatchArgs& a, int* flags /* [count] */, hipStream_t st);
hipError_t launch_batch_axpy(const BatchArgs& a, const double* cpk, const double* rho, hipStream_t st);
hipError_t launch_batch_accept(const BatchArgs& a, double* cpk, hipStream_t st);
hipError_t launch_batch_pack(const BatchArgs& a, double* Jpk, double* Fpk, hipStream_t st);

}  // namespace dse

// The context behind the opaque dse_ctx handle of the C ABI.
struct dse_ctx {
  dse_params p;
  dse::Views v;
  dse::Phys ph;
  hipStream_t st;
  int device;
  char* ws;
  size_t ws_bytes;
  bool timing;
  // event ring: per timed dse_jacobian, events before dressing, before the
  // gluon point kernel, between gluon and ghost, after ghost, after the
  // contraction, after the assembly
  static constexpr int kRing = 64;
  static constexpr int kEv = 6;
  hipEvent_t ev[kRing][kEv];
  // device time of the assembly and LU phases of dse_newton_solve
  hipEvent_t nev[4] = {nullptr, nullptr, nullptr, nullptr};
  // pinned host words for the small reads the host waits on (norms, pivot
  // flag): a copy to pageable memory would wait for the stream by itself
  double* hpin = nullptr;  // [0..3] norms, [4] flag (as int32)
  int32_t* hflag() { return reinterpret_cast<int32_t*>(hpin + 4); }
  int ring_count;
  double acc_ms[5];
  int acc_n;
  // Newton matrix, residual and scale held in the workspace (v.J, v.F, v.S)
  // for the coefficients at this device pointer (nullptr: nothing held)
  const double* jac_at = nullptr;
  // recorded Newton steps (dse_newton_step): the launch sequence for one set
  // of pointers, relaxation and kind (with or without the assembly at d_c),
  // replayed as a HIP graph; a few are kept (alternating buffers need two)
  bool graphs = false;
  hipStream_t cap_st = nullptr;  // private stream the graphs are recorded on (the
                                 // caller's stream may be the null stream, which
                                 // cannot be captured); replays go to st
  struct StepGraph {
    hipGraphExec_t exec = nullptr;
    const void* key[4] = {nullptr, nullptr, nullptr, nullptr};
    double rho = 0.0;
    bool reuse = false;
    unsigned long long used = 0;
  };
  static constexpr int kSteps = 4;
  StepGraph steps[kSteps];
  unsigned long long step_clock = 0;
  char err[512];
};
