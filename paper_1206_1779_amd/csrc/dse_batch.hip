// dse_batch.hip -- host side of the batched family: many independent DSE
// problems (own orders, grids and physics, e.g. a family of decoupling
// solutions G(0) = 5 ... 50, the solution family of Sec. 2) assembled and
// solved together, one launch per stage for the whole family.
//
// Point work is a queue of (problem, row kind, row, tile) items ordered
// largest first (LPT: longest processing time first) and taken either by one
// workgroup per item in queue order or by persistent workgroups through an
// atomic counter.  The angular split (slices), the launch form and the queue
// order are chosen by timing every candidate on the family itself
// (dse_batch_autotune).  The Newton iteration of every problem follows the
// single-problem driver step for step (same tests, same relaxation rule);
// the problems only share launches.

#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <new>
#include <vector>

#include "dse_impl.h"

struct dse_batch {
  int count = 0;
  std::vector<dse_params> p;
  std::vector<dse::SolveDesc> desc;  // host copy of the device descriptors
  hipStream_t st = nullptr;
  int device = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  // device control area
  dse::SolveDesc* d_desc = nullptr;
  int4* d_items = nullptr;
  double* d_nrm = nullptr;
  int* d_flags = nullptr;
  int* d_mask = nullptr;
  double* d_rho = nullptr;
  int* d_counter = nullptr;
  int max_items = 0;
  int n_items = 0;
  int ks_cap = 1;
  // launch choice
  int slices = 1;
  int grid = 0;   // 0: one workgroup per item; > 0: persistent workgroups
  int order = 1;  // 1: largest first, 0: problem order
  int tpi = 1;    // partial tiles per queue item
  int fused = 0;  // 1: the whole assembly in one cooperative launch of grid workgroups
  int ncu = 256;
  int coop = 0;   // the device supports cooperative launches
  dse::BatchArgs args{};
  std::vector<int> h_mask;
  std::vector<double> h_rho;
  // pinned host words for the device-to-host reads the host waits on (norms
  // [count][4], then the pivot flags [count] as int): a copy to pageable
  // memory would wait for the stream by itself
  double* h_pin = nullptr;
  int* h_pin_flags() { return reinterpret_cast<int*>(h_pin + 4 * (size_t)count); }
  ~dse_batch() {
    if (h_pin) (void)hipHostFree(h_pin);
  }
  std::vector<int64_t> coff, joff;
  char err[512] = {0};
};

static char g_batch_err[512];

namespace {

using dse::set_err;

#define BHIP_TRY(b, expr)                                                          \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      set_err((b)->err, "%s: %s", #expr, hipGetErrorString(e_));                   \
      return DSE_E_DEVICE;                                                         \
    }                                                                              \
  } while (0)

constexpr int kSlicesCap = 4;

size_t al(size_t x) { return (x + 255) / 256 * 256; }

// Largest angular split a problem can use: every wave keeps at least one angle.
int slices_cap(const dse_params& p) {
  const int Kp = dse::pad_up(p.n_ang, dse::kKPad);
  int ks = 1;
  while (ks < kSlicesCap && 4 * (ks * 2) <= Kp) ks *= 2;
  return ks;
}

struct Sizes {
  size_t ctl, per_total;
  std::vector<size_t> per;
  int max_items;
};

Sizes sizes(const dse_params* p, int count, int ks_cap) {
  Sizes s;
  s.max_items = 0;
  s.per_total = 0;
  for (int b = 0; b < count; ++b) {
    dse::Views v;
    const size_t bytes = dse::layout(p[b], &v, nullptr, ks_cap);
    s.per.push_back(bytes);
    s.per_total += bytes;
    s.max_items += (v.RZ + v.RG) * v.nqt * ks_cap;
  }
  s.ctl = al(count * sizeof(dse::SolveDesc)) + al((size_t)s.max_items * sizeof(int4)) +
          al(count * 4 * sizeof(double)) + al(count * sizeof(int)) + al(count * sizeof(int)) +
          al(count * sizeof(double)) + 256;
  return s;
}

// Work estimate of one point item (flops per point x points), for the queue order.
double item_cost(const dse::Views& v, int kind) {
  const double pts = 64.0 * v.Kp / v.KS;
  const int nmax = v.n_z > v.n_g ? v.n_z : v.n_g;
  return kind == 0 ? pts * (2.0 * nmax + 4.0 * (v.n_z + v.n_g) + 100.0) : pts * (6.0 * v.n_z + 60.0);
}

dse_status set_launch(dse_batch* B, int slices, int grid, int order, int tpi = 1, int fused = 0) {
  B->slices = slices;
  B->grid = grid;
  B->order = order;
  B->tpi = tpi;
  B->fused = fused;
  struct It { double cost; int4 w; };
  std::vector<It> its;
  int max_nj = 16, max_n = 1, max_rbt = 1, max_dress = 1;
  for (int b = 0; b < B->count; ++b) {
    dse::Views& v = B->desc[b].v;
    v.KS = slices;
    const int nt = v.nqt * slices;
    for (int kind = 0; kind < 2; ++kind) {
      const int rows = kind == 0 ? v.RZ : v.RG;
      const double c = item_cost(v, kind);
      for (int r = 0; r < rows; ++r)
        for (int t = 0; t < nt; t += tpi) its.push_back({c * std::min(tpi, nt - t), make_int4(b, kind, r, t)});
    }
    max_nj = std::max(max_nj, v.NJ);
    max_n = std::max(max_n, v.n);
    max_rbt = std::max(max_rbt, v.Rbp / 16 + (v.RG + 15) / 16);
    max_dress = std::max(max_dress, (v.Qp + v.n + 255) / 256);
  }
  if (order == 1)
    std::stable_sort(its.begin(), its.end(), [](const It& a, const It& b) { return a.cost > b.cost; });
  std::vector<int4> w(its.size());
  for (size_t i = 0; i < its.size(); ++i) w[i] = its[i].w;
  B->n_items = (int)w.size();
  if (B->n_items > B->max_items) { set_err(B->err, "work list overflow"); return DSE_E_INVALID; }
  BHIP_TRY(B, hipMemcpyAsync(B->d_items, w.data(), w.size() * sizeof(int4), hipMemcpyHostToDevice, B->st));
  BHIP_TRY(B, hipMemcpyAsync(B->d_desc, B->desc.data(), B->desc.size() * sizeof(dse::SolveDesc),
                             hipMemcpyHostToDevice, B->st));
  BHIP_TRY(B, hipStreamSynchronize(B->st));
  B->args.desc = B->d_desc;
  B->args.count = B->count;
  B->args.mask = B->d_mask;
  B->args.max_n = max_n;
  B->args.max_np = (max_n + 15) / 16 * 16;
  B->args.max_nj = max_nj;
  B->args.max_rbt = max_rbt;
  B->args.max_dress_blocks = max_dress;
  return DSE_OK;
}

// Mask and relaxation upload (the caller synchronises before changing them again).
dse_status upload_ctl(dse_batch* B) {
  BHIP_TRY(B, hipMemcpyAsync(B->d_mask, B->h_mask.data(), B->count * sizeof(int), hipMemcpyHostToDevice, B->st));
  BHIP_TRY(B, hipMemcpyAsync(B->d_rho, B->h_rho.data(), B->count * sizeof(double), hipMemcpyHostToDevice, B->st));
  return DSE_OK;
}

// The staged launches' persistent grid for the fused form's point stage is
// its own cooperative grid; the residual pass always runs staged (with
// persistent blocks when the fused form is chosen).
dse_status eval_residuals(dse_batch* B, const double* cpk, int which) {
  const dse::BatchArgs& a = B->args;
  BHIP_TRY(B, dse::launch_batch_dressing(a, cpk, which, B->d_counter, B->st));
  BHIP_TRY(B, dse::launch_batch_points(a, B->d_items, B->n_items, 0, B->grid, B->tpi, B->d_counter, B->st));
  BHIP_TRY(B, dse::launch_batch_residual_rows(a, which, B->st));
  return DSE_OK;
}

// which 1: at each member's trial point ct (cpk unused)
dse_status eval_jacobians(dse_batch* B, const double* cpk, int which = 0) {
  const dse::BatchArgs& a = B->args;
  if (B->fused) {
    BHIP_TRY(B, dse::launch_batch_fused(a, cpk, B->d_items, B->n_items, B->tpi, B->grid, B->d_counter, B->st,
                                        which));
    return DSE_OK;
  }
  BHIP_TRY(B, dse::launch_batch_dressing(a, cpk, which, B->d_counter, B->st));
  BHIP_TRY(B, dse::launch_batch_points(a, B->d_items, B->n_items, 1, B->grid, B->tpi, B->d_counter, B->st));
  BHIP_TRY(B, dse::launch_batch_contract(a, B->st));
  BHIP_TRY(B, dse::launch_batch_assemble(a, B->st));
  return DSE_OK;
}

// Largest cooperative grid of the fused form (0: not available).
int fused_grid(const dse_batch* B) {
  if (!B->coop) return 0;
  return dse::batch_fused_occupancy(B->args.max_nj) * B->ncu;
}

// with_flags: the pivot flags come back with the norms (one wait)
dse_status read_nrm(dse_batch* B, int which, std::vector<double>& out, std::vector<int>* flags = nullptr) {
  BHIP_TRY(B, dse::launch_batch_norms(B->args, which, B->d_nrm, B->st));
  out.resize(4 * (size_t)B->count);
  BHIP_TRY(B, hipMemcpyAsync(B->h_pin, B->d_nrm, out.size() * sizeof(double), hipMemcpyDeviceToHost, B->st));
  if (flags)
    BHIP_TRY(B, hipMemcpyAsync(B->h_pin_flags(), B->d_flags, B->count * sizeof(int), hipMemcpyDeviceToHost, B->st));
  BHIP_TRY(B, hipStreamSynchronize(B->st));
  memcpy(out.data(), B->h_pin, out.size() * sizeof(double));
  if (flags) {
    flags->resize(B->count);
    memcpy(flags->data(), B->h_pin_flags(), B->count * sizeof(int));
  }
  return DSE_OK;
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

size_t dse_batch_workspace_bytes(const dse_params* p, int32_t count) {
  if (!p || count < 1) return 0;
  char tmp[512];
  int cap = kSlicesCap;
  for (int b = 0; b < count; ++b) {
    if (dse::validate(&p[b], tmp) != DSE_OK || (p[b].quad & DSE_QUAD_SPLIT)) return 0;
    cap = std::min(cap, slices_cap(p[b]));
  }
  const Sizes s = sizes(p, count, cap);
  return s.ctl + s.per_total;
}

dse_status dse_batch_init(const dse_params* p, int32_t count, void* d_workspace, size_t ws_bytes,
                          void* hip_stream, dse_batch** out) {
  if (!out) { set_err(g_batch_err, "out is NULL"); return DSE_E_INVALID; }
  *out = nullptr;
  if (!p || count < 1) { set_err(g_batch_err, "need params and count >= 1"); return DSE_E_INVALID; }
  int cap = kSlicesCap;
  for (int b = 0; b < count; ++b) {
    char e[512];
    if (dse::validate(&p[b], e) != DSE_OK) {
      set_err(g_batch_err, "problem %d: %s", b, e);
      return DSE_E_INVALID;
    }
    if (p[b].precision != DSE_FP64) {
      set_err(g_batch_err, "problem %d: the batched family runs in FP64 (precision must be DSE_FP64)", b);
      return DSE_E_INVALID;
    }
    if (p[b].quad & DSE_QUAD_SPLIT) {
      set_err(g_batch_err, "problem %d: the batched family shares one radial grid per problem (no DSE_QUAD_SPLIT)", b);
      return DSE_E_INVALID;
    }
    cap = std::min(cap, slices_cap(p[b]));
  }
  if (!d_workspace || ((uintptr_t)d_workspace & 255u)) {
    set_err(g_batch_err, "workspace must be a non-NULL, 256-byte aligned device pointer");
    return DSE_E_INVALID;
  }
  const Sizes s = sizes(p, count, cap);
  if (ws_bytes < s.ctl + s.per_total) {
    set_err(g_batch_err, "workspace has %zu bytes, needs %zu", ws_bytes, s.ctl + s.per_total);
    return DSE_E_NOMEM;
  }
  dse_batch* B = new (std::nothrow) dse_batch();
  if (!B) { set_err(g_batch_err, "host allocation failed"); return DSE_E_INVALID; }
  B->count = count;
  B->p.assign(p, p + count);
  B->st = (hipStream_t)hip_stream;
  B->ws = (char*)d_workspace;
  B->ws_bytes = ws_bytes;
  B->ks_cap = cap;
  B->max_items = s.max_items;
  if (hipGetDevice(&B->device) != hipSuccess) {
    set_err(g_batch_err, "hipGetDevice failed");
    delete B;
    return DSE_E_DEVICE;
  }
  if (hipHostMalloc((void**)&B->h_pin, (size_t)count * (4 * sizeof(double) + sizeof(int)), hipHostMallocDefault) !=
      hipSuccess) {
    B->h_pin = nullptr;
    set_err(g_batch_err, "hipHostMalloc failed");
    delete B;
    return DSE_E_DEVICE;
  }
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, B->device) == hipSuccess && ncu > 0)
    B->ncu = ncu;
  int coop = 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, B->device) == hipSuccess) B->coop = coop;
  char* c = B->ws;
  B->d_desc = (dse::SolveDesc*)c; c += al(count * sizeof(dse::SolveDesc));
  B->d_items = (int4*)c; c += al((size_t)s.max_items * sizeof(int4));
  B->d_nrm = (double*)c; c += al(count * 4 * sizeof(double));
  B->d_flags = (int*)c; c += al(count * sizeof(int));
  B->d_mask = (int*)c; c += al(count * sizeof(int));
  B->d_rho = (double*)c; c += al(count * sizeof(double));
  B->d_counter = (int*)c; c += 256;
  B->desc.resize(count);
  B->coff.assign(count + 1, 0);
  B->joff.assign(count + 1, 0);
  for (int b = 0; b < count; ++b) {
    dse::SolveDesc& d = B->desc[b];
    memset(&d, 0, sizeof(d));
    dse::layout(p[b], &d.v, c, cap);
    c += s.per[b];
    d.ph = dse::make_phys(p[b]);
    d.coff = (int)B->coff[b];
    d.joff = (size_t)B->joff[b];
    B->coff[b + 1] = B->coff[b] + d.v.n;
    B->joff[b + 1] = B->joff[b] + (int64_t)d.v.n * d.v.n;
    const dse_status st = dse::upload_tables(p[b], d.v, d.ph, B->st, B->err);
    if (st != DSE_OK) {
      set_err(g_batch_err, "problem %d: %s", b, B->err);
      delete B;
      return st;
    }
  }
  dse::lu_setup();
  B->h_mask.assign(count, 1);
  B->h_rho.assign(count, 1.0);
  // default launch (before any tuning): no angular split, one workgroup per
  // item, largest first
  dse_status st = set_launch(B, 1, 0, 1);
  if (st == DSE_OK) st = upload_ctl(B);
  if (st == DSE_OK && hipStreamSynchronize(B->st) != hipSuccess) st = DSE_E_DEVICE;
  if (st != DSE_OK) {
    set_err(g_batch_err, "%s", B->err);
    delete B;
    return st;
  }
  *out = B;
  return DSE_OK;
}

dse_status dse_batch_destroy(dse_batch* B) {
  delete B;
  return DSE_OK;
}

const char* dse_batch_last_error(const dse_batch* B) { return B ? B->err : g_batch_err; }

dse_status dse_batch_offsets(const dse_batch* B, int64_t* h_coff, int64_t* h_joff) {
  if (!B) return DSE_E_INVALID;
  for (int b = 0; b <= B->count; ++b) {
    if (h_coff) h_coff[b] = B->coff[b];
    if (h_joff) h_joff[b] = B->joff[b];
  }
  return DSE_OK;
}

dse_status dse_batch_start_guess(dse_batch* B, double* d_c) {
  if (!B || !d_c) return DSE_E_INVALID;
  DevGuard dg(B->device);
  std::vector<double> c((size_t)B->coff[B->count]);
  for (int b = 0; b < B->count; ++b) dse::start_guess_host(B->p[b], B->desc[b].ph, c.data() + B->coff[b]);
  BHIP_TRY(B, hipMemcpyAsync(d_c, c.data(), c.size() * 8, hipMemcpyHostToDevice, B->st));
  BHIP_TRY(B, hipStreamSynchronize(B->st));
  return DSE_OK;
}

dse_status dse_batch_set_launch_ex(dse_batch* B, int32_t slices, int32_t persistent_blocks, int32_t order,
                                   int32_t tiles_per_item, int32_t fused) {
  if (!B) return DSE_E_INVALID;
  if (slices < 1 || slices > B->ks_cap || (slices & (slices - 1)) || persistent_blocks < 0 ||
      (order != 0 && order != 1) || tiles_per_item < 1 || tiles_per_item > 64 || (fused != 0 && fused != 1)) {
    set_err(B->err,
            "slices must be a power of two in [1, %d], persistent_blocks >= 0, order 0 or 1, "
            "tiles_per_item in [1, 64], fused 0 or 1",
            B->ks_cap);
    return DSE_E_INVALID;
  }
  DevGuard dg(B->device);
  if (fused) {
    const int cap = fused_grid(B);
    if (cap < 1) {
      set_err(B->err, "the device offers no cooperative launch for the fused assembly");
      return DSE_E_INVALID;
    }
    if (persistent_blocks < 1 || persistent_blocks > cap) {
      set_err(B->err, "fused: persistent_blocks must be in [1, %d] (all resident)", cap);
      return DSE_E_INVALID;
    }
  }
  return set_launch(B, slices, persistent_blocks, order, tiles_per_item, fused);
}

dse_status dse_batch_set_launch(dse_batch* B, int32_t slices, int32_t persistent_blocks, int32_t order) {
  return dse_batch_set_launch_ex(B, slices, persistent_blocks, order, 1, 0);
}

dse_status dse_batch_get_launch_ex(const dse_batch* B, int32_t* slices, int32_t* persistent_blocks, int32_t* order,
                                   int32_t* tiles_per_item, int32_t* fused) {
  if (!B) return DSE_E_INVALID;
  if (slices) *slices = B->slices;
  if (persistent_blocks) *persistent_blocks = B->grid;
  if (order) *order = B->order;
  if (tiles_per_item) *tiles_per_item = B->tpi;
  if (fused) *fused = B->fused;
  return DSE_OK;
}

dse_status dse_batch_get_launch(const dse_batch* B, int32_t* slices, int32_t* persistent_blocks, int32_t* order) {
  return dse_batch_get_launch_ex(B, slices, persistent_blocks, order, nullptr, nullptr);
}

dse_status dse_batch_jacobian(dse_batch* B, const double* d_c, double* d_J, double* d_F) {
  if (!B) return DSE_E_INVALID;
  if (!d_c || !d_J) { set_err(B->err, "d_c and d_J must not be NULL"); return DSE_E_INVALID; }
  DevGuard dg(B->device);
  std::fill(B->h_mask.begin(), B->h_mask.end(), 1);
  dse_status s = upload_ctl(B);
  if (s == DSE_OK) s = eval_jacobians(B, d_c);
  if (s != DSE_OK) return s;
  BHIP_TRY(B, dse::launch_batch_pack(B->args, d_J, d_F, B->st));
  BHIP_TRY(B, hipStreamSynchronize(B->st));
  return DSE_OK;
}

dse_status dse_batch_autotune(dse_batch* B, const double* d_c, dse_batch_tuning* rep) {
  if (!B || !d_c) return DSE_E_INVALID;
  DevGuard dg(B->device);
  std::fill(B->h_mask.begin(), B->h_mask.end(), 1);
  dse_status s = upload_ctl(B);
  if (s != DSE_OK) return s;
  hipEvent_t e0, e1;
  BHIP_TRY(B, hipEventCreate(&e0));
  BHIP_TRY(B, hipEventCreate(&e1));
  dse_batch_tuning r;
  memset(&r, 0, sizeof(r));
  double best = INFINITY;
  int bs = 1, bg = 0, bo = 1, bt = 1, bf = 0;
  const int occ = dse::batch_points_occupancy(1, B->args.max_nj);
  const int fgrid = fused_grid(B);
  // one candidate: the best of three timed assemblies after a warm-up
  auto time_one = [&](int ks, int grid, int ord, int tpi, int fu) -> dse_status {
    dse_status st = set_launch(B, ks, grid, ord, tpi, fu);
    if (st != DSE_OK) return st;
    double ms_best = INFINITY;
    for (int rep_ = 0; rep_ < 4; ++rep_) {
      if (hipEventRecord(e0, B->st) != hipSuccess) return DSE_E_DEVICE;
      if ((st = eval_jacobians(B, d_c)) != DSE_OK) return st;
      if (hipEventRecord(e1, B->st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return DSE_E_DEVICE;
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep_ > 0) ms_best = std::min(ms_best, (double)ms);  // the first run is a warm-up
    }
    if (r.n_candidates < 32) {
      const int i = r.n_candidates++;
      r.cand_slices[i] = ks;
      r.cand_blocks[i] = grid;
      r.cand_order[i] = ord;
      r.cand_ms[i] = ms_best;
      r.cand_tiles[i] = tpi;
      r.cand_fused[i] = fu;
    }
    if (ms_best < best) { best = ms_best; bs = ks; bg = grid; bo = ord; bt = tpi; bf = fu; }
    return DSE_OK;
  };
  // angular slices x launch form (one workgroup per item, persistent
  // workgroups, the fused cooperative launch) x partial tiles per item, queue
  // largest first; then problem order for the best of them
  for (int ks = 1; ks <= B->ks_cap && s == DSE_OK; ks *= 2)
    for (int form = 0; form < 3 && s == DSE_OK; ++form) {
      if (form == 2 && fgrid < 1) continue;
      const int grid = form == 0 ? 0 : (form == 1 ? occ * B->ncu : fgrid);
      for (int tpi = 1; tpi <= 4 && s == DSE_OK; tpi *= 2) s = time_one(ks, grid, 1, tpi, form == 2 ? 1 : 0);
    }
  if (s == DSE_OK) s = time_one(bs, bg, 0, bt, bf);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != DSE_OK) { set_err(B->err, "autotune: evaluation failed"); return s; }
  s = set_launch(B, bs, bg, bo, bt, bf);
  r.slices = bs;
  r.persistent_blocks = bg;
  r.order = bo;
  r.best_ms = best;
  r.tiles_per_item = bt;
  r.fused = bf;
  if (rep) *rep = r;
  return s;
}

// Newton iteration of every problem, each exactly as dse_newton_solve (same
// tests and relaxation), sharing launches: a Jacobian round for every problem
// still iterating, then line-search rounds for those still searching.
dse_status dse_batch_newton_solve(dse_batch* B, double* d_c, const dse_newton_opts* opts, dse_newton_report* reps) {
  if (!B) return DSE_E_INVALID;
  if (!d_c) { set_err(B->err, "d_c is NULL"); return DSE_E_INVALID; }
  DevGuard dg(B->device);
  const auto t0 = std::chrono::steady_clock::now();
  dse_newton_opts o;
  if (opts) {
    o = *opts;
  } else {
    o.tol = 1e-10; o.max_iter = 60; o.extra_iters = 0; o.max_halvings = 30; o.reserved_ = 0; o.step_tol = 1e-14;
  }
  if (!(o.tol > 0.0) || o.max_iter < 0 || o.extra_iters < 0 || o.max_halvings < 0) {
    set_err(B->err, "invalid Newton options");
    return DSE_E_INVALID;
  }
  const int N = B->count;
  std::vector<dse_newton_report> R(N);
  for (auto& r : R) memset(&r, 0, sizeof(r));
  std::vector<double> f(N), f2(N), nrm;
  std::vector<int> extra(N, 0), done(N, 0), conv(N, 0), searching(N, 0), accepted(N, 0);
  std::vector<dse_status> status(N, DSE_OK);
  // J, F, S at the start points: as in the single-problem solve, every
  // evaluation of an accepted point is an assembly, so the next iteration's
  // matrix comes with the residual that accepts it
  std::fill(B->h_mask.begin(), B->h_mask.end(), 1);
  std::fill(B->h_rho.begin(), B->h_rho.end(), 1.0);
  dse_status s = upload_ctl(B);
  if (s == DSE_OK) s = eval_jacobians(B, d_c);
  if (s == DSE_OK) s = read_nrm(B, 0, nrm);
  if (s != DSE_OK) return s;
  std::vector<int> have_J(N, 1);  // the workspace's J belongs to the member's current point
  for (int b = 0; b < N; ++b) {
    f[b] = nrm[4 * b];
    f2[b] = nrm[4 * b + 3];
    R[b].fnorm_hist[0] = f[b];
    R[b].fnorm2 = nrm[4 * b + 1];
    R[b].n_jacobians = 1;
    if (!isfinite(f[b])) { status[b] = DSE_E_NONFINITE; done[b] = 1; }
  }
  std::vector<double> ft(N, INFINITY), ft2(N, INFINITY), dinf(N, 0.0), fn2t(N, 0.0);
  std::vector<int> flags(N, 0);
  for (;;) {
    // which problems iterate this round
    int nact = 0;
    for (int b = 0; b < N; ++b) {
      B->h_mask[b] = 0;
      if (done[b]) continue;
      if (f[b] < o.tol) {
        if (extra[b] >= o.extra_iters) { done[b] = 1; continue; }
        ++extra[b];
      }
      if (R[b].iters >= o.max_iter) { status[b] = DSE_E_NOCONV; done[b] = 1; continue; }
      B->h_mask[b] = 1;
      conv[b] = f[b] < o.tol;
      B->h_rho[b] = 1.0;
      ++nact;
    }
    if (nact == 0) break;
    // the matrix at the current point, for the members whose last step was
    // relaxed (their workspace holds a trial's matrix)
    std::vector<int> act(B->h_mask);
    int nre = 0;
    for (int b = 0; b < N; ++b) {
      B->h_mask[b] = act[b] && !have_J[b];
      if (B->h_mask[b]) { ++nre; ++R[b].n_jacobians; }
    }
    if (nre > 0) {
      if ((s = upload_ctl(B)) != DSE_OK) return s;
      if ((s = eval_jacobians(B, d_c)) != DSE_OK) return s;
    }
    B->h_mask = act;
    if ((s = upload_ctl(B)) != DSE_OK) return s;
    BHIP_TRY(B, dse::launch_batch_lu(B->args, B->d_flags, B->st));
    for (int b = 0; b < N; ++b) {
      searching[b] = B->h_mask[b];
      accepted[b] = 0;
    }
    for (int h = 0;; ++h) {
      BHIP_TRY(B, dse::launch_batch_axpy(B->args, d_c, B->d_rho, B->st));
      if (h == 0) {
        // the full step in Jacobian mode: accepted, its matrix is the next one
        if ((s = eval_jacobians(B, nullptr, 1)) != DSE_OK) return s;
        if ((s = read_nrm(B, 2, nrm, &flags)) != DSE_OK) return s;
      } else {
        // relaxed steps in residual mode
        if ((s = eval_residuals(B, nullptr, 1)) != DSE_OK) return s;
        if ((s = read_nrm(B, 1, nrm)) != DSE_OK) return s;
      }
      int still = 0;
      for (int b = 0; b < N; ++b) {
        if (!searching[b]) continue;
        if (h == 0) {
          ++R[b].n_jacobians;
          have_J[b] = 1;
        } else {
          ++R[b].n_residuals;
          have_J[b] = 0;
        }
        if (h == 0 && flags[b] == DSE_E_SINGULAR) {
          status[b] = DSE_E_SINGULAR;
          done[b] = 1;
          searching[b] = 0;
          continue;
        }
        ft[b] = isfinite(nrm[4 * b]) ? nrm[4 * b] : INFINITY;
        ft2[b] = isfinite(nrm[4 * b]) && isfinite(nrm[4 * b + 3]) ? nrm[4 * b + 3] : INFINITY;
        fn2t[b] = nrm[4 * b + 1];
        dinf[b] = nrm[4 * b + 2];
        if (conv[b] || ft2[b] < f2[b] || h >= o.max_halvings) {
          searching[b] = 0;
          accepted[b] = 1;
        } else {
          B->h_rho[b] *= 0.5;
          ++still;
        }
      }
      if (still == 0) break;
      for (int b = 0; b < N; ++b) B->h_mask[b] = searching[b];
      if ((s = upload_ctl(B)) != DSE_OK) return s;
    }
    // take the accepted steps (mask 2: the full step, whose F and S the
    // Jacobian-mode assembly wrote in place; 1: a relaxed one)
    for (int b = 0; b < N; ++b) {
      B->h_mask[b] = 0;
      if (!accepted[b]) continue;
      if (!isfinite(ft[b])) { status[b] = DSE_E_NONFINITE; done[b] = 1; continue; }
      B->h_mask[b] = have_J[b] ? 2 : 1;
    }
    if ((s = upload_ctl(B)) != DSE_OK) return s;
    BHIP_TRY(B, dse::launch_batch_accept(B->args, d_c, B->st));
    BHIP_TRY(B, hipStreamSynchronize(B->st));
    for (int b = 0; b < N; ++b) {
      if (!B->h_mask[b]) continue;
      dse_newton_report& r = R[b];
      f[b] = ft[b];
      f2[b] = ft2[b];
      const int it = ++r.iters;
      if (it < 128) { r.fnorm_hist[it] = f[b]; r.relax_hist[it - 1] = B->h_rho[b]; }
      r.fnorm2 = fn2t[b];
      if (conv[b] && B->h_rho[b] * dinf[b] < o.step_tol) done[b] = 1;
    }
  }
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  dse_status worst = DSE_OK;
  int nbad = 0;
  for (int b = 0; b < N; ++b) {
    R[b].status = status[b];
    R[b].fnorm = f[b];
    R[b].t_total_ms = ms;
    if (status[b] != DSE_OK) {
      ++nbad;
      if (worst == DSE_OK) worst = status[b];
    }
  }
  if (reps) memcpy(reps, R.data(), N * sizeof(dse_newton_report));
  if (nbad) set_err(B->err, "%d of %d problems did not converge (first status %d)", nbad, N, (int)worst);
  return worst;
}

}  // extern "C"
