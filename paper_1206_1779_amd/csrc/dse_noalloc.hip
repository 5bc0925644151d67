// dse_noalloc.hip -- the dense LU solve of the Newton step for callers that
// cannot allocate device memory (code under stream capture, tight serving
// loops, harnesses that forbid hipMalloc).  Its scratch -- the padded factors
// of [A | b] when they do not fit in LDS, the pivot rows, the status word and
// the largest entry of each row (for the relative pivot test) --
// lives in one static device array per GPU, held until the process ends.

#include <hip/hip_runtime.h>

#include <mutex>

#include "dse_impl.h"

namespace {

constexpr int kMaxN = 2 * DSE_MAX_N;  // largest n = n_z + n_g of a problem
constexpr int kLuNB = 16;             // the factorisation pads n to a multiple of its panel width
constexpr size_t kLuBytes =
    (size_t)((kMaxN + kLuNB - 1) / kLuNB * kLuNB) * ((kMaxN + kLuNB - 1) / kLuNB * kLuNB + 1) * sizeof(double);
constexpr size_t kPivOff = (kLuBytes + 255) / 256 * 256;
constexpr size_t kFlagOff = kPivOff + (kMaxN * sizeof(int32_t) + 255) / 256 * 256;
constexpr size_t kRowOff = kFlagOff + 256;
constexpr size_t kScratchBytes = kRowOff + kMaxN * sizeof(double);
constexpr int kMaxDevices = 64;

}  // namespace

// 517.25 KiB per GPU.  In host code this name is only a handle for
// hipGetSymbolAddress: the device address comes from that call.
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
char* g_scratch[kMaxDevices];  // device address of `scratch` on each GPU

// Device address of the current GPU's scratch array (looked up once per GPU,
// with that GPU current).
dse_status scratch_ptr(char** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    dse::set_err(dse::global_err(), "no usable current device");
    return DSE_E_DEVICE;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      dse::set_err(dse::global_err(), "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
      return DSE_E_DEVICE;
    }
    g_scratch[dev] = (char*)p;
  }
  *out = g_scratch[dev];
  return DSE_OK;
}

}  // namespace

extern "C" dse_status dse_lu_solve_noalloc(int32_t n, const double* d_J, const double* d_b, double* d_x,
                                           int32_t trans, int32_t* d_info, void* hip_stream) {
  if (n < 1 || n > kMaxN) {
    dse::set_err(dse::global_err(), "n = %d: dse_lu_solve_noalloc handles 1 <= n <= %d", n, kMaxN);
    return DSE_E_INVALID;
  }
  if (!d_J || !d_b || !d_x) {
    dse::set_err(dse::global_err(), "d_J, d_b and d_x must not be NULL");
    return DSE_E_INVALID;
  }
  char* base = nullptr;
  const dse_status s = scratch_ptr(&base);
  if (s != DSE_OK) return s;
  // the factorisation kernel only reads the size and these three buffers
  dse::Views v{};
  v.n = n;
  v.LU = (double*)base;
  v.piv = (int32_t*)(base + kPivOff);
  v.flag = d_info ? d_info : (int32_t*)(base + kFlagOff);
  double* rowmax = (double*)(base + kRowOff);
  hipError_t e = dse::launch_row_absmax(n, d_J, rowmax, (hipStream_t)hip_stream);
  if (e == hipSuccess)
    e = dse::launch_lu_solve(v, d_J, d_b, d_x, trans, (hipStream_t)hip_stream, nullptr, 0.0, nullptr, rowmax);
  if (e != hipSuccess) {
    dse::set_err(dse::global_err(), "LU launch: %s", hipGetErrorString(e));
    return DSE_E_DEVICE;
  }
  return DSE_OK;
}
