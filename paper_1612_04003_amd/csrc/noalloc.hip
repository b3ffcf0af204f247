// cabcd_gram_noalloc: the gathered-row Gram of cabcd_gram for callers that
// cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc).  Its split-K partial Grams and the
// checked copy of the indices live in one fixed device array of this file;
// the call allocates nothing, copies nothing to the host and never
// synchronises.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "internal.h"

namespace cabcd {
namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;   // per GPU, held until process exit
constexpr size_t kHeadBytes = 2048;                  // checked indices (<= 256 int32)
constexpr size_t kScratchDoubles = kScratchBytes / sizeof(double);
constexpr size_t kPartialDoubles = (kScratchBytes - kHeadBytes) / sizeof(double);
constexpr int kMaxRows = 256;
constexpr int kMaxDevices = 64;

// The scratch of every cabcd_gram_noalloc call on a GPU (each GPU holds its
// own copy).  Host code never passes this name to a kernel: it stands for a
// host-side shadow there; the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};   // device address of `scratch`, per device

// Looks the array's device address up once per device, with that device current.
cabcd_status scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    set_error("cabcd_gram_noalloc: hipGetDevice failed");
    return CABCD_EHIP;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("cabcd_gram_noalloc: device %d beyond the supported %d", dev, kMaxDevices);
    return CABCD_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[dev] == nullptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      set_error("cabcd_gram_noalloc: hipGetSymbolAddress of the scratch array failed: %s",
                hipGetErrorString(e));
      return CABCD_EHIP;
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return CABCD_OK;
}

// Copies idx[0..m) into `out` with every index outside [0, rows) replaced by
// row 0, and writes CABCD_EINVAL or CABCD_OK to *status.  One workgroup of
// kMaxRows threads (m <= kMaxRows).
__global__ __launch_bounds__(kMaxRows) void check_idx_kernel(const int32_t* __restrict__ idx,
                                                             int m, int64_t rows,
                                                             int32_t* __restrict__ out,
                                                             int32_t* __restrict__ status) {
  const int t = threadIdx.x;
  int bad = 0;
  if (t < m) {
    const int32_t v = idx[t];
    bad = (v < 0 || (int64_t)v >= rows) ? 1 : 0;
    out[t] = bad ? 0 : v;
  }
  bad = __syncthreads_or(bad);
  if (t == 0 && status != nullptr) *status = bad ? CABCD_EINVAL : CABCD_OK;
}

// The Gram plan with its partials cut to fit the scratch: the column slabs
// are widened (chunk doubled, so it stays a multiple of the tile width) until
// the partial sets fit.
GramPlan fit_plan(GramPlan p, int64_t cols) {
  while (gram_partial_doubles(p) > kPartialDoubles && p.nsplit > 1) {
    p.chunk *= 2;
    p.nsplit = (int)((cols + p.chunk - 1) / p.chunk);
  }
  return p;
}

}  // namespace
}  // namespace cabcd

using namespace cabcd;

extern "C" cabcd_status cabcd_gram_noalloc(const cabcd_matrix* A, const int32_t* idx,
                                           int32_t m, double scale, double shift,
                                           const double* u, double* G, double* Yu,
                                           int32_t* status, void* stream) {
  clear_error();
  if (A == nullptr || idx == nullptr || G == nullptr) {
    set_error("cabcd_gram_noalloc: A, idx and G must be non-NULL");
    return CABCD_EINVAL;
  }
  if (A->kind != CABCD_DENSE) {
    set_error("cabcd_gram_noalloc: dense matrices only (CSR needs a structure check that "
              "synchronises; use cabcd_gram)");
    return CABCD_EUNSUPPORTED;
  }
  if (A->dtype != CABCD_F64 && A->dtype != CABCD_BF16 && A->dtype != CABCD_FP8_E4M3) {
    set_error("cabcd_gram_noalloc: unknown dtype %d", A->dtype);
    return CABCD_EINVAL;
  }
  if (A->rows < 1 || A->cols < 1 || A->rows > INT32_MAX || A->cols > INT32_MAX ||
      A->data == nullptr || A->ld < A->cols) {
    set_error("cabcd_gram_noalloc: need 1 <= rows, cols < 2^31, non-NULL data and ld >= cols");
    return CABCD_EINVAL;
  }
  if (m < 1) {
    set_error("cabcd_gram_noalloc: need m >= 1");
    return CABCD_EINVAL;
  }
  if (m > kMaxRows) {
    set_error("cabcd_gram_noalloc: m = %d exceeds the maximum %d of the fixed scratch", m,
              kMaxRows);
    return CABCD_EUNSUPPORTED;
  }
  void* base = nullptr;
  cabcd_status rc = scratch_address(&base);
  if (rc != CABCD_OK) return rc;
  int32_t* idx_ok = static_cast<int32_t*>(base);
  double* partials = reinterpret_cast<double*>(static_cast<char*>(base) + kHeadBytes);
  hipStream_t st = static_cast<hipStream_t>(stream);

  hipLaunchKernelGGL(check_idx_kernel, dim3(1), dim3(kMaxRows), 0, st, idx, m, A->rows, idx_ok,
                     status);
  hipError_t e = hipGetLastError();
  const bool want_u = u != nullptr && Yu != nullptr;
  if (e == hipSuccess) {
    if (A->dtype == CABCD_F64) {
      const double* X = static_cast<const double*>(A->data);
      const GramPlan plan = fit_plan(plan_gram_f64(m, A->cols), A->cols);
      e = launch_gram_f64(plan, X, A->ld, A->cols, idx_ok, m, want_u ? u : nullptr, partials, st);
      if (e == hipSuccess)
        e = launch_gram_reduce(plan, partials, idx_ok, m, scale, shift, false, G,
                               want_u ? Yu : nullptr, st);
    } else {
      const GramPlan plan = fit_plan(plan_gram_lp(m, A->cols, A->dtype), A->cols);
      e = launch_gram_lp(plan, A->dtype, A->data, A->ld, A->cols, idx_ok, m,
                         want_u ? u : nullptr, partials, st);
      if (e == hipSuccess)
        e = launch_gram_reduce(plan, partials, idx_ok, m, scale, shift, false, G,
                               want_u ? Yu : nullptr, st,
                               gram_lp_partial_layout(plan, A->dtype, A->data, A->ld),
                               A->row_scale);
    }
  }
  if (e != hipSuccess) {
    set_error("cabcd_gram_noalloc: kernel launch failed: %s", hipGetErrorString(e));
    return CABCD_EHIP;
  }
  return CABCD_OK;
}
