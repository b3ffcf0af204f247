// C-ABI of libcabcd: argument checking, workspace, and the outer-step drivers
// of CA-BCD (Alg. 2) and CA-BDCD (Alg. 4).  Everything numeric runs in the HIP
// kernels of this library; this file only validates, plans and enqueues.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace cabcd {

namespace {
thread_local std::string g_err;
}

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

void clear_error() { g_err.clear(); }

namespace {

constexpr int kMaxSB = 256;       // s*b handled by one Gram launch and one solve
constexpr int kMaxB = 32;         // block size handled by the fused solve
constexpr int64_t kIdxChunkSteps = 4096;   // outer steps whose indices are drawn at once

__global__ void set_int_kernel(int* p, int v) { *p = v; }

// ----------------------------------------------------------------- workspace
struct Pool {
  void* ptr = nullptr;
  size_t cap = 0;
};
std::mutex g_pool_mu;
std::vector<Pool> g_pools;

cabcd_status pool_get(size_t bytes, void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    set_error("hipGetDevice failed");
    return CABCD_EHIP;
  }
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if ((int)g_pools.size() <= dev) g_pools.resize(dev + 1);
  Pool& p = g_pools[dev];
  if (p.cap < bytes) {
    if (p.ptr != nullptr) {
      (void)hipDeviceSynchronize();
      (void)hipFree(p.ptr);
      p.ptr = nullptr;
      p.cap = 0;
    }
    size_t want = std::max(bytes, (size_t)1 << 20);
    if (hipMalloc(&p.ptr, want) != hipSuccess) {
      p.ptr = nullptr;
      set_error("hipMalloc of %zu workspace bytes failed", want);
      return CABCD_ENOMEM;
    }
    p.cap = want;
  }
  *out = p.ptr;
  return CABCD_OK;
}

// Bump allocator over one workspace block (256-byte aligned pieces).
struct Carve {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
    off += count * sizeof(T);
    return p;
  }
};

#define HIP_TRY(expr)                                                         \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess) {                                                   \
      set_error("%s failed: %s", #expr, hipGetErrorString(e_));               \
      return CABCD_EHIP;                                                      \
    }                                                                         \
  } while (0)

cabcd_status check_dense(const cabcd_matrix* A, const char* name) {
  if (A == nullptr) {
    set_error("%s is NULL", name);
    return CABCD_EINVAL;
  }
  if (A->rows < 1 || A->cols < 1) {
    set_error("%s must have rows >= 1 and cols >= 1 (got %lld x %lld)", name,
              (long long)A->rows, (long long)A->cols);
    return CABCD_EINVAL;
  }
  if (A->kind != CABCD_DENSE && A->kind != CABCD_CSR) {
    set_error("%s: unknown kind %d", name, A->kind);
    return CABCD_EINVAL;
  }
  if (A->kind == CABCD_CSR) {
    set_error("%s: CSR storage is not supported by this entry point yet", name);
    return CABCD_EUNSUPPORTED;
  }
  if (A->dtype != CABCD_F64) {
    if (A->dtype == CABCD_BF16 || A->dtype == CABCD_FP8_E4M3) {
      set_error("%s: low-precision storage is not supported by this entry point yet", name);
      return CABCD_EUNSUPPORTED;
    }
    set_error("%s: unknown dtype %d", name, A->dtype);
    return CABCD_EINVAL;
  }
  if (A->data == nullptr || A->ld < A->cols) {
    set_error("%s: data is NULL or ld (%lld) < cols (%lld)", name, (long long)A->ld,
              (long long)A->cols);
    return CABCD_EINVAL;
  }
  if (A->rows > INT32_MAX) {
    set_error("%s: more than 2^31-1 rows", name);
    return CABCD_EINVAL;
  }
  return CABCD_OK;
}

cabcd_status finish(hipStream_t st, int* status_dev, bool async) {
  if (async) return CABCD_OK;
  int h = 0;
  HIP_TRY(hipMemcpyAsync(&h, status_dev, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (h == DEV_NOTSPD) {
    set_error("a b x b diagonal block of the Gram was not positive definite");
    return CABCD_ENOTSPD;
  }
  if (h == DEV_NONFINITE) {
    set_error("a non-finite value appeared in the iterates or the objective");
    return CABCD_ENONFINITE;
  }
  return CABCD_OK;
}

// Host-side validation of caller indices (copied back once; explicit index
// lists are a testing and replay feature).
cabcd_status check_explicit(const int32_t* idx_dev, int64_t H, int b, int64_t range,
                            hipStream_t st) {
  if (H == 0) return CABCD_OK;
  std::vector<int32_t> h((size_t)(H * b));
  HIP_TRY(hipMemcpyAsync(h.data(), idx_dev, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                         st));
  HIP_TRY(hipStreamSynchronize(st));
  for (int64_t i = 0; i < H; ++i) {
    const int32_t* blk = h.data() + i * b;
    for (int u = 0; u < b; ++u) {
      if (blk[u] < 0 || blk[u] >= range) {
        set_error("explicit_idx[%lld] = %d outside [0, %lld)", (long long)(i * b + u), blk[u],
                  (long long)range);
        return CABCD_EINVAL;
      }
      for (int v = 0; v < u; ++v)
        if (blk[v] == blk[u]) {
          set_error("explicit_idx block %lld repeats index %d", (long long)i, blk[u]);
          return CABCD_EINVAL;
        }
    }
  }
  return CABCD_OK;
}

// Optional per-phase timing with HIP events on the call's stream.
class PhaseTimer {
 public:
  PhaseTimer(double* out, hipStream_t st) : out_(out), st_(st) {}
  ~PhaseTimer() {
    for (auto& r : recs_) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
  }
  template <class F>
  hipError_t run(int phase, F&& f) {
    if (out_ == nullptr) return f();
    Rec r{phase, nullptr, nullptr};
    hipError_t e = hipEventCreate(&r.a);
    if (e == hipSuccess) e = hipEventCreate(&r.b);
    if (e != hipSuccess) return e;
    recs_.push_back(r);
    e = hipEventRecord(r.a, st_);
    if (e != hipSuccess) return e;
    e = f();
    if (e != hipSuccess) return e;
    return hipEventRecord(r.b, st_);
  }
  // Call after the stream has been synchronised.
  hipError_t collect() {
    if (out_ == nullptr) return hipSuccess;
    for (auto& r : recs_) {
      float ms = 0.f;
      hipError_t e = hipEventElapsedTime(&ms, r.a, r.b);
      if (e != hipSuccess) return e;
      out_[r.phase] += ms;
      out_[CABCD_NPHASES + r.phase] += 1.0;
    }
    return hipSuccess;
  }

 private:
  struct Rec {
    int phase;
    hipEvent_t a, b;
  };
  double* out_;
  hipStream_t st_;
  std::vector<Rec> recs_;
};

struct StepBuffers {
  int* status;
  int32_t* idx;      // kIdxChunkSteps * s * b
  double* G;         // sb x sb
  double* Yu;        // sb
  double* delta;     // sb
  double* partials;  // Gram partials
  double* scratch;   // gemv row-group partials
  double* obj;       // objective scratch
  double* fval;      // 1 double
  double* rtmp;      // companion-length temporary (monitoring)
};

size_t max_partials(int sb_max, int64_t cols) {
  size_t best = 0;
  for (int m = 1; m <= sb_max; m = (m < 16 ? 16 : m * 2)) {
    GramPlan p = plan_gram_f64(std::min(m, sb_max), cols);
    best = std::max(best, gram_partial_doubles(p));
    if (m >= sb_max) break;
  }
  GramPlan p = plan_gram_f64(sb_max, cols);
  return std::max(best, gram_partial_doubles(p));
}

// Layout of the step workspace.  rows/cols are those of A; comp_len is the
// length of the companion vector (cols for both methods); rtmp_len the length
// of the monitoring temporary.
size_t layout(Carve& c, StepBuffers& B, int64_t rows, int64_t cols, int b, int s,
              int64_t rtmp_len) {
  const int sb = s * b;
  B.status = c.take<int>(1);
  B.idx = c.take<int32_t>((size_t)kIdxChunkSteps * sb);
  B.G = c.take<double>((size_t)sb * sb);
  B.Yu = c.take<double>(sb);
  B.delta = c.take<double>(sb);
  B.partials = c.take<double>(max_partials(sb, cols));
  const size_t sc = std::max(gemv_t_scratch_doubles(sb, cols),
                             std::max(gemv_t_scratch_doubles(rows, cols), (size_t)1));
  B.scratch = c.take<double>(sc);
  B.obj = c.take<double>(objective_scratch_doubles(0, 0));
  B.fval = c.take<double>(1);
  B.rtmp = c.take<double>(std::max<int64_t>(rtmp_len, 1));
  return c.off + 256;
}

cabcd_status get_workspace(const cabcd_opts* o, size_t need, void** ws) {
  if (o != nullptr && o->workspace != nullptr) {
    if (o->workspace_bytes < need) {
      set_error("workspace of %zu bytes is smaller than the %zu needed", o->workspace_bytes,
                need);
      return CABCD_ENOMEM;
    }
    *ws = o->workspace;
    return CABCD_OK;
  }
  return pool_get(need, ws);
}

cabcd_status check_common(const cabcd_matrix* A, double lambda, int b, int s, int64_t H,
                          int64_t range) {
  if (!(lambda > 0.0) || !std::isfinite(lambda)) {
    set_error("lambda must be a positive finite number (got %g)", lambda);
    return CABCD_EINVAL;
  }
  if (b < 1 || (int64_t)b > range) {
    set_error("block size b = %d must satisfy 1 <= b <= %lld", b, (long long)range);
    return CABCD_EINVAL;
  }
  if (s < 1) {
    set_error("s = %d must be >= 1", s);
    return CABCD_EINVAL;
  }
  if (H < 0) {
    set_error("H = %lld must be >= 0", (long long)H);
    return CABCD_EINVAL;
  }
  if (b > kMaxB) {
    set_error("block size b = %d exceeds the supported maximum %d", b, kMaxB);
    return CABCD_EUNSUPPORTED;
  }
  if ((int64_t)s * b > kMaxSB) {
    set_error("s*b = %lld exceeds the supported maximum %d", (long long)s * b, kMaxSB);
    return CABCD_EUNSUPPORTED;
  }
  (void)A;
  return CABCD_OK;
}

// One driver for both methods (they differ in the scalars and the role of the
// vectors, see the fused solve).  primal: coord = w (d), comp = r (n).
// dual: coord = alpha (n), comp = w (d).
cabcd_status run_bcd(bool dual, const cabcd_matrix* A, const double* y, double lambda, int b,
                     int s, int64_t H, uint64_t seed, double* coord, double* comp,
                     const cabcd_opts* opts, hipStream_t st) {
  cabcd_opts o;
  cabcd_opts_init(&o);
  if (opts != nullptr) o = *opts;
  const int64_t rows = A->rows, cols = A->cols;
  const double n = dual ? (double)rows : (double)cols;
  const double* X = static_cast<const double*>(A->data);
  const int64_t ld = A->ld;
  if (y == nullptr || coord == nullptr || comp == nullptr) {
    set_error("y, the coordinate vector and the companion vector must be non-NULL");
    return CABCD_EINVAL;
  }
  if (o.h0 < 0) {
    set_error("opts.h0 must be >= 0");
    return CABCD_EINVAL;
  }
  if (o.monitor_every > 0 && (o.trace == nullptr || o.trace_len < 0)) {
    set_error("monitor_every > 0 needs a trace buffer");
    return CABCD_EINVAL;
  }
  if (o.resid_every < 0 || o.monitor_every < 0) {
    set_error("resid_every and monitor_every must be >= 0");
    return CABCD_EINVAL;
  }
  if (o.explicit_idx != nullptr) {
    cabcd_status e = check_explicit(o.explicit_idx, H, b, rows, st);
    if (e != CABCD_OK) return e;
  }
  // monitoring needs the residual of length n (primal: cols, dual: rows)
  const int64_t rtmp_len = o.monitor_every > 0 ? (dual ? rows : cols) : 1;
  StepBuffers B{};
  Carve probe{nullptr};
  const size_t need = layout(probe, B, rows, cols, b, s, rtmp_len);
  void* ws = nullptr;
  cabcd_status e = get_workspace(&o, need, &ws);
  if (e != CABCD_OK) return e;
  Carve carve{static_cast<char*>(ws)};
  layout(carve, B, rows, cols, b, s, rtmp_len);

  hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, st, B.status, 0);
  HIP_TRY(hipGetLastError());

  const double scale = dual ? 1.0 / (lambda * n * n) : 1.0 / n;
  const double shift = dual ? 1.0 / n : lambda;
  const double gamma = dual ? -1.0 / (lambda * n) : 1.0;

  auto exact_companion = [&]() -> hipError_t {
    if (dual)   // w = -X alpha / (lambda n)
      return launch_gemv_t(X, ld, cols, nullptr, rows, coord, -1.0 / (lambda * n), nullptr,
                           0.0, false, comp, B.scratch, st);
    // r = X^T w - y
    return launch_gemv_t(X, ld, cols, nullptr, rows, coord, 1.0, y, -1.0, false, comp,
                         B.scratch, st);
  };
  auto monitor = [&](int64_t slot) -> hipError_t {
    hipError_t he;
    if (dual) {   // f(w) with r = X^T w - y computed from the X^T layout
      he = launch_gemv_n(X, ld, rows, cols, comp, y, -1.0, B.rtmp, st);
      if (he != hipSuccess) return he;
      return launch_objective(B.rtmp, rows, 0.5 / n, comp, cols, 0.5 * lambda, o.trace + slot,
                              B.obj, B.status, st);
    }
    he = launch_gemv_t(X, ld, cols, nullptr, rows, coord, 1.0, y, -1.0, false, B.rtmp,
                       B.scratch, st);
    if (he != hipSuccess) return he;
    return launch_objective(B.rtmp, cols, 0.5 / n, coord, rows, 0.5 * lambda, o.trace + slot,
                            B.obj, B.status, st);
  };

  if (o.timing != nullptr && (o.flags & CABCD_FLAG_ASYNC)) {
    set_error("opts.timing needs a synchronising call");
    return CABCD_EINVAL;
  }
  PhaseTimer timer(o.timing, st);
  if (!(o.flags & CABCD_FLAG_STATE_VALID))
    HIP_TRY(timer.run(CABCD_PHASE_RECOMPUTE, exact_companion));

  int64_t h = 0, k = 0, slot = 0;
  int64_t chunk_begin = -1, chunk_end = -1;
  const int64_t chunk_iters = kIdxChunkSteps * (int64_t)s;
  while (h < H) {
    const int sk = (int)std::min<int64_t>(s, H - h);
    const int m = sk * b;
    const int32_t* idx;
    if (o.explicit_idx != nullptr) {
      idx = o.explicit_idx + h * b;
    } else {
      if (h >= chunk_end) {
        chunk_begin = h;
        chunk_end = std::min(H, h + chunk_iters);
        HIP_TRY(timer.run(CABCD_PHASE_SAMPLE, [&] {
          return launch_sample(seed, o.h0 + chunk_begin, chunk_end - chunk_begin, b, rows, B.idx,
                               st);
        }));
      }
      idx = B.idx + (h - chunk_begin) * b;
    }
    const GramPlan plan = plan_gram_f64(m, cols);
    HIP_TRY(timer.run(CABCD_PHASE_GRAM, [&] {
      return launch_gram_f64(plan, X, ld, cols, idx, m, comp, B.partials, st);
    }));
    HIP_TRY(timer.run(CABCD_PHASE_REDUCE, [&] {
      return launch_gram_reduce(plan, B.partials, idx, m, scale, shift, true, B.G, B.Yu, st);
    }));
    SolveArgs sa{};
    sa.G = B.G;
    sa.Yu = B.Yu;
    sa.idx = idx;
    sa.y = y;
    sa.x = coord;
    sa.delta = B.delta;
    sa.status = B.status;
    sa.m = m;
    sa.b = b;
    sa.s = sk;
    sa.mode = dual ? 1 : 0;
    sa.lambda = lambda;
    sa.n = n;
    HIP_TRY(timer.run(CABCD_PHASE_SOLVE, [&] { return launch_solve(sa, st); }));
    HIP_TRY(timer.run(CABCD_PHASE_UPDATE, [&] {
      return launch_gemv_t(X, ld, cols, idx, m, B.delta, gamma, nullptr, 0.0, true, comp,
                           B.scratch, st);
    }));
    h += sk;
    ++k;
    if (o.resid_every > 0 && k % o.resid_every == 0)
      HIP_TRY(timer.run(CABCD_PHASE_RECOMPUTE, exact_companion));
    if (o.monitor_every > 0 && k % o.monitor_every == 0 && slot < o.trace_len) {
      const int64_t sl = slot++;
      HIP_TRY(timer.run(CABCD_PHASE_MONITOR, [&] { return monitor(sl); }));
    }
  }
  const cabcd_status fs = finish(st, B.status, (o.flags & CABCD_FLAG_ASYNC) != 0);
  HIP_TRY(timer.collect());
  return fs;
}

}  // namespace
}  // namespace cabcd

using namespace cabcd;

extern "C" {

void cabcd_opts_init(cabcd_opts* o) {
  if (o == nullptr) return;
  std::memset(o, 0, sizeof *o);
}

const char* cabcd_last_error(void) { return g_err.c_str(); }

const char* cabcd_version(void) { return "cabcd 0.1 (gfx950)"; }

cabcd_status cabcd_sample(uint64_t seed, int64_t h0, int64_t count, int32_t b, int64_t range,
                          int32_t* idx, void* stream) {
  clear_error();
  if (count < 0 || h0 < 0 || b < 1 || range < b || range > INT32_MAX ||
      (count > 0 && idx == nullptr)) {
    set_error("cabcd_sample: need count >= 0, h0 >= 0, 1 <= b <= range <= 2^31-1, idx != NULL");
    return CABCD_EINVAL;
  }
  HIP_TRY(launch_sample(seed, h0, count, b, range, idx, (hipStream_t)stream));
  return CABCD_OK;
}

cabcd_status cabcd_gram(const cabcd_matrix* A, const int32_t* idx, int32_t m, double scale,
                        double shift, const double* u, double* G, double* Yu, void* stream) {
  clear_error();
  cabcd_status e = check_dense(A, "A");
  if (e != CABCD_OK) return e;
  if (m < 1 || idx == nullptr || G == nullptr) {
    set_error("cabcd_gram: need m >= 1 and non-NULL idx and G");
    return CABCD_EINVAL;
  }
  if (m > kMaxSB) {
    set_error("cabcd_gram: m = %d exceeds the supported maximum %d", m, kMaxSB);
    return CABCD_EUNSUPPORTED;
  }
  hipStream_t st = (hipStream_t)stream;
  {
    std::vector<int32_t> h(m);
    HIP_TRY(hipMemcpyAsync(h.data(), idx, m * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int i = 0; i < m; ++i)
      if (h[i] < 0 || h[i] >= A->rows) {
        set_error("cabcd_gram: idx[%d] = %d outside [0, %lld)", i, h[i], (long long)A->rows);
        return CABCD_EINVAL;
      }
  }
  const GramPlan plan = plan_gram_f64(m, A->cols);
  void* ws = nullptr;
  e = pool_get(gram_partial_doubles(plan) * sizeof(double), &ws);
  if (e != CABCD_OK) return e;
  double* part = static_cast<double*>(ws);
  const bool want_u = u != nullptr && Yu != nullptr;
  HIP_TRY(launch_gram_f64(plan, static_cast<const double*>(A->data), A->ld, A->cols, idx, m,
                          want_u ? u : nullptr, part, st));
  HIP_TRY(launch_gram_reduce(plan, part, idx, m, scale, shift, false, G, want_u ? Yu : nullptr,
                             st));
  HIP_TRY(hipStreamSynchronize(st));
  return CABCD_OK;
}

cabcd_status cabcd_primal_bcd(const cabcd_matrix* X, const double* y, double lambda, int32_t b,
                              int32_t s, int64_t H, uint64_t seed, double* w, double* r,
                              const cabcd_opts* opts, void* stream) {
  clear_error();
  cabcd_status e = check_dense(X, "X");
  if (e != CABCD_OK) return e;
  e = check_common(X, lambda, b, s, H, X->rows);
  if (e != CABCD_OK) return e;
  return run_bcd(false, X, y, lambda, b, s, H, seed, w, r, opts, (hipStream_t)stream);
}

cabcd_status cabcd_dual_bcd(const cabcd_matrix* XT, const double* y, double lambda, int32_t b,
                            int32_t s, int64_t H, uint64_t seed, double* alpha, double* w,
                            const cabcd_opts* opts, void* stream) {
  clear_error();
  cabcd_status e = check_dense(XT, "XT");
  if (e != CABCD_OK) return e;
  e = check_common(XT, lambda, b, s, H, XT->rows);
  if (e != CABCD_OK) return e;
  return run_bcd(true, XT, y, lambda, b, s, H, seed, alpha, w, opts, (hipStream_t)stream);
}

cabcd_status cabcd_primal_objective(const cabcd_matrix* X, const double* y, double lambda,
                                    const double* w, double* r, double* f, void* stream) {
  clear_error();
  cabcd_status e = check_dense(X, "X");
  if (e != CABCD_OK) return e;
  if (y == nullptr || w == nullptr || !(lambda >= 0.0)) {
    set_error("cabcd_primal_objective: y and w must be non-NULL and lambda >= 0");
    return CABCD_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  Carve probe{nullptr};
  double* rt = probe.take<double>(X->cols);
  double* sc = probe.take<double>(std::max<size_t>(gemv_t_scratch_doubles(X->rows, X->cols), 1));
  double* ob = probe.take<double>(objective_scratch_doubles(0, 0));
  void* ws = nullptr;
  e = pool_get(probe.off + 256, &ws);
  if (e != CABCD_OK) return e;
  Carve c{static_cast<char*>(ws)};
  rt = c.take<double>(X->cols);
  sc = c.take<double>(std::max<size_t>(gemv_t_scratch_doubles(X->rows, X->cols), 1));
  ob = c.take<double>(objective_scratch_doubles(0, 0));
  double* rr = r != nullptr ? r : rt;
  const double* A = static_cast<const double*>(X->data);
  HIP_TRY(launch_gemv_t(A, X->ld, X->cols, nullptr, X->rows, w, 1.0, y, -1.0, false, rr, sc, st));
  if (f != nullptr)
    HIP_TRY(launch_objective(rr, X->cols, 0.5 / (double)X->cols, w, X->rows, 0.5 * lambda, f, ob,
                             nullptr, st));
  HIP_TRY(hipStreamSynchronize(st));
  return CABCD_OK;
}

cabcd_status cabcd_primal_objective_t(const cabcd_matrix* XT, const double* y, double lambda,
                                      const double* w, double* r, double* f, void* stream) {
  clear_error();
  cabcd_status e = check_dense(XT, "XT");
  if (e != CABCD_OK) return e;
  if (y == nullptr || w == nullptr || !(lambda >= 0.0)) {
    set_error("cabcd_primal_objective_t: y and w must be non-NULL and lambda >= 0");
    return CABCD_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  Carve probe{nullptr};
  probe.take<double>(XT->rows);
  probe.take<double>(objective_scratch_doubles(0, 0));
  void* ws = nullptr;
  e = pool_get(probe.off + 256, &ws);
  if (e != CABCD_OK) return e;
  Carve c{static_cast<char*>(ws)};
  double* rt = c.take<double>(XT->rows);
  double* ob = c.take<double>(objective_scratch_doubles(0, 0));
  double* rr = r != nullptr ? r : rt;
  const double* A = static_cast<const double*>(XT->data);
  HIP_TRY(launch_gemv_n(A, XT->ld, XT->rows, XT->cols, w, y, -1.0, rr, st));
  if (f != nullptr)
    HIP_TRY(launch_objective(rr, XT->rows, 0.5 / (double)XT->rows, w, XT->cols, 0.5 * lambda, f,
                             ob, nullptr, st));
  HIP_TRY(hipStreamSynchronize(st));
  return CABCD_OK;
}

cabcd_status cabcd_dual_to_primal(const cabcd_matrix* XT, const double* alpha, double lambda,
                                  double* w, void* stream) {
  clear_error();
  cabcd_status e = check_dense(XT, "XT");
  if (e != CABCD_OK) return e;
  if (alpha == nullptr || w == nullptr || !(lambda > 0.0)) {
    set_error("cabcd_dual_to_primal: alpha and w must be non-NULL and lambda > 0");
    return CABCD_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  void* ws = nullptr;
  e = pool_get(std::max<size_t>(gemv_t_scratch_doubles(XT->rows, XT->cols), 1) * sizeof(double),
               &ws);
  if (e != CABCD_OK) return e;
  const double n = (double)XT->rows;
  HIP_TRY(launch_gemv_t(static_cast<const double*>(XT->data), XT->ld, XT->cols, nullptr,
                        XT->rows, alpha, -1.0 / (lambda * n), nullptr, 0.0, false, w,
                        static_cast<double*>(ws), st));
  HIP_TRY(hipStreamSynchronize(st));
  return CABCD_OK;
}

size_t cabcd_workspace_bytes(const cabcd_matrix* A, int32_t b, int32_t s) {
  if (A == nullptr || b < 1 || s < 1 || (int64_t)s * b > kMaxSB) return 0;
  StepBuffers B{};
  Carve probe{nullptr};
  const int64_t rt = std::max(A->rows, A->cols);
  return layout(probe, B, A->rows, A->cols, b, s, rt);
}

}  // extern "C"
