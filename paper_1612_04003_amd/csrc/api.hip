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

constexpr int kMaxSBDense = 512;            // s*b of a dense Gram (above 256: four-part form)
constexpr int kGramRows = 256;              // rows of one dense Gram launch
constexpr int64_t kIdxChunkSteps = 4096;    // outer steps whose indices are drawn at once
constexpr int kCsrAhead = 64;               // CSR: outer-step Grams computed per launch (max)
constexpr int kDenseAhead = 32;             // dense: the same, when one Gram is too small
constexpr int kDenseFill = 512;             // workgroups that fill the GPU (two per CU)
constexpr int64_t kAheadRowBytes = 8 << 20; // dense: gathered rows small enough to read twice
constexpr int64_t kAheadDoubles = (int64_t)8 << 20;   // their buffers (64 MiB at most)
constexpr int kSplitMinRows = 256;          // CSR: the split Gram from this many rows a step
constexpr int kSplitMaxRows = 512;
constexpr int kSplitAhead = 16;             // steps per split Gram launch (at most)
constexpr size_t kSplitBudget = (size_t)512 << 20;   // its scratch (bytes, at most)
constexpr int64_t kSplitMaxCols = (int64_t)1 << 22;   // its per-step tables index columns
constexpr int kSplitMaxRowLen = 1 << 22;              // entries of a row, below

__global__ void set_int_kernel(int* p, int v) { *p = v; }

// ----------------------------------------------------------------- workspace
struct Pool {
  void* ptr = nullptr;
  size_t cap = 0;
};
std::mutex g_pool_mu;
std::vector<Pool> g_pools[2];   // [0]: step buffers, [1]: the split sparse Gram's scratch

cabcd_status pool_get(size_t bytes, void** out, int which = 0) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    set_error("hipGetDevice failed");
    return CABCD_EHIP;
  }
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if ((int)g_pools[which].size() <= dev) g_pools[which].resize(dev + 1);
  Pool& p = g_pools[which][dev];
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

// ----------------------------------------------------------------- matrices
// The library's view of A: dense FP64 / BF16 / FP8 (row-major) or CSR FP64.
struct Mat {
  bool csr = false;
  int dtype = CABCD_F64;
  const double* X = nullptr;     // dense FP64
  const void* Q = nullptr;       // dense BF16 / FP8 codes
  const float* rs = nullptr;     // their row scales (NULL = 1)
  int64_t ld = 0;
  CsrView C{};
  int64_t rows = 0, cols = 0;
  bool lowp() const { return !csr && dtype != CABCD_F64; }
};

cabcd_status check_matrix(const cabcd_matrix* A, const char* name, Mat* M) {
  if (A == nullptr) {
    set_error("%s is NULL", name);
    return CABCD_EINVAL;
  }
  if (A->rows < 1 || A->cols < 1) {
    set_error("%s must have rows >= 1 and cols >= 1 (got %lld x %lld)", name,
              (long long)A->rows, (long long)A->cols);
    return CABCD_EINVAL;
  }
  if (A->rows > INT32_MAX || A->cols > INT32_MAX) {
    set_error("%s: rows and cols must be below 2^31", name);
    return CABCD_EINVAL;
  }
  if (A->dtype != CABCD_F64 && A->dtype != CABCD_BF16 && A->dtype != CABCD_FP8_E4M3) {
    set_error("%s: unknown dtype %d", name, A->dtype);
    return CABCD_EINVAL;
  }
  M->rows = A->rows;
  M->cols = A->cols;
  if (A->kind == CABCD_CSR) {
    if (A->dtype != CABCD_F64) {
      set_error("%s: CSR storage holds FP64 values only", name);
      return CABCD_EINVAL;
    }
    if (A->rowptr == nullptr || A->nnz < 0 || (A->nnz > 0 && (A->colidx == nullptr ||
                                                              A->vals == nullptr))) {
      set_error("%s: CSR needs rowptr, and colidx and vals when nnz > 0", name);
      return CABCD_EINVAL;
    }
    M->csr = true;
    M->C = CsrView{A->rowptr, A->colidx, A->vals, A->rows, A->cols, A->nnz};
    return CABCD_OK;
  }
  if (A->kind != CABCD_DENSE) {
    set_error("%s: unknown kind %d", name, A->kind);
    return CABCD_EINVAL;
  }
  if (A->data == nullptr || A->ld < A->cols) {
    set_error("%s: data is NULL or ld (%lld) < cols (%lld)", name, (long long)A->ld,
              (long long)A->cols);
    return CABCD_EINVAL;
  }
  M->dtype = A->dtype;
  M->ld = A->ld;
  if (A->dtype == CABCD_F64) {
    M->X = static_cast<const double*>(A->data);
  } else {
    M->Q = A->data;
    M->rs = A->row_scale;
  }
  return CABCD_OK;
}

// Device-side structure check of a CSR matrix (one synchronisation).
cabcd_status check_csr_device(const Mat& M, int* flag_dev, hipStream_t st) {
  if (!M.csr) return CABCD_OK;
  int h = 0;
  hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, st, flag_dev, 0);
  HIP_TRY(hipGetLastError());
  HIP_TRY(launch_csr_check(M.C, flag_dev, st));
  HIP_TRY(hipMemcpyAsync(&h, flag_dev, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (h != 0) {
    set_error("malformed CSR: rowptr must start at 0, be non-decreasing and end at nnz; "
              "columns strictly increasing within a row and below cols");
    return CABCD_EINVAL;
  }
  return CABCD_OK;
}

int max_rows_per_gram(const Mat& M) { return M.csr ? kCsrMaxRows : kMaxSBDense; }

// Plan of one dense Gram launch of m rows (at most kGramRows: larger Grams
// are assembled from launches of kGramRows rows).
GramPlan plan_for(const Mat& M, int m) {
  m = std::min(m, kGramRows);
  return M.lowp() ? plan_gram_lp(m, M.cols, M.dtype) : plan_gram_f64(m, M.cols);
}

// A Gram of more than kGramRows rows: six partial sets of the 256-row plan
// (two diagonal blocks, up to four cross blocks) and the two index lists.
size_t big_partials(const Mat& M) {
  return 6 * gram_partial_doubles(plan_for(M, kGramRows)) + (512 + 4 * 256) / 2;
}

size_t max_partials(const Mat& M, int sb_max) {
  if (M.csr) return 1;
  size_t best = 0;
  for (int m = 1;; m = (m < 16 ? 16 : m * 2)) {
    best = std::max(best, gram_partial_doubles(plan_for(M, std::min(m, sb_max))));
    if (m >= sb_max) break;
  }
  if (sb_max > kGramRows) best = std::max(best, big_partials(M));
  return best;
}

// out = [beta base | out] + gamma * sum_p A[row(p)]^T v[p]
hipError_t mat_scatter(const Mat& M, const int32_t* idx, int64_t m, const double* v,
                       double gamma, const double* base, double beta, bool accumulate,
                       double* out, double* scratch, hipStream_t st) {
  if (M.lowp())
    return launch_gemv_t_lp(M.dtype, M.Q, M.ld, M.cols, M.rs, idx, m, v, gamma, base, beta,
                            accumulate, out, st);
  if (!M.csr)
    return launch_gemv_t(M.X, M.ld, M.cols, idx, m, v, gamma, base, beta, accumulate, out,
                         scratch, st);
  if (!accumulate) {
    hipError_t e = launch_fill(out, M.cols, base, beta, st);
    if (e != hipSuccess) return e;
  }
  return launch_csr_scatter(M.C, idx, m, v, gamma, out, st);
}

// out[p] = A[p] . v + beta base[p]
hipError_t mat_rowdot(const Mat& M, const double* v, const double* base, double beta,
                      double* out, double* scratch, hipStream_t st) {
  if (!M.csr)
    return launch_rowdot(M.dtype, M.lowp() ? M.Q : static_cast<const void*>(M.X), M.ld, M.rows,
                         M.cols, M.rs, v, base, beta, out, scratch, st);
  return launch_csr_rowdot(M.C, v, base, beta, out, st);
}

// Scratch of the streaming passes over all rows of A or over sb gathered rows.
size_t mat_scratch_doubles(const Mat& M, int64_t sb) {
  if (M.csr) return 1;
  size_t sc = std::max(gemv_t_scratch_doubles(sb, M.cols), gemv_t_scratch_doubles(M.rows, M.cols));
  sc = std::max(sc, rowdot_scratch_doubles(M.rows, M.cols, M.dtype));
  sc = std::max(sc, rowdot_scratch_doubles(sb, M.cols, M.dtype));
  return std::max<size_t>(sc, 1);
}

// out[p] = A[idx[p]] . u for p < m (row scales applied): the Y u of a step
// whose Gram was computed ahead.
hipError_t mat_rows_dot(const Mat& M, const int32_t* idx, int m, const double* u, double* out,
                        double* scratch, hipStream_t st) {
  if (M.csr) return launch_csr_rowdot_rows(M.C, idx, m, u, out, st);
  return launch_rowdot_rows(M.dtype, M.lowp() ? M.Q : static_cast<const void*>(M.X), M.ld, idx,
                            m, M.cols, M.rs, u, out, scratch, st);
}

// The full residual of the stopping test (Section 5.1.5) and its 2-norm
// (device scalar), from the vectors the iteration maintains:
//   primal (A = X, coord = w, comp = r = z - y):  rho = -lambda w - 1/n X r
//   dual (A = X^T, coord = alpha, comp = w):      rho = -X^T w + alpha + y
// rho (length rows) receives the vector; it may be the temporary itself.
hipError_t full_residual(bool dual, const Mat& M, const double* y, double lambda,
                         const double* coord, const double* comp, double* rho, double* norm,
                         double* scratch, double* obj_scratch, int* status, hipStream_t st) {
  hipError_t e;
  if (!dual) {
    const double n = (double)M.cols;
    e = mat_rowdot(M, comp, coord, lambda * n, rho, scratch, st);   // X r + lambda n w
    if (e != hipSuccess) return e;
    return launch_resid_norm(rho, -1.0 / n, nullptr, 0.0, M.rows, rho, norm, obj_scratch, status,
                             st);
  }
  e = mat_rowdot(M, comp, y, -1.0, rho, scratch, st);   // X^T w - y
  if (e != hipSuccess) return e;
  return launch_resid_norm(coord, 1.0, rho, -1.0, M.rows, rho, norm, obj_scratch, status, st);
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
  PhaseTimer(double* out, uint32_t mask, hipStream_t st)
      : out_(out), mask_(mask == 0 ? ~0u : mask), st_(st) {}
  ~PhaseTimer() {
    for (auto& r : recs_) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto& r : dropped_) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
  }
  // Called from inside a phase that enqueued nothing (an update left to the
  // next step's Gram or made moot by a recomputation): the phase is not
  // counted.
  void drop() { drop_ = true; }
  template <class F>
  hipError_t run(int phase, F&& f) {
    return run_on(st_, phase, f);
  }
  // The same for work enqueued on another stream (the events go there).
  template <class F>
  hipError_t run_on(hipStream_t st, int phase, F&& f) {
    if (out_ == nullptr || !((mask_ >> phase) & 1u)) return f();
    Rec r{phase, nullptr, nullptr};
    hipError_t e = hipEventCreate(&r.a);
    if (e == hipSuccess) e = hipEventCreate(&r.b);
    if (e != hipSuccess) return e;
    recs_.push_back(r);
    e = hipEventRecord(r.a, st);
    if (e != hipSuccess) return e;
    drop_ = false;
    e = f();
    if (e != hipSuccess) return e;
    if (drop_) {
      drop_ = false;
      dropped_.push_back(r);
      recs_.pop_back();
      return hipSuccess;
    }
    return hipEventRecord(r.b, st);
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
  uint32_t mask_;
  hipStream_t st_;
  bool drop_ = false;
  std::vector<Rec> dropped_;   // events of dropped phases, destroyed at the end
  std::vector<Rec> recs_;
};

// The second stream of a device (created once, default priority): Grams
// computed ahead run there beside the steps of the previous batch.
hipStream_t side_stream() {
  static std::mutex mu;
  static hipStream_t streams[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(mu);
  if (streams[dev] == nullptr &&
      hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
    streams[dev] = nullptr;
  return streams[dev];
}

// The two events of one call's hand-offs between the streams.
struct StreamEvents {
  hipEvent_t issued = nullptr, ready = nullptr;
  hipError_t create() {
    hipError_t e = hipEventCreateWithFlags(&issued, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ready, hipEventDisableTiming);
    return e;
  }
  ~StreamEvents() {
    if (issued != nullptr) (void)hipEventDestroy(issued);
    if (ready != nullptr) (void)hipEventDestroy(ready);
  }
};

// Layout of the Gram partials a launch of `plan` writes for the dense M.
int partial_layout(const Mat& M, const GramPlan& plan) {
  return M.lowp() ? gram_lp_partial_layout(plan, M.dtype, M.Q, M.ld) : 0;
}

// scale * Y Y^T + shift * E and Y u for the rows idx[0..m) of A.
hipError_t mat_gram(const Mat& M, const int32_t* idx, int m, const double* u, double scale,
                    double shift, bool overlap, double* G, double* Yu, double* partials,
                    hipStream_t st, PhaseTimer* timer) {
  if (M.csr) {
    auto f = [&] { return launch_csr_gram(M.C, idx, m, u, scale, shift, overlap, G, Yu, st); };
    return timer ? timer->run(CABCD_PHASE_GRAM, f) : f();
  }
  if (m > kGramRows) {
    // rows [0, 256) and [256, m): the two diagonal blocks as two 256-row
    // Grams (with Y u), the cross block from the 256-row Grams of pairs of
    // 128-row halves (their off-diagonal quarter)
    const GramPlan plan = plan_for(M, kGramRows);
    const size_t set = gram_partial_doubles(plan);
    int32_t* ia = reinterpret_cast<int32_t*>(partials + 6 * set);
    int32_t* ib = ia + 512;
    const int nc = big_cross_steps(m);
    auto g = [&]() -> hipError_t {
      hipError_t e = launch_big_index(idx, m, ia, ib, st);
      if (e != hipSuccess) return e;
      if (M.lowp()) {
        e = launch_gram_lp(plan, M.dtype, M.Q, M.ld, M.cols, ia, kGramRows, u, partials, st, 2);
        if (e != hipSuccess) return e;
        return launch_gram_lp(plan, M.dtype, M.Q, M.ld, M.cols, ib, kGramRows, nullptr,
                              partials + 2 * set, st, nc);
      }
      e = launch_gram_f64(plan, M.X, M.ld, M.cols, ia, kGramRows, u, partials, st, 2);
      if (e != hipSuccess) return e;
      return launch_gram_f64(plan, M.X, M.ld, M.cols, ib, kGramRows, nullptr, partials + 2 * set,
                             st, nc);
    };
    auto r = [&] {
      return launch_gram_reduce_big(plan, partials, idx, m, scale, shift, overlap, G, Yu, st,
                                    partial_layout(M, plan), M.lowp() ? M.rs : nullptr);
    };
    hipError_t e = timer ? timer->run(CABCD_PHASE_GRAM, g) : g();
    if (e != hipSuccess) return e;
    return timer ? timer->run(CABCD_PHASE_REDUCE, r) : r();
  }
  const GramPlan plan = plan_for(M, m);
  auto g = [&] {
    return M.lowp() ? launch_gram_lp(plan, M.dtype, M.Q, M.ld, M.cols, idx, m, u, partials, st)
                    : launch_gram_f64(plan, M.X, M.ld, M.cols, idx, m, u, partials, st);
  };
  auto r = [&] {
    return launch_gram_reduce(plan, partials, idx, m, scale, shift, overlap, G, Yu, st,
                              partial_layout(M, plan), M.lowp() ? M.rs : nullptr);
  };
  hipError_t e = timer ? timer->run(CABCD_PHASE_GRAM, g) : g();
  if (e != hipSuccess) return e;
  return timer ? timer->run(CABCD_PHASE_REDUCE, r) : r();
}

// Gram slots of the step buffers: the Grams of several future outer steps are
// computed in one launch (they depend on the sampled indices only) when one
// step's Gram cannot fill the GPU: always for CSR (a latency-bound walk per
// row), and for dense rows too short to give the split-K Gram enough slabs.
// Y u then takes a second pass over the gathered rows, so dense look-ahead is
// kept to gathered rows of a few MiB.
int gram_slots(const Mat& M, int64_t sb) {
  if (M.csr)
    return (int)std::max<int64_t>(1, std::min<int64_t>(kCsrAhead, kAheadDoubles / (sb * sb)));
  const int64_t elem = M.dtype == CABCD_F64 ? 8 : (M.dtype == CABCD_BF16 ? 2 : 1);
  if (sb > kGramRows || sb * M.cols * elem > kAheadRowBytes) return 1;
  const GramPlan p = plan_for(M, (int)sb);
  if (p.nsplit >= kDenseFill) return 1;
  const int64_t per = (int64_t)gram_partial_doubles(p) + sb * sb;   // partials and G
  int64_t k = (kDenseFill + p.nsplit - 1) / p.nsplit;
  k = std::min<int64_t>(k, kDenseAhead);
  k = std::min<int64_t>(k, kAheadDoubles / per);
  return (int)std::max<int64_t>(k, 1);
}

// The Grams of nsteps full outer steps (indices idx + k m for step k) into G +
// k m^2, without Y u.
hipError_t mat_gram_steps(const Mat& M, const int32_t* idx, int m, int nsteps, double scale,
                          double shift, double* G, double* partials, hipStream_t st,
                          PhaseTimer* timer) {
  if (M.csr)
    return timer->run_on(st, CABCD_PHASE_GRAM, [&] {
      return launch_csr_gram_steps(M.C, idx, m, nsteps, scale, shift, true, G, st);
    });
  const GramPlan plan = plan_for(M, m);
  hipError_t e = timer->run_on(st, CABCD_PHASE_GRAM, [&] {
    return M.lowp() ? launch_gram_lp(plan, M.dtype, M.Q, M.ld, M.cols, idx, m, nullptr, partials,
                                     st, nsteps)
                    : launch_gram_f64(plan, M.X, M.ld, M.cols, idx, m, nullptr, partials, st,
                                      nsteps);
  });
  if (e != hipSuccess) return e;
  return timer->run_on(st, CABCD_PHASE_REDUCE, [&] {
    return launch_gram_reduce(plan, partials, idx, m, scale, shift, true, G, nullptr, st,
                              partial_layout(M, plan), M.lowp() ? M.rs : nullptr, nsteps);
  });
}

// CSR steps of kSplitMinRows..kSplitMaxRows rows whose Grams are computed
// ahead take the split Gram (heavy columns dense, light ones by column lists).
bool use_split(const Mat& M, int64_t sb) {
  return M.csr && sb >= kSplitMinRows && sb <= kSplitMaxRows && M.cols <= kSplitMaxCols &&
         gram_slots(M, sb) > 1;
}

struct StepBuffers {
  int* split_prep;   // the split Gram's per-matrix numbering of heavy columns
  int* status;
  int32_t* idx;      // kIdxChunkSteps * s * b
  double* G;         // gram_slots x sb x sb (twice when computed ahead)
  double* G2;        // the second buffer of Grams computed ahead (or G)
  double* Yu;        // sb
  double* delta;     // sb
  double* partials;  // dense Gram partials
  double* partials2; // the second buffer of the ahead path's partials (or partials)
  double* scratch;   // gemv row-group partials
  double* obj;       // objective scratch
  double* rtmp;      // residual temporary (monitoring)
  double* rho;       // full residual of the stopping test (rows)
  double* rnorm;     // its norm
};

// Layout of the step workspace.
size_t layout(Carve& c, StepBuffers& B, const Mat& M, int b, int s, int64_t rtmp_len,
              bool checks) {
  const int sb = s * b;
  B.split_prep = c.take<int>(use_split(M, sb) ? csr_split_prepare_ints(M.C) : 1);
  B.status = c.take<int>(1);
  B.idx = c.take<int32_t>((size_t)kIdxChunkSteps * sb);
  const int slots = gram_slots(M, sb);
  const int nbuf = slots > 1 ? 2 : 1;   // Grams computed ahead: the next batch's buffer too
  B.G = c.take<double>((size_t)nbuf * slots * sb * sb);
  B.G2 = B.G + (size_t)(nbuf - 1) * slots * sb * sb;
  B.Yu = c.take<double>(sb);
  B.delta = c.take<double>(sb);
  const size_t ahead_p =
      M.csr || slots == 1 ? (size_t)0 : (size_t)slots * gram_partial_doubles(plan_for(M, sb));
  B.partials = c.take<double>(std::max(max_partials(M, sb), nbuf * ahead_p));
  B.partials2 = B.partials + (nbuf - 1) * ahead_p;
  B.scratch = c.take<double>(mat_scratch_doubles(M, sb));
  B.obj = c.take<double>(objective_scratch_doubles(0, 0));
  B.rtmp = c.take<double>(std::max<int64_t>(rtmp_len, 1));
  B.rho = c.take<double>(checks ? M.rows : 1);
  B.rnorm = c.take<double>(1);
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

cabcd_status check_common(const Mat& M, double lambda, int b, int s, int64_t H) {
  if (!(lambda > 0.0) || !std::isfinite(lambda)) {
    set_error("lambda must be a positive finite number (got %g)", lambda);
    return CABCD_EINVAL;
  }
  if (b < 1 || (int64_t)b > M.rows) {
    set_error("block size b = %d must satisfy 1 <= b <= %lld", b, (long long)M.rows);
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
  if (b > kSolveMaxB) {
    set_error("block size b = %d exceeds the supported maximum %d", b, kSolveMaxB);
    return CABCD_EUNSUPPORTED;
  }
  const int64_t sb = (int64_t)s * b;
  if (sb > max_rows_per_gram(M)) {
    set_error("s*b = %lld exceeds the supported maximum %d for %s storage", (long long)sb,
              max_rows_per_gram(M), M.csr ? "CSR" : "dense");
    return CABCD_EUNSUPPORTED;
  }
  if (b > 16 && sb > 512) {   // the 32-lane block solves hold at most 512 rows
    set_error("s*b = %lld with b = %d > 16 exceeds the supported maximum 512", (long long)sb, b);
    return CABCD_EUNSUPPORTED;
  }
  if (solve_lds_bytes((int)sb, b) > kSolveMaxLds) {
    set_error("s*b = %lld with b = %d needs more LDS than one workgroup has", (long long)sb, b);
    return CABCD_EUNSUPPORTED;
  }
  return CABCD_OK;
}

// One driver for both methods (they differ in the scalars and the role of the
// vectors, see the fused solve).  primal: coord = w (d), comp = r (n).
// dual: coord = alpha (n), comp = w (d).
cabcd_status run_bcd(bool dual, const Mat& M, const double* y, double lambda, int b, int s,
                     int64_t H, uint64_t seed, double* coord, double* comp,
                     const cabcd_opts* opts, hipStream_t st) {
  cabcd_opts o;
  cabcd_opts_init(&o);
  if (opts != nullptr) o = *opts;
  const int64_t rows = M.rows, cols = M.cols;
  const double n = dual ? (double)rows : (double)cols;
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
  if (o.timing != nullptr && (o.flags & CABCD_FLAG_ASYNC)) {
    set_error("opts.timing needs a synchronising call");
    return CABCD_EINVAL;
  }
  if (!(o.tol >= 0.0) || std::isinf(o.tol) || o.check_every < 0 ||
      (o.tol > 0.0 && o.check_every == 0)) {
    set_error("opts.tol must be finite and >= 0, opts.check_every >= 0, and a tolerance "
              "needs check_every >= 1");
    return CABCD_EINVAL;
  }
  if (o.check_every > 0 && (o.flags & CABCD_FLAG_ASYNC)) {
    set_error("residual checks (opts.check_every) need a synchronising call");
    return CABCD_EINVAL;
  }
  if (o.explicit_idx != nullptr) {
    cabcd_status e = check_explicit(o.explicit_idx, H, b, rows, st);
    if (e != CABCD_OK) return e;
  }
  // monitoring needs the residual X^T w - y of length n (primal: cols, dual: rows)
  const int64_t rtmp_len = o.monitor_every > 0 ? (dual ? rows : cols) : 1;
  StepBuffers B{};
  Carve probe{nullptr};
  const bool checks = o.check_every > 0;
  const size_t need = layout(probe, B, M, b, s, rtmp_len, checks);
  void* ws = nullptr;
  cabcd_status e = get_workspace(&o, need, &ws);
  if (e != CABCD_OK) return e;
  Carve carve{static_cast<char*>(ws)};
  layout(carve, B, M, b, s, rtmp_len, checks);
  if (o.iters_done != nullptr) *o.iters_done = 0;
  if (o.resid_norm != nullptr) *o.resid_norm = std::nan("");
  e = check_csr_device(M, B.status, st);
  if (e != CABCD_OK) return e;

  // The split sparse Gram: heavy columns numbered once for this matrix, its
  // data-dependent scratch from the second pool (or from a caller workspace
  // that has room for it beyond `need`; otherwise the Grams stay on the
  // row-pair kernel).
  const int64_t sb_full = (int64_t)s * b;
  bool split = use_split(M, sb_full);
  CsrSplitInfo sinfo{};
  int ksplit = 0;
  double* split_d[2] = {nullptr, nullptr};   // the scratch of two launches (see the loop)
  int* split_i[2] = {nullptr, nullptr};
  if (split) {
    HIP_TRY(csr_split_prepare(M.C, B.split_prep, &sinfo, st));
  }
  if (split && sinfo.maxrow >= kSplitMaxRowLen) split = false;   // entry keys need < 2^22
  if (split) {
    ksplit = std::min(gram_slots(M, sb_full), kSplitAhead);
    // a launch takes 1..ksplit steps; its doubles, then its ints, must fit
    size_t dmax = 0, imax = 0;
    auto bytes_of = [&](int k) {
      dmax = imax = 0;
      for (int j = 1; j <= k; ++j) {
        const SplitLayout L = csr_split_layout(sinfo, M.cols, (int)sb_full, j);
        dmax = std::max(dmax, L.doubles);
        imax = std::max(imax, L.ints);
      }
      return dmax * sizeof(double) + imax * sizeof(int) + 512;
    };
    while (ksplit > 1 && bytes_of(ksplit) > kSplitBudget) ksplit /= 2;
    const size_t sbytes = (bytes_of(ksplit) + 255) & ~(size_t)255;   // one launch's
    void* sp = nullptr;
    if (sbytes > kSplitBudget) {
      split = false;   // rows too long for the per-step entry tables
    } else if (o.workspace != nullptr) {
      // the split scratch starts at the first 256-byte boundary past `need`
      const uintptr_t w0 = reinterpret_cast<uintptr_t>(o.workspace);
      const uintptr_t s0 = (w0 + need + 255) & ~(uintptr_t)255;
      if (s0 + 2 * sbytes <= w0 + o.workspace_bytes) sp = reinterpret_cast<void*>(s0);
      split = sp != nullptr;
    } else {
      e = pool_get(2 * sbytes, &sp, 1);
      if (e != CABCD_OK) return e;
    }
    if (split) {
      for (int q = 0; q < 2; ++q) {
        split_d[q] = reinterpret_cast<double*>(static_cast<char*>(sp) + q * sbytes);
        split_i[q] = reinterpret_cast<int*>(split_d[q] + dmax);
      }
    }
  }

  hipLaunchKernelGGL(set_int_kernel, dim3(1), dim3(1), 0, st, B.status, 0);
  HIP_TRY(hipGetLastError());

  const double scale = dual ? 1.0 / (lambda * n * n) : 1.0 / n;
  const double shift = dual ? 1.0 / n : lambda;
  const double gamma = dual ? -1.0 / (lambda * n) : 1.0;

  auto exact_companion = [&]() -> hipError_t {
    if (dual)   // w = -X alpha / (lambda n)
      return mat_scatter(M, nullptr, rows, coord, -1.0 / (lambda * n), nullptr, 0.0, false,
                         comp, B.scratch, st);
    // r = X^T w - y
    return mat_scatter(M, nullptr, rows, coord, 1.0, y, -1.0, false, comp, B.scratch, st);
  };
  // f(w) at a monitor point.  fresh: the primal residual comp was recomputed
  // exactly in this outer step, so it is used instead of another full pass;
  // CABCD_FLAG_MONITOR_MAINTAINED asks for the maintained residual always.
  auto monitor = [&](int64_t slot, bool fresh) -> hipError_t {
    hipError_t he;
    if (!dual && (fresh || (o.flags & CABCD_FLAG_MONITOR_MAINTAINED)))
      return launch_objective(comp, cols, 0.5 / n, coord, rows, 0.5 * lambda, o.trace + slot,
                              B.obj, B.status, st);
    if (dual) {   // f(w) with r = X^T w - y computed from the X^T layout
      he = mat_rowdot(M, comp, y, -1.0, B.rtmp, B.scratch, st);
      if (he != hipSuccess) return he;
      return launch_objective(B.rtmp, rows, 0.5 / n, comp, cols, 0.5 * lambda, o.trace + slot,
                              B.obj, B.status, st);
    }
    he = mat_scatter(M, nullptr, rows, coord, 1.0, y, -1.0, false, B.rtmp, B.scratch, st);
    if (he != hipSuccess) return he;
    return launch_objective(B.rtmp, cols, 0.5 / n, coord, rows, 0.5 * lambda, o.trace + slot,
                            B.obj, B.status, st);
  };

  PhaseTimer timer(o.timing, o.timing_mask, st);
  if (!(o.flags & CABCD_FLAG_STATE_VALID))
    HIP_TRY(timer.run(CABCD_PHASE_RECOMPUTE, exact_companion));

  const int K = gram_slots(M, (int64_t)s * b);   // Grams per launch (computed ahead)
  // Grams computed ahead get their diagonal blocks inverted in one launch, and
  // the one-barrier solves (b <= 16, s BP <= 512 lanes) skip their own
  // inversion: sparse dual solve at b = 16, s = 1 / 8 / 32: 11.9 -> 8.9 /
  // 15.9 -> 12.3 / 43 -> 34 us (the 512-thread solve without the inversion
  // code also stops spilling registers).
  int bp = 1;
  while (bp < b) bp *= 2;
  const bool pre_inv = K > 1 && bp <= 16 && (int64_t)s * bp <= 512;
  // CABCD_FLAG_FOLD_UPDATE: the dense 256-row Gram applies the previous
  // step's companion update on its way (one pass over both steps' rows, the
  // update's traffic beside the matrix cores' work instead of a pass of its
  // own): a full step leaves its update pending when the next step is a full
  // one with nothing in between that reads the companion (check, monitor
  // point, exact recomputation) and keeps its indices in place.  Every such
  // step's update runs through that device code, folded or alone, so a
  // column's rounding does not depend on how a run is split into calls.
  const GramPlan fplan = plan_for(M, kGramRows);
  const bool fuse_kind = (o.flags & CABCD_FLAG_FOLD_UPDATE) != 0 && K == 1 && !M.csr &&
                         !M.lowp() && (int64_t)s * b == kGramRows &&
                         gram_f64_takes_update(fplan, M.X, M.ld, kGramRows);
  bool pending = false;
  const int32_t* pend_idx = nullptr;
  int ahead = 0, gslot = 0;                       // precomputed Grams left, next slot
  int split_nst = 0;                              // steps of the current batch
  int64_t h = 0, k = 0, slot = 0;
  int64_t chunk_begin = -1, chunk_end = -1;
  const int64_t chunk_iters = kIdxChunkSteps * (int64_t)s;

  // Grams computed ahead come in batches of up to K (ksplit) full outer steps.
  // While the steps of one batch run on the call's stream, the next batch's
  // Grams (whose indices are at hand) are computed on a second stream into
  // the other of two buffers; the first step of that batch waits for them.
  double* const Gbuf[2] = {B.G, B.G2};
  double* const Pbuf[2] = {B.partials, B.partials2};
  int cur = 0;                                    // buffer of the current batch
  bool pf_ready = false;                          // next batch launched on the side stream
  int64_t pf_h = -1;
  int pf_nst = 0;
  hipStream_t side = nullptr;
  StreamEvents ev;
  if (K > 1) {
    side = side_stream();
    if (side == nullptr || ev.create() != hipSuccess) {
      set_error("creating the second stream or its events failed");
      return CABCD_EHIP;
    }
  }
  // steps of the batch starting at iteration hb whose indices are at hand (0: none)
  auto batch_steps = [&](int64_t hb) -> int {
    int64_t avail = (H - hb) / s;
    if (o.explicit_idx == nullptr) avail = std::min(avail, (chunk_end - hb) / s);
    return (int)std::min<int64_t>(split ? ksplit : K, std::max<int64_t>(avail, 0));
  };
  auto launch_batch = [&](int64_t hb, int nst, int buf, hipStream_t bs) -> hipError_t {
    const int32_t* ib = o.explicit_idx != nullptr ? o.explicit_idx + hb * b
                                                  : B.idx + (hb - chunk_begin) * b;
    const int mb = s * b;
    hipError_t he;
    if (split)
      he = timer.run_on(bs, CABCD_PHASE_GRAM, [&] {
        return launch_csr_gram_split(M.C, sinfo, ib, mb, nst, scale, shift, true, Gbuf[buf],
                                     split_d[buf], split_i[buf], bs);
      });
    else
      he = mat_gram_steps(M, ib, mb, nst, scale, shift, Gbuf[buf], Pbuf[buf], bs, &timer);
    if (he != hipSuccess) return he;
    // their diagonal blocks inverted together, off the solves' chains
    if (pre_inv)
      he = timer.run_on(bs, CABCD_PHASE_SOLVE, [&] {
        return launch_invert_diag(Gbuf[buf], nst, mb, b, B.status, bs);
      });
    return he;
  };
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
    const double* Gk = B.G;
    const bool from_ahead = K > 1 && sk == s;
    if (from_ahead) {
      if (ahead == 0) {
        if (pf_ready && pf_h == h) {   // computed on the side stream
          HIP_TRY(hipStreamWaitEvent(st, ev.ready, 0));
          cur ^= 1;
          ahead = pf_nst;
          pf_ready = false;
        } else {                       // computed here
          ahead = std::max(batch_steps(h), 1);
          HIP_TRY(launch_batch(h, ahead, cur, st));
        }
        split_nst = ahead;
        gslot = 0;
        // the next batch on the side stream, after everything enqueued so far
        // (the previous batch's steps used its buffer)
        const int64_t h2 = h + (int64_t)ahead * s;
        const int n2 = batch_steps(h2);
        if (n2 > 0) {
          HIP_TRY(hipEventRecord(ev.issued, st));
          HIP_TRY(hipStreamWaitEvent(side, ev.issued, 0));
          HIP_TRY(launch_batch(h2, n2, cur ^ 1, side));
          HIP_TRY(hipEventRecord(ev.ready, side));
          pf_ready = true;
          pf_h = h2;
          pf_nst = n2;
        }
      }
      Gk = Gbuf[cur] + (size_t)gslot * m * m;
      ++gslot;
      --ahead;
      HIP_TRY(timer.run(CABCD_PHASE_YU, [&] {
        return mat_rows_dot(M, idx, m, comp, B.Yu, B.scratch, st);
      }));
    } else if (pending) {
      HIP_TRY(timer.run(CABCD_PHASE_GRAM, [&] {
        return launch_gram_f64_upd(fplan, M.X, M.ld, M.cols, idx, m, B.partials,
                                   D16Upd{pend_idx, B.delta, gamma, comp}, st);
      }));
      HIP_TRY(timer.run(CABCD_PHASE_REDUCE, [&] {
        return launch_gram_reduce(fplan, B.partials, idx, m, scale, shift, true, B.G, B.Yu, st,
                                  partial_layout(M, fplan), nullptr);
      }));
      pending = false;
    } else {
      HIP_TRY(
          mat_gram(M, idx, m, comp, scale, shift, true, B.G, B.Yu, B.partials, st, &timer));
    }
    SolveArgs sa{};
    sa.G = Gk;
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
    sa.pre_inverted = from_ahead && pre_inv ? 1 : 0;
    HIP_TRY(timer.run(CABCD_PHASE_SOLVE, [&] { return launch_solve(sa, st); }));
    HIP_TRY(timer.run(CABCD_PHASE_UPDATE, [&] {
      // an exact recomputation right after this step rebuilds the companion
      // from the coordinates alone, so the update would be overwritten
      if (o.resid_every > 0 && (k + 1) % o.resid_every == 0) {
        timer.drop();
        return hipSuccess;
      }
      // steps whose Gram came from a split launch: the deterministic update
      // from its panel and sorted lists
      if (from_ahead && split)
        return launch_csr_update_split(M.C, sinfo, idx, m, split_nst, gslot - 1, B.delta, gamma,
                                       comp, split_d[cur], split_i[cur], st);
      if (fuse_kind && m == kGramRows) {
        const int64_t h1 = h + sk, k1 = k + 1;
        const bool reads_comp =
            (o.resid_every > 0 && k1 % o.resid_every == 0) ||
            (o.monitor_every > 0 && k1 % o.monitor_every == 0 && slot < o.trace_len) ||
            (checks && k1 % o.check_every == 0);
        if (H - h1 >= s && !reads_comp && (o.explicit_idx != nullptr || h1 < chunk_end)) {
          pending = true;
          pend_idx = idx;
          timer.drop();
          return hipSuccess;
        }
        return launch_update_f64(fplan, M.X, M.ld, M.cols, D16Upd{idx, B.delta, gamma, comp}, st);
      }
      return mat_scatter(M, idx, m, B.delta, gamma, nullptr, 0.0, true, comp, B.scratch, st);
    }));
    h += sk;
    ++k;
    const bool fresh = o.resid_every > 0 && k % o.resid_every == 0;
    if (fresh) HIP_TRY(timer.run(CABCD_PHASE_RECOMPUTE, exact_companion));
    if (o.monitor_every > 0 && k % o.monitor_every == 0 && slot < o.trace_len) {
      const int64_t sl = slot++;
      HIP_TRY(timer.run(CABCD_PHASE_MONITOR, [&] { return monitor(sl, fresh); }));
    }
    if (checks && k % o.check_every == 0) {
      // Section 5.1.5: the full residual, formed now and then, decides when to
      // stop (its norm bounds the objective error).
      HIP_TRY(timer.run(CABCD_PHASE_CHECK, [&] {
        return full_residual(dual, M, y, lambda, coord, comp, B.rho, B.rnorm, B.scratch, B.obj,
                             B.status, st);
      }));
      double nrm = 0.0;
      HIP_TRY(hipMemcpyAsync(&nrm, B.rnorm, sizeof nrm, hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      if (o.resid_norm != nullptr) *o.resid_norm = nrm;
      if (!std::isfinite(nrm) || nrm <= o.tol) break;   // non-finite: reported by finish
    }
  }
  if (o.iters_done != nullptr) *o.iters_done = h;
  // a batch computed ahead and not used (the run stopped early) still ends
  // before the call's stream moves on
  if (pf_ready) HIP_TRY(hipStreamWaitEvent(st, ev.ready, 0));
  const cabcd_status fs = finish(st, B.status, (o.flags & CABCD_FLAG_ASYNC) != 0);
  HIP_TRY(timer.collect());
  return fs;
}

// Workspace for the single-pass helpers (residual, objective, dual map).
struct AuxBuffers {
  int* flag;
  double* r;
  double* scratch;
  double* obj;
};
size_t aux_layout(Carve& c, AuxBuffers& B, const Mat& M, int64_t rlen) {
  B.flag = c.take<int>(1);
  B.r = c.take<double>(std::max<int64_t>(rlen, 1));
  B.scratch = c.take<double>(mat_scratch_doubles(M, 1));
  B.obj = c.take<double>(objective_scratch_doubles(0, 0) + 1);   // + one norm
  return c.off + 256;
}
cabcd_status aux_get(const Mat& M, int64_t rlen, AuxBuffers& B) {
  Carve probe{nullptr};
  const size_t need = aux_layout(probe, B, M, rlen);
  void* ws = nullptr;
  cabcd_status e = pool_get(need, &ws);
  if (e != CABCD_OK) return e;
  Carve c{static_cast<char*>(ws)};
  aux_layout(c, B, M, rlen);
  return CABCD_OK;
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

const char* cabcd_version(void) { return "cabcd 0.2 (gfx950)"; }

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
  Mat M;
  cabcd_status e = check_matrix(A, "A", &M);
  if (e != CABCD_OK) return e;
  if (m < 1 || idx == nullptr || G == nullptr) {
    set_error("cabcd_gram: need m >= 1 and non-NULL idx and G");
    return CABCD_EINVAL;
  }
  if (m > max_rows_per_gram(M)) {
    set_error("cabcd_gram: m = %d exceeds the supported maximum %d", m, max_rows_per_gram(M));
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
  Carve probe{nullptr};
  int* flag = probe.take<int>(1);
  double* part = probe.take<double>(max_partials(M, m));
  void* ws = nullptr;
  e = pool_get(probe.off + 256, &ws);
  if (e != CABCD_OK) return e;
  Carve c{static_cast<char*>(ws)};
  flag = c.take<int>(1);
  part = c.take<double>(max_partials(M, m));
  e = check_csr_device(M, flag, st);
  if (e != CABCD_OK) return e;
  const bool want_u = u != nullptr && Yu != nullptr;
  HIP_TRY(mat_gram(M, idx, m, want_u ? u : nullptr, scale, shift, false, G,
                   want_u ? Yu : nullptr, part, st, nullptr));
  HIP_TRY(hipStreamSynchronize(st));
  return CABCD_OK;
}

cabcd_status cabcd_primal_bcd(const cabcd_matrix* X, const double* y, double lambda, int32_t b,
                              int32_t s, int64_t H, uint64_t seed, double* w, double* r,
                              const cabcd_opts* opts, void* stream) {
  clear_error();
  Mat M;
  cabcd_status e = check_matrix(X, "X", &M);
  if (e != CABCD_OK) return e;
  e = check_common(M, lambda, b, s, H);
  if (e != CABCD_OK) return e;
  return run_bcd(false, M, y, lambda, b, s, H, seed, w, r, opts, (hipStream_t)stream);
}

cabcd_status cabcd_dual_bcd(const cabcd_matrix* XT, const double* y, double lambda, int32_t b,
                            int32_t s, int64_t H, uint64_t seed, double* alpha, double* w,
                            const cabcd_opts* opts, void* stream) {
  clear_error();
  Mat M;
  cabcd_status e = check_matrix(XT, "XT", &M);
  if (e != CABCD_OK) return e;
  e = check_common(M, lambda, b, s, H);
  if (e != CABCD_OK) return e;
  return run_bcd(true, M, y, lambda, b, s, H, seed, alpha, w, opts, (hipStream_t)stream);
}

cabcd_status cabcd_primal_objective(const cabcd_matrix* X, const double* y, double lambda,
                                    const double* w, double* r, double* f, void* stream) {
  clear_error();
  Mat M;
  cabcd_status e = check_matrix(X, "X", &M);
  if (e != CABCD_OK) return e;
  if (y == nullptr || w == nullptr || !(lambda >= 0.0)) {
    set_error("cabcd_primal_objective: y and w must be non-NULL and lambda >= 0");
    return CABCD_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  AuxBuffers B{};
  e = aux_get(M, M.cols, B);
  if (e != CABCD_OK) return e;
  e = check_csr_device(M, B.flag, st);
  if (e != CABCD_OK) return e;
  double* rr = r != nullptr ? r : B.r;
  HIP_TRY(mat_scatter(M, nullptr, M.rows, w, 1.0, y, -1.0, false, rr, B.scratch, st));
  if (f != nullptr)
    HIP_TRY(launch_objective(rr, M.cols, 0.5 / (double)M.cols, w, M.rows, 0.5 * lambda, f, B.obj,
                             nullptr, st));
  HIP_TRY(hipStreamSynchronize(st));
  return CABCD_OK;
}

cabcd_status cabcd_primal_objective_t(const cabcd_matrix* XT, const double* y, double lambda,
                                      const double* w, double* r, double* f, void* stream) {
  clear_error();
  Mat M;
  cabcd_status e = check_matrix(XT, "XT", &M);
  if (e != CABCD_OK) return e;
  if (y == nullptr || w == nullptr || !(lambda >= 0.0)) {
    set_error("cabcd_primal_objective_t: y and w must be non-NULL and lambda >= 0");
    return CABCD_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  AuxBuffers B{};
  e = aux_get(M, M.rows, B);
  if (e != CABCD_OK) return e;
  e = check_csr_device(M, B.flag, st);
  if (e != CABCD_OK) return e;
  double* rr = r != nullptr ? r : B.r;
  HIP_TRY(mat_rowdot(M, w, y, -1.0, rr, B.scratch, st));
  if (f != nullptr)
    HIP_TRY(launch_objective(rr, M.rows, 0.5 / (double)M.rows, w, M.cols, 0.5 * lambda, f, B.obj,
                             nullptr, st));
  HIP_TRY(hipStreamSynchronize(st));
  return CABCD_OK;
}

cabcd_status cabcd_dual_to_primal(const cabcd_matrix* XT, const double* alpha, double lambda,
                                  double* w, void* stream) {
  clear_error();
  Mat M;
  cabcd_status e = check_matrix(XT, "XT", &M);
  if (e != CABCD_OK) return e;
  if (alpha == nullptr || w == nullptr || !(lambda > 0.0)) {
    set_error("cabcd_dual_to_primal: alpha and w must be non-NULL and lambda > 0");
    return CABCD_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  AuxBuffers B{};
  e = aux_get(M, 1, B);
  if (e != CABCD_OK) return e;
  e = check_csr_device(M, B.flag, st);
  if (e != CABCD_OK) return e;
  const double n = (double)M.rows;
  HIP_TRY(mat_scatter(M, nullptr, M.rows, alpha, -1.0 / (lambda * n), nullptr, 0.0, false, w,
                      B.scratch, st));
  HIP_TRY(hipStreamSynchronize(st));
  return CABCD_OK;
}

cabcd_status cabcd_primal_residual(const cabcd_matrix* X, double lambda, const double* w,
                                   const double* r, double* rho, double* norm, void* stream) {
  clear_error();
  Mat M;
  cabcd_status e = check_matrix(X, "X", &M);
  if (e != CABCD_OK) return e;
  if (w == nullptr || r == nullptr || !(lambda >= 0.0) || std::isinf(lambda) ||
      (rho == nullptr && norm == nullptr)) {
    set_error("cabcd_primal_residual: w and r must be non-NULL, lambda finite and >= 0, and "
              "rho or norm requested");
    return CABCD_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  AuxBuffers B{};
  e = aux_get(M, M.rows, B);
  if (e != CABCD_OK) return e;
  e = check_csr_device(M, B.flag, st);
  if (e != CABCD_OK) return e;
  HIP_TRY(full_residual(false, M, nullptr, lambda, w, r, rho != nullptr ? rho : B.r,
                        norm != nullptr ? norm : B.obj + objective_scratch_doubles(0, 0), B.scratch,
                        B.obj, nullptr, st));
  HIP_TRY(hipStreamSynchronize(st));
  return CABCD_OK;
}

cabcd_status cabcd_dual_residual(const cabcd_matrix* XT, const double* y, const double* alpha,
                                 const double* w, double* rho, double* norm, void* stream) {
  clear_error();
  Mat M;
  cabcd_status e = check_matrix(XT, "XT", &M);
  if (e != CABCD_OK) return e;
  if (y == nullptr || alpha == nullptr || w == nullptr || (rho == nullptr && norm == nullptr)) {
    set_error("cabcd_dual_residual: y, alpha and w must be non-NULL, and rho or norm requested");
    return CABCD_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  AuxBuffers B{};
  e = aux_get(M, M.rows, B);
  if (e != CABCD_OK) return e;
  e = check_csr_device(M, B.flag, st);
  if (e != CABCD_OK) return e;
  HIP_TRY(full_residual(true, M, y, 0.0, alpha, w, rho != nullptr ? rho : B.r,
                        norm != nullptr ? norm : B.obj + objective_scratch_doubles(0, 0), B.scratch,
                        B.obj, nullptr, st));
  HIP_TRY(hipStreamSynchronize(st));
  return CABCD_OK;
}

cabcd_status cabcd_quantize(const double* A, int64_t rows, int64_t cols, int64_t lda,
                            int32_t dtype, void* Q, int64_t ldq, float* row_scale,
                            void* stream) {
  clear_error();
  if (A == nullptr || Q == nullptr || rows < 1 || cols < 1 || lda < cols || ldq < cols) {
    set_error("cabcd_quantize: need non-NULL A and Q, rows, cols >= 1, lda and ldq >= cols");
    return CABCD_EINVAL;
  }
  if (dtype != CABCD_BF16 && dtype != CABCD_FP8_E4M3) {
    set_error("cabcd_quantize: dtype must be CABCD_BF16 or CABCD_FP8_E4M3");
    return CABCD_EINVAL;
  }
  if (dtype == CABCD_FP8_E4M3 && row_scale == nullptr) {
    set_error("cabcd_quantize: FP8 storage needs row_scale");
    return CABCD_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(launch_quantize(A, rows, cols, lda, dtype, Q, ldq, row_scale, st));
  HIP_TRY(hipStreamSynchronize(st));
  return CABCD_OK;
}

int64_t cabcd_leading_dim(int64_t cols, int32_t dtype) {
  clear_error();
  if (cols < 1 || (dtype != CABCD_F64 && dtype != CABCD_BF16 && dtype != CABCD_FP8_E4M3)) {
    set_error("cabcd_leading_dim: need cols >= 1 and dtype CABCD_F64, CABCD_BF16 or CABCD_FP8_E4M3");
    return -1;
  }
  const int64_t es = dtype == CABCD_F64 ? 8 : dtype == CABCD_BF16 ? 2 : 1;
  int64_t bytes = (cols * es + 255) / 256 * 256;
  // A row stride that is a multiple of 64 KiB sends the same columns of the
  // gathered rows to the same HBM channels: measured on 256 gathered rows of
  // 2 MiB, the LDS-DMA stream of the Gram ran at 5.2 TB/s against 5.9 TB/s
  // with the stride 256 bytes longer.
  if (bytes % 65536 == 0) bytes += 256;
  return bytes / es;
}

size_t cabcd_workspace_bytes(const cabcd_matrix* A, int32_t b, int32_t s) {
  clear_error();
  Mat M;
  if (check_matrix(A, "A", &M) != CABCD_OK) return 0;
  if (b < 1 || s < 1 || (int64_t)s * b > max_rows_per_gram(M)) return 0;
  StepBuffers B{};
  Carve probe{nullptr};
  return layout(probe, B, M, b, s, std::max(A->rows, A->cols), true);
}

}  // extern "C"
