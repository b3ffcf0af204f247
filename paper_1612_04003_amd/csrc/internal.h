// Internal declarations shared by the translation units of libcabcd.
// Not part of the public interface (that is include/cabcd.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/cabcd.h"

namespace cabcd {

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...);
void clear_error();

// Device status word values written by kernels (0 = fine).
enum DeviceStatus : int { DEV_OK = 0, DEV_NOTSPD = 1, DEV_NONFINITE = 2 };

// ------------------------------------------------------------------ sampler
hipError_t launch_sample(uint64_t seed, int64_t h0, int64_t count, int b, int64_t range,
                         int32_t* idx, hipStream_t st);

// ------------------------------------------------------------------ dense FP64 Gram
// Plan of one Gram launch over the gathered rows of a dense FP64 matrix.
struct GramPlan {
  int nb;          // 16-row blocks covering m rows (1, 2, 4, 8 or 16)
  int nblk;        // lower-triangular 16x16 blocks: nb*(nb+1)/2
  int kt;          // columns per LDS tile
  int64_t chunk;   // columns per workgroup (multiple of kt)
  int nsplit;      // workgroups along the reduction dimension
};
GramPlan plan_gram_f64(int m, int64_t cols);
size_t gram_partial_doubles(const GramPlan& p);   // partial G + partial Yu
// partials: nsplit * (nblk*256 + 16*nb) doubles.
hipError_t launch_gram_f64(const GramPlan& p, const double* A, int64_t ld, int64_t cols,
                           const int32_t* idx, int m, const double* u, double* partials,
                           hipStream_t st);
// G (m x m, ld m, both triangles) = scale * sum(partials) + shift * E,
// E = I (overlap = false) or E_pq = [idx_p == idx_q] (overlap = true).
// Yu (may be NULL) = sum of the partial Yu.
hipError_t launch_gram_reduce(const GramPlan& p, const double* partials, const int32_t* idx,
                              int m, double scale, double shift, bool overlap, double* G,
                              double* Yu, hipStream_t st);

// ------------------------------------------------------------------ fused solve
// One outer step's s block solves through the unrolled recurrence, followed by
// the coordinate scatter-add x[idx] += delta (single writer per coordinate,
// block order).  Gov is the overlap-augmented Gram (m x m, ld m).
//   mode 0 (primal): c_p = -lambda x[idx_p] - Yu_p / n
//   mode 1 (dual)  : c_p = (Yu_p - x[idx_p] - y[idx_p]) / n
struct SolveArgs {
  const double* G;
  const double* Yu;
  const int32_t* idx;
  const double* y;     // dual only
  double* x;           // coordinate vector (w primal, alpha dual), updated
  double* delta;       // out, m
  int* status;         // device status word
  int m, b, s;
  int mode;
  double lambda, n;
};
hipError_t launch_solve(const SolveArgs& a, hipStream_t st);

// ------------------------------------------------------------------ vector kernels
// out[k] = (accumulate ? out[k] : beta*base[k]) + gamma * sum_p A[row(p)][k] * v[p]
// for k < cols, p < m, row(p) = idx ? idx[p] : p.  Deterministic order.
// Needs a scratch of gemv_t_scratch_doubles(m, cols) doubles (may be 0).
size_t gemv_t_scratch_doubles(int64_t m, int64_t cols);
hipError_t launch_gemv_t(const double* A, int64_t ld, int64_t cols, const int32_t* idx,
                         int64_t m, const double* v, double gamma, const double* base,
                         double beta, bool accumulate, double* out, double* scratch,
                         hipStream_t st);
// out[p] = sum_k A[p][k] v[k] + beta*base[p], p < rows.
hipError_t launch_gemv_n(const double* A, int64_t ld, int64_t rows, int64_t cols,
                         const double* v, const double* base, double beta, double* out,
                         hipStream_t st);
// *out = c1 * ||a||^2 + c2 * ||b||^2 (b may be NULL), deterministic; sets the
// status word to DEV_NONFINITE when the result is not finite (status may be NULL).
size_t objective_scratch_doubles(int64_t na, int64_t nb);
hipError_t launch_objective(const double* a, int64_t na, double c1, const double* b,
                            int64_t nb, double c2, double* out, double* scratch, int* status,
                            hipStream_t st);

}  // namespace cabcd
