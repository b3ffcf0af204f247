// Internal declarations shared by the translation units of libcabcd.
// Not part of the public interface (that is include/cabcd.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/cabcd.h"

namespace cabcd {

// Workgroup barrier that orders LDS traffic only.  __syncthreads() also waits
// for every outstanding global load of the wave, which would drain register
// prefetches issued ahead of the barrier.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Global-memory view of a device pointer.  A pointer that reaches device code
// through memory or through a non-inlined call is generic to the compiler, and
// generic (flat) accesses also count against the LDS wait counter, so an LDS
// barrier would wait for global prefetches still in flight.  Accesses through
// the cast compile to global_* instructions.
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> glb(T* p) {
  return (gptr<T>)p;
}

// Exact decoding of BF16 storage to FP64.  (E4M3 codes are decoded by the
// hardware conversion v_cvt_pk_f32_fp8, which reads 0x7F / 0xFF as NaN, the same
// reading as the FP8 matrix instructions.)
__device__ __forceinline__ double decode_bf16(uint32_t b) {
  return (double)__uint_as_float((b & 0xFFFFu) << 16);
}

// ------------------------------------------------------------------ errors
void set_error(const char* fmt, ...);
void clear_error();

// Device status word values written by kernels (0 = fine).  A larger value
// outranks a smaller one: a block that is not positive definite makes its
// solve and every later value non-finite, and the status must name the cause.
enum DeviceStatus : int { DEV_OK = 0, DEV_NONFINITE = 1, DEV_NOTSPD = 2 };

// Records a device-detected error in the status word, keeping the highest
// ranked one (integer atomic maximum, so concurrent writers agree).
__device__ __forceinline__ void raise_status(int* status, int code) {
  atomicMax(status, code);
}

// ------------------------------------------------------------------ sampler
// Counter-based block sampler (the sampling step of Alg. 1-4): b distinct
// coordinates per inner iteration, uniform without replacement, keyed by
// (seed, h) only, so every consumer of the same seed draws the same blocks.
//   SplitMix64 output t of a stream seeded with x: mix64(x + GAMMA*(t+1))
//     (Steele, Lea & Flood, OOPSLA 2014; finaliser constants of that paper)
//   key(h) = output h of the stream seeded with `seed`
//   word t = upper 32 bits of output t of the stream seeded with key(h)
//   bounded(range): Lemire's multiply-shift with rejection (TOMACS 2019)
//   block: Floyd's algorithm (Bentley & Floyd, CACM 1987), insertion order.
namespace smp {
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t stream_out(uint64_t seed, uint64_t t) {
  return mix64(seed + kGamma * (t + 1));
}

// The b indices of inner iteration h into out[0..b) (out may be in LDS).
__device__ __forceinline__ void sample_block(uint64_t seed, int64_t h, int b, int64_t range,
                                             int32_t* out) {
  const uint64_t key = stream_out(seed, (uint64_t)h);
  uint64_t t = 0;
  int filled = 0;
  for (int64_t j = range - b; j < range; ++j) {
    const uint64_t m = (uint64_t)(j + 1);          // draw uniformly from [0, j]
    uint64_t x = stream_out(key, t++) >> 32;
    uint64_t prod = x * m;
    uint32_t low = (uint32_t)prod;
    if (low < m) {
      const uint32_t thr = (uint32_t)((0x100000000ull - m) % m);
      while (low < thr) {
        x = stream_out(key, t++) >> 32;
        prod = x * m;
        low = (uint32_t)prod;
      }
    }
    const int32_t v = (int32_t)(prod >> 32);
    bool seen = false;
    for (int q = 0; q < filled; ++q) seen |= (out[q] == v);
    out[filled++] = seen ? (int32_t)j : v;
  }
}
}  // namespace smp

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
  int rpw;         // block rows per wave (2: eight waves, 4: four waves)
};
GramPlan plan_gram_f64(int m, int64_t cols);
// The deferred companion update of the previous outer step (Alg. 2: r += gamma
// Y^T delta with the previous step's rows and delta; Alg. 4 the same for w):
// its 256 rows idx (all valid), delta (256), the scale gamma, and the
// companion r, read and then rewritten in place, each column by the one
// workgroup whose slab holds it.
struct D16Upd {
  const int32_t* idx;
  const double* delta;
  double gamma;
  double* r;
};
// The dense 256-row Gram can take the previous step's update along
// (launch_gram_f64_upd) when its plan runs the LDS-DMA kernel: 16-byte
// aligned rows with an even ld, m = 256.
bool gram_f64_takes_update(const GramPlan& p, const double* A, int64_t ld, int m);
// The 256-row Gram (nsteps = 1) of gram_f64 with the previous step's update
// applied to r first; the Y r partials use the updated r.
hipError_t launch_gram_f64_upd(const GramPlan& p, const double* A, int64_t ld, int64_t cols,
                               const int32_t* idx, int m, double* partials, const D16Upd& up,
                               hipStream_t st);
// The same update alone, by the same device code (so its rounding matches).
hipError_t launch_update_f64(const GramPlan& p, const double* A, int64_t ld, int64_t cols,
                             const D16Upd& up, hipStream_t st);
size_t gram_partial_doubles(const GramPlan& p);   // partial G + partial Yu
// partials: nsplit * (nblk*256 + 16*nb) doubles.
// nsteps > 1: the Grams of nsteps row lists in one launch (step k reads
// idx + k m, writes partials + k gram_partial_doubles(p), its Y u with the
// same u).
hipError_t launch_gram_f64(const GramPlan& p, const double* A, int64_t ld, int64_t cols,
                           const int32_t* idx, int m, const double* u, double* partials,
                           hipStream_t st, int nsteps = 1);
// G (m x m, ld m, both triangles) = scale * sum(partials) + shift * E,
// E = I (overlap = false) or E_pq = [idx_p == idx_q] (overlap = true).
// Yu (may be NULL) = sum of the partial Yu.
// layout 0: partial block entries in the FP64 MFMA output order; 1: in the FP32
// MFMA output order; 2: as 1, the block entries stored as FP32 (the first
// nblk*256 floats of each partial set; Y u stays FP64 at its place).  rs (may be NULL) are row scales of A applied as
// rs[idx_p] rs[idx_q] to G and rs[idx_p] to Y u.
// nsteps > 1: step k reduces partials + k gram_partial_doubles(p) into
// G + k m^2 (Yu must be NULL).
// add (may be NULL): nsteps m x m row-major terms (read at row >= col) added
// to the partial sums before scaling.
hipError_t launch_gram_reduce(const GramPlan& p, const double* partials, const int32_t* idx,
                              int m, double scale, double shift, bool overlap, double* G,
                              double* Yu, hipStream_t st, int layout = 0,
                              const float* rs = nullptr, int nsteps = 1,
                              const double* add = nullptr);
// Grams of m in (256, 512] rows from 256-row Grams (plan p of 256 rows, nb 16),
// for ngram row lists idx + k m: launch_big_index builds per Gram the index
// lists ia (512: the rows padded with the first) and ib (nc = big_cross_steps(m)
// lists of 256: half-bands [rows 128 x.. ; rows 256 + 128 y..]); the Gram
// launches then write 2 ngram partial sets (ia as 2 ngram steps, with Y u for
// a single Gram) followed by nc ngram sets (ib), each of
// gram_partial_doubles(p), which launch_gram_reduce_big sums into G + k m^2
// (adding add + k m^2 when given) and Y u.
hipError_t launch_big_index(const int32_t* idx, int m, int32_t* ia, int32_t* ib, hipStream_t st,
                            int ngram = 1);
int big_cross_steps(int m);
hipError_t launch_gram_reduce_big(const GramPlan& p, const double* partials, const int32_t* idx,
                                  int m, double scale, double shift, bool overlap, double* G,
                                  double* Yu, hipStream_t st, int layout = 0,
                                  const float* rs = nullptr, int ngram = 1,
                                  const double* add = nullptr);

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
  int pre_inverted;    // 1: the diagonal blocks of G hold Gamma_j^-1 (launch_invert_diag)
};
constexpr int kSolveMaxRows = 1024;
constexpr int kSolveMaxB = 32;
constexpr size_t kSolveMaxLds = 160 * 1024;
size_t solve_lds_bytes(int m, int b);   // dynamic LDS of one solve launch
hipError_t launch_solve(const SolveArgs& a, hipStream_t st);
// Inverts in place the diagonal b x b blocks (Gamma_j, b <= 16) of nsteps
// consecutive m x m Grams (s = m / b blocks each), as the solve would; a pivot
// that is not positive sets *status to "not positive definite".
hipError_t launch_invert_diag(double* G, int nsteps, int m, int b, int* status, hipStream_t st);

// ------------------------------------------------------------------ low precision
// Codes of A (rows x cols, FP64, ld lda) into Q (ld ldq elements) with FP32
// row scales (FP8: amax/448; BF16: 1, row_scale may be NULL).
hipError_t launch_quantize(const double* A, int64_t rows, int64_t cols, int64_t lda, int dtype,
                           void* Q, int64_t ldq, float* row_scale, hipStream_t st);
GramPlan plan_gram_lp(int m, int64_t cols, int dtype);
// Partial layout a low-precision Gram launch of plan p writes for A (ld in
// elements): 1 = FP64 entries in the FP32 MFMA output order, 2 = the same
// entries stored as FP32 (the LDS-DMA kernel); Y u is FP64 in both.
int gram_lp_partial_layout(const GramPlan& p, int dtype, const void* A, int64_t ld);
// Gram partials of stored codes (FP32 MFMA accumulation, FP64 partials; the
// partial blocks use the FP32 MFMA output layout) plus Y u of the codes in FP64.
hipError_t launch_gram_lp(const GramPlan& p, int dtype, const void* A, int64_t ld, int64_t cols,
                          const int32_t* idx, int m, const double* u, double* partials,
                          hipStream_t st, int nsteps = 1);
// out = [beta base | out] + gamma sum_p s[row(p)] v[p] decode(Q[row(p)]), FP64.
hipError_t launch_gemv_t_lp(int dtype, const void* A, int64_t ld, int64_t cols, const float* rs,
                            const int32_t* idx, int64_t m, const double* v, double gamma,
                            const double* base, double beta, bool accumulate, double* out,
                            hipStream_t st);

// ------------------------------------------------------------------ CSR kernels
struct CsrView {
  const int64_t* rowptr;
  const int32_t* colidx;
  const double* vals;
  int64_t rows, cols, nnz;
};
constexpr int kCsrMaxRows = 1024;   // gathered rows one CSR Gram launch handles
// Gov (or plain G) and Y u of the rows idx[0..m) of a CSR matrix, m <= 1024.
hipError_t launch_csr_gram(const CsrView& A, const int32_t* idx, int m, const double* u,
                           double scale, double shift, bool overlap, double* G, double* Yu,
                           hipStream_t st);
// out[col] += gamma * v[p] * A[row(p)][col], row(p) = idx ? idx[p] : p (atomic adds).
// The Grams of nsteps outer steps of m rows each in one launch (step k uses
// idx + k m and writes G + k m^2; no Y u): the Gram depends on the indices only.
hipError_t launch_csr_gram_steps(const CsrView& A, const int32_t* idx, int m, int nsteps,
                                 double scale, double shift, bool overlap, double* G,
                                 hipStream_t st);
// out[p] = A[idx[p]] . v for p < m (the Y u of a step whose Gram came from
// launch_csr_gram_steps).
hipError_t launch_csr_rowdot_rows(const CsrView& A, const int32_t* idx, int64_t m,
                                  const double* v, double* out, hipStream_t st);
// The Grams of nsteps outer steps computed ahead, split by column popularity
// (csr_split.hip): the heavy columns (at most 512 of the most popular) through
// a dense panel on the matrix cores, the light ones through per-step column
// lists (per-step tables indexed by column: scratch grows with cols).  csr_split_prepare numbers the heavy columns (once per matrix; ws
// holds csr_split_prepare_ints(A) ints) and reads the statistics the layout
// needs back to the host.  m <= 512.
struct CsrSplitInfo {
  const int* hmap;   // per column: heavy slot (column order) or -1
  const int* hcol;   // per heavy slot: its column
  int heavy;         // heavy columns
  int maxrow;        // longest row
  int maxlight;      // most light entries in one row
};
struct SplitLayout {
  int hp;            // panel width (heavy rounded up to 16; 0 without heavy columns)
  int nblk;          // scan workgroups over the columns
  int64_t cs;        // per-step column-table stride (nblk whole scan workgroups)
  int64_t lcap;      // light list capacity per step
  GramPlan plan;     // the panel Gram's plan
  size_t doubles, ints;   // scratch of one launch
};
size_t csr_split_prepare_ints(const CsrView& A);
hipError_t csr_split_prepare(const CsrView& A, int* ws, CsrSplitInfo* info, hipStream_t st);
SplitLayout csr_split_layout(const CsrSplitInfo& info, int64_t cols, int m, int nsteps);
hipError_t launch_csr_gram_split(const CsrView& A, const CsrSplitInfo& info, const int32_t* idx,
                                 int m, int nsteps, double scale, double shift, bool overlap,
                                 double* G, double* dws, int* iws, hipStream_t st);
// The companion update out += gamma Y^T delta of step `step` of the split
// launch of nsteps steps that is still in (dws, iws): one writer per column,
// fixed summation order (heavy columns from the step's dense panel, light ones
// from its row-sorted column lists).
hipError_t launch_csr_update_split(const CsrView& A, const CsrSplitInfo& info,
                                   const int32_t* idx, int m, int nsteps, int step,
                                   const double* delta, double gamma, double* out, double* dws,
                                   int* iws, hipStream_t st);
hipError_t launch_csr_scatter(const CsrView& A, const int32_t* idx, int64_t m, const double* v,
                              double gamma, double* out, hipStream_t st);
// out[p] = A[p] . v + beta * base[p] for every row.
hipError_t launch_csr_rowdot(const CsrView& A, const double* v, const double* base, double beta,
                             double* out, hipStream_t st);
// out[i] = beta * base[i] (base may be NULL: zero).
hipError_t launch_fill(double* out, int64_t n, const double* base, double beta, hipStream_t st);
// Sets *bad (device int) if the CSR structure is malformed.
hipError_t launch_csr_check(const CsrView& A, int* bad, hipStream_t st);

// ------------------------------------------------------------------ vector kernels
// out[k] = (accumulate ? out[k] : beta*base[k]) + gamma * sum_p A[row(p)][k] * v[p]
// for k < cols, p < m, row(p) = idx ? idx[p] : p.  Deterministic order.
// Needs a scratch of gemv_t_scratch_doubles(m, cols) doubles (may be 0).
size_t gemv_t_scratch_doubles(int64_t m, int64_t cols);
hipError_t launch_gemv_t(const double* A, int64_t ld, int64_t cols, const int32_t* idx,
                         int64_t m, const double* v, double gamma, const double* base,
                         double beta, bool accumulate, double* out, double* scratch,
                         hipStream_t st);
// out[p] = s_p sum_k A[p][k] v[k] + beta*base[p], p < rows, for dense A of
// element type dtype (row scales rs for BF16 / FP8, NULL = 1; ignored for
// FP64).  Needs a scratch of rowdot_scratch_doubles(rows, cols, dtype) doubles
// (may be 0).  Deterministic.
size_t rowdot_scratch_doubles(int64_t rows, int64_t cols, int dtype);
hipError_t launch_rowdot(int dtype, const void* A, int64_t ld, int64_t rows, int64_t cols,
                         const float* rs, const double* v, const double* base, double beta,
                         double* out, double* scratch, hipStream_t st);
// The same for the gathered rows idx[0..m): out[p] = s_row A[idx[p]] . v.
hipError_t launch_rowdot_rows(int dtype, const void* A, int64_t ld, const int32_t* idx,
                              int64_t m, int64_t cols, const float* rs, const double* v,
                              double* out, double* scratch, hipStream_t st);
// t = ca a + cb b (b may be NULL), written to vec when non-NULL, and *norm =
// ||t||_2 (device scalar); scratch holds objective_scratch_doubles() doubles;
// a non-finite norm sets the status word (status may be NULL).  Deterministic.
hipError_t launch_resid_norm(const double* a, double ca, const double* b, double cb, int64_t n,
                             double* vec, double* norm, double* scratch, int* status,
                             hipStream_t st);
// *out = c1 * ||a||^2 + c2 * ||b||^2 (b may be NULL), deterministic; sets the
// status word to DEV_NONFINITE when the result is not finite (status may be NULL).
size_t objective_scratch_doubles(int64_t na, int64_t nb);
hipError_t launch_objective(const double* a, int64_t na, double c1, const double* b,
                            int64_t nb, double c2, double* out, double* scratch, int* status,
                            hipStream_t st);

}  // namespace cabcd
