// Streaming vector passes over A (HBM-bound, FP64 accumulation).
//
// gemv_t: out = [beta base | out] + gamma * sum_p A[row(p)]^T v[p]
//   * the deferred companion update of an outer step: primal z += X^T sum_t
//     I_t dw_t (Alg. 2 update after eq. recur), dual w -= 1/(lambda n) X sum_t
//     I_t da_t (Alg. 4 update), with row(p) = idx[p];
//   * the exact recomputation of the full residual (Section 5.1.5): primal
//     r = X^T w - y, dual w = -X a/(lambda n), with row(p) = p.
//   Each thread owns two adjacent columns (16-byte loads) and walks its rows in
//   order; when there are few columns the rows are split over workgroups and
//   the row groups are summed afterwards in group order, so the result is
//   deterministic.
// rowdot: out[p] = s_p A[p] . v + beta base[p] for every row p of dense A
//   (FP64, or BF16 / FP8 codes with row scales s_p): the primal residual from
//   the X^T layout, and the full residuals of the stopping test (Section
//   5.1.5): X r for the primal, X^T w for the dual.  One wave per (row, part);
//   rows longer than one part are cut into parts whose sums are added in
//   part order by a second pass, so the result is deterministic.
// objective: c1 ||a||^2 + c2 ||b||^2 in two deterministic passes.
// resid_norm: t = ca a + cb b (optionally written out) and ||t||_2.
#include "internal.h"
#include "lowp_dev.h"

#include <algorithm>
#include <cmath>

namespace cabcd {
namespace {

constexpr int kVecThreads = 256;
constexpr int kColsPerWG = 2 * kVecThreads;

struct GemvT {
  const double* A;
  int64_t ld, cols;
  const int32_t* idx;
  int64_t m;
  const double* v;
  double gamma;
  const double* base;
  double beta;
  int accumulate;
  double* out;
  double* scratch;   // rg x cols partials when the rows are split
  int64_t rows_per_group;
  int aligned;
};

// VEC: 16-byte loads of column pairs (A 16-byte aligned, even ld).  Eight rows
// at a time: their indices and coefficients (the same for every thread) are
// fetched first, then the eight loads go out together with no branch between
// them, so each thread keeps eight loads in flight (sixteen measured the same).
template <bool VEC>
__global__ __launch_bounds__(kVecThreads) void gemv_t_kernel(GemvT g) {
  constexpr int U = 8;
  const int64_t k = ((int64_t)blockIdx.x * kVecThreads + threadIdx.x) * 2;
  const int64_t p0 = (int64_t)blockIdx.y * g.rows_per_group;
  const int64_t p1 = std::min(g.m, p0 + g.rows_per_group);
  if (k >= g.cols) return;
  const bool two = k + 1 < g.cols;
  const bool vec = VEC && two;
  const gptr<const double> A = glb(g.A) + k;
  typedef double dv2 __attribute__((ext_vector_type(2)));
  double s0 = 0.0, s1 = 0.0;
  int64_t p = p0;
  // the row of entry p: idx[p] (gathered rows) or p; one loop per case keeps
  // the loop body free of branches
  auto batches = [&](auto row) {
    for (; p + U <= p1; p += U) {
      int64_t off[U];
      double c[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        off[q] = row(p + q) * g.ld;
        c[q] = g.v[p + q];
      }
      dv2 x[U];
      if (vec) {
#pragma unroll
        for (int q = 0; q < U; ++q) x[q] = *reinterpret_cast<gptr<const dv2>>(A + off[q]);
      } else {
#pragma unroll
        for (int q = 0; q < U; ++q) {
          x[q].x = A[off[q]];
          x[q].y = two ? A[off[q] + 1] : 0.0;
        }
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        s0 = fma(x[q].x, c[q], s0);
        s1 = fma(x[q].y, c[q], s1);
      }
    }
  };
  if (g.idx != nullptr)
    batches([&](int64_t r) { return (int64_t)g.idx[r]; });
  else
    batches([&](int64_t r) { return r; });
  for (; p < p1; ++p) {
    const gptr<const double> a = A + (g.idx ? (int64_t)g.idx[p] : p) * g.ld;
    const double c = g.v[p];
    s0 = fma(a[0], c, s0);
    if (two) s1 = fma(a[1], c, s1);
  }
  if (g.scratch != nullptr) {
    double* o = g.scratch + (int64_t)blockIdx.y * g.cols + k;
    o[0] = s0;
    if (two) o[1] = s1;
    return;
  }
  double* o = g.out + k;
  const double b0 = g.accumulate ? o[0] : (g.base ? g.beta * g.base[k] : 0.0);
  o[0] = b0 + g.gamma * s0;
  if (two) {
    const double b1 = g.accumulate ? o[1] : (g.base ? g.beta * g.base[k + 1] : 0.0);
    o[1] = b1 + g.gamma * s1;
  }
}

__global__ __launch_bounds__(kVecThreads) void gemv_t_combine_kernel(GemvT g, int groups) {
  const int64_t k = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  if (k >= g.cols) return;
  double s = 0.0;
  for (int r = 0; r < groups; ++r) s += g.scratch[(int64_t)r * g.cols + k];
  const double b0 = g.accumulate ? g.out[k] : (g.base ? g.beta * g.base[k] : 0.0);
  g.out[k] = b0 + g.gamma * s;
}

int gemv_t_groups(int64_t m, int64_t cols) {
  // Split the rows (partials + a combine pass) only when there are too few
  // column tiles to give every CU work; a split pass measured slower than one
  // pass at 256+ tiles.
  const int64_t tiles = (cols + kColsPerWG - 1) / kColsPerWG;
  int64_t rg = (256 + tiles - 1) / tiles;
  rg = std::min<int64_t>(rg, std::max<int64_t>(1, m / 16));
  rg = std::min<int64_t>(rg, 4096);
  return (int)std::max<int64_t>(rg, 1);
}

// Row parts: 64 KiB of A per wave and part (8192 FP64, 32768 BF16, 65536 FP8
// elements), a multiple of the 1 KiB a wave reads per load.
constexpr int64_t kRowPartBytes = 64 * 1024;

struct RowDot {
  const uint8_t* A;
  int64_t ld;          // elements
  const int32_t* idx;  // gathered rows (row p is idx[p]) or NULL
  int64_t rows, cols;
  const float* rs;     // low precision: row scales (NULL = 1)
  const double* v;
  const double* base;
  double beta;
  double* out;
  double* part;        // rows x parts partial sums when parts > 1
  int64_t chunk;       // elements per part
  int parts;
  int vec;             // A rows and v 16-byte aligned
};

// Lane l of a wave reads the 16-byte chunks l, l + 64, ... of its row part,
// four in flight; the lane sums are combined by a butterfly.
template <int FMT>
__global__ __launch_bounds__(kVecThreads) void rowdot_kernel(RowDot g) {
  constexpr int ES = FMT == CABCD_F64 ? 8 : (FMT == CABCD_BF16 ? 2 : 1);
  constexpr int EPC = 16 / ES;     // elements per 16-byte chunk
  constexpr int U = 4;
  const int lane = threadIdx.x & 63;
  const int64_t wv = (int64_t)blockIdx.x * (kVecThreads / 64) + (threadIdx.x >> 6);
  if (wv >= g.rows * g.parts) return;   // wave-uniform
  const int64_t p = wv / g.parts;
  const int q = (int)(wv - p * g.parts);
  const int64_t k0 = (int64_t)q * g.chunk;
  const int64_t k1 = std::min(g.cols, k0 + g.chunk);
  const int64_t ar = g.idx ? (int64_t)g.idx[p] : p;   // row of A
  const gptr<const uint8_t> row = glb(g.A) + ar * g.ld * ES;
  const gptr<const double> v = glb(g.v);
  typedef double dv2 __attribute__((ext_vector_type(2)));
  double acc = 0.0;
  auto chunk_dot = [&](const uint4& x, int64_t k) {
    double e[EPC];
    if constexpr (FMT == CABCD_F64) {
      __builtin_memcpy(e, &x, 16);
    } else {
      ldev::lp_decode_all<FMT>(x, e);
    }
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < EPC; j += 2) {
      const dv2 c = *(gptr<const dv2>)(v + k + j);
      t = fma(e[j], c.x, t);
      t = fma(e[j + 1], c.y, t);
    }
    return t;
  };
  int64_t k = k0 + (int64_t)lane * EPC;
  if (g.vec) {
    typedef unsigned int uv4 __attribute__((ext_vector_type(4)));
    for (; k + (int64_t)(U - 1) * 64 * EPC + EPC <= k1; k += (int64_t)U * 64 * EPC) {
      uint4 x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uv4 t = *(gptr<const uv4>)(row + (k + (int64_t)u * 64 * EPC) * ES);
        x[u] = make_uint4(t.x, t.y, t.z, t.w);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) acc += chunk_dot(x[u], k + (int64_t)u * 64 * EPC);
    }
    for (; k + EPC <= k1; k += 64 * EPC) {
      const uv4 t = *(gptr<const uv4>)(row + k * ES);
      acc += chunk_dot(make_uint4(t.x, t.y, t.z, t.w), k);
    }
  }
  // element by element: unaligned rows, and the ragged end of the part
  for (; k < k1; k += 64 * EPC) {
    const int64_t ke = std::min<int64_t>(k + EPC, k1);
    double t = 0.0;
    for (int64_t kk = k; kk < ke; ++kk) {
      double a;
      if constexpr (FMT == CABCD_F64) {
        a = *(gptr<const double>)(row + kk * 8);
      } else if constexpr (FMT == CABCD_BF16) {
        a = decode_bf16((uint32_t)row[2 * kk] | ((uint32_t)row[2 * kk + 1] << 8));
      } else {
        a = (double)__builtin_amdgcn_cvt_pk_f32_fp8((int)row[kk], false)[0];
      }
      t = fma(a, v[kk], t);
    }
    acc += t;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane != 0) return;
  if (g.parts > 1) {
    g.part[p * g.parts + q] = acc;
    return;
  }
  const double sc = g.rs ? (double)g.rs[ar] : 1.0;
  g.out[p] = sc * acc + (g.base ? g.beta * g.base[p] : 0.0);
}

__global__ __launch_bounds__(kVecThreads) void rowdot_combine_kernel(RowDot g) {
  const int64_t p = (int64_t)blockIdx.x * kVecThreads + threadIdx.x;
  if (p >= g.rows) return;
  double acc = 0.0;
  for (int q = 0; q < g.parts; ++q) acc += g.part[p * g.parts + q];
  const double sc = g.rs ? (double)g.rs[g.idx ? (int64_t)g.idx[p] : p] : 1.0;
  g.out[p] = sc * acc + (g.base ? g.beta * g.base[p] : 0.0);
}

int rowdot_parts(int64_t rows, int64_t cols, int es, int64_t* chunk) {
  const int64_t per = kRowPartBytes / es;
  // Split long rows only when the rows alone give fewer than 8192 waves.
  int64_t parts = (cols + per - 1) / per;
  if (rows >= 8192) parts = 1;
  parts = std::max<int64_t>(1, std::min<int64_t>(parts, 4096));
  int64_t c = (cols + parts - 1) / parts;
  c = (c + 1023) / 1024 * 1024;   // whole 16-byte chunks of every element size
  *chunk = c;
  return (int)((cols + c - 1) / c);
}

constexpr int kObjBlocks = 512;

__global__ __launch_bounds__(kVecThreads) void sumsq_kernel(const double* __restrict__ a,
                                                            int64_t na,
                                                            const double* __restrict__ b,
                                                            int64_t nb,
                                                            double* __restrict__ part) {
  __shared__ double red[kVecThreads];
  for (int which = 0; which < 2; ++which) {
    const double* x = which == 0 ? a : b;
    const int64_t n = which == 0 ? na : nb;
    double s = 0.0;
    if (x != nullptr)
      for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n;
           i += (int64_t)gridDim.x * kVecThreads)
        s = fma(x[i], x[i], s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kVecThreads / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[which * gridDim.x + blockIdx.x] = red[0];
    __syncthreads();
  }
}

__global__ __launch_bounds__(kVecThreads) void objective_final_kernel(
    const double* __restrict__ part, int blocks, double c1, double c2, double* __restrict__ out,
    int* __restrict__ status) {
  __shared__ double red[2][kVecThreads];
  for (int which = 0; which < 2; ++which) {
    double s = 0.0;
    for (int i = threadIdx.x; i < blocks; i += kVecThreads) s += part[which * blocks + i];
    red[which][threadIdx.x] = s;
  }
  __syncthreads();
  for (int w = kVecThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double f = c1 * red[0][0] + c2 * red[1][0];
    *out = f;
    if (status != nullptr && !isfinite(f)) raise_status(status, DEV_NONFINITE);
  }
}

// t = ca a + cb b (b may be NULL); t written to vec when non-NULL; per-block
// sums of t^2 to part.
__global__ __launch_bounds__(kVecThreads) void comb_sumsq_kernel(
    const double* __restrict__ a, double ca, const double* __restrict__ b, double cb, int64_t n,
    double* __restrict__ vec, double* __restrict__ part) {
  __shared__ double red[kVecThreads];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kVecThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kVecThreads) {
    const double t = ca * a[i] + (b ? cb * b[i] : 0.0);
    if (vec) vec[i] = t;
    s = fma(t, t, s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kVecThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kVecThreads) void norm_final_kernel(
    const double* __restrict__ part, int blocks, double* __restrict__ out,
    int* __restrict__ status) {
  __shared__ double red[kVecThreads];
  double s = 0.0;
  for (int i = threadIdx.x; i < blocks; i += kVecThreads) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kVecThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double r = sqrt(red[0]);
    *out = r;
    if (status != nullptr && !isfinite(r)) raise_status(status, DEV_NONFINITE);
  }
}

}  // namespace

size_t rowdot_scratch_doubles(int64_t rows, int64_t cols, int dtype) {
  int64_t chunk = 0;
  const int es = dtype == CABCD_F64 ? 8 : (dtype == CABCD_BF16 ? 2 : 1);
  const int parts = rowdot_parts(rows, cols, es, &chunk);
  return parts > 1 ? (size_t)parts * (size_t)rows : 0;
}

static hipError_t launch_rowdot_any(int dtype, const void* A, int64_t ld, const int32_t* idx,
                                    int64_t rows, int64_t cols, const float* rs,
                                    const double* v, const double* base, double beta,
                                    double* out, double* scratch, hipStream_t st);

hipError_t launch_rowdot(int dtype, const void* A, int64_t ld, int64_t rows, int64_t cols,
                         const float* rs, const double* v, const double* base, double beta,
                         double* out, double* scratch, hipStream_t st) {
  return launch_rowdot_any(dtype, A, ld, nullptr, rows, cols, rs, v, base, beta, out, scratch,
                           st);
}

hipError_t launch_rowdot_rows(int dtype, const void* A, int64_t ld, const int32_t* idx,
                              int64_t m, int64_t cols, const float* rs, const double* v,
                              double* out, double* scratch, hipStream_t st) {
  return launch_rowdot_any(dtype, A, ld, idx, m, cols, rs, v, nullptr, 0.0, out, scratch, st);
}

static hipError_t launch_rowdot_any(int dtype, const void* A, int64_t ld, const int32_t* idx,
                                    int64_t rows, int64_t cols, const float* rs,
                                    const double* v, const double* base, double beta,
                                    double* out, double* scratch, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  const int es = dtype == CABCD_F64 ? 8 : (dtype == CABCD_BF16 ? 2 : 1);
  RowDot g{};
  g.A = static_cast<const uint8_t*>(A);
  g.ld = ld;
  g.idx = idx;
  g.rows = rows;
  g.cols = cols;
  g.rs = dtype == CABCD_F64 ? nullptr : rs;
  g.v = v;
  g.base = base;
  g.beta = beta;
  g.out = out;
  g.parts = rowdot_parts(rows, cols, es, &g.chunk);
  g.part = g.parts > 1 ? scratch : nullptr;
  if (g.parts > 1 && scratch == nullptr) return hipErrorInvalidValue;
  g.vec = ((reinterpret_cast<uintptr_t>(A) & 15) == 0 && ((ld * es) & 15) == 0 &&
           (reinterpret_cast<uintptr_t>(v) & 15) == 0)
              ? 1
              : 0;
  const int64_t waves = rows * g.parts;
  const int64_t per = kVecThreads / 64;
  const dim3 grid((unsigned)((waves + per - 1) / per));
  if (dtype == CABCD_F64)
    hipLaunchKernelGGL(rowdot_kernel<CABCD_F64>, grid, dim3(kVecThreads), 0, st, g);
  else if (dtype == CABCD_BF16)
    hipLaunchKernelGGL(rowdot_kernel<CABCD_BF16>, grid, dim3(kVecThreads), 0, st, g);
  else
    hipLaunchKernelGGL(rowdot_kernel<CABCD_FP8_E4M3>, grid, dim3(kVecThreads), 0, st, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || g.parts == 1) return e;
  hipLaunchKernelGGL(rowdot_combine_kernel, dim3((unsigned)((rows + kVecThreads - 1) / kVecThreads)),
                     dim3(kVecThreads), 0, st, g);
  return hipGetLastError();
}

hipError_t launch_resid_norm(const double* a, double ca, const double* b, double cb, int64_t n,
                             double* vec, double* norm, double* scratch, int* status,
                             hipStream_t st) {
  hipLaunchKernelGGL(comb_sumsq_kernel, dim3(kObjBlocks), dim3(kVecThreads), 0, st, a, ca, b, cb,
                     n, vec, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(norm_final_kernel, dim3(1), dim3(kVecThreads), 0, st, scratch, kObjBlocks,
                     norm, status);
  return hipGetLastError();
}

size_t gemv_t_scratch_doubles(int64_t m, int64_t cols) {
  const int rg = gemv_t_groups(m, cols);
  return rg > 1 ? (size_t)rg * (size_t)cols : 0;
}

hipError_t launch_gemv_t(const double* A, int64_t ld, int64_t cols, const int32_t* idx,
                         int64_t m, const double* v, double gamma, const double* base,
                         double beta, bool accumulate, double* out, double* scratch,
                         hipStream_t st) {
  if (cols <= 0) return hipSuccess;
  GemvT g{};
  g.A = A;
  g.ld = ld;
  g.cols = cols;
  g.idx = idx;
  g.m = m;
  g.v = v;
  g.gamma = gamma;
  g.base = base;
  g.beta = beta;
  g.accumulate = accumulate ? 1 : 0;
  g.out = out;
  g.aligned = ((reinterpret_cast<uintptr_t>(A) & 15) == 0 && (ld & 1) == 0) ? 1 : 0;
  const int rg = gemv_t_groups(m, cols);
  g.rows_per_group = (m + rg - 1) / rg;
  g.scratch = rg > 1 ? scratch : nullptr;
  if (rg > 1 && scratch == nullptr) return hipErrorInvalidValue;
  const int64_t tiles = (cols + kColsPerWG - 1) / kColsPerWG;
  if (g.aligned)
    hipLaunchKernelGGL(gemv_t_kernel<true>, dim3((unsigned)tiles, (unsigned)rg),
                       dim3(kVecThreads), 0, st, g);
  else
    hipLaunchKernelGGL(gemv_t_kernel<false>, dim3((unsigned)tiles, (unsigned)rg),
                       dim3(kVecThreads), 0, st, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || rg == 1) return e;
  hipLaunchKernelGGL(gemv_t_combine_kernel,
                     dim3((unsigned)((cols + kVecThreads - 1) / kVecThreads)),
                     dim3(kVecThreads), 0, st, g, rg);
  return hipGetLastError();
}

size_t objective_scratch_doubles(int64_t, int64_t) { return 2 * kObjBlocks; }

hipError_t launch_objective(const double* a, int64_t na, double c1, const double* b,
                            int64_t nb, double c2, double* out, double* scratch, int* status,
                            hipStream_t st) {
  hipLaunchKernelGGL(sumsq_kernel, dim3(kObjBlocks), dim3(kVecThreads), 0, st, a, na, b, nb,
                     scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(objective_final_kernel, dim3(1), dim3(kVecThreads), 0, st, scratch,
                     kObjBlocks, c1, c2, out, status);
  return hipGetLastError();
}

}  // namespace cabcd
