// Low-precision storage of A for the mixed-precision path: quantisation,
// decoding, and the FP64-accumulating streaming passes over BF16 / FP8 rows.
//
// Storage formats (rounding FP64 directly to nearest, ties to even):
//   BF16      1 sign, 8 exponent (bias 127), 7 fraction bits; overflow -> inf.
//   FP8 E4M3  OCP "fn" variant: 1 sign, 4 exponent (bias 7), 3 fraction bits,
//             largest finite 448, no infinities; rounding saturates at +-448.
//             Row i is stored as q = E4M3(x / s_i), s_i = fp32(amax_i / 448)
//             (1 for an all-zero row), so the stored matrix is X^ = diag(s) Q.
// The method then runs on X^ (exact in FP64): the Gram uses the stored codes on
// the matrix cores with FP32 accumulation and applies s_p s_q in FP64, while
// Y u, the companion updates and the exact recomputation decode to FP64.
#include "lowp_dev.h"

#include <algorithm>
#include <cmath>

namespace cabcd {
namespace {

using namespace ldev;

constexpr int kQThreads = 256;

// Nearest value on a grid with `mant` fraction bits and minimum normal
// exponent `emin` (subnormal spacing below it), ties to even.
__device__ __forceinline__ double round_grid(double v, int mant, int emin) {
  if (v == 0.0) return v;
  int ex;
  (void)frexp(v, &ex);                 // |v| = f 2^ex, 0.5 <= f < 1
  const int e = max(ex - 1, emin);
  return ldexp(rint(ldexp(v, mant - e)), e - mant);
}

__device__ __forceinline__ uint16_t encode_bf16(double v) {
  double q = round_grid(v, 7, -126);
  const double mx = 0x1.fep127;       // (2 - 2^-7) 2^127
  if (fabs(q) > mx) q = copysign(INFINITY, q);
  const float f = (float)q;           // exact: BF16 values are FP32 values
  return (uint16_t)(__float_as_uint(f) >> 16);
}

__device__ __forceinline__ uint8_t encode_e4m3(double v) {
  double q = round_grid(v, 3, -6);
  q = fmin(fmax(q, -448.0), 448.0);
  const uint8_t sign = signbit(q) ? 0x80 : 0;
  const double a = fabs(q);
  if (a < 0x1p-6) return sign | (uint8_t)rint(a * 512.0);          // E = 0: a = M 2^-9
  int ex;
  const double f = frexp(a, &ex);                                    // a = f 2^ex
  const int e = ex - 1;                                              // a = (2f) 2^e
  const int frac = (int)rint((2.0 * f - 1.0) * 8.0);
  return sign | (uint8_t)(((e + 7) << 3) | frac);
}

__global__ __launch_bounds__(kQThreads) void quantize_kernel(const double* __restrict__ A,
                                                             int64_t cols, int64_t lda,
                                                             int dtype, void* __restrict__ Q,
                                                             int64_t ldq,
                                                             float* __restrict__ row_scale) {
  __shared__ double red[kQThreads];
  const int64_t r = blockIdx.x;
  const double* a = A + r * lda;
  if (dtype == CABCD_BF16) {
    uint16_t* q = static_cast<uint16_t*>(Q) + r * ldq;
    for (int64_t k = threadIdx.x; k < cols; k += kQThreads) q[k] = encode_bf16(a[k]);
    if (row_scale != nullptr && threadIdx.x == 0) row_scale[r] = 1.0f;
    return;
  }
  double mx = 0.0;
  for (int64_t k = threadIdx.x; k < cols; k += kQThreads) mx = fmax(mx, fabs(a[k]));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = kQThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  const double amax = red[0];
  const float s = amax == 0.0 ? 1.0f : (float)(amax / 448.0);
  const double sd = (double)s;
  uint8_t* q = static_cast<uint8_t*>(Q) + r * ldq;
  for (int64_t k = threadIdx.x; k < cols; k += kQThreads) q[k] = encode_e4m3(a[k] / sd);
  if (threadIdx.x == 0) row_scale[r] = s;
}

template <int NB, int FMT>
__global__ __launch_bounds__(kLpThreads) void gram_lp_kernel(
    const uint8_t* __restrict__ A, int64_t ld, int64_t cols, const int32_t* __restrict__ idx,
    int m, const double* __restrict__ u, int64_t chunk, double* __restrict__ partials,
    int64_t pstride, int aligned) {
  using C = LpCfg<NB, FMT>;
  __shared__ __attribute__((aligned(16))) uint8_t lds[C::LDS];
  idx += (int64_t)blockIdx.y * m;            // several outer steps per launch
  partials += (int64_t)blockIdx.y * pstride;
  const int64_t k_begin = (int64_t)blockIdx.x * chunk;
  const int64_t k_end = std::min(cols, k_begin + chunk);
  gram_lp_slab<NB, FMT>(A, ld, k_begin, k_end, idx, m, u,
                        partials + (int64_t)blockIdx.x * (C::NBLK * 256 + C::SBP), aligned, lds);
}

template <int NB, int FMT>
hipError_t launch_lp_nb(const GramPlan& p, const void* A, int64_t ld, int64_t cols,
                        const int32_t* idx, int m, int nsteps, const double* u,
                        double* partials, hipStream_t st) {
  using C = LpCfg<NB, FMT>;
  const int aligned =
      ((reinterpret_cast<uintptr_t>(A) & 15) == 0 && ((ld * C::ES) & 15) == 0) ? 1 : 0;
  hipLaunchKernelGGL((gram_lp_kernel<NB, FMT>), dim3((unsigned)p.nsplit, (unsigned)nsteps),
                     dim3(kLpThreads), 0, st, static_cast<const uint8_t*>(A), ld, cols, idx, m, u,
                     p.chunk, partials, (int64_t)gram_partial_doubles(p), aligned);
  return hipGetLastError();
}

template <int FMT>
hipError_t launch_lp_fmt(const GramPlan& p, const void* A, int64_t ld, int64_t cols,
                         const int32_t* idx, int m, int nsteps, const double* u,
                         double* partials, hipStream_t st) {
  switch (p.nb) {
    case 1: return launch_lp_nb<1, FMT>(p, A, ld, cols, idx, m, nsteps, u, partials, st);
    case 2: return launch_lp_nb<2, FMT>(p, A, ld, cols, idx, m, nsteps, u, partials, st);
    case 4: return launch_lp_nb<4, FMT>(p, A, ld, cols, idx, m, nsteps, u, partials, st);
    case 8: return launch_lp_nb<8, FMT>(p, A, ld, cols, idx, m, nsteps, u, partials, st);
    case 16: return launch_lp_nb<16, FMT>(p, A, ld, cols, idx, m, nsteps, u, partials, st);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------- streaming pass
// out[k] = (accumulate ? out[k] : beta base[k]) + gamma sum_p s[row(p)] v[p] dec(Q[row(p)][k])
constexpr int kLvThreads = 256;

template <int FMT>
__global__ __launch_bounds__(kLvThreads) void gemv_t_lp_kernel(
    const uint8_t* __restrict__ A, int64_t ld, int64_t cols, const float* __restrict__ rs,
    const int32_t* __restrict__ idx, int64_t m, const double* __restrict__ v, double gamma,
    const double* __restrict__ base, double beta, int accumulate, double* __restrict__ out,
    int aligned) {
  constexpr int ES = FMT == CABCD_BF16 ? 2 : 1;
  constexpr int EPC = 16 / ES;
  const int64_t k = ((int64_t)blockIdx.x * kLvThreads + threadIdx.x) * EPC;
  if (k >= cols) return;
  double acc[EPC];
#pragma unroll
  for (int e = 0; e < EPC; ++e) acc[e] = 0.0;
  int64_t p = 0;
  for (; p + 4 <= m; p += 4) {
    uint4 x[4];
    double c[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t row = idx ? (int64_t)idx[p + q] : p + q;
      c[q] = v[p + q] * (rs ? (double)rs[row] : 1.0);
      x[q] = lp_load<FMT>(A + row * ld * ES, k, cols, aligned != 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double dv[EPC];
      lp_decode_all<FMT>(x[q], dv);
#pragma unroll
      for (int e = 0; e < EPC; ++e) acc[e] = fma(dv[e], c[q], acc[e]);
    }
  }
  for (; p < m; ++p) {
    const int64_t row = idx ? (int64_t)idx[p] : p;
    const double cq = v[p] * (rs ? (double)rs[row] : 1.0);
    const uint4 x = lp_load<FMT>(A + row * ld * ES, k, cols, aligned != 0);
    double dv[EPC];
    lp_decode_all<FMT>(x, dv);
#pragma unroll
    for (int e = 0; e < EPC; ++e) acc[e] = fma(dv[e], cq, acc[e]);
  }
#pragma unroll
  for (int e = 0; e < EPC; ++e) {
    if (k + e < cols) {
      const double b0 = accumulate ? out[k + e] : (base ? beta * base[k + e] : 0.0);
      out[k + e] = b0 + gamma * acc[e];
    }
  }
}

}  // namespace

GramPlan plan_gram_lp(int m, int64_t cols, int dtype) {
  GramPlan p{};
  int nb = 1;
  while (16 * nb < m) nb *= 2;
  p.nb = nb;
  p.nblk = nb * (nb + 1) / 2;
  const int es = dtype == CABCD_BF16 ? 2 : 1;
  p.kt = (2048 / nb) / es;
  p.rpw = 2;
  // HBM-bound: about two workgroups per CU, and slabs long enough that the
  // partial blocks (nblk*2 KiB per workgroup) stay small next to the slab.
  const int64_t min_chunk = std::max<int64_t>(p.kt, (int64_t)p.nblk * 2048 * 8 / (16 * nb * es));
  int64_t chunk = std::max<int64_t>(min_chunk, (cols + 511) / 512);
  chunk = ((chunk + p.kt - 1) / p.kt) * p.kt;
  p.chunk = chunk;
  p.nsplit = (int)((cols + chunk - 1) / chunk);
  return p;
}

hipError_t launch_gram_lp(const GramPlan& p, int dtype, const void* A, int64_t ld, int64_t cols,
                          const int32_t* idx, int m, const double* u, double* partials,
                          hipStream_t st, int nsteps) {
  if (nsteps < 1 || nsteps > 65535 || (nsteps > 1 && u != nullptr)) return hipErrorInvalidValue;
  if (dtype == CABCD_BF16)
    return launch_lp_fmt<CABCD_BF16>(p, A, ld, cols, idx, m, nsteps, u, partials, st);
  return launch_lp_fmt<CABCD_FP8_E4M3>(p, A, ld, cols, idx, m, nsteps, u, partials, st);
}

hipError_t launch_gemv_t_lp(int dtype, const void* A, int64_t ld, int64_t cols, const float* rs,
                            const int32_t* idx, int64_t m, const double* v, double gamma,
                            const double* base, double beta, bool accumulate, double* out,
                            hipStream_t st) {
  if (cols <= 0) return hipSuccess;
  const int es = dtype == CABCD_BF16 ? 2 : 1;
  const int epc = 16 / es;
  const int aligned = ((reinterpret_cast<uintptr_t>(A) & 15) == 0 && ((ld * es) & 15) == 0);
  const int64_t blocks = (cols + (int64_t)kLvThreads * epc - 1) / ((int64_t)kLvThreads * epc);
  if (dtype == CABCD_BF16)
    hipLaunchKernelGGL(gemv_t_lp_kernel<CABCD_BF16>, dim3((unsigned)blocks), dim3(kLvThreads), 0,
                       st, static_cast<const uint8_t*>(A), ld, cols, rs, idx, m, v, gamma, base,
                       beta, accumulate ? 1 : 0, out, aligned);
  else
    hipLaunchKernelGGL(gemv_t_lp_kernel<CABCD_FP8_E4M3>, dim3((unsigned)blocks),
                       dim3(kLvThreads), 0, st, static_cast<const uint8_t*>(A), ld, cols, rs, idx,
                       m, v, gamma, base, beta, accumulate ? 1 : 0, out, aligned);
  return hipGetLastError();
}

hipError_t launch_quantize(const double* A, int64_t rows, int64_t cols, int64_t lda, int dtype,
                           void* Q, int64_t ldq, float* row_scale, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(quantize_kernel, dim3((unsigned)rows), dim3(kQThreads), 0, st, A, cols, lda,
                     dtype, Q, ldq, row_scale);
  return hipGetLastError();
}

}  // namespace cabcd
