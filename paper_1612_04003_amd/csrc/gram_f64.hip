// Dense FP64 Gram of gathered rows on the CDNA4 matrix cores.
//
// Computes the s-step Gram Y Y^T of Alg. 2 (Y = [I_1..I_s]^T X, rows of X) and
// Alg. 4 (Y = X[I_1..I_s], rows of X^T), together with Y u for the companion
// vector u (the residual products of eq. recur / the dual recurrence).  The
// paper forms this with MKL on CSR on every MPI rank (Section 5.2); here it is
// one launch per outer step:
//
// * The reduction dimension (cols of A) is split into `chunk`-wide slabs, one
//   workgroup each (split-K), so that hundreds of workgroups cover a thin
//   m x m output with K in the hundreds of thousands.
// * A workgroup streams its slab through LDS in KT-wide tiles: the m gathered
//   rows are read with 16-byte coalesced loads, double-buffered, and Y u is
//   accumulated in FP64 from the same registers while the tile is written to
//   LDS, so Y is read from HBM exactly once.
// * The lower triangle of 16x16 output blocks is computed with
//   v_mfma_f64_16x16x4_f64.  Each wave owns the blocks of two block rows
//   (r, NB-1-r), so every wave has NB+1 accumulators and reads at most NB
//   fragments per k-step.  For small NB the waves also split the k-steps of a
//   tile and are summed through LDS at the end.
// * The MFMA reduction index is permuted: lane group g of a 128-bit fragment
//   read supplies columns 8p+2g and 8p+2g+1 to two consecutive MFMAs.  Any
//   bijection of k works because both operands use the same one.
// * Each workgroup writes its partial blocks; a second kernel sums them in
//   split order (deterministic), applies scale and shift in FP64 and mirrors
//   the result into both triangles.
#include "internal.h"

#include <algorithm>
#include <cmath>

namespace cabcd {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 512;   // 8 waves

template <int NB>
struct Cfg {
  static constexpr int SBP = 16 * NB;                 // padded rows
  static constexpr int NBLK = NB * (NB + 1) / 2;      // lower 16x16 blocks
  static constexpr int KT = 256 / NB;                 // tile width: SBP*KT = 4096
  static constexpr int RS = KT + 2;                   // LDS row stride (doubles)
  static constexpr int CH = KT / 2;                   // 16-byte chunks per row
  static constexpr int NCH = SBP * CH / kThreads;     // chunks per thread (= 4)
  static constexpr int BW = NB >= 2 ? NB / 2 : 1;     // waves sharing the blocks
  static constexpr int KG = 8 / BW;                   // waves splitting the k-steps
  static constexpr int PAIRS = KT / 8;                // 128-bit fragment reads per tile
  static constexpr int NACC = NB >= 2 ? NB + 1 : 1;   // accumulators per wave
  static constexpr int TILE = SBP * RS;
  static constexpr int RED = (KG - 1) * NBLK * 256;
  static constexpr int YUS = SBP * CH;
  static constexpr int LDS = std::max(std::max(2 * TILE, RED), YUS);
  static_assert(NCH * kThreads == SBP * CH, "tile must split evenly");
  static_assert(PAIRS % KG == 0, "k-steps must split evenly");
};

// Index of lower block (r, c) in row-major lower-triangular order.
__host__ __device__ constexpr int blk_index(int r, int c) { return r * (r + 1) / 2 + c; }

// Block index of accumulator a of the wave that owns block rows bw and NB-1-bw.
template <int NB>
__device__ __forceinline__ int acc_block(int bw, int a) {
  if (NB == 1) return 0;
  const int r1 = bw, r2 = NB - 1 - bw;
  return a <= r1 ? blk_index(r1, a) : blk_index(r2, a - r1 - 1);
}

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int NB, int W>
__device__ __forceinline__ void mma_tile(const double* __restrict__ tile, int lane, int kg,
                                         d4 (&acc)[Cfg<NB>::NACC]) {
  using C = Cfg<NB>;
  constexpr int R1 = NB >= 2 ? W : 0;
  constexpr int R2 = NB >= 2 ? NB - 1 - W : 0;
  const double* base = tile + (lane & 15) * C::RS + 2 * (lane >> 4);
#pragma unroll
  for (int p = 0; p < C::PAIRS / C::KG; ++p) {
    const int col = 8 * (kg + p * C::KG);
    auto frag = [&](int r) {
      return *reinterpret_cast<const double2*>(base + r * 16 * C::RS + col);
    };
    // The wave's two block rows stay in registers; the column fragments are
    // streamed, so at most a few fragments are live next to the accumulators.
    const double2 f1 = frag(R1);
    const double2 f2 = NB >= 2 ? frag(R2) : f1;
#pragma unroll
    for (int c = 0; c <= R2; ++c) {
      const double2 fc = c == R1 ? f1 : (c == R2 ? f2 : frag(c));
      if (c <= R1) {
        acc[c] = mfma(f1.x, fc.x, acc[c]);
        acc[c] = mfma(f1.y, fc.y, acc[c]);
      }
      if constexpr (NB >= 2) {
        acc[R1 + 1 + c] = mfma(f2.x, fc.x, acc[R1 + 1 + c]);
        acc[R1 + 1 + c] = mfma(f2.y, fc.y, acc[R1 + 1 + c]);
      }
    }
  }
}

template <int NB, int W = 0>
__device__ __forceinline__ void mma_dispatch(int bw, const double* __restrict__ tile, int lane,
                                             int kg, d4 (&acc)[Cfg<NB>::NACC]) {
  if constexpr (W < Cfg<NB>::BW) {
    if (bw == W)
      mma_tile<NB, W>(tile, lane, kg, acc);
    else
      mma_dispatch<NB, W + 1>(bw, tile, lane, kg, acc);
  }
}

__device__ __forceinline__ double2 load2(const double* __restrict__ p, int64_t k, int64_t k_end,
                                         bool aligned) {
  double2 v;
  if (k + 1 < k_end) {
    if (aligned) {
      v = *reinterpret_cast<const double2*>(p + k);
    } else {
      v.x = p[k];
      v.y = p[k + 1];
    }
  } else {
    v.x = k < k_end ? p[k] : 0.0;
    v.y = 0.0;
  }
  return v;
}

template <int NB>
__global__ __launch_bounds__(kThreads) void gram_f64_kernel(
    const double* __restrict__ A, int64_t ld, int64_t cols, const int32_t* __restrict__ idx,
    int m, const double* __restrict__ u, int64_t chunk, double* __restrict__ partials,
    int aligned) {
  using C = Cfg<NB>;
  __shared__ __attribute__((aligned(16))) double lds[C::LDS];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int bw = wave % C::BW;
  const int kg = wave / C::BW;
  const int c = tid % C::CH;
  const int64_t k_begin = (int64_t)blockIdx.x * chunk;
  const int64_t k_end = std::min(cols, k_begin + chunk);
  const int ntiles = (int)((k_end - k_begin + C::KT - 1) / C::KT);

  int rho[C::NCH];
  const double* rowp[C::NCH];
#pragma unroll
  for (int i = 0; i < C::NCH; ++i) {
    rho[i] = tid / C::CH + (kThreads / C::CH) * i;
    rowp[i] = rho[i] < m ? A + (int64_t)idx[rho[i]] * ld : nullptr;
  }
  const bool want_u = u != nullptr;
  double yu[C::NCH];
  double2 buf[C::NCH];
  double2 ub = {0.0, 0.0};
#pragma unroll
  for (int i = 0; i < C::NCH; ++i) yu[i] = 0.0;

  auto load_tile = [&](int t) {
    const int64_t k = k_begin + (int64_t)t * C::KT + 2 * c;
    if (want_u) ub = load2(u, k, k_end, true);
#pragma unroll
    for (int i = 0; i < C::NCH; ++i) {
      if (rowp[i] != nullptr) {
        buf[i] = load2(rowp[i], k, k_end, aligned != 0);
      } else {
        buf[i].x = 0.0;
        buf[i].y = 0.0;
      }
    }
  };
  auto store_tile = [&](int slot) {
    double* T = lds + slot * C::TILE;
#pragma unroll
    for (int i = 0; i < C::NCH; ++i) {
      *reinterpret_cast<double2*>(T + rho[i] * C::RS + 2 * c) = buf[i];
      if (want_u) {
        yu[i] = fma(buf[i].x, ub.x, yu[i]);
        yu[i] = fma(buf[i].y, ub.y, yu[i]);
      }
    }
  };

  d4 acc[C::NACC];
#pragma unroll
  for (int a = 0; a < C::NACC; ++a) acc[a] = d4{0.0, 0.0, 0.0, 0.0};

  load_tile(0);
  store_tile(0);
  __syncthreads();
  for (int t = 0; t < ntiles; ++t) {
    const bool more = t + 1 < ntiles;
    if (more) load_tile(t + 1);
    mma_dispatch<NB>(bw, lds + (t & 1) * C::TILE, lane, kg, acc);
    if (more) store_tile((t + 1) & 1);
    __syncthreads();
  }

  double* part = partials + (int64_t)blockIdx.x * (C::NBLK * 256 + C::SBP);

  // Sum the k-groups (waves with the same blocks) through LDS, in group order.
  if constexpr (C::KG > 1) {
    if (kg > 0) {
#pragma unroll
      for (int a = 0; a < C::NACC; ++a) {
        double* dst = lds + ((kg - 1) * C::NBLK + acc_block<NB>(bw, a)) * 256 + lane;
        dst[0] = acc[a][0];
        dst[64] = acc[a][1];
        dst[128] = acc[a][2];
        dst[192] = acc[a][3];
      }
    }
    __syncthreads();
    if (kg == 0) {
      for (int g = 1; g < C::KG; ++g) {
#pragma unroll
        for (int a = 0; a < C::NACC; ++a) {
          const double* src = lds + ((g - 1) * C::NBLK + acc_block<NB>(bw, a)) * 256 + lane;
          acc[a][0] += src[0];
          acc[a][1] += src[64];
          acc[a][2] += src[128];
          acc[a][3] += src[192];
        }
      }
    }
  }
  if (kg == 0) {
#pragma unroll
    for (int a = 0; a < C::NACC; ++a) {
      double* dst = part + acc_block<NB>(bw, a) * 256 + lane;
      dst[0] = acc[a][0];
      dst[64] = acc[a][1];
      dst[128] = acc[a][2];
      dst[192] = acc[a][3];
    }
  }

  if (want_u) {
    __syncthreads();   // LDS is reused for the row sums of Y u
#pragma unroll
    for (int i = 0; i < C::NCH; ++i) lds[rho[i] * C::CH + c] = yu[i];
    __syncthreads();
    if (tid < C::SBP) {
      double s = 0.0;
      for (int q = 0; q < C::CH; ++q) s += lds[tid * C::CH + q];
      part[C::NBLK * 256 + tid] = s;
    }
  }
}

// Element e of a partial block (lane-major: e = item*64 + lane) sits at
// row 4*item + lane/16, column lane%16 of its 16x16 block: the output layout
// of v_mfma_f64_16x16x4_f64 on gfx950 (checked on the hardware with a probe of
// known integer matrices).
__global__ void gram_reduce_kernel(const double* __restrict__ partials, int nsplit, int nb,
                                   const int32_t* __restrict__ idx, int m, double scale,
                                   double shift, int overlap, double* __restrict__ G,
                                   double* __restrict__ Yu) {
  const int nblk = nb * (nb + 1) / 2;
  const int64_t pstride = (int64_t)nblk * 256 + 16 * nb;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < nblk * 256) {
    double s = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) s += partials[sp * pstride + e];
    const int q = e >> 8;
    int r = 0;
    while (blk_index(r + 1, 0) <= q) ++r;
    const int cb = q - blk_index(r, 0);
    const int item = (e >> 6) & 3;
    const int lane = e & 63;
    const int row = 16 * r + 4 * item + (lane >> 4);
    const int col = 16 * cb + (lane & 15);
    if (row < m && col < m && (r != cb || row >= col)) {
      const bool on = overlap ? (idx[row] == idx[col]) : (row == col);
      const double v = scale * s + (on ? shift : 0.0);
      G[(int64_t)row * m + col] = v;
      G[(int64_t)col * m + row] = v;
    }
  }
  if (Yu != nullptr && e < m) {
    double s = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) s += partials[sp * pstride + nblk * 256 + e];
    Yu[e] = s;
  }
}

template <int NB>
hipError_t launch_nb(const GramPlan& p, const double* A, int64_t ld, int64_t cols,
                     const int32_t* idx, int m, const double* u, double* partials,
                     hipStream_t st) {
  const int aligned = ((reinterpret_cast<uintptr_t>(A) & 15) == 0 && (ld & 1) == 0) ? 1 : 0;
  hipLaunchKernelGGL(gram_f64_kernel<NB>, dim3(p.nsplit), dim3(kThreads), 0, st, A, ld, cols,
                     idx, m, u, p.chunk, partials, aligned);
  return hipGetLastError();
}

}  // namespace

GramPlan plan_gram_f64(int m, int64_t cols) {
  GramPlan p{};
  int nb = 1;
  while (16 * nb < m) nb *= 2;
  p.nb = nb;
  p.nblk = nb * (nb + 1) / 2;
  p.kt = 256 / nb;
  const int bw = nb >= 2 ? nb / 2 : 1;
  const int kg = 8 / bw;
  const int nacc = nb >= 2 ? nb + 1 : 1;
  // Cost model (alpha-beta-gamma style, eq. comm): matrix-core time of the
  // slowest round of workgroups, HBM time of the gathered rows, and the traffic
  // of writing and re-reading the partial Grams.  Pick the cheapest chunk.
  const double clock = 2.4e9, hbm = 6.0e12;
  // The plan depends on m only through nb, so every m of one class gets the
  // same split and the workspace bound over classes is exact.
  const double ybytes = 16.0 * nb * (double)cols * 8.0;
  const double pbytes_per = ((double)p.nblk * 256 + 16.0 * nb) * 8.0;
  double best = 1e300;
  int64_t best_chunk = cols;
  for (int64_t chunk = p.kt; ; chunk *= 2) {
    const int64_t nsplit = (cols + chunk - 1) / chunk;
    const double per_wg = 2.0 * ((double)chunk / (4.0 * kg)) * nacc * 64.0 / clock;
    const double rounds = std::ceil((double)nsplit / 256.0);
    const double t = std::max(rounds * per_wg, ybytes / hbm) +
                     2.0 * nsplit * pbytes_per / hbm + (nsplit > 1024 ? 1e-3 : 0.0);
    if (t < best) {
      best = t;
      best_chunk = chunk;
    }
    if (nsplit <= 1) break;
  }
  // Also try the chunk that gives exactly one workgroup per CU.
  {
    int64_t chunk = (cols + 255) / 256;
    chunk = ((chunk + p.kt - 1) / p.kt) * p.kt;
    const int64_t nsplit = (cols + chunk - 1) / chunk;
    const double per_wg = 2.0 * ((double)chunk / (4.0 * kg)) * nacc * 64.0 / clock;
    const double t = std::max(per_wg, ybytes / hbm) + 2.0 * nsplit * pbytes_per / hbm;
    if (t < best) {
      best = t;
      best_chunk = chunk;
    }
  }
  p.chunk = best_chunk;
  p.nsplit = (int)((cols + best_chunk - 1) / best_chunk);
  return p;
}

size_t gram_partial_doubles(const GramPlan& p) {
  return (size_t)p.nsplit * ((size_t)p.nblk * 256 + 16 * (size_t)p.nb);
}

hipError_t launch_gram_f64(const GramPlan& p, const double* A, int64_t ld, int64_t cols,
                           const int32_t* idx, int m, const double* u, double* partials,
                           hipStream_t st) {
  switch (p.nb) {
    case 1: return launch_nb<1>(p, A, ld, cols, idx, m, u, partials, st);
    case 2: return launch_nb<2>(p, A, ld, cols, idx, m, u, partials, st);
    case 4: return launch_nb<4>(p, A, ld, cols, idx, m, u, partials, st);
    case 8: return launch_nb<8>(p, A, ld, cols, idx, m, u, partials, st);
    case 16: return launch_nb<16>(p, A, ld, cols, idx, m, u, partials, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gram_reduce(const GramPlan& p, const double* partials, const int32_t* idx,
                              int m, double scale, double shift, bool overlap, double* G,
                              double* Yu, hipStream_t st) {
  const int n = std::max(p.nblk * 256, m);
  const int threads = 256;
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((n + threads - 1) / threads), dim3(threads), 0, st,
                     partials, p.nsplit, p.nb, idx, m, scale, shift, overlap ? 1 : 0, G, Yu);
  return hipGetLastError();
}

}  // namespace cabcd
