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
#include <cstdlib>

namespace cabcd {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// Wave layouts.  RPW = block rows owned by one wave: 2 (rows r and NB-1-r, 8
// waves, two per SIMD) or 4 (rows r, NB-1-r, NB/2-1-r, NB/2+r, 4 waves, one
// per SIMD with the accumulators in AGPRs).  Either way every wave owns
// the same number of lower blocks.  Waves that own the same rows (KG > 1, small
// NB) split the k-steps of a tile instead.
template <int NB, int RPW>
struct Cfg {
  static constexpr int SBP = 16 * NB;                       // padded rows
  static constexpr int NBLK = NB * (NB + 1) / 2;            // lower 16x16 blocks
  static constexpr int KT = 256 / NB;                       // tile width: SBP*KT = 4096
  static constexpr int RS = KT + 2;                         // LDS row stride (doubles)
  static constexpr int CH = KT / 2;                         // 16-byte chunks per row
  static constexpr int R = NB >= RPW ? RPW : 1;             // rows per wave
  static constexpr int BW = NB >= RPW ? NB / RPW : 1;       // waves splitting the blocks
  static constexpr int WAVES = RPW == 2 ? 8 : 4;
  static constexpr int KG = WAVES / BW;                     // waves splitting the k-steps
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int NCH = SBP * CH / THREADS;            // chunks per thread per tile
  static constexpr int PAIRS = KT / 8;                      // 128-bit fragment reads per tile
  static constexpr int NACC = NB >= RPW ? NBLK / BW : 1;    // accumulators per wave
  static constexpr int TILE = SBP * RS;
  static constexpr int RED = (KG - 1) * NBLK * 256;
  static constexpr int YUS = SBP * CH;
  static constexpr int LDS = std::max(std::max(2 * TILE, RED), YUS);
  static_assert(NCH * THREADS == SBP * CH, "tile must split evenly");
  static_assert(PAIRS % KG == 0, "k-steps must split evenly");
  static_assert(NB < RPW || NACC * BW == NBLK, "blocks must split evenly");
};

// Index of lower block (r, c) in row-major lower-triangular order.
__host__ __device__ constexpr int blk_index(int r, int c) { return r * (r + 1) / 2 + c; }

// i-th block row owned by wave w.
__host__ __device__ constexpr int owned_row(int NB, int RPW, int w, int i) {
  if (NB < RPW) return NB == 1 ? 0 : (i == 0 ? 0 : 1);
  const int pair = RPW == 2 ? w : (i < 2 ? w : NB / 2 - 1 - w);
  return (i % 2 == 0) ? pair : NB - 1 - pair;
}

// First accumulator of owned row i (accumulators of row r are its r+1 blocks).
__host__ __device__ constexpr int acc_offset(int NB, int RPW, int w, int i) {
  int off = 0;
  for (int k = 0; k < i; ++k) off += owned_row(NB, RPW, w, k) + 1;
  return off;
}

// Block index of accumulator a of wave bw.
template <int NB, int RPW>
__device__ __forceinline__ int acc_block(int bw, int a) {
  using C = Cfg<NB, RPW>;
  if (NB < RPW) return a;   // the whole (tiny) triangle, in row-major order
  for (int i = 0; i < C::R; ++i) {
    const int r = owned_row(NB, RPW, bw, i);
    if (a <= r) return blk_index(r, a);
    a -= r + 1;
  }
  return 0;
}

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int NB, int RPW, int W>
__device__ __forceinline__ void mma_tile(const double* __restrict__ tile, int lane, int kg,
                                         d4 (&acc)[Cfg<NB, RPW>::NACC]) {
  using C = Cfg<NB, RPW>;
  constexpr int NR = NB >= RPW ? C::R : (NB == 1 ? 1 : 2);
  const double* base = tile + (lane & 15) * C::RS + 2 * (lane >> 4);
#pragma unroll
  for (int p = 0; p < C::PAIRS / C::KG; ++p) {
    const int col = 8 * (kg + p * C::KG);
    auto frag = [&](int r) {
      return *reinterpret_cast<const double2*>(base + r * 16 * C::RS + col);
    };
    // The wave's own block rows stay in registers; the column fragments are
    // streamed so only a few are live next to the accumulators.
    double2 fo[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) fo[i] = frag(owned_row(NB, RPW, W, i));
    constexpr int CMAX = NB >= RPW ? NB - 1 - W : NB - 1;   // largest owned row
#pragma unroll
    for (int c = 0; c <= CMAX; ++c) {
      double2 fc = {0.0, 0.0};
      bool own = false;
#pragma unroll
      for (int i = 0; i < NR; ++i)
        if (owned_row(NB, RPW, W, i) == c) {
          fc = fo[i];
          own = true;
        }
      if (!own) fc = frag(c);
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        const int r = owned_row(NB, RPW, W, i);
        if (c <= r) {
          const int a = acc_offset(NB, RPW, W, i) + c;
          acc[a] = mfma(fo[i].x, fc.x, acc[a]);
          acc[a] = mfma(fo[i].y, fc.y, acc[a]);
        }
      }
    }
  }
}

template <int NB, int RPW, int W = 0>
__device__ __forceinline__ void mma_dispatch(int bw, const double* __restrict__ tile, int lane,
                                             int kg, d4 (&acc)[Cfg<NB, RPW>::NACC]) {
  if constexpr (W < Cfg<NB, RPW>::BW) {
    if (bw == W)
      mma_tile<NB, RPW, W>(tile, lane, kg, acc);
    else
      mma_dispatch<NB, RPW, W + 1>(bw, tile, lane, kg, acc);
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

template <int NB, int RPW>
__global__ __launch_bounds__((Cfg<NB, RPW>::THREADS)) void gram_f64_kernel(
    const double* __restrict__ A, int64_t ld, int64_t cols, const int32_t* __restrict__ idx,
    int m, const double* __restrict__ u, int64_t chunk, double* __restrict__ partials,
    int aligned) {
  using C = Cfg<NB, RPW>;
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
    rho[i] = tid / C::CH + (C::THREADS / C::CH) * i;
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
    mma_dispatch<NB, RPW>(bw, lds + (t & 1) * C::TILE, lane, kg, acc);
    if (more) store_tile((t + 1) & 1);
    __syncthreads();
  }

  double* part = partials + (int64_t)blockIdx.x * (C::NBLK * 256 + C::SBP);

  // Sum the k-groups (waves with the same blocks) through LDS, in group order.
  if constexpr (C::KG > 1) {
    if (kg > 0) {
#pragma unroll
      for (int a = 0; a < C::NACC; ++a) {
        double* dst = lds + ((kg - 1) * C::NBLK + acc_block<NB, RPW>(bw, a)) * 256 + lane;
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
          const double* src = lds + ((g - 1) * C::NBLK + acc_block<NB, RPW>(bw, a)) * 256 + lane;
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
      double* dst = part + acc_block<NB, RPW>(bw, a) * 256 + lane;
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
// column lane%16 of its 16x16 block and row 4*item + lane/16 (layout 0: the
// output order of v_mfma_f64_16x16x4_f64 on gfx950) or 4*(lane/16) + item
// (layout 1: the FP32-output MFMAs).  Both were checked on the hardware with
// probes of known integer matrices.
constexpr int kRedElems = 64;    // partial entries per reduction workgroup
constexpr int kRedGroups = 4;    // split groups per entry (one wave each)

__global__ __launch_bounds__(kRedElems * kRedGroups) void gram_reduce_kernel(
    const double* __restrict__ partials, int nsplit, int nb, const int32_t* __restrict__ idx,
    int m, double scale, double shift, int overlap, double* __restrict__ G,
    double* __restrict__ Yu, int layout, const float* __restrict__ rs) {
  __shared__ double red[kRedGroups][kRedElems];
  const int nblk = nb * (nb + 1) / 2;
  const int64_t pstride = (int64_t)nblk * 256 + 16 * nb;
  const int el = threadIdx.x % kRedElems;
  const int grp = threadIdx.x / kRedElems;
  const int64_t e = (int64_t)blockIdx.x * kRedElems + el;
  // Each wave sums a contiguous range of splits for 64 consecutive entries;
  // the ranges are then added in group order, so the result is deterministic.
  const int per = (nsplit + kRedGroups - 1) / kRedGroups;
  const int sp0 = grp * per;
  const int sp1 = min(nsplit, sp0 + per);
  double s = 0.0;
  if (e < pstride) {
    const double* p = partials + e;
    int sp = sp0;
    for (; sp + 8 <= sp1; sp += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = p[(int64_t)(sp + q) * pstride];
#pragma unroll
      for (int q = 0; q < 8; ++q) s += v[q];
    }
    for (; sp < sp1; ++sp) s += p[(int64_t)sp * pstride];
  }
  red[grp][el] = s;
  __syncthreads();
  if (grp != 0 || e >= pstride) return;
  double t = red[0][el];
#pragma unroll
  for (int g = 1; g < kRedGroups; ++g) t += red[g][el];
  if (e >= (int64_t)nblk * 256) {          // the Y u entries follow the blocks
    const int p = (int)(e - (int64_t)nblk * 256);
    if (Yu != nullptr && p < m) Yu[p] = rs ? (double)rs[idx[p]] * t : t;
    return;
  }
  const int q = (int)(e >> 8);
  int r = 0;
  while (blk_index(r + 1, 0) <= q) ++r;
  const int cb = q - blk_index(r, 0);
  const int item = (int)(e >> 6) & 3;
  const int lane = (int)e & 63;
  const int row = 16 * r + (layout == 0 ? 4 * item + (lane >> 4) : 4 * (lane >> 4) + item);
  const int col = 16 * cb + (lane & 15);
  if (row < m && col < m && (r != cb || row >= col)) {
    const bool on = overlap ? (idx[row] == idx[col]) : (row == col);
    const double sc = rs ? scale * (double)rs[idx[row]] * (double)rs[idx[col]] : scale;
    const double v = sc * t + (on ? shift : 0.0);
    G[(int64_t)row * m + col] = v;
    G[(int64_t)col * m + row] = v;
  }
}

template <int NB, int RPW>
hipError_t launch_nb(const GramPlan& p, const double* A, int64_t ld, int64_t cols,
                     const int32_t* idx, int m, const double* u, double* partials,
                     hipStream_t st) {
  const int aligned = ((reinterpret_cast<uintptr_t>(A) & 15) == 0 && (ld & 1) == 0) ? 1 : 0;
  hipLaunchKernelGGL((gram_f64_kernel<NB, RPW>), dim3(p.nsplit), dim3(Cfg<NB, RPW>::THREADS), 0,
                     st, A, ld, cols, idx, m, u, p.chunk, partials, aligned);
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
  // Eight waves with two block rows each.  Four waves with four rows each (one
  // wave per SIMD, accumulators in AGPRs) measured slower at nb = 8 (30.9 vs
  // 38.3 TFLOP/s) and does not fit the registers at nb = 16.
  p.rpw = 2;
  return p;
}

size_t gram_partial_doubles(const GramPlan& p) {
  return (size_t)p.nsplit * ((size_t)p.nblk * 256 + 16 * (size_t)p.nb);
}

hipError_t launch_gram_f64(const GramPlan& p, const double* A, int64_t ld, int64_t cols,
                           const int32_t* idx, int m, const double* u, double* partials,
                           hipStream_t st) {
  switch (p.nb) {
    case 1: return launch_nb<1, 2>(p, A, ld, cols, idx, m, u, partials, st);
    case 2: return launch_nb<2, 2>(p, A, ld, cols, idx, m, u, partials, st);
    case 4: return launch_nb<4, 2>(p, A, ld, cols, idx, m, u, partials, st);
    case 8: return launch_nb<8, 2>(p, A, ld, cols, idx, m, u, partials, st);
    case 16: return launch_nb<16, 2>(p, A, ld, cols, idx, m, u, partials, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gram_reduce(const GramPlan& p, const double* partials, const int32_t* idx,
                              int m, double scale, double shift, bool overlap, double* G,
                              double* Yu, hipStream_t st, int layout, const float* rs) {
  const int64_t entries = (int64_t)p.nblk * 256 + 16 * p.nb;
  const int64_t blocks = (entries + kRedElems - 1) / kRedElems;
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)blocks), dim3(kRedElems * kRedGroups), 0,
                     st, partials, p.nsplit, p.nb, idx, m, scale, shift, overlap ? 1 : 0, G, Yu,
                     layout, rs);
  return hipGetLastError();
}

}  // namespace cabcd
