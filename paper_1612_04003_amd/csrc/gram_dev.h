// Device code of the dense FP64 Gram of gathered rows on the CDNA4 matrix
// cores, shared by the one-problem kernels and the batched persistent kernel.
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
// * Each workgroup writes its partial blocks; they are summed in split order
//   (deterministic) by a second kernel or, in the batched persistent kernel,
//   by the problem's last workgroup, which applies scale and shift in FP64 and
//   mirrors the result into both triangles.
#pragma once

#include "internal.h"

#include <algorithm>

namespace cabcd {
namespace gdev {

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

template <class PTR>
__device__ __forceinline__ double2 load2(PTR p, int64_t k, int64_t k_end, bool aligned) {
  double2 v;
  if (k + 1 < k_end) {
    if (aligned) {
      typedef double dv2 __attribute__((ext_vector_type(2)));
      const dv2 t = *reinterpret_cast<gptr<const dv2>>(p + k);
      v.x = t.x;
      v.y = t.y;
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

// One workgroup's slab of the Gram: columns [k_begin, k_end) of the rows
// idx[0..m) of A (m <= 16 NB; idx may point to LDS), u indexed by absolute
// column (NULL: no Y u).  Writes the partial blocks and the partial Y u to
// part[0 .. NBLK*256 + SBP).  lds holds Cfg::LDS doubles.  Every thread of the
// workgroup must call it.
template <int NB, int RPW>
__device__ __forceinline__ void gram_slab(const double* __restrict__ A, int64_t ld,
                                          int64_t k_begin, int64_t k_end, const int32_t* idx,
                                          int m, const double* __restrict__ u,
                                          double* __restrict__ part, int aligned, double* lds) {
  using C = Cfg<NB, RPW>;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int bw = wave % C::BW;
  const int kg = wave / C::BW;
  const int c = tid % C::CH;
  const int ntiles = (int)((k_end - k_begin + C::KT - 1) / C::KT);

  int rho[C::NCH];
  gptr<const double> rowp[C::NCH];
  const gptr<const double> Ag = glb(A);
  const gptr<const double> ug = glb(u);
#pragma unroll
  for (int i = 0; i < C::NCH; ++i) {
    rho[i] = tid / C::CH + (C::THREADS / C::CH) * i;
    rowp[i] = rho[i] < m ? Ag + (int64_t)idx[rho[i]] * ld : nullptr;
  }
  const bool want_u = u != nullptr;
  const bool u_aligned = (reinterpret_cast<uintptr_t>(u) & 15) == 0;   // k is even
  double yu[C::NCH];
  double2 buf[C::NCH];
  double2 ub = {0.0, 0.0};
#pragma unroll
  for (int i = 0; i < C::NCH; ++i) yu[i] = 0.0;

  auto load_tile = [&](int t) {
    const int64_t k = k_begin + (int64_t)t * C::KT + 2 * c;
    if (want_u) ub = load2(ug, k, k_end, u_aligned);
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
      gptr<double> dst = glb(part) + acc_block<NB, RPW>(bw, a) * 256 + lane;
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
      glb(part)[C::NBLK * 256 + tid] = s;
    }
  }
}


// Element e of a partial block (lane-major: e = item*64 + lane) sits at
// column lane%16 of its 16x16 block and row 4*item + lane/16 (layout 0: the
// output order of v_mfma_f64_16x16x4_f64 on gfx950) or 4*(lane/16) + item
// (layout 1: the FP32-output MFMAs).  Both were checked on the hardware with
// probes of known integer matrices.
__device__ __forceinline__ void entry_rc(int64_t e, int layout, int& row, int& col, bool& lower) {
  const int q = (int)(e >> 8);
  int r = 0;
  while (blk_index(r + 1, 0) <= q) ++r;
  const int cb = q - blk_index(r, 0);
  const int item = (int)(e >> 6) & 3;
  const int lane = (int)e & 63;
  row = 16 * r + (layout == 0 ? 4 * item + (lane >> 4) : 4 * (lane >> 4) + item);
  col = 16 * cb + (lane & 15);
  lower = r != cb || row >= col;
}

// Writes the reduced entry e (sum t of its partials) to Gov / Yu.
__device__ __forceinline__ void store_entry(int64_t e, double t, int nblk, const int32_t* idx,
                                            int m, double scale, double shift, int overlap,
                                            double* __restrict__ G, double* __restrict__ Yu,
                                            int layout, const float* __restrict__ rs) {
  if (e >= (int64_t)nblk * 256) {          // the Y u entries follow the blocks
    const int p = (int)(e - (int64_t)nblk * 256);
    if (Yu != nullptr && p < m) glb(Yu)[p] = rs ? (double)glb(rs)[idx[p]] * t : t;
    return;
  }
  int row, col;
  bool lower;
  entry_rc(e, layout, row, col, lower);
  if (row < m && col < m && lower) {
    const bool on = overlap ? (idx[row] == idx[col]) : (row == col);
    const double sc =
        rs ? scale * (double)glb(rs)[idx[row]] * (double)glb(rs)[idx[col]] : scale;
    const double v = sc * t + (on ? shift : 0.0);
    glb(G)[(int64_t)row * m + col] = v;
    glb(G)[(int64_t)col * m + row] = v;
  }
}

// The whole reduction by one workgroup of T threads: partial sets 0..nsplit-1
// (stride nblk*256 + 16 nb) are added in set order for every entry.
template <int T>
__device__ __forceinline__ void reduce_wg(const double* __restrict__ partials, int nsplit, int nb,
                                          const int32_t* idx, int m, double scale, double shift,
                                          double* __restrict__ G, double* __restrict__ Yu,
                                          int layout, const float* __restrict__ rs) {
  const int nblk = nb * (nb + 1) / 2;
  const int64_t pstride = (int64_t)nblk * 256 + 16 * nb;
  for (int64_t e = threadIdx.x; e < pstride; e += T) {
    const gptr<const double> p = glb(partials) + e;
    double s = 0.0;
    int sp = 0;
    for (; sp + 8 <= nsplit; sp += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = p[(int64_t)(sp + q) * pstride];
#pragma unroll
      for (int q = 0; q < 8; ++q) s += v[q];
    }
    for (; sp < nsplit; ++sp) s += p[(int64_t)sp * pstride];
    store_entry(e, s, nblk, idx, m, scale, shift, 1, G, Yu, layout, rs);
  }
}

}  // namespace gdev
}  // namespace cabcd
