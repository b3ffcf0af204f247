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


// ---------------------------------------------------------------------------
// NB <= 8 fed by LDS-DMA (the decomposition of gram_slab<NB, 2>: waves own
// block-row pairs and split a tile's k-steps): a 32 KiB tile of SBP rows x
// KT = 256 / NB columns goes from HBM straight into LDS, rows unpadded with the
// 16-byte chunks of each aligned group of sixteen XOR-swizzled by the row
// (chunk c of row r at c ^ (r & 15)), so the sixteen rows of a fragment read
// fall in distinct banks; a thread forms Y u for its four (row, chunk) pairs
// from LDS after the tile lands.  Rows of 256 bytes (NB = 8) to 2 KiB (NB = 1)
// per tile keep the HBM pages busy.
template <int NB>
struct DN {
  using C = Cfg<NB, 2>;
  static constexpr int DMA_PER_WAVE = C::SBP * C::CH / 64 / 8;   // 4 instructions
  static constexpr int UDMA = (C::KT / 2 + 63) / 64;              // u slots, 64 a time
  static constexpr int TILE = C::SBP * C::KT + C::KT;            // doubles: rows, then u
  static constexpr int LDS = std::max(std::max(2 * TILE, C::RED), C::YUS);
};

template <int NB, int W>
__device__ __forceinline__ void mma_tile_dma(const double* __restrict__ tile, int lane, int kg,
                                             d4 (&acc)[Cfg<NB, 2>::NACC]) {
  using C = Cfg<NB, 2>;
  constexpr int NR = NB >= 2 ? 2 : 1;
  const int rl = lane & 15, g = lane >> 4;
#pragma unroll
  for (int p = 0; p < C::PAIRS / C::KG; ++p) {
    const int ch = 4 * (kg + p * C::KG) + g;            // chunk (two columns) of this lane
    const double* base = tile + rl * C::KT + 2 * (ch ^ rl);
    auto frag = [&](int r) { return *reinterpret_cast<const double2*>(base + r * 16 * C::KT); };
    double2 fo[NR];
#pragma unroll
    for (int i = 0; i < NR; ++i) fo[i] = frag(owned_row(NB, 2, W, i));
    constexpr int CMAX = NB >= 2 ? NB - 1 - W : 0;        // largest owned row
#pragma unroll
    for (int c = 0; c <= CMAX; ++c) {
      double2 fc = {0.0, 0.0};
      bool own = false;
#pragma unroll
      for (int i = 0; i < NR; ++i)
        if (owned_row(NB, 2, W, i) == c) {
          fc = fo[i];
          own = true;
        }
      if (!own) fc = frag(c);
#pragma unroll
      for (int i = 0; i < NR; ++i) {
        const int r = owned_row(NB, 2, W, i);
        if (c <= r) {
          const int a = acc_offset(NB, 2, W, i) + c;
          acc[a] = mfma(fo[i].x, fc.x, acc[a]);
          acc[a] = mfma(fo[i].y, fc.y, acc[a]);
        }
      }
    }
  }
}

template <int NB, int W = 0>
__device__ __forceinline__ void mma_dispatch_dma(int bw, const double* __restrict__ tile, int lane,
                                                 int kg, d4 (&acc)[Cfg<NB, 2>::NACC]) {
  if constexpr (W < Cfg<NB, 2>::BW) {
    if (bw == W)
      mma_tile_dma<NB, W>(tile, lane, kg, acc);
    else
      mma_dispatch_dma<NB, W + 1>(bw, tile, lane, kg, acc);
  }
}

// The slab of gram_slab<NB, 2> on the DMA path (A 16-byte aligned with an even
// ld); same arguments and partial layout.  lds holds DN<NB>::LDS doubles.
template <int NB>
__device__ __forceinline__ void gram_slab_dma(const double* __restrict__ A, int64_t ld,
                                              int64_t k_begin, int64_t k_end, const int32_t* idx,
                                              int m, const double* __restrict__ u,
                                              double* __restrict__ part, double* lds) {
  using C = Cfg<NB, 2>;
  using D = DN<NB>;
  typedef __attribute__((address_space(3))) void* lds_vptr;
  typedef __attribute__((address_space(1))) const void* glb_vptr;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int bw = __builtin_amdgcn_readfirstlane(wave % C::BW);
  const int kg = __builtin_amdgcn_readfirstlane(wave / C::BW);
  const int ntiles = (int)((k_end - k_begin + C::KT - 1) / C::KT);

  // DMA instruction i of this wave fills slots (4 wave + i) * 64 + lane:
  // row slot / CH, position slot % CH, chunk position ^ (row % 16).
  // Rows past m (padding of the last block row) are never loaded: they are
  // zeroed once in both buffers.
  gptr<const double> src[D::DMA_PER_WAVE];
  int cofs[D::DMA_PER_WAVE];
  bool live[D::DMA_PER_WAVE];
  const gptr<const double> Ag = glb(A);
#pragma unroll
  for (int i = 0; i < D::DMA_PER_WAVE; ++i) {
    const int q = (D::DMA_PER_WAVE * wave + i) * 64 + lane;
    const int r = q / C::CH;
    cofs[i] = 2 * ((q % C::CH) ^ (r & 15));
    live[i] = r < m;
    src[i] = Ag + (int64_t)idx[r < m ? r : 0] * ld;
    if (!live[i]) {
#pragma unroll
      for (int sl = 0; sl < 2; ++sl)
        *reinterpret_cast<double2*>(lds + sl * D::TILE + (D::DMA_PER_WAVE * wave + i) * 128 +
                                    2 * lane) = double2{0.0, 0.0};
    }
  }
  const bool want_u = u != nullptr;
  const gptr<const double> ug = glb(u);
  const bool u_dma = want_u && (reinterpret_cast<uintptr_t>(u) & 15) == 0;
  auto issue = [&](int t, int slot) {
    const int64_t k0 = k_begin + (int64_t)t * C::KT;
    double* T = lds + slot * D::TILE;
    const bool full = k0 + C::KT <= k_end;
#pragma unroll
    for (int i = 0; i < D::DMA_PER_WAVE; ++i) {
      double* dst = T + (D::DMA_PER_WAVE * wave + i) * 128;   // 64 slots of 2 doubles
      const int64_t k = k0 + cofs[i];
      if (!live[i]) {
        // padding row: stays zero
      } else if (full) {
        __builtin_amdgcn_global_load_lds((glb_vptr)(src[i] + k), (lds_vptr)dst, 16, 0, 0);
      } else {
        double2 v;
        v.x = k < k_end ? src[i][k] : 0.0;
        v.y = k + 1 < k_end ? src[i][k + 1] : 0.0;
        *reinterpret_cast<double2*>(dst + 2 * lane) = v;
      }
    }
    if (want_u && wave == 7) {   // the tile's KT entries of u, unswizzled after the rows
#pragma unroll
      for (int j = 0; j < D::UDMA; ++j) {
        if (64 * j + lane < C::KT / 2) {
          double* dst = T + C::SBP * C::KT + 128 * j;
          const int64_t k = k0 + 2 * (64 * j + lane);
          if (full && u_dma) {
            __builtin_amdgcn_global_load_lds((glb_vptr)(ug + k), (lds_vptr)dst, 16, 0, 0);
          } else {
            double2 v;
            v.x = k < k_end ? ug[k] : 0.0;
            v.y = k + 1 < k_end ? ug[k + 1] : 0.0;
            *reinterpret_cast<double2*>(dst + 2 * lane) = v;
          }
        }
      }
    }
  };

  // Y u: chunk c of rows tid / CH + (THREADS / CH) i, as in gram_slab
  const int c = tid % C::CH;
  int rho[C::NCH];
#pragma unroll
  for (int i = 0; i < C::NCH; ++i) rho[i] = tid / C::CH + (C::THREADS / C::CH) * i;
  double yu[C::NCH];
#pragma unroll
  for (int i = 0; i < C::NCH; ++i) yu[i] = 0.0;

  d4 acc[C::NACC];
#pragma unroll
  for (int a = 0; a < C::NACC; ++a) acc[a] = d4{0.0, 0.0, 0.0, 0.0};

  issue(0, 0);
  __builtin_amdgcn_s_waitcnt(0);   // the LDS-DMA writes count on the vector memory counter
  __syncthreads();
  for (int t = 0; t < ntiles; ++t) {
    if (t + 1 < ntiles) issue(t + 1, (t + 1) & 1);
    const double* tile = lds + (t & 1) * D::TILE;
    mma_dispatch_dma<NB>(bw, tile, lane, kg, acc);
    if (want_u) {
      const double2 ub = *reinterpret_cast<const double2*>(tile + C::SBP * C::KT + 2 * c);
#pragma unroll
      for (int i = 0; i < C::NCH; ++i) {
        const int r = rho[i];
        const double2 v =
            *reinterpret_cast<const double2*>(tile + r * C::KT + 2 * (c ^ (r & 15)));
        yu[i] = fma(v.x, ub.x, yu[i]);
        yu[i] = fma(v.y, ub.y, yu[i]);
      }
    }
    __builtin_amdgcn_s_waitcnt(0);   // tile t + 1 is in LDS
    __syncthreads();
  }

  // Sum the k-groups (waves with the same blocks) through LDS, in group order.
  if constexpr (C::KG > 1) {
    if (kg > 0) {
#pragma unroll
      for (int a = 0; a < C::NACC; ++a) {
        double* dst = lds + ((kg - 1) * C::NBLK + acc_block<NB, 2>(bw, a)) * 256 + lane;
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
          const double* srcp = lds + ((g - 1) * C::NBLK + acc_block<NB, 2>(bw, a)) * 256 + lane;
          acc[a][0] += srcp[0];
          acc[a][1] += srcp[64];
          acc[a][2] += srcp[128];
          acc[a][3] += srcp[192];
        }
      }
    }
  }
  if (kg == 0) {
#pragma unroll
    for (int a = 0; a < C::NACC; ++a) {
      gptr<double> dst = glb(part) + acc_block<NB, 2>(bw, a) * 256 + lane;
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
      double sum = 0.0;
      for (int q = 0; q < C::CH; ++q) sum += lds[tid * C::CH + q];
      glb(part)[C::NBLK * 256 + tid] = sum;
    }
  }
}

// ---------------------------------------------------------------------------
// NB = 16 fed by LDS-DMA loads (gfx950 global_load_lds_dwordx4): the tile goes
// from global memory straight into LDS, so there are no staging registers and
// no ds_write instructions.  A DMA instruction writes 64 consecutive 16-byte
// LDS slots (lane l at base + 16 l); the slots hold unpadded 128-byte rows
// whose eight 16-byte chunks are XOR-swizzled, chunk c of row r at position
// c ^ ((r >> 1) & 7), so the sixteen rows of a fragment read fall in distinct
// banks.  Y u is accumulated from the waves' own-row fragments (each block row
// is owned by exactly one wave) and summed over the four lane groups at the
// end.  Needs A 16-byte aligned with an even ld; chunks that cross the end of
// the slab are written with ordinary LDS stores (zero-filled).
struct D16 {
  static constexpr int NB = 16, SBP = 256, NBLK = 136, KT = 16, CH = KT / 2;
  static constexpr int PP = KT / 8;                  // 128-bit fragment reads per tile
  static constexpr int THREADS = 512;
  static constexpr int TILE = SBP * KT + KT;         // doubles per buffer: rows, then u
  static constexpr int DMA_PER_WAVE = SBP * CH / THREADS;   // 4 instructions
  static constexpr int LDS = 2 * TILE;
  // With the previous step's companion update folded in: two more buffers
  // for the previous step's rows (and the tile's old companion entries), then
  // gamma * delta of the previous step.
  static constexpr int YT = SBP * KT + KT;           // doubles per update buffer
  static constexpr int YOFF = 2 * TILE;
  static constexpr int DOFF = 2 * TILE + 2 * YT;
  static constexpr int LDS_UPD = DOFF + SBP;
};


// x of the lane N places along in the lane's row of sixteen (DPP row_ror),
// as two 32-bit moves
template <int N>
__device__ __forceinline__ double d16_ror(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x120 + N, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x120 + N, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// The sum over a row of sixteen lanes, in every lane of the row.
__device__ __forceinline__ double d16_row_sum(double x) {
  x += d16_ror<8>(x);
  x += d16_ror<4>(x);
  x += d16_ror<2>(x);
  x += d16_ror<1>(x);
  return x;
}
// x of lane l (the same l in every lane) in every lane.
__device__ __forceinline__ double d16_read_lane(double x, int l) {
  const long long b = __double_as_longlong(x);
  return __hiloint2double(__builtin_amdgcn_readlane((int)(b >> 32), l),
                          __builtin_amdgcn_readlane((int)b, l));
}

// Chunk swizzle of row r: the sixteen rows of a fragment read land on
// distinct banks (8 chunks a row: (r >> 1) & 7; 16 chunks a row: r & 15).
__device__ __forceinline__ int d16_swz(int r) { return D16::CH == 8 ? (r >> 1) & 7 : r & 15; }

// The whole slab for wave W (block rows W and 15 - W); gram_slab_dma16 picks
// the instantiation once, so each wave's tile loop is one straight-line path
// for the register allocator.
// MODE 0: the Gram slab (and Y u with u given).  MODE 1: the same, with the
// previous step's companion update applied to the slab's columns first; Y u
// then uses the updated companion (u is ignored).  MODE 2: the update alone
// (the last step of a call, or one followed by a check), by the same code, so
// a column's update has the same rounding whichever way it runs.
//
// The update of tile t's 16 columns: wave W sums column pair W over the 256
// rows (lane l: rows l + 64 j, then a butterfly over the wave, lane 0's total
// kept), adds the old entries, writes the companion and, in MODE 1, the
// tile's u slot.  In MODE 1 it runs one tile ahead of the Gram (tile t + 1
// during tile t), so the end-of-tile barrier publishes the u slot; the
// previous step's rows are DMA'd two tiles ahead, their chunks swizzled as
// the Gram's tiles are ((r >> 1) & 7), so the column-pair reads of sixteen
// consecutive rows fall in distinct banks.
template <int W, int MODE>
__device__ __forceinline__ void d16_slab(const double* __restrict__ A, int64_t ld,
                                         int64_t k_begin, int64_t k_end, const int32_t* idx,
                                         int m, const double* __restrict__ u,
                                         double* __restrict__ part, double* lds,
                                         const D16Upd up) {
  using C = D16;
  typedef __attribute__((address_space(3))) void* lds_vptr;
  typedef __attribute__((address_space(1))) const void* glb_vptr;
  constexpr int R0 = W, R1 = 15 - W;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int ntiles = (int)((k_end - k_begin + C::KT - 1) / C::KT);

  // DMA instruction i of this wave fills slots (4 W + i) * 64 + lane.
  gptr<const double> src[C::DMA_PER_WAVE];
  int cofs[C::DMA_PER_WAVE];
  const gptr<const double> Ag = glb(A);
#pragma unroll
  for (int i = 0; i < C::DMA_PER_WAVE; ++i) {
    const int q = (C::DMA_PER_WAVE * W + i) * 64 + lane;
    const int r = q / C::CH;
    cofs[i] = 2 * ((q % C::CH) ^ d16_swz(r));
    // rows past m: any valid row (MODE 2 reads no Gram rows)
    src[i] = MODE == 2 ? Ag : Ag + (int64_t)idx[r < m ? r : 0] * ld;
  }
  const bool want_u = MODE == 1 || u != nullptr;
  const gptr<const double> ug = glb(u);
  const bool u_dma = MODE == 0 && want_u && (reinterpret_cast<uintptr_t>(u) & 15) == 0;

  // The previous step's rows (MODE 1 and 2): DMA instruction i of this wave
  // fills slots q = (4 W + i) * 64 + lane of an update buffer: row q / 8 =
  // 8 (4 W + i) + lane / 8, chunk (q % 8) ^ ((row >> 1) & 7), the swizzle
  // being (4 i + lane / 16) & 7.  The rows are kept as indices and the
  // addresses formed at each issue, to spare registers.
  int yrow[C::DMA_PER_WAVE];
  const gptr<double> rg = glb(up.r);
  const bool r_dma = (reinterpret_cast<uintptr_t>(up.r) & 15) == 0;
  if constexpr (MODE != 0) {
#pragma unroll
    for (int i = 0; i < C::DMA_PER_WAVE; ++i)
      yrow[i] = up.idx[8 * (C::DMA_PER_WAVE * W + i) + (lane >> 3)];
    if (tid < C::SBP) lds[C::DOFF + tid] = up.gamma * up.delta[tid];
  }
  auto issue_y = [&](int t, int slot) {
    const int64_t k0 = k_begin + (int64_t)t * C::KT;
    double* Y = lds + C::YOFF + slot * C::YT;
#pragma unroll
    for (int i = 0; i < C::DMA_PER_WAVE; ++i) {
      double* dst = Y + (C::DMA_PER_WAVE * W + i) * 128;
      const int64_t k = k0 + 2 * ((lane & 7) ^ ((4 * i + (lane >> 4)) & 7));
      const gptr<const double> row = Ag + (int64_t)yrow[i] * ld;
      if (k + 1 < k_end) {
        __builtin_amdgcn_global_load_lds((glb_vptr)(row + k), (lds_vptr)dst, 16, 0, 0);
      } else {
        double2 v;
        v.x = k < k_end ? row[k] : 0.0;
        v.y = 0.0;
        *reinterpret_cast<double2*>(dst + 2 * lane) = v;
      }
    }
    // the old companion entries of the tile's columns: lanes 0..CH-1 of wave 7
    if (W == 7 && lane < C::CH) {
      double* dst = Y + C::SBP * C::KT;
      const int64_t k = k0 + 2 * lane;
      if (r_dma && k + 1 < k_end) {
        __builtin_amdgcn_global_load_lds((glb_vptr)(rg + k), (lds_vptr)dst, 16, 0, 0);
      } else {
        double2 v;
        v.x = k < k_end ? rg[k] : 0.0;
        v.y = k + 1 < k_end ? rg[k + 1] : 0.0;
        *reinterpret_cast<double2*>(dst + 2 * lane) = v;
      }
    }
  };
  // tile t's update from update buffer yslot; MODE 1 also fills the u slot
  // of Gram buffer uslot
  auto update = [&](int t, int yslot, int uslot) {
    const double* Y = lds + C::YOFF + yslot * C::YT;
    const double* dl = lds + C::DOFF;
    double p0 = 0.0, p1 = 0.0;
#pragma unroll 2
    for (int j = 0; j < C::SBP / 64; ++j) {
      const int r = lane + 64 * j;
      const double2 y = *reinterpret_cast<const double2*>(Y + r * C::KT + 2 * (W ^ d16_swz(r)));
      const double dj = dl[r];
      p0 = fma(y.x, dj, p0);
      p1 = fma(y.y, dj, p1);
    }
    // the wave's total: each row of 16 lanes by DPP rotations, then the four
    // row sums (lanes 0, 16, 32, 48) in a fixed order
    p0 = d16_row_sum(p0);
    p1 = d16_row_sum(p1);
    p0 = (d16_read_lane(p0, 0) + d16_read_lane(p0, 16)) +
         (d16_read_lane(p0, 32) + d16_read_lane(p0, 48));
    p1 = (d16_read_lane(p1, 0) + d16_read_lane(p1, 16)) +
         (d16_read_lane(p1, 32) + d16_read_lane(p1, 48));
    if (lane == 0) {
      const int64_t k = k_begin + (int64_t)t * C::KT + 2 * W;
      const double* ro = Y + C::SBP * C::KT;
      const double n0 = ro[2 * W] + p0, n1 = ro[2 * W + 1] + p1;
      if (k < k_end) rg[k] = n0;
      if (k + 1 < k_end) rg[k + 1] = n1;
      if constexpr (MODE == 1) {
        double* us = lds + uslot * C::TILE + C::SBP * C::KT;
        us[2 * W] = k < k_end ? n0 : 0.0;
        us[2 * W + 1] = k + 1 < k_end ? n1 : 0.0;
      }
    }
  };
  if constexpr (MODE == 2) {
    issue_y(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    for (int t = 0; t < ntiles; ++t) {
      if (t + 1 < ntiles) issue_y(t + 1, (t + 1) & 1);
      update(t, t & 1, -1);
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
    return;
  }

  auto issue = [&](int t, int slot) {
    const int64_t k0 = k_begin + (int64_t)t * C::KT;
    double* T = lds + slot * C::TILE;
#pragma unroll
    for (int i = 0; i < C::DMA_PER_WAVE; ++i) {
      double* dst = T + (C::DMA_PER_WAVE * W + i) * 128;   // 64 slots of 2 doubles
      const int64_t k = k0 + cofs[i];
      if (k + 1 < k_end) {
        __builtin_amdgcn_global_load_lds((glb_vptr)(src[i] + k), (lds_vptr)dst, 16, 0, 0);
      } else {
        double2 v;
        v.x = k < k_end ? src[i][k] : 0.0;
        v.y = 0.0;
        *reinterpret_cast<double2*>(dst + 2 * lane) = v;
      }
    }
    // the tile's KT entries of u (zeros without u): lanes 0..CH-1 of wave 7
    // (MODE 1: the update writes them)
    if (MODE == 0 && W == 7 && lane < C::CH) {
      double* dst = T + C::SBP * C::KT;
      const int64_t k = k0 + 2 * lane;
      if (u_dma && k + 1 < k_end) {
        __builtin_amdgcn_global_load_lds((glb_vptr)(ug + k), (lds_vptr)dst, 16, 0, 0);
      } else {
        double2 v;
        v.x = want_u && k < k_end ? ug[k] : 0.0;
        v.y = want_u && k + 1 < k_end ? ug[k + 1] : 0.0;
        *reinterpret_cast<double2*>(dst + 2 * lane) = v;
      }
    }
  };

  // This lane's fragment offsets (doubles) for the two k-pairs of a tile: row
  // lane & 15 of every block row, chunk 4 pp + lane / 16, swizzled.
  const int g = lane >> 4;
  const int rl = lane & 15;
  int lane_off[C::PP];
#pragma unroll
  for (int pp = 0; pp < C::PP; ++pp) lane_off[pp] = rl * C::KT + 2 * ((4 * pp + g) ^ d16_swz(rl));

  d4 acc[17];
#pragma unroll
  for (int a = 0; a < 17; ++a) acc[a] = d4{0.0, 0.0, 0.0, 0.0};
  double yua[2] = {0.0, 0.0};

  issue(0, 0);
  if constexpr (MODE == 1) {
    issue_y(0, 0);
    if (ntiles > 1) issue_y(1, 1);
  }
  __builtin_amdgcn_s_waitcnt(0);   // the LDS-DMA writes count on the vector memory counter
  __syncthreads();
  if constexpr (MODE == 1) {
    update(0, 0, 0);
    __syncthreads();
  }
  for (int t = 0; t < ntiles; ++t) {
    if (t + 1 < ntiles) issue(t + 1, (t + 1) & 1);
    if constexpr (MODE == 1) {
      // update buffer t & 1 held tile t (updated during tile t - 1); tile t + 1
      // arrived during tile t - 1.  Waves 0-3 update before their matrix
      // instructions, waves 4-7 (the other wave of each SIMD) after them, so
      // the update's latency runs beside the other wave's MFMA chain.
      if (t + 2 < ntiles) issue_y(t + 2, t & 1);
      if (W < 4 && t + 1 < ntiles) update(t + 1, (t + 1) & 1, (t + 1) & 1);
    }
    const double* tile = lds + (t & 1) * C::TILE;
#pragma unroll
    for (int pp = 0; pp < C::PP; ++pp) {
      const double* base = tile + lane_off[pp];
      auto frag = [&](int r) {   // rows 16 r .. 16 r + 15, this lane's chunk of pair pp
        return *reinterpret_cast<const double2*>(base + r * 16 * C::KT);
      };
      const double2 f0 = frag(R0);
      const double2 f1 = frag(R1);
      const double2 ut =   // u at the same two columns (unswizzled, after the rows)
          *reinterpret_cast<const double2*>(tile + C::SBP * C::KT + 8 * pp + 2 * g);
      yua[0] = fma(f0.x, ut.x, yua[0]);
      yua[0] = fma(f0.y, ut.y, yua[0]);
      yua[1] = fma(f1.x, ut.x, yua[1]);
      yua[1] = fma(f1.y, ut.y, yua[1]);
#pragma unroll
      for (int c = 0; c <= R1; ++c) {
        const double2 fc = c == R0 ? f0 : (c == R1 ? f1 : frag(c));
        if (c <= R0) {
          acc[c] = mfma(f0.x, fc.x, acc[c]);
          acc[c] = mfma(f0.y, fc.y, acc[c]);
        }
        acc[R0 + 1 + c] = mfma(f1.x, fc.x, acc[R0 + 1 + c]);
        acc[R0 + 1 + c] = mfma(f1.y, fc.y, acc[R0 + 1 + c]);
      }
    }
    if constexpr (MODE == 1) {
      if (W >= 4 && t + 1 < ntiles) update(t + 1, (t + 1) & 1, (t + 1) & 1);
    }
    __builtin_amdgcn_s_waitcnt(0);   // tile t + 1 is in LDS
    __syncthreads();
  }

  gptr<double> pg = glb(part);
#pragma unroll
  for (int a = 0; a < 17; ++a) {
    const int blk = a <= R0 ? blk_index(R0, a) : blk_index(R1, a - R0 - 1);
    gptr<double> dst = pg + blk * 256 + lane;
    dst[0] = acc[a][0];
    dst[64] = acc[a][1];
    dst[128] = acc[a][2];
    dst[192] = acc[a][3];
  }
  if (want_u) {   // Y u of the two owned block rows: sum the four lane groups
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      double v = yua[i];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      if (lane < 16) pg[C::NBLK * 256 + 16 * (i == 0 ? R0 : R1) + lane] = v;
    }
  }
}

// The NB = 16 slab of gram_slab<16, 2> on the DMA path; same arguments and
// partial layout (A must be 16-byte aligned with an even ld).
template <int MODE = 0>
__device__ __forceinline__ void gram_slab_dma16(const double* __restrict__ A, int64_t ld,
                                                int64_t k_begin, int64_t k_end,
                                                const int32_t* idx, int m,
                                                const double* __restrict__ u,
                                                double* __restrict__ part, double* lds,
                                                const D16Upd up = D16Upd{}) {
  switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {
    case 0: d16_slab<0, MODE>(A, ld, k_begin, k_end, idx, m, u, part, lds, up); break;
    case 1: d16_slab<1, MODE>(A, ld, k_begin, k_end, idx, m, u, part, lds, up); break;
    case 2: d16_slab<2, MODE>(A, ld, k_begin, k_end, idx, m, u, part, lds, up); break;
    case 3: d16_slab<3, MODE>(A, ld, k_begin, k_end, idx, m, u, part, lds, up); break;
    case 4: d16_slab<4, MODE>(A, ld, k_begin, k_end, idx, m, u, part, lds, up); break;
    case 5: d16_slab<5, MODE>(A, ld, k_begin, k_end, idx, m, u, part, lds, up); break;
    case 6: d16_slab<6, MODE>(A, ld, k_begin, k_end, idx, m, u, part, lds, up); break;
    default: d16_slab<7, MODE>(A, ld, k_begin, k_end, idx, m, u, part, lds, up); break;
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

// Writes the reduced entry e (sum t of its partials) to Gov / Yu.  add (may be
// NULL): an m x m row-major term added to the sum before scaling, read at
// (row, col) with row >= col (the light-column part of a split sparse Gram).
__device__ __forceinline__ void store_entry(int64_t e, double t, int nblk, const int32_t* idx,
                                            int m, double scale, double shift, int overlap,
                                            double* __restrict__ G, double* __restrict__ Yu,
                                            int layout, const float* __restrict__ rs,
                                            const double* __restrict__ add = nullptr) {
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
    if (add != nullptr) t += glb(add)[(int64_t)row * m + col];
    const double v = sc * t + (on ? shift : 0.0);
    glb(G)[(int64_t)row * m + col] = v;
    glb(G)[(int64_t)col * m + row] = v;
  }
}

// Index lists of a Gram of m in (256, 512] rows: ia = the m indices padded to
// 512 with idx[0] (two 256-row Grams: the diagonal blocks); ib[t] (t < nc,
// nc = 4 when m > 384, else 2) = idx[128 x .. 128 x + 128) followed by
// ia[256 + 128 y .. 256 + 128 y + 128), x = t % 2, y = t / 2, whose 256-row
// Gram holds the cross block of rows 256 + 128 y.. and columns 128 x.. .
// Padding rows are multiplied and never stored.  Thread t of nthreads.
__device__ __forceinline__ void big_lists(const int32_t* idx, int m, int32_t* ia, int32_t* ib,
                                          int t, int nthreads) {
  const int nc = m - 256 > 128 ? 4 : 2;
  const int i0 = idx[0];
  for (int q = t; q < 512; q += nthreads) ia[q] = idx[q < m ? q : 0];
  for (int slot = t; slot < 256 * nc; slot += nthreads) {
    const int list = slot >> 8, pos = slot & 255;
    const int x = list & 1, y = list >> 1;
    int v;
    if (pos < 128) {
      v = idx[128 * x + pos];
    } else {
      const int r = 256 + 128 * y + (pos - 128);
      v = r < m ? idx[r] : i0;
    }
    ib[slot] = v;
  }
}

// Where the reduced entry e of step `step` of a Gram of more than 256 rows
// goes (m in (256, 512], assembled from 256-row Grams; see
// launch_big_index): set 0 holds the two diagonal 256 x 256 blocks (step k:
// rows and columns 256 k + local) and Y u; set 1 holds the cross blocks, step
// t giving rows 256 + 128 (t / 2) + (local row - 128) and columns
// 128 (t % 2) + local column from the local block rows 8..15 x columns 0..7.
__device__ __forceinline__ void store_entry_big(int64_t e, double t, int set, int step,
                                                const int32_t* idx, int m, double scale,
                                                double shift, int overlap,
                                                double* __restrict__ G, double* __restrict__ Yu,
                                                int layout, const float* __restrict__ rs,
                                                const double* __restrict__ add) {
  constexpr int kNblk = 136;
  if (e >= (int64_t)kNblk * 256) {          // the Y u entries follow the blocks
    const int p = 256 * step + (int)(e - (int64_t)kNblk * 256);
    if (set == 0 && Yu != nullptr && p < m) glb(Yu)[p] = rs ? (double)glb(rs)[idx[p]] * t : t;
    return;
  }
  int row, col;
  bool lower;
  entry_rc(e, layout, row, col, lower);
  if (!lower) return;
  int gr, gc;
  if (set == 0) {
    gr = 256 * step + row;
    gc = 256 * step + col;
  } else {
    if (row < 128 || col >= 128) return;
    gr = 256 + 128 * (step >> 1) + (row - 128);
    gc = 128 * (step & 1) + col;
  }
  if (gr >= m || gc >= m) return;
  const bool on = overlap ? (idx[gr] == idx[gc]) : (gr == gc);
  const double sc = rs ? scale * (double)glb(rs)[idx[gr]] * (double)glb(rs)[idx[gc]] : scale;
  if (add != nullptr) t += glb(add)[(int64_t)gr * m + gc];
  const double v = sc * t + (on ? shift : 0.0);
  glb(G)[(int64_t)gr * m + gc] = v;
  glb(G)[(int64_t)gc * m + gr] = v;
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

// The reduction of a Gram of m <= 512 rows assembled from 256-row Grams, by
// one workgroup of T threads: slab q's partial set g (g < 2: the diagonal
// blocks, then the cross blocks; nsets = 2 + big_cross_steps(m)) is at
// partials + q sstride + g pstride16; every entry sums its slabs in slab order
// and is stored once (store_entry_big).
template <int T>
__device__ __forceinline__ void reduce_wg_big(const double* __restrict__ partials, int nslab,
                                              int64_t sstride, int nsets, const int32_t* idx,
                                              int m, double scale, double shift,
                                              double* __restrict__ G, double* __restrict__ Yu,
                                              int layout, const float* __restrict__ rs) {
  constexpr int64_t pstride = (int64_t)136 * 256 + 16 * 16;
  for (int g = 0; g < nsets; ++g) {
    const int cls = g < 2 ? 0 : 1, step = g < 2 ? g : g - 2;
    for (int64_t e = threadIdx.x; e < pstride; e += T) {
      const gptr<const double> p = glb(partials) + (int64_t)g * pstride + e;
      double s = 0.0;
      int q = 0;
      for (; q + 8 <= nslab; q += 8) {
        double v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = p[(int64_t)(q + j) * sstride];
#pragma unroll
        for (int j = 0; j < 8; ++j) s += v[j];
      }
      for (; q < nslab; ++q) s += p[(int64_t)q * sstride];
      store_entry_big(e, s, cls, step, idx, m, scale, shift, 1, G, Yu, layout, rs, nullptr);
    }
  }
}

}  // namespace gdev
}  // namespace cabcd
