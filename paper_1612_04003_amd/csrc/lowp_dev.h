// Device code of the low-precision (BF16 / FP8-E4M3 storage) Gram on the
// CDNA4 matrix cores with FP32 accumulation, shared by the one-problem kernel
// and the batched persistent kernel.  Same decomposition as the FP64 Gram
// (split-K slabs, 32 KiB LDS tiles, two block rows per wave); the partial
// blocks are stored in the FP32 MFMA output order.
#pragma once

#include "internal.h"

#include <algorithm>

namespace cabcd {
namespace ldev {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kLpThreads = 512;   // 8 waves, two block rows each

// FMT: CABCD_BF16 (2-byte elements, one MFMA per 16-byte fragment) or
// CABCD_FP8_E4M3 (1-byte elements, one K = 128 MFMA per two 16-byte fragments).
// TB: tile bytes per row times NB (a tile of SBP rows holds 16 TB bytes).
template <int NB, int FMT, int TB = 2048>
struct LpCfg {
  static constexpr int ES = FMT == CABCD_BF16 ? 2 : 1;      // element bytes
  static constexpr int SBP = 16 * NB;
  static constexpr int NBLK = NB * (NB + 1) / 2;
  static constexpr int RB = TB / NB;                        // tile row bytes: tile = 16 TB
  static constexpr int RSB = RB + 16;                       // LDS row stride in bytes
  static constexpr int KT = RB / ES;                        // tile width in elements
  static constexpr int EPC = 16 / ES;                       // elements per 16-byte chunk
  static constexpr int CH = RB / 16;                        // chunks per row
  static constexpr int NCH = SBP * CH / kLpThreads;         // chunks per thread (= 4)
  static constexpr int WIN = RB / 64;                       // 64-byte windows per tile row
  static constexpr int BW = NB >= 2 ? NB / 2 : 1;
  static constexpr int KG = 8 / BW;
  static constexpr int NACC = NB >= 2 ? NB + 1 : 1;
  static constexpr int TILE = SBP * RSB;                    // bytes
  static constexpr int RED = (KG - 1) * NBLK * 256 * 4;     // bytes (FP32 partial blocks)
  static constexpr int YUS = SBP * CH * 8;                  // bytes
  static constexpr int LDS = std::max(std::max(2 * TILE, RED), YUS);
  static_assert(NCH * kLpThreads == SBP * CH, "tile must split evenly");
  static_assert(WIN % KG == 0, "windows must split evenly");
};

__device__ __forceinline__ int lp_blk_index(int r, int c) { return r * (r + 1) / 2 + c; }

template <int NB>
__device__ __forceinline__ int lp_acc_block(int bw, int a) {
  if (NB == 1) return 0;
  const int r1 = bw, r2 = NB - 1 - bw;
  return a <= r1 ? lp_blk_index(r1, a) : lp_blk_index(r2, a - r1 - 1);
}

// BF16 x BF16, K = 32: each lane brings 8 codes of its row.
__device__ __forceinline__ f4 lp_mma_bf16(const uint4& a, const uint4& b, f4 c) {
  bf16x8 x, y;
  __builtin_memcpy(&x, &a, 16);
  __builtin_memcpy(&y, &b, 16);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
}

typedef int lp_i8v __attribute__((ext_vector_type(8)));

// E4M3 x E4M3 on the gfx950 K = 128 instruction (format 0 for both operands,
// no block scaling): each lane brings 32 codes of its row.
__device__ __forceinline__ f4 lp_mma_k128(const lp_i8v& a, const lp_i8v& b, f4 c) {
  return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
}

template <int NB, int FMT, int W, int TB>
__device__ __forceinline__ void lp_tile(const uint8_t* __restrict__ tile, int lane, int kg,
                                        f4 (&acc)[LpCfg<NB, FMT, TB>::NACC]) {
  using C = LpCfg<NB, FMT, TB>;
  constexpr int R1 = NB >= 2 ? W : 0;
  constexpr int R2 = NB >= 2 ? NB - 1 - W : 0;
  const uint8_t* base = tile + (lane & 15) * C::RSB + 16 * (lane >> 4);
  if constexpr (FMT == CABCD_BF16) {
#pragma unroll
    for (int p = 0; p < C::WIN / C::KG; ++p) {
      const int off = 64 * (kg + p * C::KG);
      auto frag = [&](int r) {
        return *reinterpret_cast<const uint4*>(base + r * 16 * C::RSB + off);
      };
      const uint4 f1 = frag(R1);
      const uint4 f2 = NB >= 2 ? frag(R2) : f1;
#pragma unroll
      for (int c = 0; c <= R2; ++c) {
        const uint4 fc = c == R1 ? f1 : (c == R2 ? f2 : frag(c));
        if (c <= R1) acc[c] = lp_mma_bf16(f1, fc, acc[c]);
        if constexpr (NB >= 2) acc[R1 + 1 + c] = lp_mma_bf16(f2, fc, acc[R1 + 1 + c]);
      }
    }
  } else {
    // FP8: two of this group's 64-byte windows per K = 128 instruction (the
    // same 32 codes of a row for both operands, so which columns pair up
    // does not matter for Y Y^T)
    static_assert((C::WIN / C::KG) % 2 == 0, "windows pair up");
#pragma unroll
    for (int p = 0; p < C::WIN / C::KG; p += 2) {
      const int off0 = 64 * (kg + p * C::KG), off1 = 64 * (kg + (p + 1) * C::KG);
      auto frag = [&](int r) {
        const uint4 x = *reinterpret_cast<const uint4*>(base + r * 16 * C::RSB + off0);
        const uint4 y = *reinterpret_cast<const uint4*>(base + r * 16 * C::RSB + off1);
        return lp_i8v{(int)x.x, (int)x.y, (int)x.z, (int)x.w, (int)y.x, (int)y.y, (int)y.z,
                      (int)y.w};
      };
      const lp_i8v f1 = frag(R1);
      const lp_i8v f2 = NB >= 2 ? frag(R2) : f1;
#pragma unroll
      for (int c = 0; c <= R2; ++c) {
        const lp_i8v fc = c == R1 ? f1 : (c == R2 ? f2 : frag(c));
        if (c <= R1) acc[c] = lp_mma_k128(f1, fc, acc[c]);
        if constexpr (NB >= 2) acc[R1 + 1 + c] = lp_mma_k128(f2, fc, acc[R1 + 1 + c]);
      }
    }
  }
}

template <int NB, int FMT, int TB, int W = 0>
__device__ __forceinline__ void lp_dispatch(int bw, const uint8_t* tile, int lane, int kg,
                                            f4 (&acc)[LpCfg<NB, FMT, TB>::NACC]) {
  if constexpr (W < LpCfg<NB, FMT, TB>::BW) {
    if (bw == W)
      lp_tile<NB, FMT, W, TB>(tile, lane, kg, acc);
    else
      lp_dispatch<NB, FMT, TB, W + 1>(bw, tile, lane, kg, acc);
  }
}

// The 16 / 8 elements of a 16-byte chunk of codes, decoded exactly to FP64.
template <int FMT>
__device__ __forceinline__ void lp_decode_all(const uint4& v, double (&out)[FMT == CABCD_BF16 ? 8 : 16]) {
  const uint32_t words[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    if constexpr (FMT == CABCD_BF16) {
      out[2 * w] = decode_bf16(words[w] & 0xFFFFu);
      out[2 * w + 1] = decode_bf16(words[w] >> 16);
    } else {
      // The hardware E4M3 -> FP32 conversion (OCP format on gfx950; exact, as
      // every E4M3 value is an FP32 value) replaces a bit-level decode that
      // made the FP8 streaming passes ALU-bound.
      const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)words[w], false);
      const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)words[w], true);
      out[4 * w] = (double)lo[0];
      out[4 * w + 1] = (double)lo[1];
      out[4 * w + 2] = (double)hi[0];
      out[4 * w + 3] = (double)hi[1];
    }
  }
}

// 16-byte chunk of row `row` starting at element k (zeros past k_end).
template <int FMT, class PTR>
__device__ __forceinline__ uint4 lp_load(PTR row, int64_t k, int64_t k_end, bool aligned) {
  constexpr int ES = FMT == CABCD_BF16 ? 2 : 1;
  constexpr int EPC = 16 / ES;
  if (k + EPC <= k_end && aligned) {
    typedef unsigned int uv4 __attribute__((ext_vector_type(4)));
    const uv4 t = *(gptr<const uv4>)(row + k * ES);
    return make_uint4(t.x, t.y, t.z, t.w);
  }
  uint8_t b[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) b[e] = (k + e / ES < k_end) ? row[k * ES + e] : 0;
  uint4 v;
  __builtin_memcpy(&v, b, 16);
  return v;
}

// One workgroup's slab of the low-precision Gram: columns [k_begin, k_end) of
// the rows idx[0..m) of the stored codes A (ld in elements), FP32 MFMA
// accumulation, partial blocks (FP32 MFMA output order) and partial Y u (FP64,
// decoded codes, row scales not applied) to part.  lds holds LpCfg::LDS bytes.
template <int NB, int FMT, int TB = 2048>
__device__ __forceinline__ void gram_lp_slab(const uint8_t* __restrict__ A, int64_t ld,
                                             int64_t k_begin, int64_t k_end, const int32_t* idx,
                                             int m, const double* __restrict__ u,
                                             double* __restrict__ part, int aligned,
                                             uint8_t* lds) {
  using C = LpCfg<NB, FMT, TB>;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int bw = wave % C::BW;
  const int kg = wave / C::BW;
  const int c = tid % C::CH;
  const int ntiles = (int)((k_end - k_begin + C::KT - 1) / C::KT);

  int rho[C::NCH];
  gptr<const uint8_t> rowp[C::NCH];
  const gptr<const double> ug = glb(u);
#pragma unroll
  for (int i = 0; i < C::NCH; ++i) {
    rho[i] = tid / C::CH + (kLpThreads / C::CH) * i;
    rowp[i] = rho[i] < m ? glb(A) + (int64_t)idx[rho[i]] * ld * C::ES : nullptr;
  }
  const bool want_u = u != nullptr;
  double yu[C::NCH];
  uint4 buf[C::NCH];
  double ub[C::EPC];
#pragma unroll
  for (int i = 0; i < C::NCH; ++i) yu[i] = 0.0;

  auto load_tile = [&](int t) {
    const int64_t k = k_begin + (int64_t)t * C::KT + (int64_t)C::EPC * c;
    if (want_u) {
#pragma unroll
      for (int e = 0; e < C::EPC; ++e) ub[e] = (k + e < k_end) ? ug[k + e] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < C::NCH; ++i)
      buf[i] = rowp[i] ? lp_load<FMT>(rowp[i], k, k_end, aligned != 0) : make_uint4(0, 0, 0, 0);
  };
  auto store_tile = [&](int slot) {
    uint8_t* T = lds + slot * C::TILE;
#pragma unroll
    for (int i = 0; i < C::NCH; ++i) {
      *reinterpret_cast<uint4*>(T + rho[i] * C::RSB + 16 * c) = buf[i];
      if (want_u) {
        double dv[C::EPC];
        lp_decode_all<FMT>(buf[i], dv);
#pragma unroll
        for (int e = 0; e < C::EPC; ++e) yu[i] = fma(dv[e], ub[e], yu[i]);
      }
    }
  };

  f4 acc[C::NACC];
#pragma unroll
  for (int a = 0; a < C::NACC; ++a) acc[a] = f4{0.f, 0.f, 0.f, 0.f};
  load_tile(0);
  store_tile(0);
  __syncthreads();
  for (int t = 0; t < ntiles; ++t) {
    const bool more = t + 1 < ntiles;
    if (more) load_tile(t + 1);
    lp_dispatch<NB, FMT, TB>(bw, lds + (t & 1) * C::TILE, lane, kg, acc);
    if (more) store_tile((t + 1) & 1);
    __syncthreads();
  }

  float* red = reinterpret_cast<float*>(lds);
  if constexpr (C::KG > 1) {
    if (kg > 0) {
#pragma unroll
      for (int a = 0; a < C::NACC; ++a) {
        float* dst = red + ((kg - 1) * C::NBLK + lp_acc_block<NB>(bw, a)) * 256 + lane;
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
          const float* src = red + ((g - 1) * C::NBLK + lp_acc_block<NB>(bw, a)) * 256 + lane;
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
      gptr<double> dst = glb(part) + lp_acc_block<NB>(bw, a) * 256 + lane;
      dst[0] = acc[a][0];
      dst[64] = acc[a][1];
      dst[128] = acc[a][2];
      dst[192] = acc[a][3];
    }
  }
  if (want_u) {
    __syncthreads();
    double* ys = reinterpret_cast<double*>(lds);
#pragma unroll
    for (int i = 0; i < C::NCH; ++i) ys[rho[i] * C::CH + c] = yu[i];
    __syncthreads();
    if (tid < C::SBP) {
      double s = 0.0;
      for (int q = 0; q < C::CH; ++q) s += ys[tid * C::CH + q];
      glb(part)[C::NBLK * 256 + tid] = s;
    }
  }
}


}  // namespace ldev
}  // namespace cabcd
