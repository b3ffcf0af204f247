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

// ---------------------------------------------------------------------------
// sb in (128, 256] (NB = 16) with 16-byte aligned rows: the slab is fed by
// LDS-DMA (gfx950 global_load_lds_dwordx4), as in the FP64 kernel.  A tile is
// 256 rows x 256 bytes of codes (128 BF16 / 256 FP8 columns): the longer row
// pieces keep the HBM pages busier than 128-byte pieces, and a 64 KiB tile
// per workgroup in flight (one workgroup per CU, double-buffered in 130 KiB
// of LDS) covers the memory latency.  The sixteen 16-byte chunks of a row
// are stored XOR-swizzled (chunk c of row r at c ^ (r & 15)), so the sixteen
// rows of a fragment read fall in distinct banks.  Y u is formed from LDS:
// thread t of waves 0-3 decodes chunk t % 16 of rows t / 16 + 16 j (j < 16)
// against the tile's u segment (DMA'd beside the rows) and keeps one FP64
// sum per row; the sixteen chunk sums of a row are added in chunk order at
// the end.
__host__ __device__ constexpr int blk_index16(int r, int c) { return r * (r + 1) / 2 + c; }

template <int FMT>
struct LD16 {
  static constexpr int ES = FMT == CABCD_BF16 ? 2 : 1;   // element bytes
  static constexpr int SBP = 256, NBLK = 136;
  static constexpr int RB = 256;                         // row bytes per tile
  static constexpr int KT = RB / ES;                     // tile width in elements
  static constexpr int EPC = 16 / ES;                    // elements per chunk
  static constexpr int TILE = SBP * RB;                  // 64 KiB of codes
  static constexpr int UB = KT * 8;                      // the tile's u segment
  static constexpr int BUF = TILE + UB;
  static constexpr int LDS = 2 * BUF;
  static constexpr int DMA_PER_WAVE = TILE / 1024 / 8;   // 8 instructions of 1 KiB
  static constexpr int UDMA = UB / 1024;                 // 1 (BF16) or 2 (FP8)
};

// Blocks of the 16 x 16 block triangle by wave, in 4 x 4 super-blocks: waves
// 0-5 take the six off-diagonal super-blocks (16 blocks, 4 row and 4 column
// fragments per k-step), waves 6 and 7 two diagonal ones each (10 + 10
// blocks, 4 + 4 fragments).  Every wave reads 8 fragments per k-step where
// block-row pairs read 18, so the tile is read from LDS less than half as
// often; waves 6 and 7 carry 20 instead of 17 blocks.
constexpr int kSbI[6] = {1, 2, 3, 2, 3, 3};
constexpr int kSbJ[6] = {0, 0, 0, 1, 1, 2};
__host__ __device__ constexpr int lp16_sb_nacc(int W) { return W < 6 ? 16 : 20; }
__host__ __device__ constexpr int lp16_sb_block(int W, int a) {
  if (W < 6) return blk_index16(4 * kSbI[W] + a / 4, 4 * kSbJ[W] + a % 4);
  const int d = a < 10 ? (W == 6 ? 0 : 1) : (W == 6 ? 3 : 2);
  const int t = a % 10;                        // t = r (r + 1) / 2 + c, c <= r < 4
  const int r = t < 1 ? 0 : t < 3 ? 1 : t < 6 ? 2 : 3;
  return blk_index16(4 * d + r, 4 * d + t - r * (r + 1) / 2);
}

// One k-step of wave W's blocks: frag(r) gives the fragment of block row r,
// mma(row, col, acc) one matrix instruction.
template <int W, class Frag, class Mma>
__device__ __forceinline__ void lp16_sb_step(Frag frag, Mma mma, f4 (&acc)[20]) {
  if constexpr (W < 6) {
    constexpr int I = kSbI[W], J = kSbJ[W];
    decltype(frag(0)) rf[4], cf[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) rf[a] = frag(4 * I + a);
#pragma unroll
    for (int b = 0; b < 4; ++b) cf[b] = frag(4 * J + b);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[4 * a + b] = mma(rf[a], cf[b], acc[4 * a + b]);
  } else {
#pragma unroll
    for (int di = 0; di < 2; ++di) {
      const int d = di == 0 ? (W == 6 ? 0 : 1) : (W == 6 ? 3 : 2);
      decltype(frag(0)) f[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) f[a] = frag(4 * d + a);
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c <= r; ++c) {
          const int i = 10 * di + r * (r + 1) / 2 + c;
          acc[i] = mma(f[r], f[c], acc[i]);
        }
    }
  }
}

template <int FMT, int W>
__device__ __forceinline__ void lp16_slab(const uint8_t* __restrict__ A, int64_t ld,
                                          int64_t k_begin, int64_t k_end, const int32_t* idx,
                                          int m, const double* __restrict__ u,
                                          double* __restrict__ part, uint8_t* lds) {
  using C = LD16<FMT>;
  typedef __attribute__((address_space(3))) void* lds_vptr;
  typedef __attribute__((address_space(1))) const void* glb_vptr;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int ntiles = (int)((k_end - k_begin + C::KT - 1) / C::KT);
  const int64_t end_b = k_end * C::ES;   // row bytes in range

  // DMA instruction i of this wave fills tile bytes (8 W + i) KiB + 16 lane:
  // row 4 (8 W + i) + lane / 16, position lane % 16, chunk (lane % 16) ^ (row % 16).
  gptr<const uint8_t> src[C::DMA_PER_WAVE];
  int cof[C::DMA_PER_WAVE];
  const gptr<const uint8_t> Ag = glb(A);
#pragma unroll
  for (int i = 0; i < C::DMA_PER_WAVE; ++i) {
    const int r = 4 * (C::DMA_PER_WAVE * W + i) + (lane >> 4);
    cof[i] = 16 * ((lane & 15) ^ (r & 15));
    src[i] = Ag + (int64_t)idx[r < m ? r : 0] * ld * C::ES;   // rows past m: any valid row
  }
  const bool want_u = u != nullptr;
  const gptr<const double> ug = glb(u);
  const bool u_dma = want_u && (reinterpret_cast<uintptr_t>(u) & 15) == 0;
  // The tile's u segment in LDS: 16-byte slot 16 q + c holds piece
  // (EPC / 2) c + q of the segment (the q-th pair of u values of chunk c), so
  // the Y u threads of the sixteen chunks read a piece from consecutive slots.
  auto upiece = [](int slot) { return (C::EPC / 2) * (slot & 15) + (slot >> 4); };
  // A tile inside the slab is all DMA; the last tile of a slab that ends
  // inside a tile is filled by a compact loop of ordinary loads (zeros past
  // the end), kept out of line of the DMA path to keep the loop body small.
  auto issue = [&](int t, int slot) {
    const int64_t k0 = k_begin + (int64_t)t * C::KT;
    uint8_t* T = lds + slot * C::BUF;
    if (k0 + C::KT <= k_end) {
#pragma unroll
      for (int i = 0; i < C::DMA_PER_WAVE; ++i)
        __builtin_amdgcn_global_load_lds((glb_vptr)(src[i] + k0 * C::ES + cof[i]),
                                         (lds_vptr)(T + (C::DMA_PER_WAVE * W + i) * 1024), 16,
                                         0, 0);
      if (want_u && W == 7) {   // the tile's u segment after the rows, pieces transposed
#pragma unroll
        for (int j = 0; j < C::UDMA; ++j) {
          uint8_t* dst = T + C::TILE + j * 1024;
          const int64_t ku = k0 + 2 * upiece(64 * j + lane);
          if (u_dma) {
            __builtin_amdgcn_global_load_lds((glb_vptr)(ug + ku), (lds_vptr)dst, 16, 0, 0);
          } else {
            double2 v;
            v.x = ug[ku];
            v.y = ug[ku + 1];
            *reinterpret_cast<double2*>(dst + 16 * lane) = v;
          }
        }
      }
      return;
    }
#pragma unroll
    for (int i = 0; i < C::DMA_PER_WAVE; ++i) {
      const int64_t kb = k0 * C::ES + cof[i];
      uint64_t lo = 0, hi = 0;
#pragma clang loop unroll(disable)
      for (int e = 0; e < 16; ++e) {
        const uint64_t v = kb + e < end_b ? (uint64_t)src[i][kb + e] : 0;
        if (e < 8)
          lo |= v << (8 * e);
        else
          hi |= v << (8 * (e - 8));
      }
      *reinterpret_cast<uint4*>(T + (C::DMA_PER_WAVE * W + i) * 1024 + 16 * lane) =
          make_uint4((uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32));
    }
    if (want_u && W == 7) {
#pragma clang loop unroll(disable)
      for (int j = 0; j < C::UDMA; ++j) {
        const int64_t ku = k0 + 2 * upiece(64 * j + lane);
        double2 v;
        v.x = ku < k_end ? ug[ku] : 0.0;
        v.y = ku + 1 < k_end ? ug[ku + 1] : 0.0;
        *reinterpret_cast<double2*>(T + C::TILE + j * 1024 + 16 * lane) = v;
      }
    }
  };

  // fragment offsets of the four 64-byte windows: row lane % 16 of a block row,
  // chunk 4 w + lane / 16, swizzled.  FP8 takes the K = 128 instruction of
  // gfx950 on 128-byte halves: chunks 8 h + 2 (lane / 16) and the next one.
  int lane_off[4];
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const int ch = FMT == CABCD_BF16 ? 4 * w + (lane >> 4)
                                     : 8 * (w >> 1) + 2 * (lane >> 4) + (w & 1);
    lane_off[w] = (lane & 15) * C::RB + 16 * (ch ^ (lane & 15));
  }

  f4 acc[20];
#pragma unroll
  for (int a = 0; a < 20; ++a) acc[a] = f4{0.f, 0.f, 0.f, 0.f};
  // Y u on waves 0-3 only (one of the two waves of each SIMD, so its vector
  // work runs beside the other wave's matrix instructions; all eight waves
  // taking a share: FP8 63.5 against 60.4 us at n = 2^20): thread t < 256
  // sums chunk yc = t % 16 of rows yr0 + 16 j, yr0 = t / 16, j < 16
  constexpr int YJ = W < 4 ? 16 : 0;
  const int yc = tid & 15, yr0 = tid >> 4;
  double yu[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) yu[j] = 0.0;

  issue(0, 0);
  __builtin_amdgcn_s_waitcnt(0);   // the LDS-DMA writes count on the vector memory counter
  __syncthreads();
  for (int t = 0; t < ntiles; ++t) {
    if (t + 1 < ntiles) issue(t + 1, (t + 1) & 1);
    const uint8_t* tile = lds + (t & 1) * C::BUF;
    // 4 windows (BF16, K = 32) or 2 halves (FP8, K = 128) per tile
#pragma unroll
    for (int h = 0; h < (FMT == CABCD_BF16 ? 4 : 2); ++h) {
      if constexpr (FMT == CABCD_BF16) {
        const uint8_t* base = tile + lane_off[h];
        lp16_sb_step<W>([&](int r) {
          return *reinterpret_cast<const uint4*>(base + r * 16 * C::RB);
        }, [](const uint4& x, const uint4& y, f4 c) { return lp_mma_bf16(x, y, c); }, acc);
      } else {
        const uint8_t* b0 = tile + lane_off[2 * h];
        const uint8_t* b1 = tile + lane_off[2 * h + 1];
        lp16_sb_step<W>([&](int r) {   // 32 codes of row r: two 16-byte chunks
          const uint4 x = *reinterpret_cast<const uint4*>(b0 + r * 16 * C::RB);
          const uint4 y = *reinterpret_cast<const uint4*>(b1 + r * 16 * C::RB);
          return lp_i8v{(int)x.x, (int)x.y, (int)x.z, (int)x.w, (int)y.x, (int)y.y, (int)y.z,
                        (int)y.w};
        }, [](const lp_i8v& x, const lp_i8v& y, f4 c) { return lp_mma_k128(x, y, c); }, acc);
      }
    }
    if (want_u) {
      // the 16-byte pieces of chunk yc sit 256 bytes apart, so the sixteen
      // chunks' reads of one piece fall in distinct banks
      double ub[C::EPC];
#pragma unroll
      for (int q = 0; q < C::EPC / 2; ++q) {
        const double2 v =
            *reinterpret_cast<const double2*>(tile + C::TILE + 16 * (16 * q + yc));
        ub[2 * q] = v.x;
        ub[2 * q + 1] = v.y;
      }
#pragma unroll
      for (int j = 0; j < YJ; ++j) {
        const int r = yr0 + 16 * j;
        const uint4 v = *reinterpret_cast<const uint4*>(tile + r * C::RB + 16 * (yc ^ (r & 15)));
        double dv[C::EPC];
        lp_decode_all<FMT>(v, dv);
#pragma unroll
        for (int e = 0; e < C::EPC; ++e) yu[j] = fma(dv[e], ub[e], yu[j]);
      }
    }
    __builtin_amdgcn_s_waitcnt(0);   // tile t + 1 is in LDS
    __syncthreads();
  }

  // partial blocks as FP32 (what the accumulators hold; half the bytes of
  // FP64), Y u as FP64 at its usual place
  gptr<double> pg = glb(part);
  const gptr<float> pf = (gptr<float>)pg;
#pragma unroll
  for (int a = 0; a < lp16_sb_nacc(W); ++a) {
    gptr<float> dst = pf + lp16_sb_block(W, a) * 256 + lane;
    dst[0] = acc[a][0];
    dst[64] = acc[a][1];
    dst[128] = acc[a][2];
    dst[192] = acc[a][3];
  }
  if (want_u) {   // the sixteen chunk sums of each row, in chunk order
    double* ys = reinterpret_cast<double*>(lds);
#pragma unroll
    for (int j = 0; j < YJ; ++j) ys[(yr0 + 16 * j) * 16 + yc] = yu[j];
    __syncthreads();
    if (tid < C::SBP) {
      double sum = 0.0;
#pragma unroll
      for (int q = 0; q < 16; ++q) sum += ys[tid * 16 + q];
      pg[C::NBLK * 256 + tid] = sum;
    }
  }
}

template <int FMT>
__global__ __launch_bounds__(kLpThreads) void gram_lp_dma16_kernel(
    const uint8_t* __restrict__ A, int64_t ld, int64_t cols, const int32_t* __restrict__ idx,
    int m, const double* __restrict__ u, int64_t chunk, double* __restrict__ partials,
    int64_t pstride) {
  using C = LD16<FMT>;
  extern __shared__ __attribute__((aligned(16))) uint8_t dyn_lds[];
  idx += (int64_t)blockIdx.y * m;            // several outer steps per launch
  partials += (int64_t)blockIdx.y * pstride;
  const int64_t k_begin = (int64_t)blockIdx.x * chunk;
  const int64_t k_end = std::min(cols, k_begin + chunk);
  double* part = partials + (int64_t)blockIdx.x * (C::NBLK * 256 + C::SBP);
  switch (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) {
    case 0: lp16_slab<FMT, 0>(A, ld, k_begin, k_end, idx, m, u, part, dyn_lds); break;
    case 1: lp16_slab<FMT, 1>(A, ld, k_begin, k_end, idx, m, u, part, dyn_lds); break;
    case 2: lp16_slab<FMT, 2>(A, ld, k_begin, k_end, idx, m, u, part, dyn_lds); break;
    case 3: lp16_slab<FMT, 3>(A, ld, k_begin, k_end, idx, m, u, part, dyn_lds); break;
    case 4: lp16_slab<FMT, 4>(A, ld, k_begin, k_end, idx, m, u, part, dyn_lds); break;
    case 5: lp16_slab<FMT, 5>(A, ld, k_begin, k_end, idx, m, u, part, dyn_lds); break;
    case 6: lp16_slab<FMT, 6>(A, ld, k_begin, k_end, idx, m, u, part, dyn_lds); break;
    default: lp16_slab<FMT, 7>(A, ld, k_begin, k_end, idx, m, u, part, dyn_lds); break;
  }
}

template <int FMT>
hipError_t launch_lp_dma16(const GramPlan& p, const void* A, int64_t ld, int64_t cols,
                           const int32_t* idx, int m, int nsteps, const double* u,
                           double* partials, hipStream_t st) {
  using C = LD16<FMT>;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(gram_lp_dma16_kernel<FMT>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, C::LDS);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((gram_lp_dma16_kernel<FMT>), dim3((unsigned)p.nsplit, (unsigned)nsteps),
                     dim3(kLpThreads), C::LDS, st, static_cast<const uint8_t*>(A), ld, cols, idx,
                     m, u, p.chunk, partials, (int64_t)gram_partial_doubles(p));
  return hipGetLastError();
}

template <int NB, int FMT>
hipError_t launch_lp_nb(const GramPlan& p, const void* A, int64_t ld, int64_t cols,
                        const int32_t* idx, int m, int nsteps, const double* u,
                        double* partials, hipStream_t st) {
  using C = LpCfg<NB, FMT>;
  const int aligned =
      ((reinterpret_cast<uintptr_t>(A) & 15) == 0 && ((ld * C::ES) & 15) == 0) ? 1 : 0;
  if constexpr (NB == 16) {
    if (aligned && p.chunk % LD16<FMT>::KT == 0)
      return launch_lp_dma16<FMT>(p, A, ld, cols, idx, m, nsteps, u, partials, st);
  }
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
//
// Each thread owns 16 bytes of codes per row (EPC columns); the RS threads of
// a column chunk split the rows into RS consecutive ranges whose sums are
// added in range order through LDS (deterministic).  FP8 takes two ranges: with
// 16 columns per thread a pass over 2^20 columns has one wave per SIMD, too few
// loads in flight to stream (3.6 TB/s; two ranges: 5.7 TB/s, four: 4.7).  BF16
// (8 columns per thread) already has two waves per SIMD and streams best with
// one range.  RIF rows are in flight per thread (16 measured slower).
constexpr int kLvThreads = 256;
template <int FMT> constexpr int kLvSlices = FMT == CABCD_BF16 ? 1 : 2;
constexpr int kLvRif = 8;

template <int FMT, int RS>
__global__ __launch_bounds__(kLvThreads) void gemv_t_lp_kernel(
    const uint8_t* __restrict__ A, int64_t ld, int64_t cols, const float* __restrict__ rs,
    const int32_t* __restrict__ idx, int64_t m, const double* __restrict__ v, double gamma,
    const double* __restrict__ base, double beta, int accumulate, double* __restrict__ out,
    int aligned) {
  constexpr int ES = FMT == CABCD_BF16 ? 2 : 1;
  constexpr int EPC = 16 / ES;
  constexpr int CPB = kLvThreads / RS;   // column chunks per workgroup
  constexpr int RIF = kLvRif;
  static_assert(CPB % 64 == 0, "a row range is a whole number of waves");
  const int tc = threadIdx.x % CPB;
  // the row range is uniform in a wave, so the row indices and coefficients
  // stay scalar loads; lanes past the last column load zeros (lp_load)
  const int sl = __builtin_amdgcn_readfirstlane(threadIdx.x / CPB);
  const int64_t k = ((int64_t)blockIdx.x * CPB + tc) * EPC;
  const bool live = k < cols;
  if constexpr (RS == 1) {
    if (!live) return;
  }
  const int64_t per = (m + RS - 1) / RS;
  const int64_t p1 = std::min<int64_t>(m, (sl + 1) * per);
  double acc[EPC];
#pragma unroll
  for (int e = 0; e < EPC; ++e) acc[e] = 0.0;
  int64_t p = sl * per;
  for (; p + RIF <= p1; p += RIF) {
    uint4 x[RIF];
    double c[RIF];
#pragma unroll
    for (int q = 0; q < RIF; ++q) {
      const int64_t row = idx ? (int64_t)idx[p + q] : p + q;
      c[q] = v[p + q] * (rs ? (double)rs[row] : 1.0);
      x[q] = lp_load<FMT>(A + row * ld * ES, k, cols, aligned != 0);
    }
#pragma unroll
    for (int q = 0; q < RIF; ++q) {
      double dv[EPC];
      lp_decode_all<FMT>(x[q], dv);
#pragma unroll
      for (int e = 0; e < EPC; ++e) acc[e] = fma(dv[e], c[q], acc[e]);
    }
  }
  for (; p < p1; ++p) {
    const int64_t row = idx ? (int64_t)idx[p] : p;
    const double cq = v[p] * (rs ? (double)rs[row] : 1.0);
    const uint4 x = lp_load<FMT>(A + row * ld * ES, k, cols, aligned != 0);
    double dv[EPC];
    lp_decode_all<FMT>(x, dv);
#pragma unroll
    for (int e = 0; e < EPC; ++e) acc[e] = fma(dv[e], cq, acc[e]);
  }
  if constexpr (RS > 1) {
    __shared__ double red[RS - 1][EPC][CPB];
    if (sl > 0) {
#pragma unroll
      for (int e = 0; e < EPC; ++e) red[sl - 1][e][tc] = acc[e];
    }
    __syncthreads();
    if (sl > 0) return;
#pragma unroll
    for (int r = 0; r < RS - 1; ++r)
#pragma unroll
      for (int e = 0; e < EPC; ++e) acc[e] += red[r][e][tc];
  }
  if (!live) return;
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
  if (nb == 16) {
    // the LDS-DMA kernel (aligned rows): one workgroup per CU, 256-byte tile
    // rows; its slabs also suit the register-fed kernel (a multiple of kt)
    const int64_t kt = 256 / es;
    int64_t chunk = std::max<int64_t>(kt, (cols + 255) / 256);
    chunk = ((chunk + kt - 1) / kt) * kt;
    p.chunk = chunk;
    p.nsplit = (int)((cols + chunk - 1) / chunk);
    return p;
  }
  // HBM-bound: about two workgroups per CU, and slabs long enough that the
  // partial blocks (nblk*2 KiB per workgroup) stay small next to the slab.
  const int64_t min_chunk = std::max<int64_t>(p.kt, (int64_t)p.nblk * 2048 * 8 / (16 * nb * es));
  int64_t chunk = std::max<int64_t>(min_chunk, (cols + 511) / 512);
  chunk = ((chunk + p.kt - 1) / p.kt) * p.kt;
  p.chunk = chunk;
  p.nsplit = (int)((cols + chunk - 1) / chunk);
  return p;
}

int gram_lp_partial_layout(const GramPlan& p, int dtype, const void* A, int64_t ld) {
  const int es = dtype == CABCD_BF16 ? 2 : 1;
  const bool aligned = (reinterpret_cast<uintptr_t>(A) & 15) == 0 && ((ld * es) & 15) == 0;
  return p.nb == 16 && aligned && p.chunk % (256 / es) == 0 ? 2 : 1;
}

hipError_t launch_gram_lp(const GramPlan& p, int dtype, const void* A, int64_t ld, int64_t cols,
                          const int32_t* idx, int m, const double* u, double* partials,
                          hipStream_t st, int nsteps) {
  if (nsteps < 1 || nsteps > 65535) return hipErrorInvalidValue;
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
  const int slices = dtype == CABCD_BF16 ? kLvSlices<CABCD_BF16> : kLvSlices<CABCD_FP8_E4M3>;
  const int64_t per_block = (int64_t)(kLvThreads / slices) * epc;
  const int64_t blocks = (cols + per_block - 1) / per_block;
  if (dtype == CABCD_BF16)
    hipLaunchKernelGGL((gemv_t_lp_kernel<CABCD_BF16, kLvSlices<CABCD_BF16>>),
                       dim3((unsigned)blocks), dim3(kLvThreads), 0, st,
                       static_cast<const uint8_t*>(A), ld, cols, rs, idx, m, v, gamma, base, beta,
                       accumulate ? 1 : 0, out, aligned);
  else
    hipLaunchKernelGGL((gemv_t_lp_kernel<CABCD_FP8_E4M3, kLvSlices<CABCD_FP8_E4M3>>),
                       dim3((unsigned)blocks), dim3(kLvThreads), 0, st,
                       static_cast<const uint8_t*>(A), ld, cols, rs, idx, m, v, gamma, base, beta,
                       accumulate ? 1 : 0, out, aligned);
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
