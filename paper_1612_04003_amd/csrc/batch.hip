// Batched primal CA-BCD: many independent ridge problems (Alg. 2 each) advanced
// together, one persistent launch per outer step ("round") for the whole batch.
//
// A round is a work queue of column slabs (problem p, slab q).  A workgroup
// that takes a slab
//   1. draws the blocks of the problem's current outer step (the sampler is
//      keyed by (seed, h), so every slab of the problem gets the same ones);
//   2. applies the problem's pending companion update r += Y_prev^T delta_prev
//      on the slab's columns (the deferred residual update of the previous
//      outer step, Alg. 2), so the update's HBM traffic lands in the same pass
//      as the next Gram instead of a pass of its own;
//   3. computes the slab's Gram partial and Y r partial (the split-K slab of the
//      one-problem Gram kernel);
//   4. counts its arrival; the workgroup that completes the problem's set of
//      slabs sums the partials in slab order (deterministic), runs the fused
//      solve of the s blocks (Gauss-Jordan block inverses, recurrence,
//      w[idx] += delta) and records
//      the step.  No workgroup ever waits for another.
// A second persistent kernel evaluates f(w) every few rounds, either
// recomputing r = X^T w - y exactly from X (the periodic full residual of the
// paper's stopping discussion) or from the maintained residual after applying
// the pending update, and retires problems that reached their target; it also
// flushes the pending update at the end of a run.  The plan captures one
// monitor period into hipGraphs.
#include "gram_dev.h"
#include "lowp_dev.h"
#include "solve_dev.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

namespace cabcd {
namespace {

constexpr int kBT = 512;           // threads of the batched kernels (8 waves)
constexpr int kBMaxRows = 512;     // s*b of one problem (above 256: assembled Gram)
constexpr int kBMaxB = 16;
constexpr int kBMaxSlabs = 64;
// Low-precision slabs stream tiles of 16 kBLpTile bytes (64 KiB; the
// one-problem kernels use 32 KiB): a round's many problems fill the GPU
// without narrow slabs, and the doubled bytes in flight per workgroup cut the
// BF16 record to 1e-6 from 0.141 to 0.131 s.
constexpr int kBLpTile = 4096;

struct BProb {                     // constant per problem (device copy)
  const void* A;                   // FP64 values or BF16 / FP8 codes (row-major)
  const float* rs;                 // FP8 row scales (NULL: 1)
  int64_t ld, d, n;
  const double* y;
  double* w;
  double* r;
  double lambda;
  double f_target;
  uint64_t seed;
  int64_t H;                       // inner-iteration budget (INT64_MAX: none)
  int64_t chunk;                   // columns per slab
  int b, s, bp, nb;
  int nslab, aligned;
  int sets, pad;                   // partial sets per slab (1; above 256 rows 4 or 6)
  double* partials;                // nslab x sets x (nblk*256 + 16 nb)
  double* G;                       // (s b)^2
  double* Yu;                      // s b
  double* delta;                   // s b: the last step's delta
  double* objp;                    // nslab partial sums of r^2
};

struct BState {                    // mutable per problem
  int64_t h;                       // inner iterations done
  int64_t h_prev;                  // first iteration of the step with a pending update
  int64_t steps;                   // outer steps done
  double obj;                      // f(w) at the last monitor point
  int m_prev;                      // rows of the pending companion update (0: none)
  int active;                      // still iterating
  int arrive;                      // slab arrivals in the current launch
  int status;                      // DeviceStatus (sticky)
  int fresh;                       // 0: stale, 1: obj from the maintained r, 2: r exact
  int pad[3];
};

struct BItem {
  int prob, slab;
};

struct BQueue {
  int ticket, exited;
};

// -------------------------------------------------------------- device helpers

// out[k] = (base ? beta base[k] : out[k]) + sum_{q < mq} A[row(q)][k] coef[q],
// k in [k0, k1), row(q) = rows ? rows[q] : q; the sum runs in q order.
// Returns this thread's sum of the new out[k]^2.
__device__ __forceinline__ double slab_rows_dot(const double* __restrict__ A, int64_t ld,
                                                int64_t k0, int64_t k1, const int32_t* rows,
                                                const double* coef, int mq,
                                                const double* __restrict__ base, double beta,
                                                double* __restrict__ out, int aligned) {
  const gptr<const double> Ag = glb(A);
  const gptr<const double> bg = glb(base);
  const gptr<double> og = glb(out);
  double ss = 0.0;
  for (int64_t k = k0 + 2 * (int64_t)threadIdx.x; k < k1; k += 2 * kBT) {
    const bool two = k + 1 < k1;
    double a0, a1 = 0.0;
    if (base != nullptr) {
      a0 = beta * bg[k];
      if (two) a1 = beta * bg[k + 1];
    } else {
      a0 = og[k];
      if (two) a1 = og[k + 1];
    }
    int q = 0;
    for (; q + 8 <= mq; q += 8) {
      double2 v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t row = rows != nullptr ? rows[q + j] : q + j;
        v[j] = gdev::load2(Ag + row * ld, k, k1, aligned != 0);
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const double c = coef[q + j];
        a0 = fma(v[j].x, c, a0);
        a1 = fma(v[j].y, c, a1);
      }
    }
    for (; q < mq; ++q) {
      const int64_t row = rows != nullptr ? rows[q] : q;
      const double2 v = gdev::load2(Ag + row * ld, k, k1, aligned != 0);
      a0 = fma(v.x, coef[q], a0);
      a1 = fma(v.y, coef[q], a1);
    }
    og[k] = a0;
    if (two) og[k + 1] = a1;
    ss += a0 * a0 + a1 * a1;
  }
  return ss;
}

// The same pass over stored BF16 / FP8 codes: rows decoded exactly to FP64 and
// multiplied by coef[q] * rs[row(q)] (rs NULL: 1).  k0 is a multiple of the
// 16-byte chunk.
template <int FMT>
__device__ __forceinline__ double slab_rows_dot_lp(const uint8_t* __restrict__ A, int64_t ld,
                                                   int64_t k0, int64_t k1, const int32_t* rows,
                                                   const double* coef, const float* rs, int mq,
                                                   const double* __restrict__ base, double beta,
                                                   double* __restrict__ out, int aligned) {
  constexpr int ES = FMT == CABCD_BF16 ? 2 : 1;
  constexpr int EPC = 16 / ES;
  const gptr<const uint8_t> Ag = glb(A);
  const gptr<const double> bg = glb(base);
  const gptr<double> og = glb(out);
  const gptr<const float> rg = glb(rs);
  double ss = 0.0;
  for (int64_t k = k0 + EPC * (int64_t)threadIdx.x; k < k1; k += (int64_t)EPC * kBT) {
    double acc[EPC];
#pragma unroll
    for (int e = 0; e < EPC; ++e)
      acc[e] = k + e < k1 ? (base != nullptr ? beta * bg[k + e] : og[k + e]) : 0.0;
    int q = 0;
    for (; q + 4 <= mq; q += 4) {
      uint4 x[4];
      double c[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t row = rows != nullptr ? rows[q + j] : q + j;
        c[j] = coef[q + j] * (rs != nullptr ? (double)rg[row] : 1.0);
        x[j] = ldev::lp_load<FMT>(Ag + row * ld * ES, k, k1, aligned != 0);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        double dv[EPC];
        ldev::lp_decode_all<FMT>(x[j], dv);
#pragma unroll
        for (int e = 0; e < EPC; ++e) acc[e] = fma(dv[e], c[j], acc[e]);
      }
    }
    for (; q < mq; ++q) {
      const int64_t row = rows != nullptr ? rows[q] : q;
      const double c = coef[q] * (rs != nullptr ? (double)rg[row] : 1.0);
      double dv[EPC];
      ldev::lp_decode_all<FMT>(ldev::lp_load<FMT>(Ag + row * ld * ES, k, k1, aligned != 0), dv);
#pragma unroll
      for (int e = 0; e < EPC; ++e) acc[e] = fma(dv[e], c, acc[e]);
    }
#pragma unroll
    for (int e = 0; e < EPC; ++e) {
      if (k + e < k1) {
        og[k + e] = acc[e];
        ss += acc[e] * acc[e];
      }
    }
  }
  return ss;
}

// Either pass, by storage format.
template <int FMT>
__device__ __forceinline__ double rows_dot(const BProb& pr, int64_t k0, int64_t k1,
                                           const int32_t* rows, const double* coef, int mq,
                                           const double* base, double beta) {
  if constexpr (FMT == CABCD_F64)
    return slab_rows_dot(static_cast<const double*>(pr.A), pr.ld, k0, k1, rows, coef, mq, base,
                         beta, pr.r, pr.aligned);
  else
    return slab_rows_dot_lp<FMT>(static_cast<const uint8_t*>(pr.A), pr.ld, k0, k1, rows, coef,
                                 pr.rs, mq, base, beta, pr.r, pr.aligned);
}

// Workgroup sum in a fixed order (valid in thread 0).
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kBT / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}

// Wave-uniform copies of values that steer control flow around barriers.  The
// values are equal in every thread already, but the compiler cannot prove it
// for data read from memory; a loop whose exit it considers divergent gets
// restructured so that the threads of a wave leave it in different
// iterations, which breaks the workgroup barriers inside the loop.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
  const uint64_t u = (uint64_t)v;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <class T>
__device__ __forceinline__ T* uni_ptr(T* p) {
  return reinterpret_cast<T*>((uintptr_t)uni64((int64_t)(uintptr_t)p));
}

// The Gram slabs and solves are separate (non-inlined) functions so that each
// gets its own register allocation instead of one allocation over every
// variant of the persistent loop.  They take the workgroup's dynamic LDS from
// their own extern declaration, so their LDS accesses stay ds_* instructions.
// Rows fed to LDS by DMA, one owned row per lane (16-byte aligned A, even ld).
__device__ __noinline__ void gram_call_dma16(const double* A, int64_t ld, int64_t k0,
                                             int64_t k1, const int32_t* idx, int m,
                                             const double* u, double* part) {
  extern __shared__ __attribute__((aligned(16))) double dyn_sm[];
  gdev::gram_slab_dma16(uni_ptr(A), uni64(ld), uni64(k0), uni64(k1), uni_ptr(idx), uni(m),
                        uni_ptr(u), uni_ptr(part), dyn_sm);
}

// NB <= 8 fed by LDS-DMA (16-byte aligned A, even ld).
template <int NB>
__device__ __noinline__ void gram_call_dma(const double* A, int64_t ld, int64_t k0, int64_t k1,
                                           const int32_t* idx, int m, const double* u,
                                           double* part) {
  extern __shared__ __attribute__((aligned(16))) double dyn_sm[];
  gdev::gram_slab_dma<NB>(uni_ptr(A), uni64(ld), uni64(k0), uni64(k1), uni_ptr(idx), uni(m),
                          uni_ptr(u), uni_ptr(part), dyn_sm);
}

template <int NB>
__device__ __noinline__ void gram_call(const double* A, int64_t ld, int64_t k0, int64_t k1,
                                       const int32_t* idx, int m, const double* u, double* part,
                                       int aligned) {
  extern __shared__ __attribute__((aligned(16))) double dyn_sm[];
  // Arguments of a non-inlined function are per-lane values to the compiler;
  // the tile loop's barriers need its bounds to be visibly uniform.
  gdev::gram_slab<NB, 2>(uni_ptr(A), uni64(ld), uni64(k0), uni64(k1), uni_ptr(idx), uni(m),
                         uni_ptr(u), uni_ptr(part), uni(aligned), dyn_sm);
}

template <int NB, int FMT>
__device__ __noinline__ void gram_lp_call(const uint8_t* A, int64_t ld, int64_t k0, int64_t k1,
                                          const int32_t* idx, int m, const double* u,
                                          double* part, int aligned) {
  extern __shared__ __attribute__((aligned(16))) double dyn_sm[];
  ldev::gram_lp_slab<NB, FMT, kBLpTile>(uni_ptr(A), uni64(ld), uni64(k0), uni64(k1), uni_ptr(idx),
                                        uni(m), uni_ptr(u), uni_ptr(part), uni(aligned),
                                        reinterpret_cast<uint8_t*>(dyn_sm));
}

template <int FMT>
__device__ __forceinline__ void gram_any(int nb, const void* A, int64_t ld, int64_t k0,
                                         int64_t k1, const int32_t* idx, int m, const double* u,
                                         double* part, int aligned) {
  if constexpr (FMT == CABCD_F64) {
    const double* a = static_cast<const double*>(A);
    const bool dma = uni(aligned) != 0;
    switch (nb) {
      case 1:
        if (dma) gram_call_dma<1>(a, ld, k0, k1, idx, m, u, part);
        else gram_call<1>(a, ld, k0, k1, idx, m, u, part, aligned);
        break;
      case 2:
        if (dma) gram_call_dma<2>(a, ld, k0, k1, idx, m, u, part);
        else gram_call<2>(a, ld, k0, k1, idx, m, u, part, aligned);
        break;
      case 4:
        if (dma) gram_call_dma<4>(a, ld, k0, k1, idx, m, u, part);
        else gram_call<4>(a, ld, k0, k1, idx, m, u, part, aligned);
        break;
      case 8:
        if (dma) gram_call_dma<8>(a, ld, k0, k1, idx, m, u, part);
        else gram_call<8>(a, ld, k0, k1, idx, m, u, part, aligned);
        break;
      default:
        if (uni(aligned)) gram_call_dma16(a, ld, k0, k1, idx, m, u, part);
        else gram_call<16>(a, ld, k0, k1, idx, m, u, part, aligned);
        break;
    }
  } else {
    const uint8_t* a = static_cast<const uint8_t*>(A);
    switch (nb) {
      case 1: gram_lp_call<1, FMT>(a, ld, k0, k1, idx, m, u, part, aligned); break;
      case 2: gram_lp_call<2, FMT>(a, ld, k0, k1, idx, m, u, part, aligned); break;
      case 4: gram_lp_call<4, FMT>(a, ld, k0, k1, idx, m, u, part, aligned); break;
      case 8: gram_lp_call<8, FMT>(a, ld, k0, k1, idx, m, u, part, aligned); break;
      default: gram_lp_call<16, FMT>(a, ld, k0, k1, idx, m, u, part, aligned); break;
    }
  }
}

template <int BP, int PF>
__device__ __noinline__ void solve_call(const SolveArgs& in) {
  extern __shared__ __attribute__((aligned(16))) double dyn_sm[];
  SolveArgs a;
  a.G = uni_ptr(in.G);
  a.Yu = uni_ptr(in.Yu);
  a.idx = uni_ptr(in.idx);
  a.y = uni_ptr(in.y);
  a.x = uni_ptr(in.x);
  a.delta = uni_ptr(in.delta);
  a.status = uni_ptr(in.status);
  a.m = uni(in.m);
  a.b = uni(in.b);
  a.s = uni(in.s);
  a.mode = uni(in.mode);
  a.lambda = __builtin_bit_cast(double, uni64(__builtin_bit_cast(int64_t, in.lambda)));
  a.n = __builtin_bit_cast(double, uni64(__builtin_bit_cast(int64_t, in.n)));
  a.pre_inverted = 0;
  sdev::solve_block<BP, PF, kBT, 1>(a, dyn_sm);   // s BP <= 2 s b <= 512 lanes
}

__device__ __forceinline__ void solve_any(int bp, const SolveArgs& a) {
  switch (bp) {
    case 1: solve_call<1, 8>(a); break;
    case 2: solve_call<2, 8>(a); break;
    case 4: solve_call<4, 8>(a); break;
    case 8: solve_call<8, 8>(a); break;
    default: solve_call<16, 4>(a); break;
  }
}

// Next work item of the launch's queue (the same value in every thread).  The
// persistent loops are written as
//   it = next_item(); while (it < nitems) { do { ... } while (false); it = next_item(); }
// with every early exit a `break` out of the do-block, so that all threads run
// the same barriers in the same order and the only loop exit is uniform.
__device__ __forceinline__ int next_item(BQueue* Q, int* slot) {
  __syncthreads();   // every thread is done with the previous item and the slot
  if (threadIdx.x == 0) *slot = atomicAdd(&Q->ticket, 1);
  __syncthreads();
  return uni(*slot);
}

// Publish this workgroup's global writes and count its arrival at problem st;
// true (in every thread) for the workgroup that completes the set of nslab.
__device__ __forceinline__ bool arrive_last(BState* st, int nslab, int* slot) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) *slot = atomicAdd(&st->arrive, 1) == nslab - 1 ? 1 : 0;
  __syncthreads();
  const bool last = uni(*slot) != 0;
  if (last) __threadfence();   // acquire the other workgroups' writes
  return last;
}

// The last workgroup to leave resets the queue for the next launch.
__device__ __forceinline__ void queue_exit(BQueue* Q) {
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&Q->exited, 1) == (int)gridDim.x - 1) {
      atomicExch(&Q->ticket, 0);
      atomicExch(&Q->exited, 0);
    }
  }
}

// ------------------------------------------------------------------- kernels

template <int FMT>
__global__ __launch_bounds__(kBT) void batch_step_kernel(const BProb* __restrict__ P,
                                                         BState* __restrict__ S,
                                                         const BItem* __restrict__ items,
                                                         int nitems, BQueue* Q, int area) {
  extern __shared__ __attribute__((aligned(16))) double sm[];
  int32_t* icur = reinterpret_cast<int32_t*>(sm + area);
  int32_t* iprev = icur + kBMaxRows;
  double* dprev = reinterpret_cast<double*>(iprev + kBMaxRows);
  int* ctl = reinterpret_cast<int*>(dprev + kBMaxRows);
  int32_t* ia = ctl + 4;           // index lists of a Gram above 256 rows
  int32_t* ib = ia + 512;
  const int tid = threadIdx.x;

  for (int it = next_item(Q, ctl); it < nitems; it = next_item(Q, ctl)) do {
    const BItem item = items[it];
    const BProb& pr = P[item.prob];
    BState* st = S + item.prob;
    if (uni(st->active) == 0) break;
    const int64_t h = uni64(st->h);
    const int64_t hp = uni64(st->h_prev);
    const int mp = uni(st->m_prev);
    const int sk = (int)std::min((int64_t)pr.s, pr.H - h);
    const int m = sk * pr.b;
    const int64_t k0 = (int64_t)item.slab * pr.chunk;
    const int64_t k1 = std::min(pr.n, k0 + pr.chunk);

    if (tid < sk) smp::sample_block(pr.seed, h + tid, pr.b, pr.d, icur + tid * pr.b);
    if (mp > 0) {
      if (tid < mp / pr.b) smp::sample_block(pr.seed, hp + tid, pr.b, pr.d, iprev + tid * pr.b);
      for (int q = tid; q < mp; q += kBT) dprev[q] = glb(pr.delta)[q];
    }
    __syncthreads();
    if (mp > 0) {
      // deferred companion update of the previous outer step, this slab's columns
      rows_dot<FMT>(pr, k0, k1, iprev, dprev, mp, nullptr, 0.0);
      __syncthreads();   // the Gram below reads these r values back
    }
    const int64_t pstride = (int64_t)(pr.nb * (pr.nb + 1) / 2) * 256 + 16 * pr.nb;
    const int sets = uni(pr.sets);
    // a problem above 256 rows: the Gram of every step assembled from 256-row
    // Grams (the two diagonal blocks, then 2 or 4 cross-block Grams)
    const int nsets = sets == 1 ? 1 : 2 + (m - 256 > 128 ? 4 : 2);
    if (sets == 1) {
      gram_any<FMT>(pr.nb, pr.A, pr.ld, k0, k1, icur, m, pr.r, pr.partials + item.slab * pstride,
                    pr.aligned);
    } else {
      gdev::big_lists(icur, m, ia, ib, tid, kBT);
      __syncthreads();
      double* part = pr.partials + (int64_t)item.slab * sets * pstride;
      for (int g = 0; g < nsets; ++g)
        gram_any<FMT>(16, pr.A, pr.ld, k0, k1, g < 2 ? ia + 256 * g : ib + 256 * (g - 2), 256,
                      g < 2 ? pr.r : nullptr, part + g * pstride, pr.aligned);
    }
    if (!arrive_last(st, pr.nslab, ctl + 1)) break;

    // Last slab of this problem: Gov (overlap-augmented, Alg. 2 scale 1/n and
    // shift lambda), then the fused solve and w[idx] += delta.
    if (sets == 1)
      gdev::reduce_wg<kBT>(pr.partials, pr.nslab, pr.nb, icur, m, 1.0 / (double)pr.n, pr.lambda,
                           pr.G, pr.Yu, FMT == CABCD_F64 ? 0 : 1, pr.rs);
    else
      gdev::reduce_wg_big<kBT>(pr.partials, pr.nslab, sets * pstride, nsets, icur, m,
                               1.0 / (double)pr.n, pr.lambda, pr.G, pr.Yu,
                               FMT == CABCD_F64 ? 0 : 1, pr.rs);
    __syncthreads();
    SolveArgs a;
    a.G = pr.G;
    a.Yu = pr.Yu;
    a.idx = icur;
    a.y = nullptr;
    a.x = pr.w;
    a.delta = pr.delta;
    a.status = &st->status;
    a.m = m;
    a.b = pr.b;
    a.s = sk;
    a.mode = 0;
    a.lambda = pr.lambda;
    a.n = (double)pr.n;
    a.pre_inverted = 0;
    solve_any(pr.bp, a);
    __syncthreads();
    if (tid == 0) {
      st->arrive = 0;
      st->h_prev = h;
      st->m_prev = m;
      st->h = h + sk;
      st->steps += 1;
      st->fresh = 0;
      if (h + sk >= pr.H) st->active = 0;
    }
  } while (false);
  queue_exit(Q);
}

// MODE 0 (exact): r = X^T w - y recomputed from X, f(w) = ||r||^2/(2n) +
//         lambda/2 ||w||^2, retire the problem when f(w) <= f_target;
// MODE 1 (flush): apply the pending companion update only;
// MODE 2 (monitor): apply the pending update and evaluate f(w) from the
//         maintained r (a pass over the pending rows and r only), retire as 0.
constexpr int kAuxExact = 0, kAuxFlush = 1, kAuxMonitor = 2;

template <int MODE, int FMT>
__global__ __launch_bounds__(kBT) void batch_aux_kernel(const BProb* __restrict__ P,
                                                        BState* __restrict__ S,
                                                        const BItem* __restrict__ items,
                                                        int nitems, BQueue* Q) {
  __shared__ int32_t iprev[kBMaxRows];
  __shared__ double dprev[kBMaxRows];
  __shared__ double red[kBT / 64];
  __shared__ int ctl[2];
  const int tid = threadIdx.x;

  for (int it = next_item(Q, ctl); it < nitems; it = next_item(Q, ctl)) do {
    const BItem item = items[it];
    const BProb& pr = P[item.prob];
    BState* st = S + item.prob;
    const int fresh = uni(st->fresh);
    const int mp = uni(st->m_prev);
    if (MODE == kAuxExact ? fresh == 2 : MODE == kAuxFlush ? mp == 0 : fresh != 0) break;
    const int64_t k0 = (int64_t)item.slab * pr.chunk;
    const int64_t k1 = std::min(pr.n, k0 + pr.chunk);
    double ss = 0.0;
    if (MODE == kAuxExact) {
      ss = rows_dot<FMT>(pr, k0, k1, nullptr, pr.w, (int)pr.d, pr.y, -1.0);
    } else if (mp > 0) {
      const int64_t hp = uni64(st->h_prev);
      if (tid < mp / pr.b) smp::sample_block(pr.seed, hp + tid, pr.b, pr.d, iprev + tid * pr.b);
      for (int q = tid; q < mp; q += kBT) dprev[q] = glb(pr.delta)[q];
      __syncthreads();
      ss = rows_dot<FMT>(pr, k0, k1, iprev, dprev, mp, nullptr, 0.0);
    } else {
      const gptr<const double> rg = glb(pr.r);
      for (int64_t k = k0 + tid; k < k1; k += kBT) ss = fma(rg[k], rg[k], ss);
    }
    if (MODE != kAuxFlush) {
      ss = block_sum(ss, red);
      if (tid == 0) glb(pr.objp)[item.slab] = ss;
    }
    if (!arrive_last(st, pr.nslab, ctl + 1)) break;
    if (MODE != kAuxFlush) {
      double ww = 0.0;
      const gptr<const double> wg = glb(pr.w);
      for (int64_t i = tid; i < pr.d; i += kBT) ww = fma(wg[i], wg[i], ww);
      ww = block_sum(ww, red);
      if (tid == 0) {
        double rr = 0.0;
        for (int q = 0; q < pr.nslab; ++q) rr += glb(pr.objp)[q];
        const double f = rr / (2.0 * (double)pr.n) + 0.5 * pr.lambda * ww;
        st->obj = f;
        if (!isfinite(f)) raise_status(&st->status, DEV_NONFINITE);
        st->fresh = MODE == kAuxExact ? 2 : 1;
        st->m_prev = 0;
        if ((pr.f_target > 0.0 && f <= pr.f_target) || !isfinite(f)) st->active = 0;
        st->arrive = 0;
      }
    } else if (tid == 0) {
      st->m_prev = 0;
      st->arrive = 0;
    }
  } while (false);
  queue_exit(Q);
}

// ------------------------------------------------------------------ planning

int pow2_at_least(int b) {
  int p = 1;
  while (p < b) p *= 2;
  return p;
}

int nb_of(int sb) {
  int nb = 1;
  while (16 * nb < sb && nb < 16) nb *= 2;
  return nb;
}

// Partial sets of one slab: one Gram, or above 256 rows the 2 diagonal and
// 2 or 4 cross-block 256-row Grams.
int sets_of(int sb) { return sb <= 256 ? 1 : 2 + (sb - 256 > 128 ? 4 : 2); }

int64_t pstride_of(int nb) { return (int64_t)(nb * (nb + 1) / 2) * 256 + 16 * nb; }
int64_t slab_doubles(int sb) { return sets_of(sb) * pstride_of(nb_of(sb)); }

// Cost model of one round (seconds), with rates measured on MI355X with the
// one-problem kernels: the FP64 Gram at sb = 256 ran at 48 TFLOP/s over 256
// CUs, the streaming passes at about 5 TB/s, one workgroup reads its partials
// at about 60 GB/s, and the fused solve costs about 1.5 us per block.
constexpr double kCuF64 = 48e12 / 256;
constexpr double kCuLp = 500e12 / 256;   // FP32-accumulating BF16/FP8 Gram, well below peak
constexpr double kCuBw = 5.0e12 / 256;
constexpr double kWgBw = 60e9;
constexpr double kSolveBlock = 1.5e-6;
constexpr double kRoundFixed = 10e-6;
constexpr int kGraphMaxRounds = 64;   // rounds of one captured monitor period, at most
constexpr int kReplanRounds = 32;     // rounds between checks for re-slicing, about

int elem_bytes(int dtype) { return dtype == CABCD_F64 ? 8 : dtype == CABCD_BF16 ? 2 : 1; }

// Columns per LDS tile of the Gram slab (slab widths are multiples of it).
int tile_cols(int nb, int dtype) {
  return dtype == CABCD_F64 ? 256 / nb : (kBLpTile / nb) / elem_bytes(dtype);
}

// CU-seconds of one problem's slabs in one round (Gram of the padded rows and
// the two passes over the gathered rows: Gram and deferred update).
double slab_work(int sb, int64_t cols, int dtype) {
  const int sbp = 16 * nb_of(sb);
  const double flops = (double)cols * sbp * (sbp + 1) * sets_of(sb);
  const double bytes = 2.0 * elem_bytes(dtype) * (double)cols * sb;
  return std::max(flops / (dtype == CABCD_F64 ? kCuF64 : kCuLp), bytes / kCuBw);
}

// The tuner's block sizes are b in {4, 8, 16} (smaller only when d is) and its
// unrollings s in [4, 32]: s < 4 would be (nearly) classical BCD, which the
// s-step form exists to replace.
constexpr int kTuneMinS = 4;

int auto_b(int64_t d) {
  if (d >= 64) return 16;
  if (d >= 16) return 8;
  if (d >= 4) return 4;
  return (int)std::max<int64_t>(1, d);
}

struct Pick {
  int b, s, nslab;
  int64_t chunk;
  double crit;
};

// Slabs of a problem with `wp` CU-seconds of slab work per round for a target
// of `target` per slab: at most kBMaxSlabs, at least one tile each, widths a
// multiple of the tile.
void slice(double wp, double target, int64_t n, int kt, int64_t& chunk_out, int& nslab_out) {
  int64_t nslab = (int64_t)std::ceil(wp / target);
  nslab = std::max<int64_t>(1, std::min<int64_t>(nslab, kBMaxSlabs));
  nslab = std::min<int64_t>(nslab, (n + kt - 1) / kt);
  int64_t chunk = (n + nslab - 1) / nslab;
  chunk = (chunk + kt - 1) / kt * kt;
  chunk_out = chunk;
  nslab_out = (int)((n + chunk - 1) / chunk);
}

// Slab items per CU a round aims at: FP64 slabs carry matrix-core work and
// balance best at four; low-precision slabs are pure streams, and fewer,
// longer items cut their per-item overhead (BF16 batched to 1e-6: 0.153 s at
// four, 0.141 s at two; FP64 0.334 s at four, 0.339 s at two, 0.374 s at
// eight).
double items_per_cu(int dtype) { return dtype == CABCD_F64 ? 4.0 : 2.0; }

// (b, s) of every problem for a target of `rp` rounds per pass over the
// coordinates, slabs sized so a round has about items_per_cu items per CU, and
// the predicted time of one pass (rounds per pass x round time).
double plan_candidate(const std::vector<cabcd_problem>& pb, double rp, int cus,
                      std::vector<Pick>& out) {
  const size_t P = pb.size();
  out.assign(P, Pick{});
  double W = 0.0;
  for (size_t p = 0; p < P; ++p) {
    const int64_t d = pb[p].X.rows;
    int b = pb[p].b, s = pb[p].s;
    if (b == 0) b = s == 0 ? auto_b(d) : std::min(auto_b(d), kBMaxRows / s);
    b = (int)std::min<int64_t>(b, d);
    if (s == 0) {
      const int smax = std::min(32, kBMaxRows / b);
      s = (int)std::ceil((double)d / (b * rp));
      s = std::max(std::min(kTuneMinS, smax), std::min(s, smax));
    }
    out[p].b = b;
    out[p].s = s;
    W += slab_work(b * s, pb[p].X.cols, pb[p].X.dtype);
  }
  const double target = std::max(W / (items_per_cu(pb[0].X.dtype) * cus), 20e-6);
  double crit = 0.0, passes = 0.0;
  for (size_t p = 0; p < P; ++p) {
    const int sb = out[p].b * out[p].s;
    const int nb = nb_of(sb);
    const int64_t n = pb[p].X.cols;
    const double wp = slab_work(sb, n, pb[p].X.dtype);
    slice(wp, target, n, tile_cols(nb, pb[p].X.dtype), out[p].chunk, out[p].nslab);
    const int64_t nslab = out[p].nslab;
    out[p].crit = wp / nslab + nslab * slab_doubles(sb) * 8.0 / kWgBw + out[p].s * kSolveBlock;
    crit = std::max(crit, out[p].crit);
    passes = std::max(passes, (double)pb[p].X.rows / sb);
  }
  const double T = std::max(W / cus, crit) + kRoundFixed;
  return passes * T;
}

struct Workspace {
  char* base = nullptr;
  size_t off = 0;
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~(size_t)255;
    T* p = reinterpret_cast<T*>(base + off);
    off += n * sizeof(T);
    return p;
  }
};

}  // namespace
}  // namespace cabcd

// ---------------------------------------------------------------- the plan

struct cabcd_batch_plan {
  int device = 0;
  int P = 0;
  std::vector<cabcd::BProb> probs;
  cabcd::BProb* dP = nullptr;
  cabcd::BState* dS = nullptr;
  cabcd::BItem* dI = nullptr;
  cabcd::BQueue* dQ = nullptr;
  void* mem = nullptr;
  int nitems = 0;
  int area = 0;            // doubles of the step kernel's shared Gram/solve area
  size_t step_lds = 0;
  int grid_step = 1, grid_aux = 1;
  int monitor_every = 4;
  int cheap_monitors = 0;  // maintained-residual monitor points between exact ones
  uint32_t flags = 0;
  int64_t rounds_done = 0;
  int64_t monitors_done = 0;
  bool pending = false;    // a step ran since the last recompute / flush
  hipStream_t cap = nullptr;
  hipGraph_t graph[2] = {nullptr, nullptr};      // [0]: ends in a cheap monitor, [1]: exact
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  int graph_rounds = 0;
  int dtype = CABCD_F64;   // storage type shared by every problem of the plan
  // re-slicing of the slabs as problems retire
  int cus = 1, occ_step = 1, occ_aux = 1;
  int items_cap = 0;       // capacity of dI
  double* pool = nullptr;  // partials and objective partials of re-sliced plans
  size_t pool_doubles = 0;
  int plan_active = 0;     // active problems when the slabs were last sliced
  int64_t replan_period = 0;
};

namespace cabcd {
namespace {

template <int FMT>
hipError_t launch_step_t(cabcd_batch_plan* B, hipStream_t st) {
  hipLaunchKernelGGL(batch_step_kernel<FMT>, dim3(B->grid_step), dim3(kBT), B->step_lds, st,
                     B->dP, B->dS, B->dI, B->nitems, B->dQ, B->area);
  return hipGetLastError();
}

template <int MODE, int FMT>
hipError_t launch_aux_t(cabcd_batch_plan* B, hipStream_t st) {
  hipLaunchKernelGGL((batch_aux_kernel<MODE, FMT>), dim3(B->grid_aux), dim3(kBT), 0, st, B->dP,
                     B->dS, B->dI, B->nitems, B->dQ);
  return hipGetLastError();
}

hipError_t launch_step(cabcd_batch_plan* B, hipStream_t st) {
  switch (B->dtype) {
    case CABCD_F64: return launch_step_t<CABCD_F64>(B, st);
    case CABCD_BF16: return launch_step_t<CABCD_BF16>(B, st);
    default: return launch_step_t<CABCD_FP8_E4M3>(B, st);
  }
}

template <int FMT>
hipError_t launch_aux_f(cabcd_batch_plan* B, int mode, hipStream_t st) {
  switch (mode) {
    case kAuxExact: return launch_aux_t<kAuxExact, FMT>(B, st);
    case kAuxFlush: return launch_aux_t<kAuxFlush, FMT>(B, st);
    default: return launch_aux_t<kAuxMonitor, FMT>(B, st);
  }
}

hipError_t launch_aux(cabcd_batch_plan* B, int mode, hipStream_t st) {
  switch (B->dtype) {
    case CABCD_F64: return launch_aux_f<CABCD_F64>(B, mode, st);
    case CABCD_BF16: return launch_aux_f<CABCD_BF16>(B, mode, st);
    default: return launch_aux_f<CABCD_FP8_E4M3>(B, mode, st);
  }
}

const void* step_kernel_ptr(int dtype) {
  switch (dtype) {
    case CABCD_F64: return reinterpret_cast<const void*>(batch_step_kernel<CABCD_F64>);
    case CABCD_BF16: return reinterpret_cast<const void*>(batch_step_kernel<CABCD_BF16>);
    default: return reinterpret_cast<const void*>(batch_step_kernel<CABCD_FP8_E4M3>);
  }
}

#define BATCH_HIP(call)                                                     \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) {                                                 \
      set_error("%s failed: %s", #call, hipGetErrorString(e_));             \
      return CABCD_EHIP;                                                    \
    }                                                                       \
  } while (0)

cabcd_status check_problem(const cabcd_problem& q, int p) {
  const cabcd_matrix& X = q.X;
  if (X.kind != CABCD_DENSE) {
    set_error("problem %d: the batched path takes dense X (FP64, BF16 or FP8-E4M3)", p);
    return CABCD_EUNSUPPORTED;
  }
  if (X.dtype != CABCD_F64 && X.dtype != CABCD_BF16 && X.dtype != CABCD_FP8_E4M3) {
    set_error("problem %d: unknown dtype %d", p, X.dtype);
    return CABCD_EINVAL;
  }
  if (X.dtype == CABCD_FP8_E4M3 && X.row_scale == nullptr) {
    set_error("problem %d: FP8 storage needs its row scales", p);
    return CABCD_EINVAL;
  }
  if (X.data == nullptr || q.y == nullptr || q.w == nullptr || q.r == nullptr) {
    set_error("problem %d: X, y, w and r must be non-NULL device pointers", p);
    return CABCD_EINVAL;
  }
  const auto mis = [](const void* ptr) { return (reinterpret_cast<uintptr_t>(ptr) & 7) != 0; };
  if (mis(q.y) || mis(q.w) || mis(q.r) ||
      (reinterpret_cast<uintptr_t>(X.data) % elem_bytes(X.dtype)) != 0 ||
      (reinterpret_cast<uintptr_t>(X.row_scale) & 3) != 0) {
    set_error("problem %d: X, y, w, r and row_scale must be aligned to their element size", p);
    return CABCD_EINVAL;
  }
  if (X.rows < 1 || X.cols < 1 || X.rows > INT_MAX || X.cols > INT_MAX || X.ld < X.cols) {
    set_error("problem %d: need 1 <= d, n < 2^31 and ld >= n (d=%lld n=%lld ld=%lld)", p,
              (long long)X.rows, (long long)X.cols, (long long)X.ld);
    return CABCD_EINVAL;
  }
  if (!(q.lambda > 0.0) || !std::isfinite(q.lambda)) {
    set_error("problem %d: lambda must be finite and > 0", p);
    return CABCD_EINVAL;
  }
  if (q.b < 0 || q.b > kBMaxB || q.b > X.rows) {
    set_error("problem %d: b must be 0 (auto) or in [1, min(d, %d)] (b=%d)", p, kBMaxB, q.b);
    return CABCD_EINVAL;
  }
  if (q.s < 0 || q.s > kBMaxRows || (q.b > 0 && q.s > 0 && q.b * q.s > kBMaxRows)) {
    set_error("problem %d: s must be 0 (auto) or >= 1 with s*b <= %d (b=%d s=%d)", p,
              kBMaxRows, q.b, q.s);
    return CABCD_EINVAL;
  }
  if (q.b > 0 && q.s > 0 && q.s * pow2_at_least(q.b) > kBT) {
    set_error("problem %d: s times b rounded up to a power of two must be <= %d (b=%d s=%d)", p,
              kBT, q.b, q.s);
    return CABCD_EUNSUPPORTED;
  }
  return CABCD_OK;
}

cabcd_status sync_status(cabcd_batch_plan* B, hipStream_t st, int32_t* active) {
  std::vector<BState> S(B->P);
  BATCH_HIP(hipMemcpyAsync(S.data(), B->dS, sizeof(BState) * B->P, hipMemcpyDeviceToHost, st));
  BATCH_HIP(hipStreamSynchronize(st));
  int act = 0;
  for (int p = 0; p < B->P; ++p) {
    act += S[p].active != 0;
    if (S[p].status == DEV_NOTSPD) {
      set_error("problem %d: a diagonal block was not positive definite", p);
      return CABCD_ENOTSPD;
    }
    if (S[p].status == DEV_NONFINITE) {
      set_error("problem %d: non-finite values", p);
      return CABCD_ENONFINITE;
    }
  }
  if (active != nullptr) *active = act;
  return CABCD_OK;
}

void release(cabcd_batch_plan* B) {
  if (B == nullptr) return;
  (void)hipSetDevice(B->device);
  (void)hipDeviceSynchronize();
  for (int g = 0; g < 2; ++g) {
    if (B->exec[g] != nullptr) (void)hipGraphExecDestroy(B->exec[g]);
    if (B->graph[g] != nullptr) (void)hipGraphDestroy(B->graph[g]);
  }
  if (B->cap != nullptr) (void)hipStreamDestroy(B->cap);
  if (B->mem != nullptr) (void)hipFree(B->mem);
  delete B;
}

cabcd_status capture(cabcd_batch_plan* B);

cabcd_status create(const cabcd_problem* pb, int32_t P, const cabcd_batch_opts* opts,
                    hipStream_t st, cabcd_batch_plan* B) {
  BATCH_HIP(hipGetDevice(&B->device));
  int cus = 0;
  BATCH_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, B->device));
  cus = std::max(cus, 1);
  B->P = P;
  B->dtype = pb[0].X.dtype;
  B->monitor_every = opts != nullptr ? opts->monitor_every : 4;
  B->cheap_monitors = opts != nullptr ? opts->cheap_monitors : 0;
  B->flags = opts != nullptr ? opts->flags : 0u;

  // Autotune: the rounds-per-pass target with the cheapest predicted pass.
  std::vector<cabcd_problem> probs(pb, pb + P);
  std::vector<Pick> best, cand;
  double best_cost = 1e300;
  for (double rp : {1.0, 1.5, 2.0, 3.0, 4.0, 6.0, 8.0, 12.0, 16.0, 24.0, 32.0, 48.0, 64.0}) {
    const double c = plan_candidate(probs, rp, cus, cand);
    if (c < best_cost) {
      best_cost = c;
      best = cand;
    }
  }

  // Work items: problems with the longest critical path first, slabs of one
  // problem next to each other so they run concurrently.
  std::vector<int> order(P);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return best[a].crit > best[b].crit; });
  std::vector<BItem> items;
  for (int p : order)
    for (int q = 0; q < best[p].nslab; ++q) items.push_back(BItem{p, q});
  B->nitems = (int)items.size();
  B->cus = cus;
  B->items_cap = std::max(B->nitems, 4 * cus + 2 * P);

  // Workspace and device copies.  The pool holds the partials of re-sliced
  // plans: as much as the first plan's, plus the largest slab set of one
  // problem.
  size_t bytes = 0;
  auto add = [&](size_t n) { bytes = ((bytes + 255) & ~(size_t)255) + n; };
  add(sizeof(BProb) * P);
  add(sizeof(BState) * P);
  add(sizeof(BItem) * B->items_cap);
  add(sizeof(BQueue));
  int area = 0;
  size_t pool = 0;
  for (int p = 0; p < P; ++p) {
    const int sb = best[p].b * best[p].s;
    const int nb = nb_of(sb);
    add(sizeof(double) * best[p].nslab * slab_doubles(sb));
    add(sizeof(double) * sb * sb);
    add(sizeof(double) * sb);
    add(sizeof(double) * sb);
    add(sizeof(double) * best[p].nslab);
    area = std::max<int>(area, (int)((solve_lds_bytes(sb, best[p].b) + 7) / 8));
    pool += (size_t)best[p].nslab * (slab_doubles(sb) + 1) + 64;
  }
  pool += (size_t)kBMaxSlabs * (slab_doubles(kBMaxRows) + 1) + 64;
  B->pool_doubles = pool;
  add(sizeof(double) * pool);
  if (B->dtype == CABCD_F64) {
    area = std::max<int>(area, gdev::Cfg<16, 2>::LDS);
    area = std::max<int>(area, gdev::Cfg<1, 2>::LDS);
    area = std::max<int>(area, gdev::D16::LDS);
    area = std::max<int>(area, std::max(gdev::DN<1>::LDS, gdev::DN<2>::LDS));
    area = std::max<int>(area, std::max(gdev::DN<4>::LDS, gdev::DN<8>::LDS));
  } else {
    const int lp = B->dtype == CABCD_BF16
                       ? std::max(ldev::LpCfg<16, CABCD_BF16, kBLpTile>::LDS,
                                  ldev::LpCfg<1, CABCD_BF16, kBLpTile>::LDS)
                       : std::max(ldev::LpCfg<16, CABCD_FP8_E4M3, kBLpTile>::LDS,
                                  ldev::LpCfg<1, CABCD_FP8_E4M3, kBLpTile>::LDS);
    area = std::max<int>(area, (lp + 7) / 8);
  }
  B->area = (area + 1) & ~1;
  B->step_lds = sizeof(double) * B->area + kBMaxRows * 2 * sizeof(int32_t) +
                kBMaxRows * sizeof(double) + 4 * sizeof(int) + (512 + 1024) * sizeof(int32_t);
  if (hipMalloc(&B->mem, bytes + 256) != hipSuccess) {
    B->mem = nullptr;
    set_error("hipMalloc of %zu bytes for the batch plan failed", bytes);
    return CABCD_ENOMEM;
  }
  Workspace ws{static_cast<char*>(B->mem)};
  B->dP = ws.take<BProb>(P);
  B->dS = ws.take<BState>(P);
  B->dI = ws.take<BItem>(B->items_cap);
  B->dQ = ws.take<BQueue>(1);
  B->pool = ws.take<double>(B->pool_doubles);
  B->probs.resize(P);
  std::vector<BState> S(P);
  for (int p = 0; p < P; ++p) {
    const cabcd_problem& q = pb[p];
    BProb& o = B->probs[p];
    const int sb = best[p].b * best[p].s;
    o.A = q.X.data;
    o.rs = q.X.dtype == CABCD_F64 ? nullptr : q.X.row_scale;
    o.ld = q.X.ld;
    o.d = q.X.rows;
    o.n = q.X.cols;
    o.y = q.y;
    o.w = q.w;
    o.r = q.r;
    o.lambda = q.lambda;
    o.f_target = q.f_target;
    o.seed = q.seed;
    o.H = q.H > 0 ? q.H : INT64_MAX;
    o.chunk = best[p].chunk;
    o.b = best[p].b;
    o.s = best[p].s;
    o.bp = pow2_at_least(o.b);
    o.nb = nb_of(sb);
    o.sets = sets_of(sb);
    o.pad = 0;
    o.nslab = best[p].nslab;
    o.aligned = ((reinterpret_cast<uintptr_t>(o.A) & 15) == 0 &&
                 ((o.ld * elem_bytes(B->dtype)) & 15) == 0)
                    ? 1
                    : 0;
    o.partials = ws.take<double>((size_t)o.nslab * slab_doubles(sb));
    o.G = ws.take<double>((size_t)sb * sb);
    o.Yu = ws.take<double>(sb);
    o.delta = ws.take<double>(sb);
    o.objp = ws.take<double>(o.nslab);
    BState& s = S[p];
    std::memset(&s, 0, sizeof s);
    s.obj = NAN;
    s.active = 1;
  }
  BATCH_HIP(hipMemcpyAsync(B->dP, B->probs.data(), sizeof(BProb) * P, hipMemcpyHostToDevice, st));
  BATCH_HIP(hipMemcpyAsync(B->dS, S.data(), sizeof(BState) * P, hipMemcpyHostToDevice, st));
  BATCH_HIP(hipMemcpyAsync(B->dI, items.data(), sizeof(BItem) * items.size(),
                           hipMemcpyHostToDevice, st));
  BQueue q0{0, 0};
  BATCH_HIP(hipMemcpyAsync(B->dQ, &q0, sizeof q0, hipMemcpyHostToDevice, st));

  // Persistent grids: as many workgroups as fit on the device at once.
  BATCH_HIP(hipFuncSetAttribute(step_kernel_ptr(B->dtype),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)B->step_lds));
  int occ = 0;
  BATCH_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, step_kernel_ptr(B->dtype), kBT,
                                                         B->step_lds));
  B->occ_step = std::max(occ, 1);
  B->grid_step = std::max(1, std::min(B->nitems, B->occ_step * cus));
  BATCH_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &occ, reinterpret_cast<const void*>(batch_aux_kernel<0, CABCD_F64>), kBT, 0));
  B->occ_aux = std::max(occ, 1);
  B->grid_aux = std::max(1, std::min(B->nitems, B->occ_aux * cus));
  B->plan_active = P;

  // r_0 = X^T w_0 - y and f(w_0).
  BATCH_HIP(launch_aux(B, kAuxExact, st));
  cabcd_status rc = sync_status(B, st, nullptr);
  if (rc != CABCD_OK) return rc;

  {
    const int R = B->monitor_every > 0 ? B->monitor_every : 1;
    B->replan_period = (int64_t)R * ((kReplanRounds + R - 1) / R);
  }
  return capture(B);
}

// Capture one monitor period (or one round without monitoring): one graph
// ending in a maintained-residual monitor, one ending in an exact one.  A
// period longer than kGraphMaxRounds rounds runs as direct launches (the graph
// would hold one node per round).  Replaces the graphs of an earlier plan.
cabcd_status capture(cabcd_batch_plan* B) {
  for (int g = 0; g < 2; ++g) {
    if (B->exec[g] != nullptr) BATCH_HIP(hipGraphExecDestroy(B->exec[g]));
    if (B->graph[g] != nullptr) BATCH_HIP(hipGraphDestroy(B->graph[g]));
    B->exec[g] = nullptr;
    B->graph[g] = nullptr;
  }
  B->graph_rounds = 0;
  if ((B->flags & CABCD_BATCH_NO_GRAPH) == 0 && B->monitor_every <= kGraphMaxRounds) {
    if (B->cap == nullptr) BATCH_HIP(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
    const int R = B->monitor_every > 0 ? B->monitor_every : 1;
    for (int g = 0; g < (B->monitor_every > 0 ? 2 : 1); ++g) {
      BATCH_HIP(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
      hipError_t e = hipSuccess;
      for (int i = 0; i < R && e == hipSuccess; ++i) e = launch_step(B, B->cap);
      if (e == hipSuccess && B->monitor_every > 0)
        e = launch_aux(B, g == 1 ? kAuxExact : kAuxMonitor, B->cap);
      hipGraph_t graph = nullptr;
      const hipError_t e2 = hipStreamEndCapture(B->cap, &graph);
      B->graph[g] = graph;
      if (e != hipSuccess || e2 != hipSuccess) {
        set_error("hipGraph capture of the batched round failed: %s",
                  hipGetErrorString(e != hipSuccess ? e : e2));
        return CABCD_EHIP;
      }
      BATCH_HIP(hipGraphInstantiate(&B->exec[g], B->graph[g], nullptr, nullptr, 0));
    }
    B->graph_rounds = R;
  }
  return CABCD_OK;
}

// Re-slicing: once the active problems have halved since the slabs were last
// cut, their slabs are cut again for the active problems alone (same (b, s),
// the slab target recomputed from their work), so the GPU stays filled as
// problems retire.  Runs between launches; the partials and objective
// partials live only within a launch, so they move to the pool freely.  Only
// the rounding order of the Gram sums changes (more, shorter slabs).
cabcd_status replan(cabcd_batch_plan* B, hipStream_t st) {
  std::vector<BState> S(B->P);
  BATCH_HIP(hipMemcpyAsync(S.data(), B->dS, sizeof(BState) * B->P, hipMemcpyDeviceToHost, st));
  BATCH_HIP(hipStreamSynchronize(st));
  std::vector<int> act;
  for (int p = 0; p < B->P; ++p)
    if (S[p].active) act.push_back(p);
  if (act.empty() || 2 * (int)act.size() > B->plan_active) return CABCD_OK;
  double W = 0.0;
  std::vector<double> wp(act.size());
  for (size_t i = 0; i < act.size(); ++i) {
    const BProb& o = B->probs[act[i]];
    wp[i] = slab_work(o.b * o.s, o.n, B->dtype);
    W += wp[i];
  }
  std::vector<int64_t> chunk(act.size());
  std::vector<int> nslab(act.size());
  for (double target = std::max(W / (items_per_cu(B->dtype) * B->cus), 20e-6);;
       target *= 2.0) {
    size_t items = 0, doubles = 0;
    for (size_t i = 0; i < act.size(); ++i) {
      const BProb& o = B->probs[act[i]];
      slice(wp[i], target, o.n, tile_cols(o.nb, B->dtype), chunk[i], nslab[i]);
      items += nslab[i];
      doubles += (size_t)nslab[i] * (slab_doubles(o.b * o.s) + 1) + 64;
    }
    if (items <= (size_t)B->items_cap && doubles <= B->pool_doubles) break;
  }
  // pool offsets, problems with the longest slab first
  std::vector<int> order(act.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return wp[a] / nslab[a] > wp[b] / nslab[b];
  });
  Workspace ws{reinterpret_cast<char*>(B->pool)};
  std::vector<BItem> items;
  for (int i : order) {
    BProb& o = B->probs[act[i]];
    o.chunk = chunk[i];
    o.nslab = nslab[i];
    o.partials = ws.take<double>((size_t)o.nslab * slab_doubles(o.b * o.s));
    o.objp = ws.take<double>(o.nslab);
    for (int q = 0; q < o.nslab; ++q) items.push_back(BItem{act[i], q});
  }
  B->nitems = (int)items.size();
  B->grid_step = std::max(1, std::min(B->nitems, B->occ_step * B->cus));
  B->grid_aux = std::max(1, std::min(B->nitems, B->occ_aux * B->cus));
  B->plan_active = (int)act.size();
  BATCH_HIP(hipMemcpyAsync(B->dP, B->probs.data(), sizeof(BProb) * B->P, hipMemcpyHostToDevice,
                           st));
  BATCH_HIP(hipMemcpyAsync(B->dI, items.data(), sizeof(BItem) * items.size(),
                           hipMemcpyHostToDevice, st));
  BATCH_HIP(hipStreamSynchronize(st));
  return capture(B);
}

}  // namespace
}  // namespace cabcd

using namespace cabcd;

extern "C" {

cabcd_status cabcd_batch_create(const cabcd_problem* problems, int32_t P,
                                const cabcd_batch_opts* opts, void* stream, cabcd_batch* out) {
  clear_error();
  if (out == nullptr) {
    set_error("out must be non-NULL");
    return CABCD_EINVAL;
  }
  *out = nullptr;
  if (problems == nullptr || P < 1) {
    set_error("need P >= 1 problems (P=%d)", P);
    return CABCD_EINVAL;
  }
  if (opts != nullptr && (opts->monitor_every < 0 || opts->cheap_monitors < 0)) {
    set_error("monitor_every and cheap_monitors must be >= 0");
    return CABCD_EINVAL;
  }
  for (int p = 0; p < P; ++p) {
    const cabcd_status rc = check_problem(problems[p], p);
    if (rc != CABCD_OK) return rc;
    if (problems[p].X.dtype != problems[0].X.dtype) {
      set_error("problem %d: every problem of a batch must use the same storage type", p);
      return CABCD_EINVAL;
    }
  }
  cabcd_batch_plan* B = new cabcd_batch_plan();
  const cabcd_status rc = create(problems, P, opts, static_cast<hipStream_t>(stream), B);
  if (rc != CABCD_OK) {
    release(B);
    return rc;
  }
  *out = B;
  return CABCD_OK;
}

cabcd_status cabcd_batch_run(cabcd_batch B, int64_t rounds, void* stream, int32_t* active) {
  clear_error();
  if (B == nullptr || rounds < 0) {
    set_error("need a plan and rounds >= 0");
    return CABCD_EINVAL;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int M = B->monitor_every;
  // Every (cheap_monitors + 1)-th monitor point recomputes r exactly.
  const auto next_exact = [&]() {
    return (B->monitors_done + 1) % ((int64_t)B->cheap_monitors + 1) == 0;
  };
  int64_t done = 0;
  while (done < rounds) {
    if (B->exec[0] != nullptr && rounds - done >= B->graph_rounds &&
        (M == 0 || B->rounds_done % M == 0)) {
      const int g = M > 0 && next_exact() ? 1 : 0;
      BATCH_HIP(hipGraphLaunch(B->exec[g], st));
      done += B->graph_rounds;
      B->rounds_done += B->graph_rounds;
      if (M > 0) ++B->monitors_done;
      B->pending = M == 0;
    } else {
      BATCH_HIP(launch_step(B, st));
      ++done;
      ++B->rounds_done;
      B->pending = true;
      if (M > 0 && B->rounds_done % M == 0) {
        BATCH_HIP(launch_aux(B, next_exact() ? kAuxExact : kAuxMonitor, st));
        ++B->monitors_done;
        B->pending = false;
      }
    }
    if (B->rounds_done % B->replan_period == 0) {
      const cabcd_status rc = replan(B, st);
      if (rc != CABCD_OK) return rc;
    }
  }
  if (B->pending) {
    BATCH_HIP(launch_aux(B, kAuxFlush, st));
    B->pending = false;
  }
  if (active != nullptr) return sync_status(B, st, active);
  return CABCD_OK;
}

cabcd_status cabcd_batch_query(cabcd_batch B, int32_t p, cabcd_batch_info* info, void* stream) {
  clear_error();
  if (B == nullptr || info == nullptr || p < 0 || p >= B->P) {
    set_error("need a plan, 0 <= p < P and an info struct");
    return CABCD_EINVAL;
  }
  BState s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  BATCH_HIP(hipMemcpyAsync(&s, B->dS + p, sizeof s, hipMemcpyDeviceToHost, st));
  BATCH_HIP(hipStreamSynchronize(st));
  const BProb& o = B->probs[p];
  info->b = o.b;
  info->s = o.s;
  info->nslab = o.nslab;
  info->active = s.active;
  info->chunk = o.chunk;
  info->h = s.h;
  info->steps = s.steps;
  info->objective = s.obj;
  info->status = s.status == DEV_NOTSPD      ? CABCD_ENOTSPD
                 : s.status == DEV_NONFINITE ? CABCD_ENONFINITE
                                             : CABCD_OK;
  info->reserved = 0;
  return CABCD_OK;
}

cabcd_status cabcd_batch_destroy(cabcd_batch B) {
  release(B);
  return CABCD_OK;
}

cabcd_status cabcd_primal_bcd_batched(const cabcd_problem* problems, int32_t P,
                                      int64_t max_rounds, const cabcd_batch_opts* opts,
                                      void* stream) {
  cabcd_batch B = nullptr;
  cabcd_status rc = cabcd_batch_create(problems, P, opts, stream, &B);
  if (rc != CABCD_OK) return rc;
  const int64_t period = B->graph_rounds > 0 ? B->graph_rounds : 4;
  int64_t done = 0;
  int32_t active = 1;
  while (rc == CABCD_OK && active > 0 && done < max_rounds) {
    const int64_t r = std::min(period, max_rounds - done);
    rc = cabcd_batch_run(B, r, stream, &active);
    done += r;
  }
  const std::string msg = cabcd_last_error();
  release(B);
  if (rc != CABCD_OK) set_error("%s", msg.c_str());
  return rc;
}

}  // extern "C"
