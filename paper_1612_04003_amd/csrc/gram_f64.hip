// Dense FP64 Gram of gathered rows: the one-problem launches (split-K Gram
// kernel and its deterministic reduction) and the launch planner.  The device
// code and its design notes are in gram_dev.h.
#include "gram_dev.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>

namespace cabcd {
namespace {

using namespace gdev;

// Several row lists per launch: step blockIdx.y reads idx + step * m and
// writes its partials (and its Y u, when u is given) at partials + step * pstride.
template <int NB, int RPW>
__global__ __launch_bounds__((Cfg<NB, RPW>::THREADS)) void gram_f64_kernel(
    const double* __restrict__ A, int64_t ld, int64_t cols, const int32_t* __restrict__ idx,
    int m, const double* __restrict__ u, int64_t chunk, double* __restrict__ partials,
    int64_t pstride, int aligned) {
  using C = Cfg<NB, RPW>;
  __shared__ __attribute__((aligned(16))) double lds[C::LDS];
  idx += (int64_t)blockIdx.y * m;
  partials += (int64_t)blockIdx.y * pstride;
  const int64_t k_begin = (int64_t)blockIdx.x * chunk;
  const int64_t k_end = std::min(cols, k_begin + chunk);
  gram_slab<NB, RPW>(A, ld, k_begin, k_end, idx, m, u,
                     partials + (int64_t)blockIdx.x * (C::NBLK * 256 + C::SBP), aligned, lds);
}

template <int NB>
__global__ __launch_bounds__((Cfg<NB, 2>::THREADS)) void gram_f64_dma_kernel(
    const double* __restrict__ A, int64_t ld, int64_t cols, const int32_t* __restrict__ idx,
    int m, const double* __restrict__ u, int64_t chunk, double* __restrict__ partials,
    int64_t pstride) {
  using C = Cfg<NB, 2>;
  __shared__ __attribute__((aligned(16))) double lds[DN<NB>::LDS];
  idx += (int64_t)blockIdx.y * m;
  partials += (int64_t)blockIdx.y * pstride;
  const int64_t k_begin = (int64_t)blockIdx.x * chunk;
  const int64_t k_end = std::min(cols, k_begin + chunk);
  gram_slab_dma<NB>(A, ld, k_begin, k_end, idx, m, u,
                    partials + (int64_t)blockIdx.x * (C::NBLK * 256 + C::SBP), lds);
}

__global__ __launch_bounds__(D16::THREADS) void gram_f64_dma16_kernel(
    const double* __restrict__ A, int64_t ld, int64_t cols, const int32_t* __restrict__ idx,
    int m, const double* __restrict__ u, int64_t chunk, double* __restrict__ partials,
    int64_t pstride) {
  __shared__ __attribute__((aligned(16))) double lds[D16::LDS];
  idx += (int64_t)blockIdx.y * m;
  partials += (int64_t)blockIdx.y * pstride;
  const int64_t k_begin = (int64_t)blockIdx.x * chunk;
  const int64_t k_end = std::min(cols, k_begin + chunk);
  gram_slab_dma16(A, ld, k_begin, k_end, idx, m, u,
                  partials + (int64_t)blockIdx.x * (D16::NBLK * 256 + D16::SBP), lds);
}

// MODE 1: the Gram with the previous step's update folded in; MODE 2: the
// update alone (one slab per workgroup, the Gram's slabs).
template <int MODE>
__global__ __launch_bounds__(D16::THREADS) void gram_f64_dma16_upd_kernel(
    const double* __restrict__ A, int64_t ld, int64_t cols, const int32_t* __restrict__ idx,
    int m, int64_t chunk, double* __restrict__ partials, D16Upd up) {
  __shared__ __attribute__((aligned(16))) double lds[D16::LDS_UPD];
  const int64_t k_begin = (int64_t)blockIdx.x * chunk;
  const int64_t k_end = std::min(cols, k_begin + chunk);
  double* part =
      MODE == 1 ? partials + (int64_t)blockIdx.x * (D16::NBLK * 256 + D16::SBP) : nullptr;
  gram_slab_dma16<MODE>(A, ld, k_begin, k_end, idx, m, nullptr, part, lds, up);
}

// A reduction workgroup has 1024 threads: GROUPS split groups (a wave or more
// each) for 1024 / GROUPS entries.  Many splits take 16 groups of 64 entries;
// a few splits take one group, each thread summing all of its entry's splits.
constexpr int kRedThreads = 1024;
int red_groups(int nsplit) { return nsplit <= 4 ? 1 : 16; }

// Partial set blockIdx.y: partials + set * nsplit * pstride.  MODE 0: the
// Gram of step blockIdx.y (idx + step * m, G and add + step * m * m; Yu is
// NULL for several steps).  MODE 1 / 2: sets 0 / 1 of Grams of m in
// (256, 512] rows (store_entry_big): `per` partial sets per Gram (2 diagonal /
// big_cross_steps(m) cross), so set q belongs to Gram q / per, whose indices,
// G and add are at step offsets as in MODE 0 (Yu only with a single Gram).
template <int MODE, int GROUPS>
__global__ __launch_bounds__(kRedThreads) void gram_reduce_kernel(
    const double* __restrict__ partials, int nsplit, int nb, const int32_t* __restrict__ idx,
    int m, double scale, double shift, int overlap, double* __restrict__ G,
    double* __restrict__ Yu, int layout, const float* __restrict__ rs,
    const double* __restrict__ add, int per) {
  constexpr int kRedElems = kRedThreads / GROUPS;
  constexpr int kRedGroups = GROUPS;
  __shared__ double red[kRedGroups][kRedElems];
  const int nblk = nb * (nb + 1) / 2;
  const int64_t pstride = (int64_t)nblk * 256 + 16 * nb;
  partials += (int64_t)blockIdx.y * nsplit * pstride;
  const int gram = MODE == 0 ? (int)blockIdx.y : (int)blockIdx.y / per;
  const int part = MODE == 0 ? 0 : (int)blockIdx.y % per;
  idx += (int64_t)gram * m;
  G += (int64_t)gram * m * m;
  if (add != nullptr) add += (int64_t)gram * m * m;
  const int el = threadIdx.x % kRedElems;
  const int grp = threadIdx.x / kRedElems;
  const int64_t e = (int64_t)blockIdx.x * kRedElems + el;
  // Each wave sums a contiguous range of splits for 64 consecutive entries;
  // the ranges are then added in group order, so the result is deterministic.
  const int spg = (nsplit + kRedGroups - 1) / kRedGroups;   // splits per group
  const int sp0 = grp * spg;
  const int sp1 = min(nsplit, sp0 + spg);
  double s = 0.0;
  if (layout == 2 && e < (int64_t)nblk * 256) {   // FP32 block entries
    const float* p = reinterpret_cast<const float*>(partials) + e;
    const int64_t fstride = 2 * pstride;
    int sp = sp0;
    for (; sp + 8 <= sp1; sp += 8) {
      float v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = p[(int64_t)(sp + q) * fstride];
#pragma unroll
      for (int q = 0; q < 8; ++q) s += (double)v[q];
    }
    for (; sp < sp1; ++sp) s += (double)p[(int64_t)sp * fstride];
  } else if (e < pstride) {
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
  if constexpr (MODE == 0)
    store_entry(e, t, nblk, idx, m, scale, shift, overlap, G, Yu, layout, rs, add);
  else
    gdev::store_entry_big(e, t, MODE - 1, part, idx, m, scale, shift, overlap, G, Yu, layout,
                          rs, add);
}

// Workgroup k builds the index lists (gdev::big_lists) of Gram k (indices
// idx + k m) at ia + 512 k and ib + 256 nc k, nc = big_cross_steps(m) lists.
__global__ __launch_bounds__(512) void big_index_kernel(const int32_t* __restrict__ idx, int m,
                                                        int32_t* __restrict__ ia,
                                                        int32_t* __restrict__ ib) {
  const int nc = m - 256 > 128 ? 4 : 2;
  gdev::big_lists(idx + (int64_t)blockIdx.x * m, m, ia + (int64_t)blockIdx.x * 512,
                  ib + (int64_t)blockIdx.x * 256 * nc, threadIdx.x, 512);
}

bool d16_ok(const GramPlan& p, const double* A, int64_t ld) {
  return p.nb == 16 && p.rpw == 1 && (reinterpret_cast<uintptr_t>(A) & 15) == 0 && (ld & 1) == 0;
}

template <int NB, int RPW>
hipError_t launch_nb(const GramPlan& p, const double* A, int64_t ld, int64_t cols,
                     const int32_t* idx, int m, int nsteps, const double* u, double* partials,
                     hipStream_t st) {
  const int aligned = ((reinterpret_cast<uintptr_t>(A) & 15) == 0 && (ld & 1) == 0) ? 1 : 0;
  const int64_t pstride = (int64_t)gram_partial_doubles(p);
  const dim3 grid((unsigned)p.nsplit, (unsigned)nsteps);
  if constexpr (NB == 16) {
    if (p.rpw == 1 && aligned) {
      hipLaunchKernelGGL(gram_f64_dma16_kernel, grid, dim3(D16::THREADS), 0, st, A, ld, cols, idx,
                         m, u, p.chunk, partials, pstride);
      return hipGetLastError();
    }
  }
  if constexpr (NB <= 8 && RPW == 2) {
    if (p.rpw == 1 && aligned) {
      hipLaunchKernelGGL((gram_f64_dma_kernel<NB>), grid, dim3(Cfg<NB, 2>::THREADS), 0, st, A,
                         ld, cols, idx, m, u, p.chunk, partials, pstride);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((gram_f64_kernel<NB, RPW>), grid, dim3(Cfg<NB, RPW>::THREADS), 0, st, A, ld,
                     cols, idx, m, u, p.chunk, partials, pstride, aligned);
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
  // A CU streams at most its share of the HBM rate, so fewer slabs than CUs
  // leave bandwidth unused.
  auto hbm_time = [&](int64_t nsplit) {
    return ybytes / (hbm * std::min(1.0, (double)nsplit / 256.0));
  };
  for (int64_t chunk = p.kt; ; chunk *= 2) {
    const int64_t nsplit = (cols + chunk - 1) / chunk;
    const double per_wg = 2.0 * ((double)chunk / (4.0 * kg)) * nacc * 64.0 / clock;
    const double rounds = std::ceil((double)nsplit / 256.0);
    const double t = std::max(rounds * per_wg, hbm_time(nsplit)) +
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
    const double t = std::max(per_wg, hbm_time(nsplit)) + 2.0 * nsplit * pbytes_per / hbm;
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
  // rpw = 1: the LDS-DMA variant of the same decomposition (aligned A only;
  // CABCD_GRAM_DMA=0 selects the register-fed kernels instead).
  const char* env = std::getenv("CABCD_GRAM_DMA");
  p.rpw = (env != nullptr && std::atoi(env) == 0) ? 2 : 1;
  return p;
}

size_t gram_partial_doubles(const GramPlan& p) {
  return (size_t)p.nsplit * ((size_t)p.nblk * 256 + 16 * (size_t)p.nb);
}

hipError_t launch_gram_f64(const GramPlan& p, const double* A, int64_t ld, int64_t cols,
                           const int32_t* idx, int m, const double* u, double* partials,
                           hipStream_t st, int nsteps) {
  if (nsteps < 1 || nsteps > 65535) return hipErrorInvalidValue;
  switch (p.nb) {
    case 1: return launch_nb<1, 2>(p, A, ld, cols, idx, m, nsteps, u, partials, st);
    case 2: return launch_nb<2, 2>(p, A, ld, cols, idx, m, nsteps, u, partials, st);
    case 4: return launch_nb<4, 2>(p, A, ld, cols, idx, m, nsteps, u, partials, st);
    case 8: return launch_nb<8, 2>(p, A, ld, cols, idx, m, nsteps, u, partials, st);
    case 16: return launch_nb<16, 2>(p, A, ld, cols, idx, m, nsteps, u, partials, st);
    default: return hipErrorInvalidValue;
  }
}

bool gram_f64_takes_update(const GramPlan& p, const double* A, int64_t ld, int m) {
  return m == D16::SBP && d16_ok(p, A, ld);
}

hipError_t launch_gram_f64_upd(const GramPlan& p, const double* A, int64_t ld, int64_t cols,
                               const int32_t* idx, int m, double* partials, const D16Upd& up,
                               hipStream_t st) {
  if (!gram_f64_takes_update(p, A, ld, m) || up.idx == nullptr || up.delta == nullptr ||
      up.r == nullptr)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL((gram_f64_dma16_upd_kernel<1>), dim3((unsigned)p.nsplit), dim3(D16::THREADS),
                     0, st, A, ld, cols, idx, m, p.chunk, partials, up);
  return hipGetLastError();
}

hipError_t launch_update_f64(const GramPlan& p, const double* A, int64_t ld, int64_t cols,
                             const D16Upd& up, hipStream_t st) {
  if (!d16_ok(p, A, ld) || up.idx == nullptr || up.delta == nullptr || up.r == nullptr)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL((gram_f64_dma16_upd_kernel<2>), dim3((unsigned)p.nsplit), dim3(D16::THREADS),
                     0, st, A, ld, cols, nullptr, 0, p.chunk, nullptr, up);
  return hipGetLastError();
}

template <int MODE>
void launch_reduce(int groups, dim3 grid, hipStream_t st, const double* partials, int nsplit,
                   int nb, const int32_t* idx, int m, double scale, double shift, int overlap,
                   double* G, double* Yu, int layout, const float* rs, const double* add,
                   int per) {
  if (groups == 1)
    hipLaunchKernelGGL((gram_reduce_kernel<MODE, 1>), grid, dim3(kRedThreads), 0, st, partials,
                       nsplit, nb, idx, m, scale, shift, overlap, G, Yu, layout, rs, add, per);
  else
    hipLaunchKernelGGL((gram_reduce_kernel<MODE, 16>), grid, dim3(kRedThreads), 0, st, partials,
                       nsplit, nb, idx, m, scale, shift, overlap, G, Yu, layout, rs, add, per);
}

hipError_t launch_gram_reduce(const GramPlan& p, const double* partials, const int32_t* idx,
                              int m, double scale, double shift, bool overlap, double* G,
                              double* Yu, hipStream_t st, int layout, const float* rs,
                              int nsteps, const double* add) {
  if (nsteps < 1 || nsteps > 65535 || (nsteps > 1 && Yu != nullptr)) return hipErrorInvalidValue;
  const int64_t entries = (int64_t)p.nblk * 256 + 16 * p.nb;
  const int groups = red_groups(p.nsplit);
  const int64_t blocks = (entries + kRedThreads / groups - 1) / (kRedThreads / groups);
  launch_reduce<0>(groups, dim3((unsigned)blocks, (unsigned)nsteps), st, partials, p.nsplit, p.nb,
                   idx, m, scale, shift, overlap ? 1 : 0, G, Yu, layout, rs, add, 1);
  return hipGetLastError();
}

hipError_t launch_big_index(const int32_t* idx, int m, int32_t* ia, int32_t* ib, hipStream_t st,
                            int ngram) {
  if (m <= 256 || m > 512 || ngram < 1 || ngram > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(big_index_kernel, dim3((unsigned)ngram), dim3(512), 0, st, idx, m, ia, ib);
  return hipGetLastError();
}

int big_cross_steps(int m) { return m - 256 > 128 ? 4 : 2; }

hipError_t launch_gram_reduce_big(const GramPlan& p, const double* partials, const int32_t* idx,
                                  int m, double scale, double shift, bool overlap, double* G,
                                  double* Yu, hipStream_t st, int layout, const float* rs,
                                  int ngram, const double* add) {
  if (p.nb != 16 || m <= 256 || m > 512 || ngram < 1 || (ngram > 1 && Yu != nullptr))
    return hipErrorInvalidValue;
  const int64_t entries = (int64_t)p.nblk * 256 + 16 * p.nb;
  const int groups = red_groups(p.nsplit);
  const int64_t blocks = (entries + kRedThreads / groups - 1) / (kRedThreads / groups);
  const size_t set = gram_partial_doubles(p);
  const int nc = big_cross_steps(m);
  launch_reduce<1>(groups, dim3((unsigned)blocks, (unsigned)(2 * ngram)), st, partials, p.nsplit,
                   p.nb, idx, m, scale, shift, overlap ? 1 : 0, G, Yu, layout, rs, add, 2);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  launch_reduce<2>(groups, dim3((unsigned)blocks, (unsigned)(nc * ngram)), st,
                   partials + 2 * ngram * set, p.nsplit, p.nb, idx, m, scale, shift,
                   overlap ? 1 : 0, G, nullptr, layout, rs, add, nc);
  return hipGetLastError();
}

}  // namespace cabcd
