// The sparse s-step Gram split by column popularity (the CSR Grams of outer
// steps computed ahead, Alg. 4 on A = X^T with power-law feature popularity).
//
// The Gram of the gathered rows is G[p][q] = sum_c Y[p][c] Y[q][c], which costs
// sum_c nnz_c(I)^2 products over the columns c of the sampled rows I.  With a
// power-law column popularity a few hundred columns carry most of that sum and
// appear in nearly every gathered row, so the output is dense although the
// rows are sparse.  The columns are therefore split once per matrix:
//   * heavy: the at most kHeavyMax most popular columns (global column counts,
//     and at least a fixed share of the rows) get a slot in a dense panel,
//     numbered in column order.  Per outer step the gathered rows' heavy
//     entries are scattered into an m x H panel and the FP64 matrix-core Gram
//     of the one-problem dense path forms its Gram (split-K, deterministic);
//   * light: the other entries of a step are grouped by column: per-step
//     tables indexed by the column id count a step's entries per column, an
//     exclusive scan of the counts lays the (row, value) lists out in column
//     order, and one wave per gathered row p adds, entry by entry in the row's
//     column order, value_p value_q into an LDS row of p's products for the
//     rows q <= p of the entry's column list (a column only p holds adds
//     value_p^2, summed by the lanes and then in a fixed tree).  Only the
//     sum_c nnz_c(I)^2 products of the light columns are formed, every sum runs
//     in a fixed order (no float atomics), and the light row is added to the
//     dense partial sums in the reduction.
// Integer atomics only count entries and hand out list positions; which
// position an entry gets does not change any sum's order (a list holds a
// gathered row at most once, so each sum meets its terms in the row's column
// order; heavy slots are numbered in column order).  The heavy columns are
// picked from the column counts of a sample of the rows: any split gives the
// same Gram, the choice only affects speed.
#include "internal.h"

#include <algorithm>

namespace cabcd {
namespace {

constexpr int kT = 256;               // threads of the helper kernels
constexpr int kHeavyMax = 512;        // panel columns at most
constexpr int kHist = 8192;           // column-count histogram bins (counts capped)
constexpr int kScanChunk = 1024;      // columns per workgroup of the slot numbering
constexpr int64_t kSampleRows = 2048; // rows whose columns estimate the popularity

__global__ __launch_bounds__(kT) void zero_ints_kernel(int* __restrict__ p, int64_t n, int v) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    p[i] = v;
}

__global__ __launch_bounds__(kT) void zero_doubles_kernel(double* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    p[i] = 0.0;
}

// Column counts over a sample of the rows (every `stride`-th row): the
// popularity estimate that picks the heavy columns.  Any split of the columns
// gives the same Gram (heavy and light parts are disjoint sums), so the
// estimate only affects speed.  One wave per sampled row.
__global__ __launch_bounds__(kT) void col_count_kernel(const int64_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ colidx,
                                                       int64_t rows, int64_t stride,
                                                       int* __restrict__ cnt) {
  const int lane = threadIdx.x & 63;
  const int64_t wv = ((int64_t)blockIdx.x * kT + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * kT) >> 6;
  for (int64_t r = wv; r * stride < rows; r += nw) {
    const int64_t i = r * stride;
    for (int64_t j = rowptr[i] + lane; j < rowptr[i + 1]; j += 64) atomicAdd(&cnt[colidx[j]], 1);
  }
}

// Histogram of the counts of the columns that can be heavy (count >= tmin).
__global__ __launch_bounds__(kT) void count_hist_kernel(const int* __restrict__ cnt, int64_t cols,
                                                        int tmin, int* __restrict__ hist) {
  for (int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x; c < cols; c += (int64_t)gridDim.x * kT) {
    const int v = cnt[c];
    if (v >= tmin) atomicAdd(&hist[min(v, kHist - 1)], 1);
  }
}

// One workgroup of 1024 threads, 8 bins each: the smallest count T >= tmin
// such that at most kHeavyMax columns have a count >= T (stats[0] = T), and
// the number of those columns (stats[3]).  The thread whose bins hold the
// crossing finds it from its suffix sum (the columns in higher bins).
constexpr int kThrT = 1024;
constexpr int kThrPer = kHist / kThrT;
__global__ __launch_bounds__(kThrT) void heavy_threshold_kernel(const int* __restrict__ hist,
                                                                int tmin, int* __restrict__ stats) {
  __shared__ int sh[kThrT / 64];
  __shared__ int res[2];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  int h[kThrPer];
  int mine = 0;
#pragma unroll
  for (int q = 0; q < kThrPer; ++q) {
    h[q] = hist[t * kThrPer + q];
    mine += h[q];
  }
  // above = sum of `mine` over the threads t' > t (inclusive scan from the top)
  int x = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_down(x, o, 64);
    if (lane + o < 64) x += v;
  }
  if (lane == 0) sh[wave] = x;
  if (t == 0) res[0] = 0;   // no crossing: every qualifying column is heavy
  __syncthreads();
  int above = x - mine;
  for (int w = wave + 1; w < kThrT / 64; ++w) above += sh[w];
  if (above <= kHeavyMax && above + mine > kHeavyMax) {
    int acc = above, T = 0;
    for (int q = kThrPer - 1; q >= 0; --q) {
      if (acc + h[q] > kHeavyMax) {
        T = t * kThrPer + q + 1;
        break;
      }
      acc += h[q];
    }
    res[0] = T;   // exactly one thread holds the crossing
  }
  __syncthreads();
  const int T = max(res[0], tmin);
  // heavy columns: those in bins >= T
  int c = 0;
#pragma unroll
  for (int q = 0; q < kThrPer; ++q) c += t * kThrPer + q >= T ? h[q] : 0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  __syncthreads();
  if (lane == 0) sh[wave] = c;
  __syncthreads();
  if (t == 0) {
    int tot = 0;
    for (int w = 0; w < kThrT / 64; ++w) tot += sh[w];
    stats[0] = T;
    stats[3] = tot;
  }
}

// Heavy columns of workgroup chunk blockIdx.x: block counts (pass 0), then slot
// numbers in column order (pass 1, with the sum of the earlier block counts).
__global__ __launch_bounds__(kScanChunk) void heavy_slots_kernel(const int* __restrict__ cnt,
                                                                 int64_t cols,
                                                                 const int* __restrict__ stats,
                                                                 int* __restrict__ blk,
                                                                 int* __restrict__ hmap, int pass) {
  __shared__ int wsum[kScanChunk / 64];
  __shared__ int bsum[kScanChunk / 64];
  const int T = stats[0];
  const int64_t c = (int64_t)blockIdx.x * kScanChunk + threadIdx.x;
  const bool heavy = c < cols && cnt[c] >= T;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long mask = __ballot(heavy);
  if (lane == 0) wsum[wave] = __popcll(mask);
  __syncthreads();
  if (pass == 0) {
    if (threadIdx.x == 0) {
      int s = 0;
      for (int w = 0; w < kScanChunk / 64; ++w) s += wsum[w];
      blk[blockIdx.x] = s;
    }
    return;
  }
  // the earlier blocks' counts, summed by the workgroup
  int e = 0;
  for (int q = threadIdx.x; q < (int)blockIdx.x; q += kScanChunk) e += blk[q];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o, 64);
  if (lane == 0) bsum[wave] = e;
  __syncthreads();
  int off = 0;
  for (int w = 0; w < kScanChunk / 64; ++w) off += bsum[w];
  for (int w = 0; w < wave; ++w) off += wsum[w];
  const int below = __popcll(mask & ((1ull << lane) - 1ull));
  if (c < cols) hmap[c] = heavy ? off + below : -1;
}

// stats[1] = longest row (the bound of a row's light entries too).
__global__ __launch_bounds__(kT) void split_stats_kernel(const int64_t* __restrict__ rowptr,
                                                         int64_t rows, int* __restrict__ stats) {
  int mx = 0;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < rows; i += (int64_t)gridDim.x * kT)
    mx = max(mx, (int)(rowptr[i + 1] - rowptr[i]));
  for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(&stats[1], mx);
}

// ----------------------------------------------------------------- per launch

// Entries of the gathered rows are handled by one wave per (step k, row p,
// chunk of 64 entries), so every entry's loads are in flight at once.
__device__ __forceinline__ bool chunk_of(int64_t wv, int m, int nchunk, int nsteps, int& k, int& p,
                                         int& ch) {
  if (wv >= (int64_t)nsteps * m * nchunk) return false;
  ch = (int)(wv % nchunk);
  const int64_t r = wv / nchunk;
  k = (int)(r / m);
  p = (int)(r % m);
  return true;
}

// Heavy entries into the dense panel row; light entries counted in the step's
// per-column counts (the column itself indexes the table).  ent[k][p][e] =
// -1 for a heavy entry, else the light column shifted up by kRankBits with
// the entry's rank in its column's list (the count before it) below: columns
// are < 2^22 and ranks < 512 rows, so the pair fits 31 bits.
constexpr int kRankBits = 9;
__global__ __launch_bounds__(kT) void split_scatter_kernel(
    const int64_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
    const double* __restrict__ vals, const int32_t* __restrict__ idx, int m, int nsteps,
    int nchunk, const int* __restrict__ hmap, double* __restrict__ Dh, int Hp,
    int* __restrict__ cnt, int64_t cs, int* __restrict__ ent, int maxrow) {
  const int lane = threadIdx.x & 63;
  const int64_t wv = ((int64_t)blockIdx.x * kT + threadIdx.x) >> 6;
  int k, p, ch;
  if (!chunk_of(wv, m, nchunk, nsteps, k, p, ch)) return;
  const int64_t row = (int64_t)k * m + p;
  const int i = idx[row];
  const int64_t a = rowptr[i], b = rowptr[i + 1];
  const int64_t j = a + 64 * ch + lane;
  if (j >= b) return;
  const int c = colidx[j];
  const int hs = hmap[c];
  int e = -1;
  if (hs >= 0)
    Dh[row * Hp + hs] = vals[j];
  else
    e = (c << kRankBits) | atomicAdd(&cnt[(int64_t)k * cs + c], 1);
  ent[row * maxrow + (j - a)] = e;
}

// Exclusive scan of the step's per-column counts into list offsets (three
// passes: workgroup sums, their scan, workgroup-local scans), so the lists
// are laid out in column order without a shared counter.  A step's table has
// a stride of whole scan workgroups (zero padding), read as int4.
constexpr int kScanT = 256;                 // threads of a scan workgroup
constexpr int kScanCols = 4096;             // its columns: 4 int4 a thread
__device__ __forceinline__ int wg_excl_scan(int v, int* sh, int& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(x, o, 64);
    if (lane >= o) x += t;
  }
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  int before = 0;
  total = 0;
#pragma unroll
  for (int w = 0; w < kScanT / 64; ++w) {
    const int t = sh[w];
    before += w < wave ? t : 0;
    total += t;
  }
  __syncthreads();   // sh is free for the next scan
  return before + x - v;
}

__global__ __launch_bounds__(kScanT) void scan_sums_kernel(const int* __restrict__ cnt,
                                                           int64_t cs, int* __restrict__ bsum,
                                                           int nblk) {
  __shared__ int sh[kScanT / 64];
  const int k = blockIdx.y;
  const int4* p = reinterpret_cast<const int4*>(cnt + (int64_t)k * cs +
                                                (int64_t)blockIdx.x * kScanCols);
  int v = 0;
#pragma unroll
  for (int q = 0; q < kScanCols / (4 * kScanT); ++q) {
    const int4 c = p[q * kScanT + threadIdx.x];
    v += c.x + c.y + c.z + c.w;
  }
  int total;
  wg_excl_scan(v, sh, total);
  if (threadIdx.x == 0) bsum[(int64_t)k * nblk + blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanT) void scan_blocks_kernel(int* __restrict__ bsum, int nblk) {
  __shared__ int sh[kScanT / 64];
  int* b = bsum + (int64_t)blockIdx.x * nblk;
  int carry = 0;
  for (int q0 = 0; q0 < nblk; q0 += kScanT) {
    const int q = q0 + (int)threadIdx.x;
    const int v = q < nblk ? b[q] : 0;
    int total;
    const int r = wg_excl_scan(v, sh, total);
    if (q < nblk) b[q] = carry + r;
    carry += total;
  }
}

__global__ __launch_bounds__(kScanT) void scan_apply_kernel(const int* __restrict__ cnt,
                                                            int64_t cs,
                                                            const int* __restrict__ bsum,
                                                            int nblk, int* __restrict__ off) {
  __shared__ int sh[kScanT / 64];
  const int k = blockIdx.y;
  const int64_t base = (int64_t)k * cs + (int64_t)blockIdx.x * kScanCols;
  const int4* p = reinterpret_cast<const int4*>(cnt + base);
  int carry = bsum[(int64_t)k * nblk + blockIdx.x];
#pragma unroll
  for (int q = 0; q < kScanCols / (4 * kScanT); ++q) {
    const int4 c = p[q * kScanT + threadIdx.x];
    int total;
    int pre = carry + wg_excl_scan(c.x + c.y + c.z + c.w, sh, total);
    int* o = off + base + (int64_t)q * 4 * kScanT + 4 * threadIdx.x;
    if (c.x > 0) o[0] = pre;
    pre += c.x;
    if (c.y > 0) o[1] = pre;
    pre += c.y;
    if (c.z > 0) o[2] = pre;
    pre += c.z;
    if (c.w > 0) o[3] = pre;
    carry += total;
  }
}

// Each light entry goes to its rank's position in its column's list (off[c]
// is the list's start).
__global__ __launch_bounds__(kT) void split_fill_kernel(
    const int64_t* __restrict__ rowptr, const double* __restrict__ vals,
    const int32_t* __restrict__ idx, int m, int nsteps, int nchunk, const int* __restrict__ off,
    int64_t cs, const int* __restrict__ ent, int maxrow, int* __restrict__ lq,
    double* __restrict__ lv, int64_t lcap) {
  const int lane = threadIdx.x & 63;
  const int64_t wv = ((int64_t)blockIdx.x * kT + threadIdx.x) >> 6;
  int k, p, ch;
  if (!chunk_of(wv, m, nchunk, nsteps, k, p, ch)) return;
  const int64_t row = (int64_t)k * m + p;
  const int i = idx[row];
  const int64_t a = rowptr[i], b = rowptr[i + 1];
  const int64_t j = a + 64 * ch + lane;
  if (j >= b) return;
  const int e = ent[row * maxrow + (j - a)];
  if (e < 0) return;
  const int pos = off[(int64_t)k * cs + (e >> kRankBits)] + (e & ((1 << kRankBits) - 1));
  lq[(int64_t)k * lcap + pos] = p;
  lv[(int64_t)k * lcap + pos] = vals[j];
}

// One wave per (step k, gathered row p): row p of the light part,
// Gl[k][p][q] = sum over the light columns c of row p, in the row's column
// order, of v_pc v_qc for q <= p.  The row's entries are taken 64 at a time
// (the next batch's columns and values are loaded while one is applied):
// their list extents are loaded by the lanes together, runs of lists that
// fit the stage are copied into LDS by the whole wave (one staged element a
// lane and load, eight loads in flight), and the entries are then applied one
// after the other from LDS.  A column's list holds a gathered row at most
// once, so the lanes of one entry add to distinct q and the order of every
// sum is the row's column order, whatever order the lists were filled in.
// The row is accumulated in LDS and written whole (zeros where no light
// column is shared).
constexpr int kSplitMaxRows = 512;
constexpr int kStage = 512;                 // staged list elements per wave
constexpr int kCopyUnroll = kStage / 64;    // loads in flight a lane while staging
constexpr int kLightWaves = kT / 64;
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__global__ __launch_bounds__(kT) void split_light_kernel(
    const int64_t* __restrict__ rowptr, const double* __restrict__ vals,
    const int32_t* __restrict__ idx, int m, int nsteps, const int* __restrict__ cnt,
    const int* __restrict__ off, int64_t cs, const int* __restrict__ ent, int maxrow,
    const int* __restrict__ lq, const double* __restrict__ lv, int64_t lcap,
    double* __restrict__ Gl) {
  __shared__ double acc[kLightWaves][kSplitMaxRows];
  __shared__ double sv[kLightWaves][kStage];
  __shared__ int sq[kLightWaves][kStage];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t wv = ((int64_t)blockIdx.x * kT + threadIdx.x) >> 6;
  if (wv >= (int64_t)nsteps * m) return;
  double* ar = acc[wave];
  double* bv = sv[wave];
  int* bq = sq[wave];
  for (int q = lane; q < m; q += 64) ar[q] = 0.0;
  wave_sync_lds();
  const int k = (int)(wv / m), p = (int)(wv % m);
  cnt += (int64_t)k * cs;
  off += (int64_t)k * cs;
  lq += (int64_t)k * lcap;
  lv += (int64_t)k * lcap;
  const int i = idx[wv];
  const int64_t a = rowptr[i], b = rowptr[i + 1];
  const int* erow = ent + wv * (int64_t)maxrow;
  // light columns no other gathered row shares give only p's own product:
  // each lane sums those of its entries (in row order), added at the end
  double self = 0.0;
  int c = a + lane < b ? erow[lane] : -1;   // the light column (or -1)
  c = c < 0 ? -1 : c >> kRankBits;
  double vp = c >= 0 ? vals[a + lane] : 0.0;
  for (int64_t e0 = a; e0 < b; e0 += 64) {
    // this batch's list extents; the next batch's columns and values
    const int nc = c >= 0 ? cnt[c] : 0;
    const int oc = c >= 0 ? off[c] : 0;
    const int64_t jn = e0 + 64 + lane;
    int cn = jn < b ? erow[jn - a] : -1;
    cn = cn < 0 ? -1 : cn >> kRankBits;
    const double vn = cn >= 0 ? vals[jn] : 0.0;
    if (nc == 1) self = fma(vp, vp, self);
    const int n = nc >= 2 ? nc : 0;
    const int s0 = oc;
    // staging positions: exclusive prefix of the list lengths
    int pre = n;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(pre, o, 64);
      if (lane >= o) pre += t;
    }
    pre -= n;
    unsigned long long todo = __ballot(n > 0);
    while (todo != 0ull) {
      // the entries staged together: from the first pending one while their
      // lists fit the stage; a longer list is applied from global memory
      const int first = __ffsll((long long)todo) - 1;
      const int base = __shfl(pre, first, 64);
      unsigned long long run = 0ull;
      {
        unsigned long long t = todo;
        while (t != 0ull) {
          const int e = __ffsll((long long)t) - 1;
          if (__shfl(pre, e, 64) + __shfl(n, e, 64) - base > kStage) break;
          run |= 1ull << e;
          t &= t - 1ull;
        }
      }
      const bool staged = run != 0ull;
      if (staged) {
        // each entry writes its elements' global positions into the stage,
        // then every lane copies staged elements lane, lane + 64, ...
        const int last = 63 - __clzll((long long)run);
        const int total = __shfl(pre, last, 64) + __shfl(n, last, 64) - base;
        if ((run >> lane) & 1ull)
          for (int t = 0; t < n; ++t) bq[pre - base + t] = s0 + t;
        wave_sync_lds();
        int g[kCopyUnroll];
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) {
          const int jj = u * 64 + lane;
          g[u] = jj < total ? bq[jj] : -1;
        }
        int qv[kCopyUnroll];
        double vv[kCopyUnroll];
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) {
          qv[u] = g[u] >= 0 ? lq[g[u]] : 0;
          vv[u] = g[u] >= 0 ? lv[g[u]] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) {
          const int jj = u * 64 + lane;
          if (jj < total) {
            bq[jj] = qv[u];
            bv[jj] = vv[u];
          }
        }
        wave_sync_lds();
      } else {
        run = 1ull << first;
      }
      todo &= ~run;
      while (run != 0ull) {
        const int e = __ffsll((long long)run) - 1;
        run &= run - 1ull;
        const int ne = __shfl(n, e, 64);
        const double ve = __shfl(vp, e, 64);
        const int se = __shfl(s0, e, 64), pe = __shfl(pre, e, 64) - base;
        for (int t0 = 0; t0 < ne; t0 += 64) {
          const int t = t0 + lane;
          const int q = t < ne ? (staged ? bq[pe + t] : lq[se + t]) : INT_MAX;
          if (q <= p) ar[q] += ve * (staged ? bv[pe + t] : lv[se + t]);
        }
        wave_sync_lds();
      }
    }
    c = cn;
    vp = vn;
  }
  // the lanes' own products in a fixed tree order
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) self += __shfl_xor(self, o, 64);
  if (lane == 0) ar[p] += self;
  wave_sync_lds();
  double* grow = Gl + wv * (int64_t)m;
  for (int q = lane; q <= p; q += 64) grow[q] = ar[q];
}

// G = scale * Gl + shift * E for steps without heavy columns (Gl lower rows).
__global__ __launch_bounds__(kT) void split_light_only_kernel(const double* __restrict__ Gl,
                                                              const int32_t* __restrict__ idx,
                                                              int m, int nsteps, double scale,
                                                              double shift, int overlap,
                                                              double* __restrict__ G) {
  const int64_t total = (int64_t)nsteps * m * m;
  for (int64_t g = (int64_t)blockIdx.x * kT + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * kT) {
    const int64_t k = g / ((int64_t)m * m);
    const int r = (int)((g / m) % m), c = (int)(g % m);
    if (c > r) continue;
    const int32_t* ix = idx + k * m;
    const bool on = overlap ? ix[r] == ix[c] : r == c;
    const double v = scale * Gl[g] + (on ? shift : 0.0);
    G[k * m * m + (int64_t)r * m + c] = v;
    G[k * m * m + (int64_t)c * m + r] = v;
  }
}

__global__ __launch_bounds__(kT) void iota_steps_kernel(int32_t* __restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    out[i] = (int32_t)i;
}

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(4096, (n + kT - 1) / kT)); }

}  // namespace

size_t csr_split_prepare_ints(const CsrView& A) {
  return (size_t)A.cols * 2 + kHist + ((A.cols + kScanChunk - 1) / kScanChunk) + 8;
}

hipError_t csr_split_prepare(const CsrView& A, int* ws, CsrSplitInfo* info, hipStream_t st) {
  int* cnt = ws;
  int* hmap = cnt + A.cols;
  int* hist = hmap + A.cols;
  const int nblk = (int)((A.cols + kScanChunk - 1) / kScanChunk);
  int* blk = hist + kHist;
  int* stats = blk + nblk;
  hipLaunchKernelGGL(zero_ints_kernel, dim3(grid_for(A.cols + kHist)), dim3(kT), 0, st, cnt,
                     (int64_t)A.cols, 0);
  hipLaunchKernelGGL(zero_ints_kernel, dim3(grid_for(kHist)), dim3(kT), 0, st, hist,
                     (int64_t)kHist, 0);
  hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(kT), 0, st, stats, (int64_t)8, 0);
  // popularity from every stride-th row (kSampleRows to 2 kSampleRows - 1
  // rows); a heavy column appears in at least 1/64 of the sampled rows (and
  // twice)
  const int64_t stride = std::max<int64_t>(1, A.rows / kSampleRows);
  const int64_t nsample = (A.rows + stride - 1) / stride;
  const int tmin = (int)std::max<int64_t>(2, nsample / 64);
  if (A.nnz > 0)
    hipLaunchKernelGGL(col_count_kernel, dim3(grid_for(nsample * 64)), dim3(kT), 0, st, A.rowptr,
                       A.colidx, A.rows, stride, cnt);
  hipLaunchKernelGGL(count_hist_kernel, dim3(grid_for(A.cols)), dim3(kT), 0, st, cnt,
                     (int64_t)A.cols, tmin, hist);
  hipLaunchKernelGGL(heavy_threshold_kernel, dim3(1), dim3(kThrT), 0, st, hist, tmin, stats);
  hipLaunchKernelGGL(heavy_slots_kernel, dim3(nblk), dim3(kScanChunk), 0, st, cnt,
                     (int64_t)A.cols, stats, blk, hmap, 0);
  hipLaunchKernelGGL(heavy_slots_kernel, dim3(nblk), dim3(kScanChunk), 0, st, cnt,
                     (int64_t)A.cols, stats, blk, hmap, 1);
  hipLaunchKernelGGL(split_stats_kernel, dim3(grid_for(A.rows)), dim3(kT), 0, st, A.rowptr,
                     A.rows, stats);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int h[4] = {0, 0, 0, 0};
  e = hipMemcpyAsync(h, stats, sizeof h, hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  info->hmap = hmap;
  info->heavy = h[3];
  info->maxrow = std::max(h[1], 1);
  info->maxlight = info->maxrow;   // a bound on a row's light entries
  return hipSuccess;
}

SplitLayout csr_split_layout(const CsrSplitInfo& info, int64_t cols, int m, int nsteps) {
  SplitLayout L{};
  L.hp = info.heavy > 0 ? (info.heavy + 15) / 16 * 16 : 0;
  L.lcap = (int64_t)m * info.maxlight;
  L.nblk = (int)((cols + kScanCols - 1) / kScanCols);
  L.cs = (int64_t)L.nblk * kScanCols;
  // the panel Gram: the nsteps Grams of a launch (their 256-row parts) with
  // enough column slabs to give every CU a workgroup
  const int sets = m > 256 ? 2 + big_cross_steps(m) : 1;
  L.plan = plan_gram_f64(std::min(m, 256), std::max(L.hp, 16));
  const int kt = L.plan.kt;
  const int64_t width = std::max(L.hp, 16);
  int want = std::max(1, (256 + nsteps * sets - 1) / (nsteps * sets));
  int64_t chunk = (width + want - 1) / want;
  chunk = std::max<int64_t>(kt, (chunk + kt - 1) / kt * kt);
  L.plan.chunk = chunk;
  L.plan.nsplit = (int)((width + chunk - 1) / chunk);
  L.doubles = (size_t)nsteps * ((size_t)m * L.hp + (size_t)m * m + (size_t)L.lcap) +
              (size_t)nsteps * sets * gram_partial_doubles(L.plan);
  L.doubles = (L.doubles + 31) / 32 * 32;   // the ints that follow start 256-byte aligned
  L.ints = (size_t)nsteps * (2 * (size_t)L.cs + L.nblk + (size_t)L.lcap +
                             (size_t)m * info.maxrow + m + 512 + 4 * 256);
  return L;
}

hipError_t launch_csr_gram_split(const CsrView& A, const CsrSplitInfo& info, const int32_t* idx,
                                 int m, int nsteps, double scale, double shift, bool overlap,
                                 double* G, double* dws, int* iws, hipStream_t st) {
  if (m < 1 || m > kSplitMaxRows || nsteps < 1 || nsteps > 65535 ||
      A.cols > ((int64_t)1 << (31 - kRankBits)) || kSplitMaxRows > (1 << kRankBits))
    return hipErrorInvalidValue;
  const SplitLayout L = csr_split_layout(info, A.cols, m, nsteps);
  const int64_t cs = L.cs;
  double* Dh = dws;
  double* Gl = Dh + (size_t)nsteps * m * L.hp;
  double* lv = Gl + (size_t)nsteps * m * m;
  double* partials = lv + (size_t)nsteps * L.lcap;
  int* cnt = iws;   // 256-byte aligned (int4 reads of the tables)
  int* off = cnt + (size_t)nsteps * cs;
  int* bsum = off + (size_t)nsteps * cs;
  int* lq = bsum + (size_t)nsteps * L.nblk;
  int* ent = lq + (size_t)nsteps * L.lcap;
  int32_t* iota = ent + (size_t)nsteps * m * info.maxrow;
  int32_t* ia = iota + (size_t)nsteps * m;
  int32_t* ib = ia + (size_t)nsteps * 512;

  const int64_t waves = (int64_t)nsteps * m;
  const int wgrid = (int)((waves * 64 + kT - 1) / kT);
  const int nchunk = (info.maxrow + 63) / 64;
  const int cgrid = (int)((waves * nchunk * 64 + kT - 1) / kT);
  if (L.hp > 0)
    hipLaunchKernelGGL(zero_doubles_kernel, dim3(grid_for((int64_t)nsteps * m * L.hp)), dim3(kT),
                       0, st, Dh, (int64_t)nsteps * m * L.hp);
  if ((reinterpret_cast<uintptr_t>(iws) & 15) != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(zero_ints_kernel, dim3(grid_for(nsteps * cs)), dim3(kT), 0, st, cnt,
                     (int64_t)nsteps * cs, 0);
  hipLaunchKernelGGL(split_scatter_kernel, dim3(cgrid), dim3(kT), 0, st, A.rowptr, A.colidx,
                     A.vals, idx, m, nsteps, nchunk, info.hmap, Dh, L.hp, cnt, cs, ent,
                     info.maxrow);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(L.nblk, nsteps), dim3(kScanT), 0, st, cnt, cs, bsum,
                     L.nblk);
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(nsteps), dim3(kScanT), 0, st, bsum, L.nblk);
  hipLaunchKernelGGL(scan_apply_kernel, dim3(L.nblk, nsteps), dim3(kScanT), 0, st, cnt, cs, bsum,
                     L.nblk, off);
  hipLaunchKernelGGL(split_fill_kernel, dim3(cgrid), dim3(kT), 0, st, A.rowptr, A.vals, idx, m,
                     nsteps, nchunk, off, cs, ent, info.maxrow, lq, lv, L.lcap);
  hipLaunchKernelGGL(split_light_kernel, dim3(wgrid), dim3(kT), 0, st, A.rowptr, A.vals, idx, m,
                     nsteps, cnt, off, cs, ent, info.maxrow, lq, lv, L.lcap, Gl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (L.hp == 0) {
    hipLaunchKernelGGL(split_light_only_kernel, dim3(grid_for((int64_t)nsteps * m * m)), dim3(kT),
                       0, st, Gl, idx, m, nsteps, scale, shift, overlap ? 1 : 0, G);
    return hipGetLastError();
  }
  // the heavy part: the Gram of each step's m x Hp panel on the matrix cores
  // (rows k m .. k m + m - 1 of the stacked panels), plus the light rows
  hipLaunchKernelGGL(iota_steps_kernel, dim3(grid_for(waves)), dim3(kT), 0, st, iota, waves);
  const GramPlan& P = L.plan;
  if (m <= 256) {
    e = launch_gram_f64(P, Dh, L.hp, L.hp, iota, m, nullptr, partials, st, nsteps);
    if (e != hipSuccess) return e;
    return launch_gram_reduce(P, partials, idx, m, scale, shift, overlap, G, nullptr, st, 0,
                              nullptr, nsteps, Gl);
  }
  const size_t set = gram_partial_doubles(P);
  const int nc = big_cross_steps(m);
  e = launch_big_index(iota, m, ia, ib, st, nsteps);
  if (e == hipSuccess)
    e = launch_gram_f64(P, Dh, L.hp, L.hp, ia, 256, nullptr, partials, st, 2 * nsteps);
  if (e == hipSuccess)
    e = launch_gram_f64(P, Dh, L.hp, L.hp, ib, 256, nullptr, partials + 2 * nsteps * set, st,
                        nc * nsteps);
  if (e != hipSuccess) return e;
  return launch_gram_reduce_big(P, partials, idx, m, scale, shift, overlap, G, nullptr, st, 0,
                                nullptr, nsteps, Gl);
}

}  // namespace cabcd
