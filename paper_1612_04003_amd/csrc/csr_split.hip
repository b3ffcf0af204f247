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
//     tables indexed by the column id count a step's entries per column (the
//     counting atomic also gives each entry a slot in its column's list), an
//     exclusive scan of the counts lays the lists of (row, value) out in
//     column order, and each list is then sorted by row (a thread per short
//     list, a wave per long one; the rows of a list are distinct, so the
//     order is unique).  One wave per gathered row p adds, entry by entry in
//     the row's column order, value_p value_q into an LDS row of p's products
//     for the rows q <= p: the first rank_p + 1 entries of the entry's sorted
//     list (a column only p holds adds value_p^2, summed by the lanes and
//     then in a fixed tree).  Only the sum_c nnz_c(I)^2 / 2 products of the
//     light columns are read, every sum runs in a fixed order (no float
//     atomics), and the light row is added to the dense partial sums in the
//     reduction.
// The companion update of such a step (out += gamma Y^T delta) reuses the
// panel and the sorted lists: one writer per column, every sum in row order.
// Heavy slots are numbered in column order; the heavy columns are picked from
// the column counts of a sample of the rows: any split gives the same Gram,
// the choice only affects speed.
#include "internal.h"

#include <algorithm>

namespace cabcd {
namespace {

constexpr int kT = 256;               // threads of the helper kernels
constexpr int kHeavyMax = 512;        // panel columns at most
constexpr int kPanelSteps = 16;       // steps per launch the panel slabs are sized for
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
                                                                 int* __restrict__ hmap,
                                                                 int* __restrict__ hcol, int pass) {
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
  if (heavy) hcol[off + below] = (int)c;
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

// The scans carry three counts per column: its entries (the list offsets),
// and whether its list is short (2..kShortList entries: sorted a thread each)
// or long (more: a wave each), so each step's two lists of lists are laid out
// in column order too.  bsum[(3 k + j) nblk + block], j = 0, 1, 2.
constexpr int kShortList = 16;
__device__ __forceinline__ int is_short(int c) { return c >= 2 && c <= kShortList ? 1 : 0; }
__device__ __forceinline__ int is_long(int c) { return c > kShortList ? 1 : 0; }

__global__ __launch_bounds__(kScanT) void scan_sums_kernel(const int* __restrict__ cnt,
                                                           int64_t cs, int* __restrict__ bsum,
                                                           int nblk) {
  __shared__ int sh[kScanT / 64];
  const int k = blockIdx.y;
  const int4* p = reinterpret_cast<const int4*>(cnt + (int64_t)k * cs +
                                                (int64_t)blockIdx.x * kScanCols);
  int v = 0, vs = 0, vl = 0;
#pragma unroll
  for (int q = 0; q < kScanCols / (4 * kScanT); ++q) {
    const int4 c = p[q * kScanT + threadIdx.x];
    v += c.x + c.y + c.z + c.w;
    vs += is_short(c.x) + is_short(c.y) + is_short(c.z) + is_short(c.w);
    vl += is_long(c.x) + is_long(c.y) + is_long(c.z) + is_long(c.w);
  }
  int t0, t1, t2;
  wg_excl_scan(v, sh, t0);
  wg_excl_scan(vs, sh, t1);
  wg_excl_scan(vl, sh, t2);
  if (threadIdx.x == 0) {
    bsum[(3 * (int64_t)k + 0) * nblk + blockIdx.x] = t0;
    bsum[(3 * (int64_t)k + 1) * nblk + blockIdx.x] = t1;
    bsum[(3 * (int64_t)k + 2) * nblk + blockIdx.x] = t2;
  }
}

// Workgroup (k, j) scans count j of step k; the list totals go to
// segn[2 k] (short) and segn[2 k + 1] (long).
__global__ __launch_bounds__(kScanT) void scan_blocks_kernel(int* __restrict__ bsum, int nblk,
                                                             int* __restrict__ segn) {
  __shared__ int sh[kScanT / 64];
  const int k = blockIdx.x, j = blockIdx.y;
  int* b = bsum + (3 * (int64_t)k + j) * nblk;
  int carry = 0;
  for (int q0 = 0; q0 < nblk; q0 += kScanT) {
    const int q = q0 + (int)threadIdx.x;
    const int v = q < nblk ? b[q] : 0;
    int total;
    const int r = wg_excl_scan(v, sh, total);
    if (q < nblk) b[q] = carry + r;
    carry += total;
  }
  if (j > 0 && threadIdx.x == 0) segn[2 * k + j - 1] = carry;
}

// A list of two or more entries: its start, length and column.
struct Seg {
  int start, n, col;
};

__global__ __launch_bounds__(kScanT) void scan_apply_kernel(const int* __restrict__ cnt,
                                                            int64_t cs,
                                                            const int* __restrict__ bsum,
                                                            int nblk, int* __restrict__ off,
                                                            Seg* __restrict__ segs,
                                                            int64_t segcap, Seg* __restrict__ lsegs,
                                                            int64_t lsegcap) {
  __shared__ int sh[kScanT / 64];
  const int k = blockIdx.y;
  segs += (int64_t)k * segcap;
  lsegs += (int64_t)k * lsegcap;
  const int64_t base = (int64_t)k * cs + (int64_t)blockIdx.x * kScanCols;
  const int4* p = reinterpret_cast<const int4*>(cnt + base);
  int carry = bsum[(3 * (int64_t)k + 0) * nblk + blockIdx.x];
  int carrys = bsum[(3 * (int64_t)k + 1) * nblk + blockIdx.x];
  int carryl = bsum[(3 * (int64_t)k + 2) * nblk + blockIdx.x];
#pragma unroll
  for (int q = 0; q < kScanCols / (4 * kScanT); ++q) {
    const int4 c = p[q * kScanT + threadIdx.x];
    const int cc[4] = {c.x, c.y, c.z, c.w};
    int t0, t1, t2;
    int pre = carry + wg_excl_scan(c.x + c.y + c.z + c.w, sh, t0);
    int ps = carrys + wg_excl_scan(is_short(c.x) + is_short(c.y) + is_short(c.z) +
                                       is_short(c.w), sh, t1);
    int pl = carryl + wg_excl_scan(is_long(c.x) + is_long(c.y) + is_long(c.z) + is_long(c.w),
                                   sh, t2);
    int* o = off + base + (int64_t)q * 4 * kScanT + 4 * threadIdx.x;
    const int col0 = blockIdx.x * kScanCols + q * 4 * kScanT + 4 * threadIdx.x;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (cc[u] > 0) o[u] = pre;
      if (is_short(cc[u])) segs[ps++] = Seg{pre, cc[u], col0 + u};
      if (is_long(cc[u])) lsegs[pl++] = Seg{pre, cc[u], col0 + u};
      pre += cc[u];
    }
    carry += t0;
    carrys += t1;
    carryl += t2;
  }
}

// Each light entry goes to its rank's position in its column's list (off[c]
// is the list's start), as the key (row << kEntryBits) | (entry's index in
// its row) with its value.
constexpr int kEntryBits = 22;   // rows have fewer than 2^22 entries
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
  lq[(int64_t)k * lcap + pos] = (p << kEntryBits) | (int)(j - a);
  lv[(int64_t)k * lcap + pos] = vals[j];
}

// One thread per short list (2..kShortList entries; workgroup row k takes
// step k's lists): its keys and values in registers, each entry's
// position = the number of smaller keys (the keys of a list are distinct),
// written back sorted; each entry's position goes to rk[k][p][e].
__global__ __launch_bounds__(kT) void split_sort_short_kernel(const Seg* __restrict__ segs,
                                                              const int* __restrict__ segn,
                                                              int64_t segcap, int nsteps,
                                                              int* __restrict__ lq,
                                                              double* __restrict__ lv,
                                                              int64_t lcap, int* __restrict__ rk,
                                                              int m, int maxrow) {
  const int64_t nt = (int64_t)gridDim.x * kT;
  const int64_t t0 = (int64_t)blockIdx.x * kT + threadIdx.x;
  const int k = blockIdx.y;   // one row of workgroups per step
  {
    const int ns = segn[2 * k];
    for (int64_t i = t0; i < ns; i += nt) {
      const Seg sg = segs[(int64_t)k * segcap + i];
      int* q = lq + (int64_t)k * lcap + sg.start;
      double* v = lv + (int64_t)k * lcap + sg.start;
      const int n = sg.n;
      int key[kShortList], pos[kShortList];
      double val[kShortList];
#pragma unroll
      for (int u = 0; u < kShortList; ++u) {
        key[u] = u < n ? q[u] : INT_MAX;
        val[u] = u < n ? v[u] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kShortList; ++u) {
        int r = 0;
#pragma unroll
        for (int w = 0; w < kShortList; ++w) r += key[w] < key[u] ? 1 : 0;
        pos[u] = r;
      }
#pragma unroll
      for (int u = 0; u < kShortList; ++u) {
        if (u < n) {
          q[pos[u]] = key[u];
          v[pos[u]] = val[u];
          rk[((int64_t)k * m + (key[u] >> kEntryBits)) * maxrow +
             (key[u] & ((1 << kEntryBits) - 1))] = pos[u];
        }
      }
    }
  }
}

// Orders one wave's LDS writes before its other lanes' reads: the LDS runs a
// wave's instructions in order, so keeping the compiler from moving memory
// accesses across this point is enough (no wait for outstanding loads).
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_wave_barrier();
  asm volatile("" ::: "memory");
}

// Lane `e` (wave-uniform) of a per-lane value.
__device__ __forceinline__ int lane_of(int v, int e) { return __builtin_amdgcn_readlane(v, e); }
__device__ __forceinline__ double lane_of(double v, int e) {
  const int64_t u = __builtin_bit_cast(int64_t, v);
  const int lo = __builtin_amdgcn_readlane((int)(uint32_t)u, e);
  const int hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), e);
  return __builtin_bit_cast(double, (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// One wave per long list (more than kShortList entries; workgroup row k takes
// step k's lists): the list is sorted by its keys, i.e. by row, and every
// entry's position in its sorted list goes to rk[k][p][e].  The keys of a
// list are distinct (a row holds a column once), so each entry's position is
// the number of smaller keys, counted against the list's keys in LDS.
constexpr int kSortMax = 512;               // list length <= rows of a step
constexpr int kSortGrid = 64;               // workgroups of a sort per step
constexpr int kUpdateGrid = 128;            // workgroups of a list pass of the update
constexpr int kSortPer = kSortMax / 64;
__global__ __launch_bounds__(kT) void split_sort_kernel(const Seg* __restrict__ segs,
                                                        const int* __restrict__ segn,
                                                        int64_t segcap, int nsteps,
                                                        int* __restrict__ lq,
                                                        double* __restrict__ lv, int64_t lcap,
                                                        int* __restrict__ rk, int m, int maxrow) {
  __shared__ int sk[kT / 64][kSortMax];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nw = (int64_t)gridDim.x * (kT / 64);
  const int64_t w0 = (int64_t)blockIdx.x * (kT / 64) + wave;
  int* keys = sk[wave];
  const int k = blockIdx.y;   // one row of workgroups per step
  {
    const int ns = segn[2 * k + 1];
    for (int64_t i = w0; i < ns; i += nw) {
      const Seg sg = segs[(int64_t)k * segcap + i];
      int* q = lq + (int64_t)k * lcap + sg.start;
      double* v = lv + (int64_t)k * lcap + sg.start;
      const int n = sg.n;
      int key[kSortPer], pos[kSortPer];
      double val[kSortPer];
#pragma unroll
      for (int u = 0; u < kSortPer; ++u) {
        const int t = lane + 64 * u;
        key[u] = t < n ? q[t] : INT_MAX;
        val[u] = t < n ? v[t] : 0.0;
        pos[u] = 0;
        if (t < n) keys[t] = key[u];
      }
      wave_sync_lds();
      for (int t = 0; t < n; ++t) {
        const int kt = keys[t];
#pragma unroll
        for (int u = 0; u < kSortPer; ++u) pos[u] += kt < key[u] ? 1 : 0;
      }
      wave_sync_lds();   // the keys are read before the next list overwrites them
#pragma unroll
      for (int u = 0; u < kSortPer; ++u) {
        if (lane + 64 * u < n) {
          q[pos[u]] = key[u];
          v[pos[u]] = val[u];
          rk[((int64_t)k * m + (key[u] >> kEntryBits)) * maxrow +
             (key[u] & ((1 << kEntryBits) - 1))] = pos[u];
        }
      }
    }
  }
}

// One wave per (step k, gathered row p): row p of the light part,
// Gl[k][p][q] = sum over the light columns c of row p, in the row's column
// order, of v_pc v_qc for q <= p.  The lists are sorted by row, so the rows
// q <= p of a list are its first rank + 1 entries, rank = p's position in it.
// The row's entries are taken 64 at a time (the next batch's columns and
// values are loaded while one is applied): their list extents and ranks are
// loaded by the lanes together, runs of list prefixes that fit the stage are
// copied into LDS by the whole wave (one staged element a lane and load,
// eight loads in flight), and the entries are then applied one after the
// other from LDS.  A column's list holds a gathered row at most once, so the
// lanes of one entry add to distinct q and the order of every sum is the
// row's column order.  The row is accumulated in LDS and written whole (zeros
// where no light column is shared).
constexpr int kSplitMaxRows = 512;
constexpr int kStage = 512;                 // staged list elements per wave
constexpr int kCopyUnroll = kStage / 64;    // loads in flight a lane while staging
constexpr int kLightWaves = kT / 64;
__global__ __launch_bounds__(kT) void split_light_kernel(
    const int64_t* __restrict__ rowptr, const double* __restrict__ vals,
    const int32_t* __restrict__ idx, int m, int nsteps, const int* __restrict__ cnt,
    const int* __restrict__ off, int64_t cs, const int* __restrict__ ent,
    const int* __restrict__ rk, int maxrow, const int* __restrict__ lq,
    const double* __restrict__ lv, int64_t lcap, double* __restrict__ Gl) {
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
  const int* rkrow = rk + wv * (int64_t)maxrow;
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
    const int rank = c >= 0 ? rkrow[e0 - a + lane] : 0;   // read only when nc >= 2
    const int64_t jn = e0 + 64 + lane;
    int cn = jn < b ? erow[jn - a] : -1;
    cn = cn < 0 ? -1 : cn >> kRankBits;
    const double vn = cn >= 0 ? vals[jn] : 0.0;
    if (nc == 1) self = fma(vp, vp, self);
    const int n = nc >= 2 ? rank + 1 : 0;   // the list's rows q <= p
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
      const int first = __builtin_amdgcn_readfirstlane(__ffsll((long long)todo) - 1);
      const int base = lane_of(pre, first);
      unsigned long long run = 0ull;
      {
        unsigned long long t = todo;
        while (t != 0ull) {
          const int e = __builtin_amdgcn_readfirstlane(__ffsll((long long)t) - 1);
          if (lane_of(pre, e) + lane_of(n, e) - base > kStage) break;
          run |= 1ull << e;
          t &= t - 1ull;
        }
      }
      const bool staged = run != 0ull;
      if (staged) {
        // each entry writes its elements' global positions into the stage,
        // then every lane copies staged elements lane, lane + 64, ...
        const int last = __builtin_amdgcn_readfirstlane(63 - __clzll((long long)run));
        const int total = lane_of(pre, last) + lane_of(n, last) - base;
        if ((run >> lane) & 1ull)
          for (int t = 0; t < n; ++t) bq[pre - base + t] = s0 + t;
        wave_sync_lds();
        int g[kCopyUnroll];
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) {
          const int jj = u * 64 + lane;
          g[u] = jj < total ? bq[jj] : -1;
        }
        // every lane loads (element 0 for the idle ones), so all loads are
        // in flight before any is used
        int qv[kCopyUnroll];
        double vv[kCopyUnroll];
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) {
          const int gi = g[u] >= 0 ? g[u] : 0;
          qv[u] = lq[gi];
          vv[u] = lv[gi];
        }
#pragma unroll
        for (int u = 0; u < kCopyUnroll; ++u) {
          const int jj = u * 64 + lane;
          if (jj < total) {
            bq[jj] = qv[u] >> kEntryBits;
            bv[jj] = vv[u];
          }
        }
        wave_sync_lds();
      } else {
        run = 1ull << first;
      }
      todo &= ~run;
      while (run != 0ull) {
        const int e = __builtin_amdgcn_readfirstlane(__ffsll((long long)run) - 1);
        run &= run - 1ull;
        const int ne = lane_of(n, e);
        const double ve = lane_of(vp, e);
        const int se = lane_of(s0, e), pe = lane_of(pre, e) - base;
        for (int t0 = 0; t0 < ne; t0 += 64) {
          const int t = t0 + lane;
          const int q = t < ne ? (staged ? bq[pe + t] : lq[se + t] >> kEntryBits) : INT_MAX;
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

// The companion update out[c] += gamma sum_p Y[p][c] delta_p of an outer step
// whose Gram came from a split launch, with one writer per column and every
// sum in a fixed order (no atomics):
//   * heavy columns: the step's dense panel, one wave per heavy slot h, lane
//     l summing rows l, l + 64, ..., then a fixed tree;
//   * light columns of one entry: added by that entry (a pass over the
//     gathered entries);
//   * short lists: a thread each, the list (sorted by row) summed in order;
//   * long lists: a wave each, lane l summing entries l, l + 64, ..., then a
//     fixed tree.
__device__ __forceinline__ double wave_tree_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

struct UpdateArgs {
  const int64_t* rowptr;
  const double* vals;
  const int32_t* idx;
  int m, nchunk, maxrow, hp, heavy;
  const double* Dh;
  const int* hcol;
  const int* ent;
  const int* cnt;
  const Seg* segs;
  const Seg* lsegs;
  const int* segn;   // [0]: short lists, [1]: long lists
  const int* lq;
  const double* lv;
  const double* delta;
  double gamma;
  double* out;
  int bh, bs, bq;    // workgroups of the heavy, single and short parts (then long)
};

// One launch, four parts by workgroup range (each writes distinct columns).
__global__ __launch_bounds__(kT) void split_update_kernel(UpdateArgs u) {
  const int lane = threadIdx.x & 63;
  int blk = blockIdx.x;
  if (blk < u.bh) {   // heavy: one wave per slot
    const int h = (int)(((int64_t)blk * kT + threadIdx.x) >> 6);
    if (h >= u.heavy) return;
    double t = 0.0;
    for (int p = lane; p < u.m; p += 64) t = fma(u.Dh[(int64_t)p * u.hp + h], u.delta[p], t);
    t = wave_tree_sum(t);
    if (lane == 0) u.out[u.hcol[h]] += u.gamma * t;
    return;
  }
  blk -= u.bh;
  if (blk < u.bs) {   // columns of one gathered entry
    const int64_t wv = ((int64_t)blk * kT + threadIdx.x) >> 6;
    if (wv >= (int64_t)u.m * u.nchunk) return;
    const int p = (int)(wv / u.nchunk), ch = (int)(wv % u.nchunk);
    const int i = u.idx[p];
    const int64_t a = u.rowptr[i], b = u.rowptr[i + 1];
    const int64_t j = a + 64 * ch + lane;
    if (j >= b) return;
    const int e = u.ent[(int64_t)p * u.maxrow + (j - a)];
    if (e < 0) return;   // a heavy column
    const int c = e >> kRankBits;
    if (u.cnt[c] == 1) u.out[c] += u.gamma * (u.vals[j] * u.delta[p]);
    return;
  }
  blk -= u.bs;
  if (blk < u.bq) {   // short lists: a thread each
    const int64_t nt = (int64_t)u.bq * kT;
    const int ns = u.segn[0];
    for (int64_t i = (int64_t)blk * kT + threadIdx.x; i < ns; i += nt) {
      const Seg sg = u.segs[i];
      int q[kShortList];
      double v[kShortList];
#pragma unroll
      for (int w = 0; w < kShortList; ++w) {
        q[w] = w < sg.n ? u.lq[sg.start + w] >> kEntryBits : 0;
        v[w] = w < sg.n ? u.lv[sg.start + w] : 0.0;
      }
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kShortList; ++w)
        if (w < sg.n) t = fma(v[w], u.delta[q[w]], t);
      u.out[sg.col] += u.gamma * t;
    }
    return;
  }
  blk -= u.bq;   // long lists: a wave each
  const int64_t nw = ((int64_t)(gridDim.x - u.bh - u.bs - u.bq) * kT) >> 6;
  const int nl = u.segn[1];
  for (int64_t i = ((int64_t)blk * kT + threadIdx.x) >> 6; i < nl; i += nw) {
    const Seg sg = u.lsegs[i];
    double t = 0.0;
    for (int w = lane; w < sg.n; w += 64)
      t = fma(u.lv[sg.start + w], u.delta[u.lq[sg.start + w] >> kEntryBits], t);
    t = wave_tree_sum(t);
    if (lane == 0) u.out[sg.col] += u.gamma * t;
  }
}

__global__ __launch_bounds__(kT) void iota_steps_kernel(int32_t* __restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    out[i] = (int32_t)i;
}

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(4096, (n + kT - 1) / kT)); }

}  // namespace

size_t csr_split_prepare_ints(const CsrView& A) {
  return (size_t)A.cols * 2 + kHist + ((A.cols + kScanChunk - 1) / kScanChunk) + 8 + kHeavyMax;
}

hipError_t csr_split_prepare(const CsrView& A, int* ws, CsrSplitInfo* info, hipStream_t st) {
  int* cnt = ws;
  int* hmap = cnt + A.cols;
  int* hist = hmap + A.cols;
  const int nblk = (int)((A.cols + kScanChunk - 1) / kScanChunk);
  int* blk = hist + kHist;
  int* stats = blk + nblk;
  int* hcol = stats + 8;
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
                     (int64_t)A.cols, stats, blk, hmap, hcol, 0);
  hipLaunchKernelGGL(heavy_slots_kernel, dim3(nblk), dim3(kScanChunk), 0, st, cnt,
                     (int64_t)A.cols, stats, blk, hmap, hcol, 1);
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
  info->hcol = hcol;
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
  // the panel Gram: the nsteps Grams of a launch (their 256-row parts), in
  // column slabs sized so that a launch of kPanelSteps steps gives every CU a
  // workgroup.  The slabs (and so every sum's order) do not depend on how many
  // steps a launch actually takes: a run gives the same result however its
  // steps are batched or split between calls.
  const int sets = m > 256 ? 2 + big_cross_steps(m) : 1;
  L.plan = plan_gram_f64(std::min(m, 256), std::max(L.hp, 16));
  const int kt = L.plan.kt;
  const int64_t width = std::max(L.hp, 16);
  const int want = std::max(1, (256 + kPanelSteps * sets - 1) / (kPanelSteps * sets));
  int64_t chunk = (width + want - 1) / want;
  chunk = std::max<int64_t>(kt, (chunk + kt - 1) / kt * kt);
  L.plan.chunk = chunk;
  L.plan.nsplit = (int)((width + chunk - 1) / chunk);
  L.doubles = (size_t)nsteps * ((size_t)m * L.hp + (size_t)m * m + (size_t)L.lcap) +
              (size_t)nsteps * sets * gram_partial_doubles(L.plan);
  L.doubles = (L.doubles + 31) / 32 * 32;   // the ints that follow start 256-byte aligned
  L.ints = (size_t)nsteps * (2 * (size_t)L.cs + 3 * (size_t)L.nblk + (size_t)L.lcap +
                             2 * (size_t)m * info.maxrow + 3 * (size_t)(L.lcap / 2 + 1) +
                             3 * (size_t)(L.lcap / (kShortList + 1) + 1) + 2 + m + 512 + 4 * 256);
  return L;
}

// The buffers of one split launch of nsteps steps inside its scratch.
struct SplitBufs {
  double *Dh, *Gl, *lv, *partials;
  int *cnt, *off, *bsum, *lq, *ent, *rk, *segn;
  Seg *segs, *lsegs;
  int64_t segcap, lsegcap;
  int32_t *iota, *ia, *ib;
};
SplitBufs split_bufs(const SplitLayout& L, const CsrSplitInfo& info, int m, int nsteps,
                     double* dws, int* iws) {
  SplitBufs B{};
  B.Dh = dws;
  B.Gl = B.Dh + (size_t)nsteps * m * L.hp;
  B.lv = B.Gl + (size_t)nsteps * m * m;
  B.partials = B.lv + (size_t)nsteps * L.lcap;
  B.cnt = iws;   // 256-byte aligned (int4 reads of the tables)
  B.off = B.cnt + (size_t)nsteps * L.cs;
  B.bsum = B.off + (size_t)nsteps * L.cs;
  B.lq = B.bsum + (size_t)nsteps * 3 * L.nblk;
  B.ent = B.lq + (size_t)nsteps * L.lcap;
  B.rk = B.ent + (size_t)nsteps * m * info.maxrow;
  B.segcap = L.lcap / 2 + 1;                    // lists of >= 2 entries
  B.lsegcap = L.lcap / (kShortList + 1) + 1;    // lists of > kShortList
  B.segs = reinterpret_cast<Seg*>(B.rk + (size_t)nsteps * m * info.maxrow);
  B.lsegs = B.segs + (size_t)nsteps * B.segcap;
  B.segn = reinterpret_cast<int*>(B.lsegs + (size_t)nsteps * B.lsegcap);
  B.iota = B.segn + 2 * nsteps;
  B.ia = B.iota + (size_t)nsteps * m;
  B.ib = B.ia + (size_t)nsteps * 512;
  return B;
}

hipError_t launch_csr_update_split(const CsrView& A, const CsrSplitInfo& info,
                                   const int32_t* idx, int m, int nsteps, int step,
                                   const double* delta, double gamma, double* out, double* dws,
                                   int* iws, hipStream_t st) {
  if (m < 1 || m > kSplitMaxRows || step < 0 || step >= nsteps) return hipErrorInvalidValue;
  const SplitLayout L = csr_split_layout(info, A.cols, m, nsteps);
  const SplitBufs B = split_bufs(L, info, m, nsteps, dws, iws);
  UpdateArgs u{};
  u.rowptr = A.rowptr;
  u.vals = A.vals;
  u.idx = idx;
  u.m = m;
  u.nchunk = (info.maxrow + 63) / 64;
  u.maxrow = info.maxrow;
  u.hp = L.hp;
  u.heavy = info.heavy;
  u.Dh = B.Dh + (size_t)step * m * L.hp;
  u.hcol = info.hcol;
  u.ent = B.ent + (size_t)step * m * info.maxrow;
  u.cnt = B.cnt + step * L.cs;
  u.segs = B.segs + step * B.segcap;
  u.lsegs = B.lsegs + step * B.lsegcap;
  u.segn = B.segn + 2 * step;
  u.lq = B.lq + step * L.lcap;
  u.lv = B.lv + step * L.lcap;
  u.delta = delta;
  u.gamma = gamma;
  u.out = out;
  u.bh = (info.heavy + kT / 64 - 1) / (kT / 64);
  u.bs = (int)(((int64_t)m * u.nchunk * 64 + kT - 1) / kT);
  u.bq = kUpdateGrid;
  hipLaunchKernelGGL(split_update_kernel, dim3(u.bh + u.bs + u.bq + kUpdateGrid), dim3(kT), 0,
                     st, u);
  return hipGetLastError();
}

hipError_t launch_csr_gram_split(const CsrView& A, const CsrSplitInfo& info, const int32_t* idx,
                                 int m, int nsteps, double scale, double shift, bool overlap,
                                 double* G, double* dws, int* iws, hipStream_t st) {
  if (m < 1 || m > kSplitMaxRows || nsteps < 1 || nsteps > 65535 ||
      A.cols > ((int64_t)1 << (31 - kRankBits)) || kSplitMaxRows > (1 << kRankBits) ||
      info.maxrow >= (1 << kEntryBits) || kSplitMaxRows > (1 << (31 - kEntryBits)))
    return hipErrorInvalidValue;
  const SplitLayout L = csr_split_layout(info, A.cols, m, nsteps);
  const int64_t cs = L.cs;
  const SplitBufs SB = split_bufs(L, info, m, nsteps, dws, iws);
  double *Dh = SB.Dh, *Gl = SB.Gl, *lv = SB.lv, *partials = SB.partials;
  int *cnt = SB.cnt, *off = SB.off, *bsum = SB.bsum, *lq = SB.lq, *ent = SB.ent, *rk = SB.rk;
  int* segn = SB.segn;
  Seg *segs = SB.segs, *lsegs = SB.lsegs;
  const int64_t segcap = SB.segcap, lsegcap = SB.lsegcap;
  int32_t *iota = SB.iota, *ia = SB.ia, *ib = SB.ib;

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
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(nsteps, 3), dim3(kScanT), 0, st, bsum, L.nblk,
                     segn);
  hipLaunchKernelGGL(scan_apply_kernel, dim3(L.nblk, nsteps), dim3(kScanT), 0, st, cnt, cs, bsum,
                     L.nblk, off, segs, segcap, lsegs, lsegcap);
  hipLaunchKernelGGL(split_fill_kernel, dim3(cgrid), dim3(kT), 0, st, A.rowptr, A.vals, idx, m,
                     nsteps, nchunk, off, cs, ent, info.maxrow, lq, lv, L.lcap);
  hipLaunchKernelGGL(split_sort_short_kernel, dim3(kSortGrid, nsteps), dim3(kT), 0, st, segs,
                     segn, segcap, nsteps, lq, lv, L.lcap, rk, m, info.maxrow);
  hipLaunchKernelGGL(split_sort_kernel, dim3(kSortGrid, nsteps), dim3(kT), 0, st, lsegs, segn,
                     lsegcap, nsteps, lq, lv, L.lcap, rk, m, info.maxrow);
  hipLaunchKernelGGL(split_light_kernel, dim3(wgrid), dim3(kT), 0, st, A.rowptr, A.vals, idx, m,
                     nsteps, cnt, off, cs, ent, rk, info.maxrow, lq, lv, L.lcap, Gl);
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
