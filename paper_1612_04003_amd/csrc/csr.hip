// CSR kernels: the sparse s-step Gram (row-gather SpGEMM), the companion
// scatter updates and the row products, for A stored as CSR with FP64 values.
//
// The paper stores X in CSR and forms the Gram with sparse BLAS on each rank
// (Section 5.2); the b x n sampled matrix has b f n non-zeros (Thm. bcd1dcol
// proof).  Here one workgroup owns one gathered row p: it loads the row into an
// LDS hash table (column -> value), and its waves take the rows q <= p, probe
// the table with q's entries and reduce the products with a fixed shuffle tree,
// giving G[p][q] directly (no partials, deterministic).  Rows longer than the
// table are processed in table-sized chunks whose dot products are added in
// chunk order.  Y u is the same pass with u gathered at the row's columns.
//
// The walks are latency-bound (each probe waits for the row's column indices),
// so a launch can cover the Grams of several future outer steps at once: the
// Gram depends on the sampled indices only, and one workgroup per (step, row)
// gives the machine enough independent walks to hide the latency.  The row
// extents of the gathered rows sit in LDS, and each lane loads four entries of
// a probed row before probing.
//
// The companion updates (primal r += Y^T delta, dual w -= Y^T delta/(lambda n))
// and the exact recomputations scatter into the columns of the gathered rows;
// columns shared by several rows (popular features) meet in FP64 atomic adds,
// so these results are reproducible up to the order of those additions.
#include "internal.h"

#include <algorithm>

namespace cabcd {
namespace {

constexpr int kCsrThreads = 256;
constexpr int kCsrWaves = kCsrThreads / 64;
constexpr int kHashSlots = 4096;            // power of two
constexpr int kChunk = kHashSlots / 2;      // row entries per table fill
constexpr int kMaxBatches = 4;              // m <= 4 * 64 * kCsrWaves = 1024
constexpr int kMaxRows = kMaxBatches * 64 * kCsrWaves;
constexpr int kProbeU = 4;                  // row entries per lane loaded together

__device__ __forceinline__ unsigned hash_col(int c) {
  return ((unsigned)c * 2654435761u) >> (32 - 12);   // log2(kHashSlots) = 12
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Step blockIdx.y uses idx + step * idx_stride and writes G + step * g_stride.
__global__ __launch_bounds__(kCsrThreads) void csr_gram_kernel(
    const int64_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
    const double* __restrict__ vals, const int32_t* __restrict__ idx, int m,
    int64_t idx_stride, const double* __restrict__ u, double scale, double shift, int overlap,
    double* __restrict__ G, int64_t g_stride, double* __restrict__ Yu) {
  __shared__ int keys[kHashSlots];
  __shared__ double hv[kHashSlots];
  __shared__ int64_t ext[2][kMaxRows];     // row extents of the gathered rows
  idx += (int64_t)blockIdx.y * idx_stride;
  G += (int64_t)blockIdx.y * g_stride;
  const int p = m - 1 - (int)blockIdx.x;   // the longest triangles start first
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int q = threadIdx.x; q <= p; q += kCsrThreads) {
    const int iq = idx[q];
    ext[0][q] = rowptr[iq];
    ext[1][q] = rowptr[iq + 1];
  }
  __syncthreads();
  const int ip = idx[p];
  const int64_t p0 = ext[0][p], p1 = ext[1][p];

  if (Yu != nullptr && wave == 0) {
    double t = 0.0;
    for (int64_t k = p0 + lane; k < p1; k += 64) t = fma(vals[k], u[colidx[k]], t);
    t = wave_sum(t);
    if (lane == 0) Yu[p] = t;
  }

  // Row q = qb + wave + W*lane of batch qb = 256*bi is summed in mine[bi] of
  // that lane; rows are handled in batches of 64*W = 256 (m <= 1024 gives at
  // most kMaxBatches).  The table of row p is filled once per chunk of row p,
  // and the chunk results are added in chunk order.
  double mine[kMaxBatches];
#pragma unroll
  for (int bi = 0; bi < kMaxBatches; ++bi) mine[bi] = 0.0;
  for (int64_t c0 = p0;; c0 += kChunk) {
    const int64_t c1 = std::min(p1, c0 + kChunk);
    for (int s = threadIdx.x; s < kHashSlots; s += kCsrThreads) keys[s] = -1;
    __syncthreads();
    for (int64_t k = c0 + threadIdx.x; k < c1; k += kCsrThreads) {
      const int col = colidx[k];
      unsigned h = hash_col(col);
      while (atomicCAS(&keys[h], -1, col) != -1) h = (h + 1) & (kHashSlots - 1);
      hv[h] = vals[k];
    }
    __syncthreads();
#pragma unroll
    for (int bi = 0; bi < kMaxBatches; ++bi) {
      const int qb = bi * 64 * kCsrWaves;
      for (int j = 0; j < 64; ++j) {
        const int q = qb + wave + kCsrWaves * j;
        if (q > p) break;
        const int64_t q0 = ext[0][q], q1 = ext[1][q];
        double t = 0.0;
        for (int64_t kb = q0 + lane; kb < q1; kb += 64 * kProbeU) {
          int col[kProbeU];
          double val[kProbeU];
#pragma unroll
          for (int e = 0; e < kProbeU; ++e) {   // entries kb, kb + 64, ... of this lane
            const int64_t k = kb + 64 * e;
            col[e] = k < q1 ? colidx[k] : -1;
            val[e] = k < q1 ? vals[k] : 0.0;
          }
#pragma unroll
          for (int e = 0; e < kProbeU; ++e) {
            if (col[e] < 0) continue;
            unsigned h = hash_col(col[e]);
            int key;
            while ((key = keys[h]) != col[e] && key != -1) h = (h + 1) & (kHashSlots - 1);
            if (key == col[e]) t = fma(val[e], hv[h], t);
          }
        }
        t = wave_sum(t);
        if (lane == j) mine[bi] += t;
      }
    }
    __syncthreads();
    if (c1 >= p1) break;
  }
#pragma unroll
  for (int bi = 0; bi < kMaxBatches; ++bi) {
    const int q = bi * 64 * kCsrWaves + wave + kCsrWaves * lane;
    if (q <= p) {
      const bool on = overlap ? (idx[q] == ip) : (q == p);
      const double v = scale * mine[bi] + (on ? shift : 0.0);
      G[(int64_t)p * m + q] = v;
      G[(int64_t)q * m + p] = v;
    }
  }
}

// The Grams of several outer steps (no Y u) with kTP gathered rows per
// workgroup: the hash table maps a column to the values of the tile's rows at
// that column (zero where a row lacks it), so each probed row q is read once
// per tile instead of once per row of the tile, and one probe feeds kTP
// products.  Lane j of wave w keeps the kTP sums of rows q = w + W j (+ 256
// per batch) across table fills; chunks of the tile's entries are added in
// chunk order, so the result is deterministic.
constexpr int kTP = 3;                      // gathered rows per workgroup
constexpr int kTSlots = 2048;               // power of two
constexpr int kTChunk = kTSlots / 2;        // tile entries per table fill
constexpr int kTMaxRows = 512;              // m of this kernel

__device__ __forceinline__ unsigned hash_col_t(int c) {
  return ((unsigned)c * 2654435761u) >> (32 - 11);   // log2(kTSlots) = 11
}

__global__ __launch_bounds__(kCsrThreads) void csr_gram_tile_kernel(
    const int64_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
    const double* __restrict__ vals, const int32_t* __restrict__ idx, int m,
    int64_t idx_stride, double scale, double shift, int overlap, double* __restrict__ G,
    int64_t g_stride) {
  __shared__ int keys[kTSlots];
  __shared__ double hv[kTSlots][kTP];
  __shared__ int64_t ext[2][kTMaxRows];     // row extents of the gathered rows
  idx += (int64_t)blockIdx.y * idx_stride;
  G += (int64_t)blockIdx.y * g_stride;
  const int ntile = (m + kTP - 1) / kTP;
  const int p0 = kTP * (ntile - 1 - (int)blockIdx.x);   // the longest triangles start first
  const int qmax = min(m, p0 + kTP);                      // rows q < qmax meet the tile
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int q = threadIdx.x; q < qmax; q += kCsrThreads) {
    const int iq = idx[q];
    ext[0][q] = rowptr[iq];
    ext[1][q] = rowptr[iq + 1];
  }
  __syncthreads();
  // the tile's entries, row after row: row i starts at tbeg[i]
  int64_t tbeg[kTP + 1];
  tbeg[0] = 0;
#pragma unroll
  for (int i = 0; i < kTP; ++i)
    tbeg[i + 1] = tbeg[i] + (p0 + i < m ? ext[1][p0 + i] - ext[0][p0 + i] : 0);
  const int64_t tot = tbeg[kTP];

  double mine[2][kTP];   // q = qb + wave + W lane, batches qb = 0, 256
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int i = 0; i < kTP; ++i) mine[bi][i] = 0.0;
  for (int64_t c0 = 0;; c0 += kTChunk) {
    const int64_t c1 = min(tot, c0 + kTChunk);
    for (int sl = threadIdx.x; sl < kTSlots; sl += kCsrThreads) {
      keys[sl] = -1;
#pragma unroll
      for (int i = 0; i < kTP; ++i) hv[sl][i] = 0.0;
    }
    __syncthreads();
    for (int64_t e = c0 + threadIdx.x; e < c1; e += kCsrThreads) {
      int i = 0;
      int64_t eb = 0;                                     // tile row of entry e
#pragma unroll
      for (int r = 1; r < kTP; ++r)
        if (e >= tbeg[r]) {
          i = r;
          eb = tbeg[r];
        }
      const int64_t k = ext[0][p0 + i] + (e - eb);
      const int col = colidx[k];
      unsigned h = hash_col_t(col);
      for (;;) {
        const int old = atomicCAS(&keys[h], -1, col);
        if (old == -1 || old == col) break;
        h = (h + 1) & (kTSlots - 1);
      }
      hv[h][i] = vals[k];   // a column appears once per row: one writer per (slot, row)
    }
    __syncthreads();
    // A wave takes four probed rows at a time, sixteen lanes each, so the
    // per-row sums need four shuffle steps inside a sixteen-lane group; lane
    // 4 jj + s then collects the sums of group s.
    const int sub = lane >> 4, l16 = lane & 15;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
      const int qb = bi * 64 * kCsrWaves;
      for (int jj = 0; jj < 16; ++jj) {
        if (qb + wave + kCsrWaves * 4 * jj >= qmax) break;   // no row of this quartet
        const int q = qb + wave + kCsrWaves * (4 * jj + sub);
        const bool live = q < qmax;
        const int64_t q0 = live ? ext[0][q] : 0, q1 = live ? ext[1][q] : 0;
        double t[kTP];
#pragma unroll
        for (int i = 0; i < kTP; ++i) t[i] = 0.0;
        for (int64_t kb = q0 + l16; kb < q1; kb += 16 * kProbeU) {
          int col[kProbeU];
          double val[kProbeU];
#pragma unroll
          for (int u = 0; u < kProbeU; ++u) {
            const int64_t k = kb + 16 * u;
            col[u] = k < q1 ? colidx[k] : -1;
            val[u] = k < q1 ? vals[k] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < kProbeU; ++u) {
            if (col[u] < 0) continue;
            unsigned h = hash_col_t(col[u]);
            int key;
            while ((key = keys[h]) != col[u] && key != -1) h = (h + 1) & (kTSlots - 1);
            if (key == col[u]) {
#pragma unroll
              for (int i = 0; i < kTP; ++i) t[i] = fma(val[u], hv[h][i], t[i]);
            }
          }
        }
#pragma unroll
        for (int i = 0; i < kTP; ++i) {
          double r = t[i];
          for (int off = 1; off < 16; off <<= 1) r += __shfl_xor(r, off, 64);
          const double g = __shfl(r, (lane & 3) << 4, 64);
          if ((lane >> 2) == jj) mine[bi][i] += g;
        }
      }
    }
    __syncthreads();
    if (c1 >= tot) break;
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi) {
    const int q = bi * 64 * kCsrWaves + wave + kCsrWaves * lane;
    if (q < qmax) {
#pragma unroll
      for (int i = 0; i < kTP; ++i) {
        const int p = p0 + i;
        if (p < m && q <= p) {
          const bool on = overlap ? (idx[q] == idx[p]) : (q == p);
          const double v = scale * mine[bi][i] + (on ? shift : 0.0);
          G[(int64_t)p * m + q] = v;
          G[(int64_t)q * m + p] = v;
        }
      }
    }
  }
}

// out[col] += gamma * v[p] * A[row(p)][col] for the entries of rows p < m.
__global__ __launch_bounds__(kCsrThreads) void csr_scatter_kernel(
    const int64_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
    const double* __restrict__ vals, const int32_t* __restrict__ idx, int64_t m,
    const double* __restrict__ v, double gamma, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * kCsrWaves + (threadIdx.x >> 6);
  if (p >= m) return;
  const int64_t row = idx ? (int64_t)idx[p] : p;
  const double c = gamma * v[p];
  if (c == 0.0) return;
  for (int64_t k = rowptr[row] + lane; k < rowptr[row + 1]; k += 64)
    unsafeAtomicAdd(out + colidx[k], c * vals[k]);   // coarse-grained memory: hardware FP64 add
}

// out[p] = A[row(p)] . v + beta * base[p], row(p) = idx ? idx[p] : p
__global__ __launch_bounds__(kCsrThreads) void csr_rowdot_kernel(
    const int64_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
    const double* __restrict__ vals, const int32_t* __restrict__ idx, int64_t rows,
    const double* __restrict__ v, const double* __restrict__ base, double beta,
    double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * kCsrWaves + (threadIdx.x >> 6);
  if (p >= rows) return;
  const int64_t r = idx ? (int64_t)idx[p] : p;
  const int64_t end = rowptr[r + 1];
  double t = 0.0;
  // kProbeU entries per lane in flight (the gathers of v depend on the column
  // loads); each lane still adds its entries in index order
  for (int64_t k0 = rowptr[r] + lane; k0 < end; k0 += 64 * kProbeU) {
    int col[kProbeU];
    double val[kProbeU];
#pragma unroll
    for (int u = 0; u < kProbeU; ++u) {
      const int64_t k = k0 + 64 * u;
      col[u] = k < end ? colidx[k] : -1;
      val[u] = k < end ? vals[k] : 0.0;
    }
    double x[kProbeU];
#pragma unroll
    for (int u = 0; u < kProbeU; ++u) x[u] = col[u] >= 0 ? v[col[u]] : 0.0;
#pragma unroll
    for (int u = 0; u < kProbeU; ++u)
      if (col[u] >= 0) t = fma(val[u], x[u], t);
  }
  t = wave_sum(t);
  if (lane == 0) out[p] = t + (base ? beta * base[p] : 0.0);
}

__global__ void fill_kernel(double* __restrict__ out, int64_t n, const double* __restrict__ base,
                            double beta) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = base ? beta * base[i] : 0.0;
}

// Structure check: rowptr[0] = 0, non-decreasing, rowptr[rows] = nnz; columns
// strictly increasing inside a row and in [0, cols).  Any violation sets *bad.
// One wave per row (wave `rows` checks the end), each lane comparing its
// entries with their predecessors.
constexpr int kCheckT = 256;
__global__ __launch_bounds__(kCheckT) void csr_check_kernel(const int64_t* __restrict__ rowptr,
                                                            const int32_t* __restrict__ colidx,
                                                            int64_t rows, int64_t cols,
                                                            int64_t nnz, int* __restrict__ bad) {
  const int lane = threadIdx.x & 63;
  const int64_t r = ((int64_t)blockIdx.x * kCheckT + threadIdx.x) >> 6;
  if (r > rows) return;
  const int64_t a = rowptr[r];
  int wrong = 0;
  if (r == rows) {
    wrong = a != nnz;
  } else {
    const int64_t e = rowptr[r + 1];
    if (e < a || e > nnz || a < 0 || (r == 0 && a != 0)) {
      wrong = 1;
    } else {
      for (int64_t k = a + lane; k < e; k += 64) {
        const int c = colidx[k];
        const int prev = k > a ? colidx[k - 1] : -1;
        if (c <= prev || c >= cols) wrong = 1;
      }
    }
  }
  if (wrong) *bad = 1;
}

}  // namespace

hipError_t launch_csr_gram(const CsrView& A, const int32_t* idx, int m, const double* u,
                           double scale, double shift, bool overlap, double* G, double* Yu,
                           hipStream_t st) {
  if (m < 1 || m > kMaxRows) return hipErrorInvalidValue;
  hipLaunchKernelGGL(csr_gram_kernel, dim3(m, 1), dim3(kCsrThreads), 0, st, A.rowptr, A.colidx,
                     A.vals, idx, m, (int64_t)0, u, scale, shift, overlap ? 1 : 0, G, (int64_t)0,
                     Yu);
  return hipGetLastError();
}

hipError_t launch_csr_gram_steps(const CsrView& A, const int32_t* idx, int m, int nsteps,
                                 double scale, double shift, bool overlap, double* G,
                                 hipStream_t st) {
  if (m < 1 || m > kMaxRows || nsteps < 1 || nsteps > 65535) return hipErrorInvalidValue;
  if (m >= 64 && m <= kTMaxRows) {   // small steps: one row per workgroup keeps more of them
    hipLaunchKernelGGL(csr_gram_tile_kernel, dim3((m + kTP - 1) / kTP, nsteps), dim3(kCsrThreads),
                       0, st, A.rowptr, A.colidx, A.vals, idx, m, (int64_t)m, scale, shift,
                       overlap ? 1 : 0, G, (int64_t)m * m);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(csr_gram_kernel, dim3(m, nsteps), dim3(kCsrThreads), 0, st, A.rowptr,
                     A.colidx, A.vals, idx, m, (int64_t)m, nullptr, scale, shift,
                     overlap ? 1 : 0, G, (int64_t)m * m, nullptr);
  return hipGetLastError();
}

hipError_t launch_csr_rowdot_rows(const CsrView& A, const int32_t* idx, int64_t m,
                                  const double* v, double* out, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(csr_rowdot_kernel, dim3((unsigned)((m + kCsrWaves - 1) / kCsrWaves)),
                     dim3(kCsrThreads), 0, st, A.rowptr, A.colidx, A.vals, idx, m, v, nullptr,
                     0.0, out);
  return hipGetLastError();
}

hipError_t launch_csr_scatter(const CsrView& A, const int32_t* idx, int64_t m, const double* v,
                              double gamma, double* out, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(csr_scatter_kernel, dim3((unsigned)((m + kCsrWaves - 1) / kCsrWaves)),
                     dim3(kCsrThreads), 0, st, A.rowptr, A.colidx, A.vals, idx, m, v, gamma, out);
  return hipGetLastError();
}

hipError_t launch_csr_rowdot(const CsrView& A, const double* v, const double* base, double beta,
                             double* out, hipStream_t st) {
  if (A.rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(csr_rowdot_kernel, dim3((unsigned)((A.rows + kCsrWaves - 1) / kCsrWaves)),
                     dim3(kCsrThreads), 0, st, A.rowptr, A.colidx, A.vals, nullptr, A.rows, v,
                     base, beta, out);
  return hipGetLastError();
}

hipError_t launch_fill(double* out, int64_t n, const double* base, double beta, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, out, n,
                     base, beta);
  return hipGetLastError();
}

hipError_t launch_csr_check(const CsrView& A, int* bad, hipStream_t st) {
  const int64_t threads = (A.rows + 1) * 64;
  hipLaunchKernelGGL(csr_check_kernel, dim3((unsigned)((threads + kCheckT - 1) / kCheckT)),
                     dim3(kCheckT), 0, st, A.rowptr, A.colidx, A.rows, A.cols, A.nnz, bad);
  return hipGetLastError();
}

}  // namespace cabcd
