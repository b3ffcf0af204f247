// Device code of the s inner b x b solves of one outer step, fused into one
// workgroup (shared by the one-problem solve kernel and the batched kernel).
//
// Primal (Alg. 2, eq. recur): with G the s-step Gram and S_jt = I_j^T I_t,
//   dw_j = Gamma_j^{-1} ( c_j - sum_{t<j} (G_jt + lambda S_jt) dw_t ),
//   c = -lambda w_I - (1/n) Y (z - y),   Gamma_j = G_jj.
// Dual (Alg. 4): writing Theta_j = G'_jj and using (1/(lambda n)) Y_j^T Y_t =
// n G'_jt, the printed recurrence becomes
//   da_j = Theta_j^{-1} ( c_j - sum_{t<j} (G'_jt + (1/n) S_jt) da_t ),
//   c = (1/n) (Y^T w - a_I - y_I).
// Both are one block forward substitution with the lower block triangle of the
// overlap-augmented Gram Gov = scale Y Y^T + shift [idx_p == idx_q], which the
// Gram reduction writes (its diagonal blocks are exactly Gamma_j / Theta_j
// because indices within a block are distinct).
//
// Phases (one workgroup; thread p owns row p of the outer step):
//  1. c, and the diagonal blocks of Gov gathered into LDS by the whole
//     workgroup (one memory round trip);
//  2. every diagonal block inverted with in-place Gauss-Jordan elimination:
//     blocks up to 8 x 8 one per lane in registers, 16 x 16 blocks four per
//     wave with one row per lane and the pivot row sent by DPP row broadcasts,
//     32 x 32 blocks by one wave with the entries spread over the lanes and
//     exchanged by shuffles (no LDS round trips, no barriers).  Blocks are padded to BP = 2^k >= b with
//     the identity, whose inverse keeps the padding.  On an SPD matrix the
//     Gauss-Jordan pivots are the LDL^T pivots, so a pivot <= 0 or NaN is
//     reported as "not positive definite";
//  3. the dependent chain over j: delta_j = Gamma_j^{-1} rhs_j, then every later
//     row subtracts its Gov row segment times delta_j.  Row segments of the
//     next PF blocks are prefetched into registers; the barriers order LDS
//     only, so the prefetches stay in flight; vectors in LDS are zero-padded to
//     BP so every read is unconditional.  The segment loads pass through the
//     CU's vector cache at its data rate, so a wave stops loading once the
//     chain has passed its last block (about half the bytes);
//  4. delta written out, and x[idx] += delta: an LDS hash of the indices gives
//     each coordinate's first occurrence and count; the rows whose index
//     repeats are compacted, in row order, into a short LDS list, and the
//     first occurrence adds its duplicates from that list in block order
//     (single writer).
#pragma once

#include "internal.h"

#include <algorithm>
#include <climits>
#include <type_traits>

namespace cabcd {
namespace sdev {


constexpr int pow2_at_least(int b) {
  int p = 1;
  while (p < b) p *= 2;
  return p;
}

template <int BP>
struct SolveCfg {
  static constexpr int EPL = BP * BP > 64 ? BP * BP / 64 : 1;   // block entries per lane
  static constexpr int SPW = BP * BP < 64 ? 64 / (BP * BP) : 1; // blocks per wave
  static constexpr int GS = BP * BP + 1;   // LDS stride of the blocks (odd: no bank conflicts
                                           // when each lane reads its own block)
};

// In-place Gauss-Jordan inversion of the SPW blocks held by one wave.
// EPL == 1: lane l holds entry (u, v) = ((l % BP^2) / BP, l % BP) of block
// l / BP^2.  EPL > 1: entry l + 64 t of the single block sits in slot t.
template <int BP>
__device__ __forceinline__ void gj_invert(double (&e)[SolveCfg<BP>::EPL], int lane, bool& bad) {
  using C = SolveCfg<BP>;
  if constexpr (C::EPL == 1) {
    const int base = (lane / (BP * BP)) * (BP * BP);
    const int idx = lane - base;
    const int u = idx / BP, v = idx % BP;
#pragma unroll
    for (int k = 0; k < BP; ++k) {
      const double piv = __shfl(e[0], base + k * BP + k, 64);
      const double akv_old = __shfl(e[0], base + k * BP + v, 64);
      const double f = __shfl(e[0], base + u * BP + k, 64);
      bad |= !(piv > 0.0);
      const double rp = 1.0 / piv;
      const double akv = (v == k ? 1.0 : akv_old) * rp;   // row k after a[k][k] = 1, / piv
      e[0] = u == k ? akv : (v == k ? 0.0 : e[0]) - f * akv;
    }
  } else {
    const int v = lane % BP;   // the same column in every slot: 64 is a multiple of BP
#pragma unroll
    for (int k = 0; k < BP; ++k) {
      const int pe = k * BP + k;
      const double piv = __shfl(e[pe / 64], pe % 64, 64);
      bad |= !(piv > 0.0);
      const double rp = 1.0 / piv;
      const double akv_old = __shfl(e[(k * BP) / 64], (k * BP + v) % 64, 64);
      const double akv = (v == k ? 1.0 : akv_old) * rp;
      double f[C::EPL];
#pragma unroll
      for (int t = 0; t < C::EPL; ++t) {
        const int u = (lane + 64 * t) / BP;
        f[t] = __shfl(e[t], (u * BP + k) % 64, 64);
      }
#pragma unroll
      for (int t = 0; t < C::EPL; ++t) {
        const int u = (lane + 64 * t) / BP;
        e[t] = u == k ? akv : (v == k ? 0.0 : e[t]) - f[t] * akv;
      }
    }
  }
}

constexpr int kHashMin = 2048;   // LDS hash slots for the scatter (>= 2 m)
constexpr int kMaxSolveWaves = 16;
// Doubles of LDS that phase 4 of the solve uses: the hash table (key, first
// row, count per slot), the list of repeated rows (two ints per row) and the
// per-wave counts.
__host__ __device__ constexpr size_t hash_doubles(int m, int slots) {
  return (((size_t)slots * 3 + (size_t)m * 2 + kMaxSolveWaves) * sizeof(int) + 7) / sizeof(double);
}

__device__ __forceinline__ unsigned hash_idx(int i, int slots) {
  return ((unsigned)i * 2654435761u) & (unsigned)(slots - 1);
}

// x of lane l (l the same in every lane) in every lane.
__device__ __forceinline__ double read_lane(double x, int l) {
  const long long bits = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)bits, l);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
  return __hiloint2double(hi, lo);
}

// The s diagonal blocks held in Gi inverted one per lane (thread j takes block
// j), each in registers with the Gauss-Jordan steps of gj_invert, so the
// results are the same; with no shuffles the cost is one block's arithmetic.
template <int BP>
__device__ __forceinline__ void gj_lane(double (&e)[BP][BP], bool& bad) {
#pragma unroll
  for (int k = 0; k < BP; ++k) {
    const double piv = e[k][k];
    bad |= !(piv > 0.0);
    const double rp = 1.0 / piv;
#pragma unroll
    for (int v = 0; v < BP; ++v) e[k][v] = (v == k ? 1.0 : e[k][v]) * rp;
#pragma unroll
    for (int u = 0; u < BP; ++u) {
      if (u == k) continue;
      const double f = e[u][k];
#pragma unroll
      for (int v = 0; v < BP; ++v) e[u][v] = (v == k ? 0.0 : e[u][v]) - f * e[k][v];
    }
  }
}

template <int BP, int THREADS>
__device__ __forceinline__ void invert_per_lane(double* Gi, int s, int tid, bool& bad) {
  using C = SolveCfg<BP>;
  for (int j = tid; j < s; j += THREADS) {
    double* g = Gi + (size_t)j * C::GS;
    double e[BP][BP];
#pragma unroll
    for (int u = 0; u < BP; ++u)
#pragma unroll
      for (int v = 0; v < BP; ++v) e[u][v] = g[u * BP + v];
    gj_lane<BP>(e, bad);
#pragma unroll
    for (int u = 0; u < BP; ++u)
#pragma unroll
      for (int v = 0; v < BP; ++v) g[u * BP + v] = e[u][v];
  }
}

// x of lane 16 (lane / 16) + K in every lane of that group of sixteen (DPP
// row broadcast: no LDS round trip).
template <int K>
__device__ __forceinline__ double bcast16(double x) {
  const long bits = __builtin_amdgcn_update_dpp(0l, (long)__double_as_longlong(x), 0x150 + K,
                                                0xF, 0xF, false);
  return __longlong_as_double((long long)bits);
}

// Gauss-Jordan step K.. of a 16 x 16 block held one row per lane (row u in
// lane u of a group of sixteen); the pivot row r comes to every lane by row
// broadcasts.  Row K becomes r / r_K, every other row u subtracts
// (a_uK / r_K) r with its column K cleared first, so column K becomes
// -a_uK / r_K: one multiply and one FMA per entry (the pivot row takes a zero
// base and the factor -1 / r_K).
template <int K>
__device__ __forceinline__ void gj_rows16(double (&e)[16], int u, bool& bad) {
  if constexpr (K < 16) {
    const double piv = bcast16<K>(e[K]);
    bad |= !(piv > 0.0);
    const double rp = 1.0 / piv;
    const bool pivot_row = u == K;
    const double keep = pivot_row ? 0.0 : 1.0;
    const double fr = pivot_row ? -rp : e[K] * rp;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const double rv = v == K ? 1.0 : bcast16<K>(e[v]);
      e[v] = fma(-fr, rv, v == K ? 0.0 : e[v] * keep);
    }
    gj_rows16<K + 1>(e, u, bad);
  }
}

// The s diagonal 16 x 16 blocks held in Gi inverted in place, four per wave at
// a time (one per group of sixteen lanes, one row per lane): the four
// elimination chains run side by side with no shuffles through LDS.
template <int WAVES>
__device__ __forceinline__ void invert_rows16(double* Gi, int s, int wave, int lane, bool& bad) {
  constexpr int GS = SolveCfg<16>::GS;
  const int u = lane & 15;
  for (int j0 = wave * 4; j0 < s; j0 += WAVES * 4) {
    const int bj = j0 + (lane >> 4);
    double e[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) e[v] = bj < s ? Gi[(size_t)bj * GS + u * 16 + v] : (u == v ? 1.0 : 0.0);
    gj_rows16<0>(e, u, bad);
    if (bj < s) {
#pragma unroll
      for (int v = 0; v < 16; ++v) Gi[(size_t)bj * GS + u * 16 + v] = e[v];
    }
  }
}

// Inverts the s diagonal blocks held in Gi ([s][BP][BP], padded with the
// identity) in place: wave w takes blocks w SPW, w SPW + WAVES SPW, ..., RND
// rounds of them per pass.
template <int BP, int RND, int WAVES>
__device__ __forceinline__ void invert_rounds(double* Gi, int s, int wave, int lane, bool& bad) {
  using C = SolveCfg<BP>;
  for (int j0 = wave * C::SPW; j0 < s; j0 += RND * WAVES * C::SPW) {
    // entry t of this lane in round r: block blk(r, t), row uu(t), column vv(t)
    auto blk = [&](int r, int t) {
      return (C::EPL == 1 ? j0 + lane / (BP * BP) : j0) + r * WAVES * C::SPW;
    };
    auto eix = [&](int t) { return C::EPL == 1 ? lane % (BP * BP) : lane + 64 * t; };
    double e[RND][C::EPL];
#pragma unroll
    for (int r = 0; r < RND; ++r)
#pragma unroll
      for (int t = 0; t < C::EPL; ++t) {
        const int bj = blk(r, t), uu = eix(t) / BP, vv = eix(t) % BP;
        e[r][t] = bj < s ? Gi[(size_t)bj * C::GS + uu * BP + vv] : (uu == vv ? 1.0 : 0.0);
      }
#pragma unroll
    for (int r = 0; r < RND; ++r) gj_invert<BP>(e[r], lane, bad);
#pragma unroll
    for (int r = 0; r < RND; ++r)
#pragma unroll
      for (int t = 0; t < C::EPL; ++t)
        if (blk(r, t) < s)
          Gi[(size_t)blk(r, t) * C::GS + eix(t)] = e[r][t];
  }
}

// One outer step's fused solve by one workgroup of THREADS threads; sm holds
// solve_lds_bytes(m, b) bytes of LDS.
//   MAP 0: thread p owns row p (THREADS >= m); per block two barriers: the
//          block's rhs goes through LDS to b threads that apply Gamma_j^-1.
//   MAP 1: thread j BP + u owns row j b + u (THREADS >= s BP), so a block's
//          rows are BP consecutive lanes of one wave: they apply Gamma_j^-1
//          (rows kept in registers) to their rhs with in-wave shuffles, and
//          one barrier per block publishes delta_j.
template <int BP, int PF, int THREADS, int MAP = 0, bool PRE = false>
__device__ __forceinline__ void solve_block(const SolveArgs& a, double* sm) {
  using C = SolveCfg<BP>;
  const int m = a.m, b = a.b, s = a.s;
  // LDS: Ginv [s][BP][BP] (reused by phase 4: hash table, list of repeated
  // indices, per-wave counts), R [BP], Dl [s][BP] (zero-padded delta)
  const int slots = std::max(kHashMin, pow2_at_least(2 * m));
  const size_t gi_doubles = std::max((size_t)s * C::GS, hash_doubles(m, slots));
  double* Gi = sm;
  double* R = Gi + gi_doubles;
  double* Dl = R + BP;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const bool active = MAP == 0 ? tid < m : (tid / BP < s && tid % BP < b);
  // block of this row (-1: no row; MAP 1 keeps padding lanes on their block)
  const int j_of = MAP == 0 ? (active ? tid / b : -1) : (tid / BP < s ? tid / BP : -1);
  const int u = MAP == 0 ? (active ? tid - j_of * b : 0) : tid % BP;
  const int p = MAP == 0 ? tid : (active ? j_of * b + u : m);   // row of the outer step

  // ---- phase 1: the loads that depend on nothing go out together (the ring
  // of Gov row segments, idx and Y u, the diagonal blocks); x[idx] follows
  // and stays in flight through the inversions.
  //
  // Prefetch ring of Gov row segments Gov[p][jb*b + v].  Gov is symmetric, so
  // they are read as Gov[jb*b + v][p]: consecutive threads then read
  // consecutive addresses (one cache line per 16 lanes instead of one per
  // lane).  Unconditional loads with the block and column clamped into range
  // keep the number of loads uniform, so the compiler waits for exactly the
  // one it needs.
  const gptr<const double> gcol = glb(a.G) + (active ? p : m - 1);
  double ring[PF][BP];
  auto ring_load = [&](int q, int jb) {
    const gptr<const double> g = gcol + (int64_t)(jb < j_of ? jb : 0) * b * m;
#pragma unroll
    for (int v = 0; v < BP; ++v) ring[q][v] = g[(int64_t)(v < b ? v : b - 1) * m];
  };
#pragma unroll
  for (int q = 0; q < PF; ++q) ring_load(q, q);
  // idx is read through a generic pointer: the batched kernel passes indices
  // that live in LDS
  const int ip = active ? a.idx[p] : 0;
  const double yu = active ? glb(a.Yu)[p] : 0.0;

  // ---- phase 2: the diagonal blocks, padded to BP x BP with the identity,
  // come into LDS through loads of the whole workgroup (four per thread in
  // flight, so about one memory round trip), then are inverted in place, SPW
  // blocks per wave at a time
  constexpr int WAVES = THREADS / 64;
  {
    constexpr int PER = 4;
    const int total = s * BP * BP;
    for (int q0 = 0; q0 < total; q0 += THREADS * PER) {
      double v[PER];
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int q = q0 + i * THREADS + tid;
        const int bj = q / (BP * BP), uu = (q / BP) % BP, vv = q % BP;
        v[i] = (q < total && uu < b && vv < b)
                   ? glb(a.G)[(int64_t)(bj * b + uu) * m + bj * b + vv]
                   : (uu == vv ? 1.0 : 0.0);
      }
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int q = q0 + i * THREADS + tid;
        if (q < total) Gi[(size_t)(q / (BP * BP)) * C::GS + q % (BP * BP)] = v[i];
      }
    }
  }
  double rhs = 0.0;
  if (active) {
    const double xi = glb(a.x)[ip];
    rhs = a.mode == 0 ? (-a.lambda * xi - yu / a.n) : ((yu - xi - glb(a.y)[ip]) / a.n);
  }
  for (int q = tid; q < s * BP; q += THREADS) Dl[q] = 0.0;
  if (tid < BP) R[tid] = 0.0;
  lds_barrier();
  // Blocks of up to 8 x 8 are inverted one per lane when the workgroup's waves
  // have registers to spare (THREADS <= 256: one wave per SIMD).  Otherwise a
  // wave inverts its blocks with the entries spread over the lanes, two at
  // once (rounds) when a block has one entry per lane: their elimination
  // chains are independent, so their latencies overlap.  Larger blocks have
  // enough independent work per round and no registers to spare.
  // PRE: launch_invert_diag has inverted them already (a compile-time choice:
  // a runtime branch here changed the register allocation of the chain)
  bool bad = false;
  if constexpr (PRE)
    ;
  else if constexpr (BP <= 8 && THREADS <= 256)
    invert_per_lane<BP, THREADS>(Gi, s, tid, bad);
  else if constexpr (BP == 16)
    invert_rows16<WAVES>(Gi, s, wave, lane, bad);
  else
    invert_rounds<BP, (C::EPL == 1 ? 2 : 1), WAVES>(Gi, s, wave, lane, bad);
  if (bad) raise_status(a.status, DEV_NOTSPD);
  lds_barrier();

  // ---- phase 3: the dependent chain over the s blocks.  Every thread runs all
  // rounds (the work of steps j >= s is switched off, the barriers and loads
  // are not), so the control flow is uniform.
  if constexpr (MAP == 1) {
    double gi[BP];   // row u of Gamma_{j_of}^-1 (identity rows for padding)
#pragma unroll
    for (int v = 0; v < BP; ++v) gi[v] = j_of >= 0 ? Gi[(size_t)j_of * C::GS + u * BP + v] : 0.0;
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    // the last block with a row in this wave: once the chain is past it, the
    // wave needs no more row segments, so it stops loading (the two loops keep
    // the load counts uniform for the waits)
    const int jlast = min(s - 1, (64 * wv + 63) / BP);
    auto rounds = [&](int j0, auto load) {
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        const int j = j0 + q;
        if (wv == (j * BP) >> 6) {   // the wave that holds block j
          // its rhs entries, read from their lanes into scalar registers
          const int lb = (j * BP) & 63;
          double rv[BP];
#pragma unroll
          for (int v = 0; v < BP; ++v) rv[v] = read_lane(rhs, lb + v);
          if (j_of == j) {
            double d[2] = {0.0, 0.0};
#pragma unroll
            for (int v = 0; v < BP; ++v) d[v & 1] = fma(gi[v], rv[v], d[v & 1]);
            Dl[j * BP + u] = u < b ? d[0] + d[1] : 0.0;
          }
        }
        lds_barrier();
        if (active && j_of > j) {
          const double* dj = Dl + j * BP;
          double acc[2] = {0.0, 0.0};
#pragma unroll
          for (int v = 0; v < BP; ++v) acc[v & 1] = fma(ring[q][v], dj[v], acc[v & 1]);
          rhs -= acc[0] + acc[1];
        }
        if constexpr (decltype(load)::value) ring_load(q, j + PF);
      }
    };
    int j0 = 0;
    for (; j0 < s && j0 + PF < jlast; j0 += PF) rounds(j0, std::true_type{});
    for (; j0 < s; j0 += PF) rounds(j0, std::false_type{});
  } else
  for (int j0 = 0; j0 < s; j0 += PF) {
#pragma unroll
    for (int q = 0; q < PF; ++q) {
      const int j = j0 + q;
      if (j_of == j) R[u] = rhs;
      lds_barrier();
      if (p < b && j < s) {
        const double* g = Gi + (size_t)j * C::GS + p * BP;
        double t = 0.0;
#pragma unroll
        for (int v = 0; v < BP; ++v) t += g[v] * R[v];
        Dl[j * BP + p] = t;
      }
      lds_barrier();
      if (j_of > j) {
        const double* dj = Dl + j * BP;
        double acc = 0.0;
#pragma unroll
        for (int v = 0; v < BP; ++v) acc += ring[q][v] * dj[v];
        rhs -= acc;
      }
      ring_load(q, j + PF);
    }
  }

  // ---- phase 4: outputs.  Gi is free now and holds the hash table, the
  // list of rows whose index repeats ({index, delta slot}, in row order) and
  // the per-wave counts of that list.
  int* hkey = reinterpret_cast<int*>(Gi);
  int* hmin = hkey + slots;
  int* hcnt = hmin + slots;
  int2* dup = reinterpret_cast<int2*>(hcnt + slots);   // slots is even: 8-byte aligned
  int* wcnt = reinterpret_cast<int*>(dup + m);
  for (int q = tid; q < slots; q += THREADS) {
    hkey[q] = -1;
    hmin[q] = INT_MAX;
    hcnt[q] = 0;
  }
  lds_barrier();
  unsigned h = 0;
  double dp = 0.0;
  const int dslot = j_of >= 0 ? j_of * BP + u : 0;
  if (active) {
    dp = Dl[dslot];
    glb(a.delta)[p] = dp;
    if (!isfinite(dp)) raise_status(a.status, DEV_NONFINITE);
    h = hash_idx(ip, slots);
    for (;;) {
      const int old = atomicCAS(&hkey[h], -1, ip);
      if (old == -1 || old == ip) break;
      h = (h + 1) & (unsigned)(slots - 1);
    }
    atomicMin(&hmin[h], p);
    atomicAdd(&hcnt[h], 1);
  }
  lds_barrier();
  // Row order is thread order (both mappings), so a ballot prefix within the
  // wave plus the counts of the lower waves places each repeated row.
  const int cnt = active ? hcnt[h] : 0;
  const uint64_t bal = __ballot(cnt > 1);
  const int below = __popcll(bal & ((1ull << lane) - 1ull));
  if (lane == 0) wcnt[wave] = __popcll(bal);
  lds_barrier();
  int pos = below, ndup = 0;
  for (int w = 0; w < WAVES; ++w) {
    const int c = wcnt[w];
    pos += w < wave ? c : 0;
    ndup += c;
  }
  if (cnt > 1) dup[pos] = make_int2(ip, dslot);
  lds_barrier();
  if (active && hmin[h] == p) {
    const gptr<double> x = glb(a.x);
    if (cnt == 1) {
      x[ip] += dp;
    } else {
      // the later occurrences follow this row in the list, in row order
      double acc = x[ip] + dp;
      int need = cnt - 1;
      for (int k = pos + 1; need > 0 && k < ndup; k += 4) {
        int2 e[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) e[t] = k + t < ndup ? dup[k + t] : make_int2(-1, 0);
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (e[t].x == ip) {
            acc += Dl[e[t].y];
            --need;
          }
      }
      x[ip] = acc;
    }
  }
}


}  // namespace sdev
}  // namespace cabcd
