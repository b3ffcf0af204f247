/*
 * cabcd.h - communication-avoiding primal and dual block coordinate descent
 * (CA-BCD / CA-BDCD) for ridge regression on AMD Instinct MI355X (gfx950).
 *
 * Problem (Section 2.2, eq. primal / eq. 6 / eq. 3): X is d x n with features
 * as rows and data points as columns, y in R^n, lambda > 0,
 *     min_w  f(w) = lambda/2 ||w||^2 + 1/(2n) ||X^T w - y||^2
 *     min_a  D(a) = lambda/2 ||X a/(lambda n)||^2 + 1/(2n) ||a + y||^2,
 *     w = -X a / (lambda n).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Matrix view.  Every routine sees the data through A, the matrix whose ROWS
 * are the coordinates that get sampled: the primal passes A = X (d x n), the
 * dual passes A = X^T (n x d).  Both methods then gather s*b rows of A, form
 * their Gram matrix and dot them with one companion vector.
 *
 * Memory.  Every array pointer is a DEVICE pointer, owned by the caller, on the
 * device that is current when the call is made; the library never frees
 * caller memory.  Scalars are passed by value; the two structs below are host
 * structs whose pointer fields are device pointers.
 *
 * Streams.  `stream` is a hipStream_t (NULL = the default stream).  All work is
 * enqueued on it in order; the one-problem drivers also compute the Grams of
 * the next batch of outer steps on a second stream of the library (one per
 * device, default priority), joined back to `stream` through events before
 * those steps and before the call returns, so the call behaves as if all of
 * its work ran on `stream` (also under graph capture).  Unless
 * CABCD_FLAG_ASYNC is set, a call synchronises the stream before returning so
 * that device-detected errors (non-SPD block, non-finite values) can be
 * returned.
 *
 * Workspace.  Scratch memory is taken from a per-device pool that the library
 * grows with hipMalloc and keeps until process exit, unless opts->workspace is
 * given (then nothing is allocated and a too small workspace is CABCD_ENOMEM;
 * cabcd_workspace_bytes() gives the size).  Concurrent calls on one device
 * that use the library pool must be serialised by the caller.
 *
 * Errors.  Every entry point returns a cabcd_status; argument errors are found
 * before anything is enqueued.  cabcd_last_error() returns a thread-local
 * message for the most recent failure.
 *
 * Block sampler.  Blocks are drawn by the counter-based sampler specified at
 * cabcd_sample(); block h (0-based global iteration) depends only on
 * (seed, h), so a run can be split into several calls (opts->h0) and give the
 * same iterates.
 */
#ifndef CABCD_H
#define CABCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum cabcd_status {
  CABCD_OK = 0,
  CABCD_EINVAL = -1,        /* invalid argument; nothing was enqueued            */
  CABCD_ENOTSPD = -2,       /* a b x b diagonal block had a pivot <= 0 or NaN     */
  CABCD_EHIP = -3,          /* a HIP runtime call failed                          */
  CABCD_ENOMEM = -4,        /* allocation failed or caller workspace too small    */
  CABCD_EUNSUPPORTED = -5,  /* valid but unsupported combination (see message)    */
  CABCD_ENONFINITE = -6     /* a monitored objective became NaN or Inf            */
} cabcd_status;

typedef enum cabcd_kind { CABCD_DENSE = 0, CABCD_CSR = 1 } cabcd_kind;

typedef enum cabcd_dtype {
  CABCD_F64 = 0,       /* IEEE binary64                                         */
  CABCD_BF16 = 1,      /* bfloat16 storage, value = bf16 * row_scale            */
  CABCD_FP8_E4M3 = 2   /* OCP FP8 E4M3 storage, value = e4m3 * row_scale        */
} cabcd_dtype;

/*
 * A, the matrix whose rows are the samplable coordinates.
 * Dense: row-major, element (i, k) at data[i*ld + k]; ld >= cols.
 *   row_scale (FP32, length rows) multiplies row i for BF16 / FP8 storage; NULL
 *   means 1.  F64 ignores it.
 * CSR: rowptr (int64, rows+1, rowptr[0] = 0), colidx (int32, nnz, strictly
 *   increasing within a row, in [0, cols)), vals (FP64, nnz).  CSR is F64 only.
 */
typedef struct cabcd_matrix {
  int32_t kind;              /* cabcd_kind                                        */
  int32_t dtype;             /* cabcd_dtype                                       */
  int64_t rows;              /* number of samplable coordinates                   */
  int64_t cols;              /* length of a row (the Gram's reduction length)     */
  const void* data;          /* dense values                                      */
  int64_t ld;                /* dense leading dimension in elements               */
  const float* row_scale;    /* dense low-precision row scales or NULL            */
  const int64_t* rowptr;     /* CSR                                               */
  const int32_t* colidx;     /* CSR                                               */
  const double* vals;        /* CSR                                               */
  int64_t nnz;               /* CSR                                               */
} cabcd_matrix;

/* flags */
#define CABCD_FLAG_STATE_VALID 1u  /* primal: r already holds X^T w - y on entry;
                                      dual: w already holds -X a/(lambda n)       */
#define CABCD_FLAG_ASYNC 2u        /* do not synchronise; device status is lost   */
#define CABCD_FLAG_MONITOR_MAINTAINED 4u  /* primal: monitor points evaluate f(w)
                                             from the maintained residual r instead
                                             of recomputing X^T w - y              */
#define CABCD_FLAG_FOLD_UPDATE 8u  /* dense FP64, s*b = 256, one Gram per outer
                                      step: apply each step's companion update
                                      inside the next step's Gram kernel (one
                                      pass over both steps' rows; the Gram kernel
                                      then runs longer, the whole step shorter).
                                      Results differ from the unfolded run in
                                      rounding only, and are reproducible bit for
                                      bit however the run is split into calls
                                      with this flag                           */

typedef struct cabcd_opts {
  int64_t h0;                /* global index of the first inner iteration (resume) */
  uint32_t flags;            /* CABCD_FLAG_*                                        */
  int32_t resid_every;       /* recompute the companion vector exactly from A every
                                this many outer steps (0 = never)                   */
  int32_t monitor_every;     /* write the primal objective f(w) to trace every this
                                many outer steps (0 = never)                        */
  uint32_t timing_mask;      /* phases bracketed by events when `timing` is set: bit
                                p = CABCD_PHASE p; 0 = every phase.  Each event pair
                                costs a few microseconds of GPU time, so a caller
                                that times one kernel should mask the others.      */
  const int32_t* explicit_idx; /* optional H*b device indices replacing the sampler:
                                  block of iteration h0+i is explicit_idx[i*b ..]  */
  double* trace;             /* device, trace_len doubles (monitor output)          */
  int64_t trace_len;
  void* workspace;           /* optional caller workspace (device)                  */
  size_t workspace_bytes;
  double* timing;            /* optional HOST array of 2*CABCD_NPHASES doubles: when
                                set, every phase is bracketed by HIP events on
                                `stream`; timing[p] accumulates its milliseconds and
                                timing[CABCD_NPHASES+p] its launch count.  Needs a
                                synchronising call (no CABCD_FLAG_ASYNC).           */
  /* Residual stopping test (Section 5.1.5).  Every check_every-th outer step
     the full residual is formed from the maintained vectors (primal:
     -lambda w - 1/n X r, i.e. -grad f(w) up to the drift of r; dual:
     -X^T w + alpha + y) and the run stops after that step when its 2-norm is
     <= tol.  tol = 0 with check_every > 0 only reports the norm.  Needs a
     synchronising call (the norm is read on the host at every check).       */
  double tol;                /* >= 0, absolute bound on the residual 2-norm        */
  int32_t check_every;       /* outer steps between checks (0 = no checks)         */
  int32_t reserved1;
  int64_t* iters_done;       /* optional HOST out: inner iterations performed (H
                                unless the test stopped the run)                   */
  double* resid_norm;        /* optional HOST out: norm at the last check (NaN if
                                there was none)                                    */
} cabcd_opts;

/* Phases reported through cabcd_opts.timing (the breakdown of one outer step). */
#define CABCD_PHASE_SAMPLE 0    /* block sampler                                   */
#define CABCD_PHASE_GRAM 1      /* gathered-row Gram (with Y u when fused; with    */
                                /* CABCD_FLAG_FOLD_UPDATE also the previous       */
                                /* step's companion update)                       */
#define CABCD_PHASE_REDUCE 2    /* sum of the Gram partials, scale and overlap     */
#define CABCD_PHASE_SOLVE 3     /* s block solves + recurrence + x[idx] += d;      */
                                /* also the launches that invert the diagonal     */
                                /* blocks of Grams computed ahead                 */
#define CABCD_PHASE_UPDATE 4    /* companion update with Y^T delta (counted only   */
                                /* when launched: not when it is left to the next */
                                /* step's Gram or made moot by the exact          */
                                /* recomputation right after the step)            */
#define CABCD_PHASE_RECOMPUTE 5 /* exact companion recomputation                   */
#define CABCD_PHASE_MONITOR 6   /* objective evaluation                            */
#define CABCD_PHASE_CHECK 7     /* full residual of the stopping test              */
#define CABCD_PHASE_YU 8        /* Y u as its own gathered-row pass (steps whose
                                   Gram was computed ahead)                        */
#define CABCD_NPHASES 9

/* Fill *o with defaults: h0 0, no flags, no recompute, no monitor, sampler on,
   no residual checks. */
void cabcd_opts_init(cabcd_opts* o);

/*
 * Block sampler (Section 1 footnote and Alg. 1-4: b indices uniformly at random
 * without replacement; Section 3.1 after eq. (recur): one shared seed).
 * Writes idx[i*b + m], i < count, m < b: the block of global iteration h0+i,
 * b distinct integers in [0, range).  Definition (integer-only):
 *   out(seed, t)  = mix64(seed + 0x9E3779B97F4A7C15 * (t+1))   [SplitMix64]
 *   key           = out(seed, h);   word t = out(key, t) >> 32
 *   bounded(m)    = Lemire multiply-shift with rejection on successive words
 *   block         = Floyd: for j = range-b .. range-1: v = bounded(j+1);
 *                   append (v already drawn ? j : v)   (insertion order)
 * Requires 1 <= b <= range <= 2^31-1, count >= 0.
 */
cabcd_status cabcd_sample(uint64_t seed, int64_t h0, int64_t count, int32_t b,
                          int64_t range, int32_t* idx, void* stream);

/*
 * Gram of gathered rows (Alg. 2 Gram step, Alg. 4 Gram step; Section 4,
 * Thm. cabcd1dcol): with Y the m x cols matrix of rows idx[0..m) of A,
 *   G  = scale * Y Y^T + shift * I     (m x m, row-major, both triangles, ld m)
 *   Yu = Y u                           (m; only if u and Yu are non-NULL)
 * Primal CA-BCD uses scale 1/n, shift lambda; dual uses 1/(lambda n^2), 1/n.
 * Dense F64 / BF16 / FP8 (m <= 512; above 256 rows the Gram is assembled from
 * 256-row Grams of the two row halves and of pairs of their 128-row quarters,
 * about 1.5x the matrix-core work) and CSR F64 (m <= 1024).  Low-precision
 * rows are multiplied in their storage type on the matrix cores with FP32
 * accumulation inside a workgroup's slab; the slabs are summed and the row
 * scales applied in FP64; Yu is computed in FP64 from the decoded values.
 * Indices may repeat.  m >= 1.
 */
cabcd_status cabcd_gram(const cabcd_matrix* A, const int32_t* idx, int32_t m,
                        double scale, double shift, const double* u, double* G,
                        double* Yu, void* stream);

/*
 * cabcd_gram for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same A, idx, m, scale, shift, u, G and Yu as cabcd_gram, for dense A (F64,
 * BF16, FP8; CSR is CABCD_EUNSUPPORTED), m <= 256.  The call allocates nothing,
 * copies nothing to the host and never synchronises: the split-K partial Grams
 * and a checked copy of idx live in a fixed 64 MiB device array of the library
 * (one per GPU, held from the first call on that GPU until the process ends).
 * The column slabs are widened so that the partials fit it, so the summation
 * order (not the result beyond rounding) may differ from cabcd_gram's.
 *   status  optional device int32: receives CABCD_OK, or CABCD_EINVAL when an
 *           index lies outside [0, rows) (that row is then read as row 0 and G,
 *           Yu are meaningless), in stream order before the Gram is formed.
 * Argument errors found on the host are returned before anything is enqueued.
 * Every call on a GPU uses that GPU's one array: calls that overlap on one GPU
 * (other streams, other threads) race and must be serialised by the caller.
 */
cabcd_status cabcd_gram_noalloc(const cabcd_matrix* A, const int32_t* idx, int32_t m,
                                double scale, double shift, const double* u, double* G,
                                double* Yu, int32_t* status, void* stream);

/*
 * Primal CA-BCD (Alg. 2; s = 1 is BCD, Alg. 1), H inner iterations.
 *   X      A = X, d x n (rows = features)
 *   y      n labels
 *   w      in: w_0, out: w_H (d)
 *   r      in (only with CABCD_FLAG_STATE_VALID): X^T w_0 - y; out: the residual
 *          z_H - y maintained by the recurrence (n).  The paper's z = X^T w is
 *          kept as r = z - y.
 * The outer loop runs ceil(H/s) steps; the last has H - s*(ceil(H/s)-1) inner
 * iterations.  Blocks come from the sampler over [0, d) or opts->explicit_idx.
 * X may be dense F64, dense BF16 / FP8 (mixed precision: the Gram on the
 * stored codes with FP32 accumulation, everything else in FP64 on X^; set
 * opts->resid_every to recompute r exactly every few outer steps) or CSR F64.
 * 1 <= b <= min(d, 32), s >= 1, s*b <= 512 dense / 1024 CSR (512 when
 * b > 16), H >= 0, lambda > 0; a larger s*b is CABCD_EUNSUPPORTED.
 * Results are reproducible bit for bit for dense storage.  For CSR, the
 * outer steps of 256 to 512 gathered rows whose Grams are computed ahead
 * update r (w for the dual) with one writer per column and are reproducible
 * too, also when the run is split into several calls (opts->h0); other CSR
 * steps add their update with FP64 atomics, whose order varies between runs.
 */
cabcd_status cabcd_primal_bcd(const cabcd_matrix* X, const double* y, double lambda,
                              int32_t b, int32_t s, int64_t H, uint64_t seed,
                              double* w, double* r, const cabcd_opts* opts,
                              void* stream);

/*
 * Dual CA-BDCD (Alg. 4; s = 1 is BDCD, Alg. 3), H inner iterations.
 *   XT     A = X^T, n x d (rows = data points)
 *   y      n labels
 *   alpha  in: a_0, out: a_H (n)
 *   w      in (only with CABCD_FLAG_STATE_VALID): -X a_0/(lambda n);
 *          out: w_H maintained by the recurrence (d)
 * X^T may be dense F64, dense BF16 / FP8 (mixed precision as for the primal:
 * the Gram on the stored codes with FP32 accumulation, everything else in
 * FP64 on the dequantised X^; one row scale per data point) or CSR F64.
 * 1 <= b <= min(n, 32), s >= 1, s*b <= 512 dense / 1024 CSR (512 when
 * b > 16), H >= 0, lambda > 0; a larger s*b is CABCD_EUNSUPPORTED.
 */
cabcd_status cabcd_dual_bcd(const cabcd_matrix* XT, const double* y, double lambda,
                            int32_t b, int32_t s, int64_t H, uint64_t seed,
                            double* alpha, double* w, const cabcd_opts* opts,
                            void* stream);

/*
 * Low-precision storage of a dense FP64 matrix for the mixed-precision mode.
 * Codes are rounded from FP64 directly to nearest, ties to even:
 *   CABCD_BF16      uint16 BF16 codes; row_scale (may be NULL) is set to 1.
 *   CABCD_FP8_E4M3  uint8 OCP E4M3 codes (largest finite 448, saturating) of
 *                   A[i][k] / s_i with s_i = fp32(amax_i / 448) (1 for an
 *                   all-zero row) written to row_scale[i] (required).
 * The stored matrix X^ = diag(s) Q is the problem the mixed-precision runs
 * solve (exact in FP64).  A: rows x cols, ld lda (FP64); Q: ld ldq elements.
 */
cabcd_status cabcd_quantize(const double* A, int64_t rows, int64_t cols, int64_t lda,
                            int32_t dtype, void* Q, int64_t ldq, float* row_scale,
                            void* stream);

/*
 * The leading dimension (in elements) to allocate a dense matrix of `cols`
 * columns with, for any storage (CABCD_F64, or cabcd_quantize's Q for
 * CABCD_BF16 / CABCD_FP8_E4M3): the row rounded up to 256 bytes, plus 256
 * bytes when that is a multiple of 64 KiB.  Such strides put the same columns
 * of every gathered row on the same HBM channels: the Gram's row gathers
 * stream about 12 % slower at a 2 MiB stride.  Any ld >= cols works; this one
 * also keeps rows on the 16-byte boundaries the vector and LDS-DMA loads need.
 * Host only, no device work.  Returns -1 (and sets the error string) for
 * cols < 1 or an unknown dtype.
 */
int64_t cabcd_leading_dim(int64_t cols, int32_t dtype);

/*
 * Exact primal residual and objective (Section 5.1.5: the full residual is
 * recomputed occasionally; eq. primal): given A = X (d x n),
 *   r = X^T w - y (n, FP64 accumulation)   and   *f = f(w)  (device scalar).
 * Either output may be NULL.
 */
cabcd_status cabcd_primal_objective(const cabcd_matrix* X, const double* y,
                                    double lambda, const double* w, double* r,
                                    double* f, void* stream);

/*
 * Primal objective f(w) evaluated with A = X^T (n x d, the dual layout; any
 * storage):
 * r = A w - y, *f = 1/(2n)||r||^2 + lambda/2 ||w||^2.  Outputs may be NULL.
 */
cabcd_status cabcd_primal_objective_t(const cabcd_matrix* XT, const double* y,
                                      double lambda, const double* w, double* r,
                                      double* f, void* stream);

/*
 * Full primal residual of the stopping test (Section 5.1.5) with A = X (d x n,
 * dense F64 / BF16 / FP8 or CSR):
 *   rho = -lambda w - (1/n) X r   (d),   *norm = ||rho||_2 (device scalar)
 * for the given r = z - y (the maintained one, or X^T w - y from
 * cabcd_primal_objective, which makes rho = -grad f(w)).  Either output may be
 * NULL, not both.  Synchronises the stream.
 */
cabcd_status cabcd_primal_residual(const cabcd_matrix* X, double lambda, const double* w,
                                   const double* r, double* rho, double* norm, void* stream);

/*
 * Full dual residual of the stopping test (Section 5.1.5) with A = X^T (n x d,
 * dense F64 / BF16 / FP8 or CSR):
 *   rho = -X^T w + alpha + y   (n),   *norm = ||rho||_2 (device scalar)
 * for the given w (the maintained one, or -X alpha/(lambda n), which makes
 * rho = n grad D(alpha)).  Either output may be NULL, not both.
 * Synchronises the stream.
 */
cabcd_status cabcd_dual_residual(const cabcd_matrix* XT, const double* y, const double* alpha,
                                 const double* w, double* rho, double* norm, void* stream);

/*
 * Primal-dual map (eq. 3) with A = X^T (n x d, any storage):
 * w = -X a / (lambda n) (d).
 */
cabcd_status cabcd_dual_to_primal(const cabcd_matrix* XT, const double* alpha,
                                  double lambda, double* w, void* stream);

/*
 * Batched primal CA-BCD: many independent ridge problems (Alg. 2 each, with
 * its own X, y, lambda, b, s and seed) advanced together.  One ROUND runs one
 * outer step of every problem that is still running; a round is ONE persistent
 * kernel launch for the whole batch (Gram slabs of all problems from one work
 * queue; the last slab of a problem to finish sums its partials, runs the
 * fused solve and records the step).  The companion update r += Y^T delta of a
 * step is applied by the next round's slabs on their own columns.  Every
 * monitor_every rounds a second persistent launch evaluates the objective f(w)
 * (recomputing r = X^T w - y exactly, or from the maintained residual, see
 * cheap_monitors) and retires problems that reached f_target.  The launches
 * of one monitor period are captured once into hipGraphs and replayed (when
 * monitor_every is at most 64; longer periods launch directly).  Every 32 or
 * so rounds (a multiple of monitor_every) cabcd_batch_run synchronises its
 * stream, and once the active problems have halved since the slabs were last
 * cut, it cuts the active problems' slabs again for them alone (same b and s,
 * more and shorter slabs) and captures the graphs again, so that the GPU stays
 * filled as problems retire; this changes only the rounding order of the Gram
 * sums, and happens at the same rounds however the rounds are split between
 * calls.
 *
 * Per problem, the iterates are those of cabcd_primal_bcd with the same X, y,
 * lambda, b, s, seed and H (the same blocks), up to rounding order.
 */
typedef struct cabcd_problem {
  cabcd_matrix X;            /* dense, rows d = features, cols n = samples: F64, or
                                BF16 / FP8 storage (Gram on the codes with FP32
                                accumulation, all else FP64 on X^); one storage
                                type per batch                                     */
  const double* y;           /* n labels                                           */
  double lambda;             /* > 0                                                */
  int32_t b;                 /* block size, 1..16; 0: chosen by the autotuner
                                (4, 8 or 16; fewer only when d is smaller)         */
  int32_t s;                 /* unrolling, s*b <= 512 and s times b rounded up to
                                a power of two <= 512 (above 256 rows the Gram is
                                assembled from 256-row Grams, as for the one-
                                problem path); 0: chosen by the autotuner
                                (4 <= s <= 32 within s*b <= 512)                   */
  uint64_t seed;             /* sampler seed (blocks over [0, d))                  */
  int64_t H;                 /* inner-iteration budget; <= 0: unlimited            */
  double f_target;           /* > 0: retire at the first monitor point with
                                f(w) <= f_target; otherwise never                  */
  double* w;                 /* d: in w_0, out w                                   */
  double* r;                 /* n: out X^T w - y (exact after a monitor point,
                                maintained by the recurrence otherwise)            */
} cabcd_problem;

#define CABCD_BATCH_NO_GRAPH 1u    /* launch every kernel directly (no hipGraph)   */

typedef struct cabcd_batch_opts {
  int32_t monitor_every;     /* rounds between monitor points (default 4; 0: never,
                                then only the budgets H end problems)              */
  uint32_t flags;            /* CABCD_BATCH_*                                      */
  int32_t cheap_monitors;    /* monitor points between two exact ones at which the
                                pending update is applied and f(w) is evaluated
                                from the maintained residual instead of
                                recomputing r = X^T w - y from X (0: every monitor
                                point is exact)                                    */
  int32_t reserved;
} cabcd_batch_opts;

/* What the plan chose for one problem and where it stands. */
typedef struct cabcd_batch_info {
  int32_t b, s;              /* block size and unrolling in use                    */
  int32_t nslab;             /* column slabs (work items) per round                */
  int32_t active;            /* 1 while the problem still runs                     */
  int64_t chunk;             /* columns per slab                                   */
  int64_t h;                 /* inner iterations done                              */
  int64_t steps;             /* outer steps done                                   */
  double objective;          /* f(w) at the last monitor point (NaN before one)    */
  int32_t status;            /* CABCD_OK, CABCD_ENOTSPD or CABCD_ENONFINITE        */
  int32_t reserved;
} cabcd_batch_info;

typedef struct cabcd_batch_plan* cabcd_batch;

/*
 * Plan a batch of P problems: validate, choose b and s where they are 0 (the
 * autotuner balances the rounds each problem needs per pass over its
 * coordinates against a cost model of the round), choose the column slabs,
 * allocate the plan's workspace (hipMalloc; released by cabcd_batch_destroy),
 * compute r = X^T w_0 - y and f(w_0), and capture the hipGraphs.  The problem
 * arrays stay owned by the caller and must outlive the plan.  Synchronises
 * `stream`.  *out is NULL on failure.
 */
cabcd_status cabcd_batch_create(const cabcd_problem* problems, int32_t P,
                                const cabcd_batch_opts* opts, void* stream,
                                cabcd_batch* out);

/*
 * Run `rounds` rounds (>= 0).  On return r of every problem holds its current
 * residual (a pending companion update is flushed).  If active is non-NULL the
 * stream is synchronised and *active receives the number of problems still
 * running; device-detected errors are then returned (the first problem with a
 * non-OK status).
 */
cabcd_status cabcd_batch_run(cabcd_batch plan, int64_t rounds, void* stream,
                             int32_t* active);

/* Copy the state of problem p (synchronises `stream`). */
cabcd_status cabcd_batch_query(cabcd_batch plan, int32_t p, cabcd_batch_info* info,
                               void* stream);

/* Release the plan (synchronises the device first).  NULL is ignored. */
cabcd_status cabcd_batch_destroy(cabcd_batch plan);

/*
 * One-shot batched solve: plan, run until no problem is active or max_rounds
 * rounds have run, destroy.  Returns the first error found.
 */
cabcd_status cabcd_primal_bcd_batched(const cabcd_problem* problems, int32_t P,
                                      int64_t max_rounds, const cabcd_batch_opts* opts,
                                      void* stream);

/* Workspace bytes a call of cabcd_primal_bcd / cabcd_dual_bcd with these
 * arguments needs when opts->workspace is supplied. */
size_t cabcd_workspace_bytes(const cabcd_matrix* A, int32_t b, int32_t s);

/* Thread-local message describing the most recent failing call ("" if none). */
const char* cabcd_last_error(void);

/* Library version string. */
const char* cabcd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CABCD_H */
