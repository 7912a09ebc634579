/*
 * cpr.h - C ABI of the MI355X (gfx950) randomized sparse CP-ALS library.
 *
 * The library computes the per-mode steps of randomized CP-ALS on a sparse
 * tensor (Alg. 1 of Bharadwaj, Malik, Murray, Buluc, Demmel, "Distributed-
 * Memory Randomized Algorithms for Sparse Tensor CP Decomposition", SPAA
 * 2024), on one GPU:
 *   - leverage-score sampling of Khatri-Rao rows with CP-ARLS-LEV (Appendix A)
 *     or STS-CP (Section 4.1, Appendix B),
 *   - extraction of the nonzeros in the sampled columns of mat(T, j) from a
 *     per-mode column-sorted index (Section 4.3),
 *   - the sampled MTTKRP mat(T, j) S^T S U_{!=j} (Eq. 7),
 *   - the normal-equation update U_j = M G^+ with G the Hadamard product of
 *     the factor Grams (Eq. 4, Eq. 5), renormalisation and sigma (Alg. 1),
 *   - the fit of Section 5.1.
 *
 * Conventions for every entry point:
 *   - "device" pointers are HIP device memory; "host" pointers are host memory.
 *   - Matrices are row-major.  Factor U_k is I_k x R.  Indices are 0-based.
 *   - A mode solve for mode j uses the modes != j in ascending order; the
 *     q-th column of a uniforms or sample-index block belongs to the q-th of
 *     them.
 *   - The column of mat(T, j) holding coordinate (i_1..i_N) is
 *       c_j = sum_{k != j} i_k * prod_{m < k, m != j} I_m
 *     (mode 1 fastest; the Khatri-Rao row order of Eq. 3).
 *   - All work is enqueued on the stream given to cp_init (a hipStream_t,
 *     passed as void*).  Calls are asynchronous unless documented as
 *     synchronising.  Data errors found by kernels (bad index, duplicate
 *     tuple, uniform outside [0,1), zero sampling mass, non-finite factor)
 *     are recorded on the device and returned by the next synchronising call.
 *   - Every call returns a cp_status; no exception crosses the ABI.  The
 *     message of the last failure is available from cp_last_error.
 *   - The library owns everything it allocates; the caller owns every
 *     buffer it passes in.  Input buffers are read during the call's
 *     enqueued work only and may be reused once the stream has reached it.
 */
#ifndef CPR_H
#define CPR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cp_ctx cp_ctx;

typedef enum {
  CP_OK = 0,
  CP_EINVAL = -1,       /* bad argument or bad input data                   */
  CP_ENOMEM = -2,       /* device allocation failed                         */
  CP_EHIP = -3,         /* HIP runtime error                                */
  CP_ESTATE = -4,       /* calls out of order (e.g. MTTKRP before sampling) */
  CP_EDEGENERATE = -5,  /* zero sampling mass (e.g. an all-zero factor)     */
  CP_ENUMERIC = -6,     /* non-finite value in a factor                     */
  CP_EUNSUPPORTED = -7  /* valid request outside what this build supports   */
} cp_status;

typedef enum {
  CP_SAMPLER_ARLS_LEV = 0, /* product of factor leverage laws (Appendix A)   */
  CP_SAMPLER_STS = 1,      /* exact leverage law by tree descent (App. B)   */
  CP_SAMPLER_EXACT = 2     /* every nonempty column at weight 1: exact ALS  */
} cp_sampler;

typedef enum {
  CP_FP64 = 0,  /* factors, sampled rows, MTTKRP and Grams in FP64          */
  CP_FP32 = 1,  /* FP32 factors / MTTKRP; FP64 Grams, sampler and solve     */
  CP_MIXED = 2  /* as CP_FP32 but factor Grams by BF16 MFMA, FP32 accumulate */
} cp_precision;

/* Sparse tensor as (N+1)-tuples (Section 2): N indices and a value. */
typedef struct {
  int32_t N;             /* order, 3 <= N <= 8                               */
  const int64_t *dims;   /* host, N mode sizes, each in [1, 2^31)            */
  int64_t nnz;           /* number of nonzeros, in [1, 2^32)                 */
  const int32_t *idx;    /* device, nnz*N, nonzero-major; distinct tuples    */
  const void *val;       /* device, nnz values (double if val_is_fp64)       */
  int32_t val_is_fp64;   /* 1: double values, 0: float values                */
} cp_tensor;

typedef struct {
  int32_t R;          /* target rank, 1 <= R <= 128                            */
  int32_t sampler;    /* cp_sampler                                            */
  int32_t precision;  /* cp_precision                                          */
  int32_t sts_leaf;   /* STS-CP tree leaf size in rows (16, 32 or 64) for
                         every tree factor; 0: per factor, from its rows,
                         the draws from it per sweep and max_J (see
                         cp_sts_leaf)                                        */
  int64_t max_J;      /* largest J any cp_sample will use, <= 2^24 (sizes    
                         workspaces); ignored by CP_SAMPLER_EXACT             */
  int32_t bucket_rows;  /* output rows per bucket of the sampled MTTKRP's
                           row-ordered placement: 0 = automatic (128, fewer
                           when 128 x R values exceed 32 KiB), else a power
                           of two in [16, 256]                             */
  int32_t solve_gram;   /* cp_solve_gram: the R x R matrix G of the update
                           U_j = M G^+                                     */
  int32_t solve_refine; /* cp_solve_refine: one step of iterative
                           refinement on the row solve X = M G^+          */
} cp_config;

typedef enum {
  CP_GRAM_EXACT = 0,    /* Hadamard product of the factor Grams (Eq. 4-5)  */
  CP_GRAM_SKETCHED = 1  /* G~ = (S U_{!=j})^T (S U_{!=j}) of the draws, the
                           sketched least-squares problem of Fig. 3: every
                           draw s adds h_s h_s^T / (J p_s); the draws still
                           follow the exact leverage laws                   */
} cp_solve_gram;

typedef enum {
  CP_REFINE_AUTO = 0,  /* on for CP_FP64, off for CP_FP32 / CP_MIXED       */
  CP_REFINE_ON = 1,    /* X = M G^+ + (M - (M G^+) G) G^+, all FP64: removes
                          the solve's own rounding (three R x R products
                          per row instead of one)                          */
  CP_REFINE_OFF = 2    /* X = M G^+ alone: FP64 MFMA in CP_FP64; in the
                          FP32 forms FP32 MFMA (G^+ rounded to FP32, FP32
                          accumulation, X kept in FP32), whose rounding is
                          of the order of what M already carries from the
                          FP32 MTTKRP                                      */
} cp_solve_refine;

/*
 * cp_init - build the per-mode column-sorted indices and allocate all state.
 * Section 4.3: one copy of the nonzeros per mode, sorted by (column of
 * mat(T, j), i_j), so that sampled columns are contiguous ranges.  The
 * tensor is validated (indices in range, tuples distinct, finite values);
 * a bad tensor returns CP_EINVAL.  The COO arrays are copied; the caller may
 * free them once cp_init returns.  Synchronising.  Column keys must fit in
 * 63 bits (prod_{k != j} I_k < 2^63 for every j), else CP_EUNSUPPORTED.
 * Factors start undefined: call cp_set_factor for every mode before use.
 */
cp_status cp_init(const cp_tensor *t, const cp_config *cfg, void *stream,
                  cp_ctx **out);
/* On failure *out is NULL (bad arguments) or a context that serves only
 * cp_last_error and cp_destroy. */

/*
 * cp_set_factor - load factor `mode` (Alg. 1, first three steps): copy U
 * (device, I_mode x R, FP64; rounded to FP32 under CP_FP32/CP_MIXED),
 * normalise its columns, set sigma = 1, form its Gram and rebuild its
 * sampler (Alg. 2 for CP-ARLS-LEV, Alg. 4 for STS-CP).  A zero column stays
 * zero.
 */
cp_status cp_set_factor(cp_ctx *ctx, int32_t mode, const double *U);

/*
 * cp_set_sigma - set sigma (device, R doubles), e.g. to resume from saved
 * factors and weights.
 */
cp_status cp_set_sigma(cp_ctx *ctx, const double *sigma);

/*
 * cp_sample - draw J Khatri-Rao rows of U_{!=mode} (Alg. 3 or Alg. 5 on one
 * device) from `uniforms` (device, J x (N-1) doubles in [0,1)).  Index of a
 * draw: min{ i : u Z < F(i) } for the (conditional) CDF F with total Z.
 * Optional outputs (device, may be NULL): idx_out J x (N-1) int32 row
 * indices, prob_out J doubles, the probability of each drawn row under the
 * sampler's law.  Also merges duplicate draws (weight count/(J p)) and
 * locates their columns in the mode's index.  1 <= J <= max_J.
 */
cp_status cp_sample(cp_ctx *ctx, int32_t mode, int64_t J,
                    const double *uniforms, int32_t *idx_out,
                    double *prob_out);

/*
 * cp_set_samples - use given draws instead of drawing (teacher forcing):
 * idx (device, J x (N-1) int32) and prob (device, J doubles, > 0).  Then
 * proceeds as cp_sample after its draws.  An index out of range or a
 * probability that is not finite and positive is a data error (CP_EINVAL
 * from the next synchronising call).
 */
cp_status cp_set_samples(cp_ctx *ctx, int32_t mode, int64_t J,
                         const int32_t *idx, const double *prob);

/*
 * cp_sampled_mttkrp - M = mat(T, mode) S^T S U_{!=mode} (Eq. 7) for the
 * last samples of `mode`: every nonzero (i, v) in a sampled column x adds
 * w_x v h_x to row i.  With CP_SAMPLER_EXACT no sample is needed and M is
 * the exact MTTKRP.  M_out (device, I_mode x R, double under CP_FP64 else
 * float) may be NULL; the library keeps M for cp_solve_factor.  If
 * nnz_extracted (host) is not NULL the call synchronises and stores the
 * number of extracted nonzeros.  CP_ESTATE if `mode` has no samples.
 */
cp_status cp_sampled_mttkrp(cp_ctx *ctx, int32_t mode, void *M_out,
                            int64_t *nnz_extracted);

/*
 * cp_solve_factor - U_mode = M G^+ (Eq. 4) with G = Hadamard of G_k,
 * k != mode (Eq. 5) and one step of iterative refinement, in FP64; then
 * sigma[r] = ||U_mode[:, r]||, column renormalisation (Alg. 1), the new
 * Gram and the sampler rebuild for `mode`.  CP_ESTATE without a preceding
 * cp_sampled_mttkrp on `mode`.
 */
cp_status cp_solve_factor(cp_ctx *ctx, int32_t mode);

/*
 * cp_sweep - nsweeps rounds of Alg. 1 (modes 0..N-1 in order), each mode
 * solve being sample -> sampled MTTKRP -> solve.  uniforms: device,
 * nsweeps x N x J x (N-1) doubles (unused for CP_SAMPLER_EXACT, may be NULL).
 */
cp_status cp_sweep(cp_ctx *ctx, int32_t nsweeps, int64_t J,
                   const double *uniforms);

/*
 * cp_fit - fit = 1 - ||[sigma; U] - T||_F / ||T||_F (Section 5.1), from
 * ||T||^2 - 2 <T, [sigma; U]> + sigma^T (Hadamard of G_k) sigma accumulated
 * in FP64 and clamped at 0.  fit: host.  Synchronising; returns pending
 * device errors.
 */
cp_status cp_fit(cp_ctx *ctx, double *fit);

/* cp_sync - wait for the stream and return pending device errors. */
cp_status cp_sync(cp_ctx *ctx);

/* Copies of the state (device outputs, FP64; asynchronous). */
cp_status cp_get_factor(cp_ctx *ctx, int32_t mode, double *U_out);
cp_status cp_get_sigma(cp_ctx *ctx, double *sigma_out);   /* R            */
cp_status cp_get_gram(cp_ctx *ctx, int32_t mode, double *G_out); /* R x R */

/*
 * cp_get_unique - the merged draws of the last cp_sample/cp_set_samples:
 * for each distinct sampled column that holds nonzeros (columns without
 * nonzeros add nothing to M), in increasing order of its first draw:
 * col_key (uint64), rep (index of its first draw), count (number of draws),
 * weight (count / (J p)).  Device outputs of capacity `cap` (any may be
 * NULL); n_out (host) receives the number of distinct columns.
 * Synchronising.
 */
cp_status cp_get_unique(cp_ctx *ctx, uint64_t *col_key, int32_t *rep,
                        int32_t *count, double *weight, int64_t cap,
                        int64_t *n_out);

/*
 * cp_get_extracted - the extracted nonzeros of the last samples of the
 * current mode, as (column key, row i_j, rep) triples in extraction order
 * (distinct columns in first-draw order, each column's nonzeros by row).
 * Device outputs of capacity `cap`; n_out (host) receives the count.
 * Synchronising.
 */
cp_status cp_get_extracted(cp_ctx *ctx, uint64_t *col_key, int32_t *row,
                           int32_t *rep, int64_t cap, int64_t *n_out);

/*
 * cp_profile - per-phase timing with HIP events on the library's stream.
 * cp_profile(ctx, 1) starts (and zeroes) accumulation, 0 stops it.
 * cp_profile_read fills ms (host, CP_NPHASE doubles: total milliseconds per
 * phase) and launches (host, CP_NPHASE int64: event pairs per phase);
 * synchronising.  Phases: see cp_phase_name.
 */
#define CP_NPHASE 8
cp_status cp_profile(cp_ctx *ctx, int32_t enable);
/*
 * cp_profile_phases - as cp_profile(ctx, 1), but events are recorded only
 * around the phases whose bit is set in mask (bit p = phase p); each event
 * pair costs the stream a few microseconds, so a timed run can restrict
 * them to the phases it reports.  mask 0 stops accumulation.
 */
cp_status cp_profile_phases(cp_ctx *ctx, uint32_t mask);
cp_status cp_profile_read(cp_ctx *ctx, double *ms, int64_t *launches);
const char *cp_phase_name(int32_t phase);

/*
 * cp_pinv - Moore-Penrose pseudo-inverse of one symmetric positive
 * semi-definite R x R matrix (Eq. 4), as used for G^+ in every mode solve:
 * Cholesky when every pivot exceeds max(R 2^-52 tr(G), 1e-9 max_i G_ii),
 * otherwise a cyclic Jacobi eigendecomposition with eigenvalues at or below
 * R 2^-52 lambda_max treated as zero.  G, Gp: device, row-major FP64.
 * stream: hipStream_t.  Synchronising; allocates its own scratch.
 * CP_ENUMERIC if G is not finite or the eigen-iteration fails.
 */
cp_status cp_pinv(const double *G, int32_t R, double *Gp, void *stream);

/*
 * cp_pinv_noalloc - cp_pinv for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, result and errors as cp_pinv (R > 128:
 * CP_EINVAL), but no allocation: its scratch (the Hadamard copy, the
 * eigen-solver work and the error word; 2 x 128 x 128 doubles + 256 bytes)
 * is a static device array, one per GPU, held until the process ends.  All
 * calls on one GPU share that array: calls that overlap on one GPU (other
 * streams, other host threads) race.  Synchronising.
 */
cp_status cp_pinv_noalloc(const double *G, int32_t R, double *Gp,
                          void *stream);

/*
 * cp_counters - cumulative work counters (host out, 4 int64): sampled mode
 * solves, distinct sampled columns, extracted nonzeros, nonzero rows of the
 * solved factors.  Synchronising; reset != 0 zeroes them afterwards.
 */
cp_status cp_counters(cp_ctx *ctx, int64_t *out, int32_t reset);

/* Index statistics for mode (host outputs): nonempty columns, longest column. */
cp_status cp_index_stats(cp_ctx *ctx, int32_t mode, int64_t *n_cols,
                         int64_t *max_col);

/*
 * cp_sts_leaf - the STS-CP tree of factor `mode` (Appendix B: a binary tree
 * over the factor's rows whose leaves hold F consecutive rows each; a draw
 * descends it, then scans one leaf's rows).  Host outputs (either may be
 * null): *leaf_rows = F, *leaves = the number of leaves (a power of two);
 * both 0 if the factor has no tree (another sampler, or a factor that is
 * always drawn first).  With cp_config.sts_leaf = 0, F is chosen per factor:
 * the tree is rebuilt once per sweep and drawn from d times (every other
 * mode's solve but those that draw it first), and F = 16, 32 or 64 nearest
 * to sqrt(94 I / (d max_J)) balances the build's memory traffic (about
 * three node Grams per leaf) against the leaf scans (F quadratic forms per
 * sample).
 */
cp_status cp_sts_leaf(cp_ctx *ctx, int32_t mode, int32_t *leaf_rows,
                      int64_t *leaves);

/*
 * Batched restarts: B independent decompositions of one tensor (Alg. 1 run
 * as independent trials, as the paper's experiments average over trials),
 * each with its own rank ranks[b] (1..128), factors, Grams, sigma and
 * sampler; the same sampler, precision, leaf size and J (cfg->max_J, the J
 * of every sweep; cfg->R is ignored) for all.  They share one copy of the
 * per-mode indices.  The restarts are spread over `nstreams` streams (0:
 * 4; by decreasing rank, round-robin): restarts of one stream run one after
 * another and share one set of workspaces, different streams run
 * concurrently.  The batch owns its streams and everything it allocates;
 * cp_batch_init is synchronising, the tensor may be freed afterwards.
 * Errors as for cp_init / cp_sweep; on failure *out still receives a batch
 * that serves cp_batch_last_error and cp_batch_destroy.
 */
typedef struct cp_batch cp_batch;
cp_status cp_batch_init(const cp_tensor *t, int32_t B, const int32_t *ranks,
                        const cp_config *cfg, int32_t nstreams, void *stream,
                        cp_batch **out);
/* cp_set_factor for restart b (device U, I_mode x ranks[b], FP64). */
cp_status cp_batch_set_factors(cp_batch *bt, int32_t b, int32_t mode,
                               const double *U);
/*
 * cp_batch_sweep - one ALS sweep (Alg. 1, modes in order) of every
 * restart.  uniforms: device, B x N x J x (N-1) doubles (restart b's block
 * is as cp_sweep's for one sweep).  The whole sweep is captured once into a
 * HIP graph and replayed with one graph launch per call; the graph reads
 * `uniforms` at this address, so pass the same buffer (refilled) to reuse
 * it (another address captures anew).  Asynchronous on the batch's stream.
 */
cp_status cp_batch_sweep(cp_batch *bt, const double *uniforms);
/* cp_fit of every restart into fits (host, B doubles); synchronising. */
cp_status cp_batch_fit(cp_batch *bt, double *fits);
/* wait for the batch's work and return pending device errors */
cp_status cp_batch_sync(cp_batch *bt);
/* copies of restart b's factor (device, I_mode x ranks[b] FP64) / sigma */
cp_status cp_batch_get_factor(cp_batch *bt, int32_t b, int32_t mode,
                              double *U_out);
cp_status cp_batch_get_sigma(cp_batch *bt, int32_t b, double *sigma_out);
/* the stream index restart b runs on (-1 if out of range) */
int32_t cp_batch_stream_of(const cp_batch *bt, int32_t b);
void cp_batch_destroy(cp_batch *bt);
const char *cp_batch_last_error(const cp_batch *bt);

void cp_destroy(cp_ctx *ctx);
const char *cp_last_error(const cp_ctx *ctx);
const char *cp_status_string(cp_status s);

#ifdef __cplusplus
}
#endif
#endif /* CPR_H */
