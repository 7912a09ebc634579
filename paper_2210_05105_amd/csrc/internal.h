// Internal declarations shared by the HIP translation units of libcpr.
// Everything here is gfx950 (CDNA4, wave64) code; nothing is portable on
// purpose.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "../../include/cpr.h"

namespace cpr {

constexpr int WAVE = 64;
constexpr int MAXN = 8;
// largest bucket shift of the sampled MTTKRP: 256-row buckets (a bucket
// record keeps row mod B in 8 bits)
constexpr int BB_MAX = 8;
constexpr int MAXR = 128;

// Bits of the device error word (kernels atomicOr them in; synchronising
// calls read and clear it).
enum : uint32_t {
  ERR_INDEX = 1u,      // coordinate outside [0, I_k)
  ERR_DUP = 2u,        // repeated coordinate tuple
  ERR_UNIFORM = 4u,    // uniform outside [0, 1) or NaN
  ERR_ZERO_MASS = 8u,  // sampling mass Z <= 0
  ERR_NONFINITE = 16u, // NaN/Inf in a factor or value
  ERR_PINV = 32u,      // Jacobi eigen solver did not converge
  ERR_CAPACITY = 64u,  // a device-sized buffer would overflow
  ERR_PROB = 128u,     // given draw probability not finite and > 0
};

// Profiling phases (order matches cp_phase_name).
enum Phase { PH_PINV = 0, PH_SAMPLE, PH_DEDUP, PH_MTTKRP, PH_SOLVE,
             PH_GRAM, PH_SAMPLER_BUILD, PH_FIT };

// Small argument block for kernels that need per-mode pointers.
struct ModeList {
  int n;                      // number of entries used
  int mode[MAXN];
  const double *G[MAXN];      // R x R Grams
  const void *U[MAXN];        // factors (float or double)
  int64_t I[MAXN];
  uint64_t stride[MAXN];      // column-key stride of each mode for mode j
  const double *lev[MAXN];    // ARLS scores
  const double *cdf[MAXN];    // ARLS inclusive prefix sums
  const double *coarse[MAXN]; // ARLS prefix sum at the end of each 64 rows
  const double *Z[MAXN];      // ARLS totals (device scalars)
  const int64_t *last[MAXN];  // ARLS last row of positive mass
  const double *tree[MAXN];   // STS trees
  int64_t P2[MAXN];           // STS leaves (power of two)
  int F[MAXN];                // STS rows per leaf
  const double *Ggt[MAXN];    // STS G_{>k} per sampled position (R x R)
};

// ---- index build (k_index.hip)
uint32_t *validate_coo(const int32_t *idx, const void *val, int val_fp64,
                       int64_t nnz, int N, const int64_t *dims,
                       uint32_t *err, hipStream_t s);
struct ModeIndex {
  int64_t I = 0, n_cols = 0, max_col = 0;
  uint64_t *col_key = nullptr;  // n_cols sorted distinct column keys
  int64_t *col_ptr = nullptr;   // n_cols + 1 offsets
  // column lookup: open addressing with linear probing over 2^hbits
  // entries, each the 32-bit id of a column (its key is col_key[id]), at
  // most half full; ~0 marks an empty entry.  4 bytes per entry: 8 to 16
  // bytes per nonempty column.
  uint32_t *hash = nullptr;
  int hbits = 0;
  // sampled MTTKRP: record region start of each output-row bucket (set up
  // by cp_init for the sampling samplers)
  int64_t *bk_start = nullptr;
  int32_t *row = nullptr;       // nnz rows i_j
  void *val = nullptr;          // nnz values (float or double)
};
// home entry of a column key in a table of 2^hbits entries (multiplicative
// hashing: the top hbits bits of key times 2^64 / golden ratio)
__device__ __forceinline__ uint64_t col_hash(uint64_t key, int hbits) {
  return (key * 0x9E3779B97F4A7C15ull) >> (64 - hbits);
}
// Returns an error message ("" on success).
std::string build_mode_index(const int32_t *idx, const void *val, int val_fp64,
                             int64_t nnz, int N, const int64_t *dims, int j,
                             int out_fp64, ModeIndex &out, uint32_t *err,
                             hipStream_t s);

// Sum of the lengths of the J longest columns (nnz if J >= n_cols); -1 on
// a HIP failure.
int64_t top_columns_total(const int64_t *col_ptr, int64_t n_cols, int64_t nnz,
                          int64_t J, hipStream_t s);

// ---- scans (k_scan.hip): deterministic reduce-then-scan
size_t scan_temp_bytes(int64_t n);
void inclusive_scan_f64(const double *in, double *out, int64_t n, void *tmp,
                        hipStream_t s);
void exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n,
                        void *tmp, hipStream_t s);
void exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n,
                        void *tmp, hipStream_t s);

// ---- dense R x R and tall-skinny kernels (k_dense.hip)
// Gram of U (I x R): partial Grams per block (FP64 MFMA), then a fixed-order
// reduction into G (R x R).
// mode: the MFMA form of the products for FP32 factors (FP64 factors always
// use GRAM_F64): FP64, FP32, or BF16 hi/lo split with three products.
enum GramMode { GRAM_F64 = 0, GRAM_F32 = 1, GRAM_BF16X3 = 2 };
size_t gram_temp_bytes(int64_t I, int R);
template <typename T>
void gram(const T *U, int64_t I, int R, double *G, void *tmp, int mode,
          hipStream_t s);
// The same after the solve: U = X / sigma written in the factor's precision
// (zero columns stay zero) by the pass that stages it, G of the stored U.
// X holds float rows when x32 (the FP32 forms' unrefined solve), else
// double.
template <typename T>
void gram_scaled(const void *X, bool x32, const double *sigma, int64_t I,
                 int R, T *U, double *G, void *tmp, int mode, hipStream_t s);
// G~ = sum_s h_s h_s^T / (J p_s) over J draws (h: J x R, factor precision),
// the sketched Gram of Fig. 3; hs: J x R FP64 scratch, tmp as for gram.
template <typename T>
void sketched_gram(const T *h, const double *prob, int64_t J, int R,
                   double *hs, double *Gs, void *tmp, hipStream_t s);
// sigma[r] = sqrt of the sum over the nblk partial rows of column r
void column_norms(const double *partial, int nblk, int R, double *sigma,
                  uint32_t *err, hipStream_t s);
// Hadamard product of the Grams in `ml` (n entries), pseudo-inverse Gp;
// for STS also the G_{>k} chain and <G^+, G> (ggt_out may be null).
void hadamard_pinv(const ModeList &ml, int R, double *Gfull, double *Gp,
                   double *ggt_out, double *trace_out, double *scratch,
                   uint32_t *err, hipStream_t s);
// X = M G^+ (FP64 MFMA, with one refinement step when `refine`, written as
// double; FP32 factors without refinement: FP32 MFMA, X written as float);
// per-block column sums of squares into partial (nblk x R).
template <typename T>
void solve_rows(const T *M, int64_t I, int R, const double *Gfull,
                const double *Gp, void *X, double *partial, int nblk,
                int64_t *rows_out, bool refine, hipStream_t s);
int solve_blocks(int64_t I);
// sigma from partial sums; U = X / sigma (zero columns stay zero).
template <typename T>
void finish_normalize(const double *X, int64_t I, int R, const double *partial,
                      int nblk, double *sigma, T *U, uint32_t *err,
                      hipStream_t s);
// U := U / ||U[:, r]|| in place (cp_set_factor), sigma unchanged.
template <typename T>
void normalize_in_place(const double *Uin, int64_t I, int R, T *U,
                        double *partial, uint32_t *err, hipStream_t s);
template <typename T>
void zero_fill(T *p, int64_t n, hipStream_t s);
void copy_to_f64(const void *src, int src_fp64, double *dst, int64_t n,
                 hipStream_t s);
void convert_values(const void *src, int src_fp64, void *dst, int dst_fp64,
                    int64_t n, hipStream_t s);

// ---- CP-ARLS-LEV (k_arls.hip)
constexpr int ARLS_CHUNK = 64;  // rows per entry of the coarse CDF
template <typename T>
void arls_build(const T *U, int64_t I, int R, const double *Gp, double *lev,
                double *cdf, double *coarse, double *Z, int64_t *last,
                void *tmp, uint32_t *err, hipStream_t s);
template <typename T>
void arls_draw(const ModeList &ml, int64_t J, int R, const double *uni,
               int32_t *sidx, double *prob, T *h, uint32_t *err, hipStream_t s);

// ---- STS-CP (k_sts.hip)
int sts_pad(int R);     // rank padded to the draw width (row stride of StsWork::h)
int64_t sts_counters(int64_t P2);
int64_t sts_top_counts(int64_t J);
int64_t sts_first_rows(int64_t I);
int64_t sts_first_sums(int64_t I);  // entries of StsWork::lc and ::rc
int sts_packed(int R);  // doubles per tree node: packed upper triangle of sts_pad(R)
template <typename T>
void sts_build(const T *U, int64_t I, int R, int F, int64_t P2, double *tree,
               hipStream_t s);
// The same after the solve: the leaf pass writes U = X / sigma in the
// factor's precision (zero columns stay zero) and builds on the stored
// values; the root, which is U^T U, is written to G (R x R) when P2 >= 2.
template <typename T>
void sts_build_scaled(const void *X, bool x32, const double *sigma, T *U,
                      int64_t I, int R, int F, int64_t P2, double *tree,
                      double *G, hipStream_t s);
// per-slot record of the level-by-level tree descent (slots grouped by node)
struct SlotBuf {
  int32_t *s;  // sample
  int32_t *v;  // current node (heap index)
  double *t;   // target inside the node
  double *m;   // mass of the node
  double *z;   // mass of the root (the sample's total for this factor)
};
struct StsWork {
  double *h;             // J x sts_pad(R): product of the rows drawn so far
  double *lev;           // sts_first_rows(I): first-factor row masses
  double *sub;           // sts_first_sums(I): their 64-row and group sums
  SlotBuf slot[2];       // J records, double-buffered across levels
  int32_t *lc, *rc;      // sts_counters(P2): samples sent left / right
  int32_t *sbeg, *send;  // 2 P2: slot range of a node
  int32_t *tcnt;         // sts_top_counts(J): samples per top node, per
                         // top-stage block
};
template <typename T>
void sts_draw(const ModeList &ml, int64_t J, int R, const double *uni,
              const double *Gp, const double *trace, int32_t *sidx,
              double *prob, T *h, const StsWork &w, uint32_t *err,
              hipStream_t s);

// ---- sample merge, extraction, MTTKRP (k_mttkrp.hip)
struct SampleWork {
  int32_t *col_id;   // J: column in the mode's index, -1 if empty
  int32_t *owner;    // n_cols_max: first draw of a column (INT_MAX = none)
  int32_t *dupcnt;   // J: extra draws merged into this first draw
  int32_t *uq_s;     // J: first draw of each distinct column
  int32_t *uq_cid;   // J: column id
  int32_t *uq_cnt;   // J: number of draws of the column
  double *uq_w;      // J: weight count/(J p)
  int64_t *uq_off;   // J+1: extracted-nonzero offsets
  int64_t *uq_base;  // J: index position of extracted nonzero e = uq_base + e
  void *hc;          // J x R (factor type): w_u h[first draw of u], by u
  int64_t *tile_first;  // bucket_tiles(rec_cap): column at each tile start
  int32_t *item_bk;  // bucket_max_items(rec_cap, buckets): bucket of an item
  int64_t max_u;     // J (bound on distinct columns)
  int64_t *counts;   // [0] = distinct columns, [1] = extracted nonzeros
  int64_t *stats;    // cumulative: solves, distinct columns, nonzeros, rows
  int64_t *scratch;  // 4 J: first-draw flags, lengths, per-block totals
  void *scan_tmp;    // scan_temp_bytes(max(J, buckets + 1))
  int64_t *bk;       // bucket_work_entries(bk_max): fill cursors (zero
                     // between calls), ends, slice starts, split buckets,
                     // plan totals
  int64_t bk_max;    // buckets of the largest mode
  void *rec;         // nnz records: extracted nonzeros in bucket regions
  void *rec1;        // nnz first-pass records (two-pass placement) or null
  int64_t *sb;       // super_work_entries(): super-bucket fill cursors (zero
                     // between calls), their copy, chunk starts
  int64_t rec_cap;
  void *part;        // per-slice blocks of split buckets (B x R each)
};
int bucket_shift(int R, int tsize);
int64_t bucket_max_items(int64_t rec_cap, int64_t nbk);
int64_t bucket_tiles(int64_t rec_cap);
// int64 entries of SampleWork::bk for a workspace of at most bk_max buckets
int64_t bucket_work_entries(int64_t bk_max);
size_t bucket_record_bytes(int tsize);
// two-pass placement of the sampled MTTKRP's records (super buckets, then
// buckets) for modes with many buckets: first-pass record size, whether a
// mode of nbk buckets takes it, and the entries of SampleWork::sb
size_t super_record_bytes(int tsize);
bool two_pass_placement(int64_t nbk);
int64_t super_work_entries();
template <typename T>
void set_sample_rows(const ModeList &ml, int64_t J, int R, const int32_t *sidx,
                     const double *prob, T *h, uint32_t *err, hipStream_t s);
void lookup_columns(const ModeList &ml, int64_t J, const int32_t *sidx,
                    const ModeIndex &ix, SampleWork &w, hipStream_t s);
void merge_samples(int64_t J, const double *prob, const int64_t *col_ptr,
                   const void *h, int R, int tsize, SampleWork &w,
                   hipStream_t s);
// bb: bucket shift (2^bb output rows per bucket, bb <= 8: a record keeps
// the row inside its bucket in 8 bits)
template <typename T>
void sampled_mttkrp(const SampleWork &w, int64_t I, const int64_t *col_ptr,
                    const int32_t *row, const T *val, const int64_t *bk_start,
                    int R, int bb, T *M, hipStream_t s);
// Fixed record regions of a mode's output-row buckets of 2^bb rows:
// starts[b] = nonzeros of the mode in buckets < b (nbk + 1 entries); cnt is
// nbk + 1 int64 of scratch.
void bucket_regions(const int32_t *row, int64_t nnz, int64_t I, int bb,
                    int64_t *starts, int64_t *cnt, void *scan_tmp,
                    hipStream_t s);
template <typename T>
void exact_mttkrp(const ModeList &ml, int64_t n_cols, const uint64_t *col_key,
                  const int64_t *col_ptr, const int32_t *row, const T *val,
                  int R, T *M, hipStream_t s);
void debug_extracted(const SampleWork &w, int64_t nz_host,
                     const int64_t *col_ptr, const uint64_t *col_key,
                     const int32_t *row, uint64_t *ck_out, int32_t *row_out,
                     int32_t *rep_out, int64_t cap, hipStream_t s);
void debug_unique(const SampleWork &w, int64_t nu_host,
                  const uint64_t *col_key, uint64_t *ck_out, int32_t *rep_out,
                  int32_t *cnt_out, double *w_out, int64_t cap, hipStream_t s);

// ---- fit (k_fit.hip)
// ml: the modes != 0 (make_ml for mode 0: strides of mode 0's column keys)
template <typename T>
void fit_inner_index(const int64_t *col_ptr, const uint64_t *col_key,
                     int64_t n_cols, const int32_t *row, const T *val,
                     int64_t nnz, const T *U0, const ModeList &ml,
                     const double *sigma, int R, double *partial, int nblk,
                     hipStream_t s);
int fit_blocks(int64_t nnz);
void fit_finish(const ModeList &ml, int N, int R, const double *sigma,
                const double *partial, int nblk, double normT2, double *out,
                hipStream_t s);
double sum_squares(const void *val, int fp64, int64_t nnz, hipStream_t s);

// ---- device helpers
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

// A lane id the compiler cannot see through: index arithmetic derived from
// it stays inside the loop that uses it instead of being hoisted out as
// loop-invariant registers (one per fragment).
__device__ __forceinline__ int opaque_lane() {
  int z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  return lane_id() + z;
}

// Factor of column r in the renormalisation U = X diag(sigma)^-1: 1 / sigma_r,
// or 0 for a zero (or non-finite) sigma_r, so a zero column stays zero.  The
// kernels multiply by it (one rounding more than a division, within an ulp).
__device__ __forceinline__ double inv_or_zero(double s) {
  return s > 0 ? 1.0 / s : 0.0;
}

// Order one wave's LDS writes before its reads of other lanes' data.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace cpr

#define CPR_LAUNCH_CHECK()                                  \
  do {                                                      \
    hipError_t e__ = hipGetLastError();                     \
    if (e__ != hipSuccess) throw cpr::HipFail(e__, __FILE__, __LINE__); \
  } while (0)

namespace cpr {
struct HipFail {
  hipError_t e;
  const char *file;
  int line;
  HipFail(hipError_t e_, const char *f, int l) : e(e_), file(f), line(l) {}
};
}  // namespace cpr
