// C ABI of libcpr: context, workspaces and the per-mode schedule of
// randomized CP-ALS (Alg. 1 with the three steps of Section 4 per mode):
//   sample (pseudo-inverse, draws, merge) -> sampled MTTKRP -> solve
//   (U_j = M G^+ with refinement, sigma, renormalisation, Gram, sampler).
// Everything is enqueued on the context's stream; only calls documented as
// synchronising wait for it.
#include "internal.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <functional>
#include <cstring>
#include <mutex>
#include <new>

using namespace cpr;

namespace {

struct ProfEv {
  int phase;
  hipEvent_t a, b;
};

}  // namespace

struct cp_ctx {
  int N = 0, R = 0, sampler = 0, precision = 0, F = 0;
  int Fk[MAXN] = {};  // STS rows per leaf of each mode's tree
  int gram_mode = GRAM_F64;  // MFMA form of the factor Grams
  bool f64 = true;
  int64_t nnz = 0, max_J = 0;
  int64_t dims[MAXN] = {};
  hipStream_t s = nullptr;
  std::string msg;
  uint32_t *d_err = nullptr;
  int64_t *d_dims = nullptr;
  double normT2 = 0;
  ModeIndex ix[MAXN];
  void *U[MAXN] = {};
  double *G[MAXN] = {};
  double *sigma = nullptr;
  double *lev[MAXN] = {}, *cdf[MAXN] = {}, *coarse[MAXN] = {}, *Zd[MAXN] = {};
  int64_t *last[MAXN] = {};
  double *tree[MAXN] = {};
  int64_t P2[MAXN] = {};
  StsWork sw{};
  double *Gfull = nullptr, *Gp = nullptr, *ggt = nullptr, *trace = nullptr;
  double *pv_scratch = nullptr, *Gp1 = nullptr, *Gfull1 = nullptr;
  int32_t *sidx = nullptr;
  double *prob = nullptr;
  void *h = nullptr;
  SampleWork w{};
  void *M = nullptr;
  double *X = nullptr, *partial = nullptr;
  void *tmp = nullptr;
  double *d_fit = nullptr, *fit_partial = nullptr;
  int64_t max_I = 0, max_cols = 0;
  bool index_owner = false;  // the per-mode indices are this context's
  int ws_R = 0;              // largest rank the workspaces serve
  int bb_fixed = -1;         // bucket shift set by the caller (-1: by rank)
  int bb = 7;                // bucket shift of this context's rank
  bool sketched = false;     // solve with the sketched Gram of the draws
  bool refine = true;        // one refinement step on the row solve
  bool x32 = false;          // the solve's rows X are FP32 (FP32 forms, no
                             // refinement), else FP64
  double *hs = nullptr;      // J x R: draws scaled by 1 / sqrt(J p)
  double *Gs = nullptr;      // R x R: their Gram
  // bucket shift of the sampled MTTKRP for rank r
  int bshift(int r) const {
    return bb_fixed >= 0 ? bb_fixed : bucket_shift(r, (int)tsize());
  }
  // bucket regions per bucket shift 0 .. BB_MAX (256-row buckets: 8)
  int64_t *bk_start_bb[BB_MAX + 1][MAXN] = {};
  int sampled_mode = -1, mttkrp_mode = -1;
  int64_t cur_J = 0;
  bool factor_set[MAXN] = {};
  bool prof = false;
  uint32_t prof_mask = 0;  // phases whose events are recorded
  std::vector<ProfEv> evs;
  size_t ev_used = 0;
  std::vector<void *> allocs;

  size_t tsize() const { return f64 ? 8 : 4; }
};

namespace {

struct Fail {
  cp_status st;
  std::string msg;
};

void require(bool ok, cp_status st, const char *msg) {
  if (!ok) throw Fail{st, msg};
}

void hip_ok(hipError_t e, const char *what) {
  if (e != hipSuccess)
    throw Fail{CP_EHIP, std::string(what) + ": " + hipGetErrorString(e)};
}

// device memory every context leaves free (runtime queues and scratch,
// the caller's own tensors)
constexpr size_t kMemReserve = size_t(4) << 30;

template <typename P>
void dalloc(cp_ctx *c, P **p, size_t bytes) {
  void *q = nullptr;
  if (hipMalloc(&q, std::max<size_t>(bytes, 16)) != hipSuccess)
    throw Fail{CP_ENOMEM, "device allocation failed"};
  // keep a reserve of device memory free for the runtime and the caller:
  // a context that would leave less is refused rather than run at capacity
  size_t fr = 0, tot = 0;
  if (bytes >= (size_t(1) << 26) && hipMemGetInfo(&fr, &tot) == hipSuccess &&
      fr < kMemReserve) {
    (void)hipFree(q);
    throw Fail{CP_ENOMEM, "device memory would fall below the reserve of " +
                              std::to_string(kMemReserve >> 30) + " GiB"};
  }
  c->allocs.push_back(q);
  *p = static_cast<P *>(q);
}

__global__ void k_fill_f64(double *p, int64_t n, double v) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}
__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}

class PhaseScope {
 public:
  PhaseScope(cp_ctx *c, int ph) : c_(c) {
    if (!c_->prof || !((c_->prof_mask >> ph) & 1u)) return;
    if (c_->ev_used == c_->evs.size()) {
      ProfEv e{ph, nullptr, nullptr};
      hip_ok(hipEventCreate(&e.a), "hipEventCreate");
      hip_ok(hipEventCreate(&e.b), "hipEventCreate");
      c_->evs.push_back(e);
    }
    idx_ = c_->ev_used++;
    c_->evs[idx_].phase = ph;
    hip_ok(hipEventRecord(c_->evs[idx_].a, c_->s), "hipEventRecord");
  }
  ~PhaseScope() {
    if (c_->prof && idx_ != (size_t)-1) (void)hipEventRecord(c_->evs[idx_].b, c_->s);
  }

 private:
  cp_ctx *c_;

  size_t idx_ = (size_t)-1;
};

ModeList make_ml(cp_ctx *c, int j) {
  ModeList ml;
  std::memset(&ml, 0, sizeof(ml));
  uint64_t st = 1;
  for (int k = 0; k < c->N; ++k) {
    if (k == j) continue;
    const int q = ml.n++;
    ml.mode[q] = k;
    ml.G[q] = c->G[k];
    ml.U[q] = c->U[k];
    ml.I[q] = c->dims[k];
    ml.stride[q] = st;
    st *= (uint64_t)c->dims[k];
    ml.lev[q] = c->lev[k];
    ml.cdf[q] = c->cdf[k];
    ml.coarse[q] = c->coarse[k];
    ml.Z[q] = c->Zd[k];
    ml.last[q] = c->last[k];
    ml.tree[q] = c->tree[k];
    ml.P2[q] = c->P2[k];
    ml.F[q] = c->Fk[k];
    ml.Ggt[q] = c->ggt ? c->ggt + (int64_t)q * c->R * c->R : nullptr;
  }
  return ml;
}

ModeList make_ml_all(cp_ctx *c) {
  ModeList ml;
  std::memset(&ml, 0, sizeof(ml));
  for (int k = 0; k < c->N; ++k) {
    ml.mode[k] = k;
    ml.G[k] = c->G[k];
    ml.U[k] = c->U[k];
    ml.I[k] = c->dims[k];
  }
  ml.n = c->N;
  return ml;
}

cp_status read_errors(cp_ctx *c) {
  uint32_t e = 0;
  hip_ok(hipMemcpyAsync(&e, c->d_err, 4, hipMemcpyDeviceToHost, c->s),
         "hipMemcpyAsync");
  hip_ok(hipStreamSynchronize(c->s), "hipStreamSynchronize");
  if (!e) return CP_OK;
  const uint32_t zero = 0;
  hip_ok(hipMemcpyAsync(c->d_err, &zero, 4, hipMemcpyHostToDevice, c->s),
         "hipMemcpyAsync");
  hip_ok(hipStreamSynchronize(c->s), "hipStreamSynchronize");
  std::string m = "device reported:";
  if (e & ERR_INDEX) m += " index out of range;";
  if (e & ERR_DUP) m += " duplicate coordinate tuple;";
  if (e & ERR_UNIFORM) m += " uniform outside [0,1);";
  if (e & ERR_ZERO_MASS) m += " zero sampling mass;";
  if (e & ERR_NONFINITE) m += " non-finite value;";
  if (e & ERR_PINV) m += " pseudo-inverse did not converge;";
  if (e & ERR_CAPACITY) m += " capacity exceeded;";
  if (e & ERR_PROB) m += " draw probability not finite and positive;";
  // a non-finite value also empties the masses it feeds: the numeric cause
  // is reported over the zero mass; bad input data over both
  cp_status st = CP_EINVAL;
  if (e & ERR_ZERO_MASS) st = CP_EDEGENERATE;
  if (e & (ERR_NONFINITE | ERR_PINV)) st = CP_ENUMERIC;
  if (e & (ERR_INDEX | ERR_DUP | ERR_UNIFORM | ERR_CAPACITY | ERR_PROB))
    st = CP_EINVAL;
  throw Fail{st, m};
}

template <typename F>
cp_status guard(cp_ctx *c, F &&fn) {
  try {
    fn();
    if (c) c->msg.clear();
    return CP_OK;
  } catch (const Fail &f) {
    if (c) c->msg = f.msg;
    return f.st;
  } catch (const HipFail &h) {
    if (c)
      c->msg = std::string("HIP launch error: ") + hipGetErrorString(h.e) +
               " at " + h.file + ":" + std::to_string(h.line);
    return CP_EHIP;
  } catch (const std::bad_alloc &) {
    if (c) c->msg = "host allocation failed";
    return CP_ENOMEM;
  }
}

bool valid_bucket_rows(int32_t b) {
  return b == 0 || b == 16 || b == 32 || b == 64 || b == 128 ||
         b == (1 << BB_MAX);
}

void check_mode(cp_ctx *c, int mode) {
  require(mode >= 0 && mode < c->N, CP_EINVAL, "mode out of range");
}

void check_factors(cp_ctx *c) {
  for (int k = 0; k < c->N; ++k)
    require(c->factor_set[k], CP_ESTATE, "cp_set_factor not called for every mode");
}

// The factors != j are drawn in ascending mode order and the first one
// (h = 1) needs no tree: mode 0 is never drawn from a tree, mode 1 only when
// some j >= 2 exists.
bool sts_tree_factor(int N, int k) { return k >= 2 || (k == 1 && N >= 3); }

// Mode solves of one sweep that draw factor k from its tree: every j != k
// for k >= 2; j >= 2 for k = 1 (mode 1 is drawn first when j = 0).
int sts_draws_per_sweep(int N, int k) {
  return k >= 2 ? N - 1 : k == 1 ? N - 2 : 0;
}

// Leaf rows F of a tree factor of I rows drawn d times per sweep with J
// samples, when the configuration leaves it open.  Per sweep the tree is
// built once, about three node Grams of memory traffic per leaf (the leaf,
// its share of the nodes above, their re-reads), and each draw scans F leaf
// rows per sample, one FP64 quadratic form per row.  Node bytes and form
// work both grow as R^2, so build + draws ~ a I / F + b d J F, minimal at
// F = sqrt((a / b) I / (d J)); a / b ~ 94 is the ratio of the sampler's
// MFMA rate (about 55 TFLOP/s on the symmetric forms) to the build's
// memory rate (about 3.5 TB/s) per node entry.  Rounded to 16, 32 or 64 at
// the geometric midpoints.
int auto_leaf(int64_t I, int d, int64_t J) {
  if (d <= 0) return 16;
  const double f = std::sqrt(94.0 * (double)I /
                             ((double)d * (double)std::max<int64_t>(J, 1)));
  return f < 22.6 ? 16 : f < 45.3 ? 32 : 64;
}

template <typename T>
void rebuild_sampler(cp_ctx *c, int k) {
  PhaseScope ps(c, PH_SAMPLER_BUILD);
  const T *U = static_cast<const T *>(c->U[k]);
  if (c->sampler == CP_SAMPLER_ARLS_LEV) {
    ModeList m1;
    std::memset(&m1, 0, sizeof(m1));
    m1.n = 1;
    m1.G[0] = c->G[k];
    hadamard_pinv(m1, c->R, c->Gfull1, c->Gp1, nullptr, nullptr, c->pv_scratch,
                  c->d_err, c->s);
    arls_build<T>(U, c->dims[k], c->R, c->Gp1, c->lev[k], c->cdf[k],
                  c->coarse[k], c->Zd[k], c->last[k], c->tmp, c->d_err, c->s);
  } else if (c->sampler == CP_SAMPLER_STS && sts_tree_factor(c->N, k)) {
    sts_build<T>(U, c->dims[k], c->R, c->Fk[k], c->P2[k], c->tree[k], c->s);
  }
}

template <typename T>
void do_set_factor(cp_ctx *c, int mode, const double *Uin) {
  const int64_t I = c->dims[mode];
  normalize_in_place<T>(Uin, I, c->R, static_cast<T *>(c->U[mode]), c->partial,
                        c->d_err, c->s);
  {
    PhaseScope ps(c, PH_GRAM);
    gram<T>(static_cast<T *>(c->U[mode]), I, c->R, c->G[mode], c->tmp,
            c->gram_mode, c->s);
  }
  rebuild_sampler<T>(c, mode);
  hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(MAXR), 0, c->s, c->sigma,
                     (int64_t)c->R, 1.0);
  CPR_LAUNCH_CHECK();
}

void pinv_for(cp_ctx *c, const ModeList &ml, bool sts) {
  PhaseScope ps(c, PH_PINV);
  hadamard_pinv(ml, c->R, c->Gfull, c->Gp, sts ? c->ggt : nullptr, c->trace,
                c->pv_scratch, c->d_err, c->s);
}

template <typename T>
void do_sample(cp_ctx *c, int mode, int64_t J, const double *uni) {
  ModeList ml = make_ml(c, mode);
  const bool sts = c->sampler == CP_SAMPLER_STS;
  pinv_for(c, ml, sts);
  {
    PhaseScope ps(c, PH_SAMPLE);
    if (sts) {
      sts_draw<T>(ml, J, c->R, uni, c->Gp, c->trace, c->sidx, c->prob,
                  static_cast<T *>(c->h), c->sw, c->d_err, c->s);
    } else {
      arls_draw<T>(ml, J, c->R, uni, c->sidx, c->prob, static_cast<T *>(c->h),
                   c->d_err, c->s);
    }
  }
  {
    PhaseScope ps(c, PH_DEDUP);
    lookup_columns(ml, J, c->sidx, c->ix[mode], c->w, c->s);
    merge_samples(J, c->prob, c->ix[mode].col_ptr, c->h, c->R, (int)sizeof(T),
                  c->w, c->s);
  }
  c->sampled_mode = mode;
  c->mttkrp_mode = -1;
  c->cur_J = J;
}

template <typename T>
void do_set_samples(cp_ctx *c, int mode, int64_t J, const int32_t *idx,
                    const double *prob) {
  const ModeList ml = make_ml(c, mode);
  pinv_for(c, ml, false);
  hip_ok(hipMemcpyAsync(c->sidx, idx, J * (c->N - 1) * 4,
                        hipMemcpyDeviceToDevice, c->s), "hipMemcpyAsync");
  hip_ok(hipMemcpyAsync(c->prob, prob, J * 8, hipMemcpyDeviceToDevice, c->s),
         "hipMemcpyAsync");
  set_sample_rows<T>(ml, J, c->R, c->sidx, c->prob, static_cast<T *>(c->h),
                     c->d_err, c->s);
  {
    PhaseScope ps(c, PH_DEDUP);
    lookup_columns(ml, J, c->sidx, c->ix[mode], c->w, c->s);
    merge_samples(J, c->prob, c->ix[mode].col_ptr, c->h, c->R, (int)sizeof(T),
                  c->w, c->s);
  }
  c->sampled_mode = mode;
  c->mttkrp_mode = -1;
  c->cur_J = J;
}

template <typename T>
void do_mttkrp(cp_ctx *c, int mode) {
  const ModeIndex &ix = c->ix[mode];
  T *M = static_cast<T *>(c->M);
  PhaseScope ps(c, PH_MTTKRP);
  if (c->sampler == CP_SAMPLER_EXACT) {
    zero_fill<T>(M, c->dims[mode] * c->R, c->s);
    const ModeList ml = make_ml(c, mode);
    exact_mttkrp<T>(ml, ix.n_cols, ix.col_key, ix.col_ptr, ix.row,
                    static_cast<const T *>(ix.val), c->R, M, c->s);
  } else {
    sampled_mttkrp<T>(c->w, c->dims[mode], ix.col_ptr, ix.row,
                      static_cast<const T *>(ix.val), ix.bk_start, c->R,
                      c->bb, M, c->s);
  }
  c->mttkrp_mode = mode;
}

template <typename T>
void do_solve(cp_ctx *c, int mode) {
  const int64_t I = c->dims[mode];
  T *U = static_cast<T *>(c->U[mode]);
  {
    PhaseScope ps(c, PH_SOLVE);
    const double *Gf = c->Gfull, *Gp = c->Gp;
    if (c->sketched && c->sampler != CP_SAMPLER_EXACT) {
      // G~ of this solve's draws (Fig. 3) and its pseudo-inverse
      sketched_gram<T>(static_cast<const T *>(c->h), c->prob, c->cur_J,
                       c->R, c->hs, c->Gs, c->tmp, c->s);
      ModeList m1;
      std::memset(&m1, 0, sizeof(m1));
      m1.n = 1;
      m1.G[0] = c->Gs;
      hadamard_pinv(m1, c->R, c->Gfull1, c->Gp1, nullptr, nullptr,
                    c->pv_scratch, c->d_err, c->s);
      Gf = c->Gfull1;
      Gp = c->Gp1;
    }
    const int nblk = solve_blocks(I);
    solve_rows<T>(static_cast<const T *>(c->M), I, c->R, Gf, Gp, c->X,
                  c->partial, nblk, c->w.stats + 3, c->refine, c->s);
    column_norms(c->partial, nblk, c->R, c->sigma, c->d_err, c->s);
  }
  // the pass that stages the new factor for its Gram (or for its tree's
  // leaves) writes it, renormalised, on the way
  if (c->sampler == CP_SAMPLER_STS && sts_tree_factor(c->N, mode) &&
      c->P2[mode] >= 2) {
    PhaseScope ps(c, PH_SAMPLER_BUILD);  // the tree's root is the Gram
    sts_build_scaled<T>(c->X, c->x32, c->sigma, U, I, c->R, c->Fk[mode],
                        c->P2[mode], c->tree[mode], c->G[mode], c->s);
  } else {
    {
      PhaseScope ps(c, PH_GRAM);
      gram_scaled<T>(c->X, c->x32, c->sigma, I, c->R, U, c->G[mode], c->tmp,
                     c->gram_mode, c->s);
    }
    rebuild_sampler<T>(c, mode);
  }
  c->sampled_mode = -1;
  c->mttkrp_mode = -1;
}

template <typename T>
void do_fit(cp_ctx *c, double *fit) {
  const ModeList ml = make_ml_all(c);
  const ModeList m0 = make_ml(c, 0);
  const ModeIndex &ix = c->ix[0];
  const int nb = fit_blocks(c->nnz);
  {
    PhaseScope ps(c, PH_FIT);
    fit_inner_index<T>(ix.col_ptr, ix.col_key, ix.n_cols, ix.row,
                       static_cast<const T *>(ix.val), c->nnz,
                       static_cast<const T *>(c->U[0]), m0, c->sigma, c->R,
                       c->fit_partial, nb, c->s);
    fit_finish(ml, c->N, c->R, c->sigma, c->fit_partial, nb, c->normT2,
               c->d_fit, c->s);
  }
  hip_ok(hipMemcpyAsync(fit, c->d_fit, 8, hipMemcpyDeviceToHost, c->s),
         "hipMemcpyAsync");
  read_errors(c);
}

int64_t next_pow2(int64_t x) {
  int64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

void set_config(cp_ctx *c, int N, const int64_t *dims, const cp_config *cfg) {
  c->N = N;
  c->R = cfg->R;
  c->sampler = cfg->sampler;
  c->precision = cfg->precision;
  c->F = cfg->sts_leaf;
  for (int k = 0; k < N; ++k)
    c->Fk[k] = c->F ? c->F : auto_leaf(dims[k], sts_draws_per_sweep(N, k),
                                       cfg->max_J);
  c->f64 = (c->precision == CP_FP64);
  c->gram_mode = c->precision == CP_FP64   ? GRAM_F64
                 : c->precision == CP_FP32 ? GRAM_F32
                                           : GRAM_BF16X3;
  c->max_J = cfg->max_J;
  c->sketched = cfg->solve_gram == CP_GRAM_SKETCHED &&
                cfg->sampler != CP_SAMPLER_EXACT;
  c->refine = cfg->solve_refine == CP_REFINE_ON ||
              (cfg->solve_refine == CP_REFINE_AUTO && c->f64);
  c->x32 = !c->f64 && !c->refine;
  c->bb_fixed = -1;
  for (int b = 4; b <= BB_MAX; ++b)
    if (cfg->bucket_rows == (1 << b)) c->bb_fixed = b;
  for (int k = 0; k < N; ++k) c->dims[k] = dims[k];
  c->max_I = 0;
  for (int k = 0; k < N; ++k) c->max_I = std::max(c->max_I, dims[k]);
}

// Validated per-mode column-sorted indices (Section 4.3) and ||T||^2.
void init_index(cp_ctx *c, const cp_tensor *t) {
  const int N = c->N;
  c->nnz = t->nnz;
  dalloc(c, &c->d_err, 4);
  dalloc(c, &c->d_dims, N * 8);
  hip_ok(hipMemsetAsync(c->d_err, 0, 4, c->s), "hipMemsetAsync");
  hip_ok(hipMemcpyAsync(c->d_dims, c->dims, N * 8, hipMemcpyHostToDevice, c->s),
         "hipMemcpyAsync");
  validate_coo(t->idx, t->val, t->val_is_fp64, t->nnz, N, c->d_dims, c->d_err,
               c->s);
  try {  // any defect of the input tensor is a bad argument
    read_errors(c);
  } catch (const Fail &f) {
    throw Fail{CP_EINVAL, "invalid tensor: " + f.msg};
  }
  for (int k = 0; k < N; ++k) {
    std::string e = build_mode_index(t->idx, t->val, t->val_is_fp64, t->nnz, N,
                                     c->dims, k, c->f64, c->ix[k], c->d_err,
                                     c->s);
    if (c->ix[k].row) c->allocs.push_back(c->ix[k].row);
    if (c->ix[k].val) c->allocs.push_back(c->ix[k].val);
    if (c->ix[k].col_key) c->allocs.push_back(c->ix[k].col_key);
    if (c->ix[k].col_ptr) c->allocs.push_back(c->ix[k].col_ptr);
    if (c->ix[k].hash) c->allocs.push_back(c->ix[k].hash);
    if (!e.empty())
      throw Fail{e.find("63 bits") != std::string::npos ? CP_EUNSUPPORTED
                                                         : CP_ENOMEM, e};
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess && fr < kMemReserve)
      throw Fail{CP_ENOMEM, "the mode indices leave less than the reserve of " +
                                std::to_string(kMemReserve >> 30) +
                                " GiB of device memory"};
    read_errors(c);
    c->max_cols = std::max(c->max_cols, c->ix[k].n_cols);
  }
  // ||T||^2 of the values in the path's precision (mode 0's copy)
  c->normT2 = sum_squares(c->ix[0].val, c->f64, c->nnz, c->s);
  require(c->normT2 > 0, CP_EINVAL, "tensor has zero norm");
  c->index_owner = true;
}

// Record regions of the sampled MTTKRP's output-row buckets of 2^bb rows,
// per mode (built once per bucket size by the context owning the index).
void ensure_bucket_regions(cp_ctx *c, int bb, int64_t *scratch,
                           void *scan_tmp) {
  require(bb >= 0 && bb <= BB_MAX, CP_EINVAL, "bucket size out of range");
  if (c->bk_start_bb[bb][0]) return;
  for (int k = 0; k < c->N; ++k) {
    const int64_t nbk_k = (c->dims[k] + (1 << bb) - 1) >> bb;
    dalloc(c, &c->bk_start_bb[bb][k], (size_t)(nbk_k + 1) * 8);
    bucket_regions(c->ix[k].row, c->nnz, c->dims[k], bb,
                   c->bk_start_bb[bb][k], scratch, scan_tmp, c->s);
  }
}

// Factors, Grams, sigma and the sampler structures of one decomposition.
void init_state(cp_ctx *c) {
  const int N = c->N, R = c->R;
  const size_t ts = c->tsize();
  if (!c->d_err) {
    dalloc(c, &c->d_err, 4);
    hip_ok(hipMemsetAsync(c->d_err, 0, 4, c->s), "hipMemsetAsync");
  }
  for (int k = 0; k < N; ++k) {
    const int64_t I = c->dims[k];
    dalloc(c, &c->U[k], (size_t)I * R * ts);
    dalloc(c, &c->G[k], (size_t)R * R * 8);
    if (c->sampler == CP_SAMPLER_ARLS_LEV) {
      dalloc(c, &c->lev[k], I * 8);
      dalloc(c, &c->cdf[k], I * 8);
      dalloc(c, &c->coarse[k], ((I + ARLS_CHUNK - 1) / ARLS_CHUNK) * 8);
      dalloc(c, &c->Zd[k], 8);
      dalloc(c, &c->last[k], 8);
    } else if (c->sampler == CP_SAMPLER_STS) {
      c->P2[k] = next_pow2((I + c->Fk[k] - 1) / c->Fk[k]);
      if (sts_tree_factor(N, k))
        dalloc(c, &c->tree[k], (size_t)2 * c->P2[k] * sts_packed(R) * 8);
    }
  }
  dalloc(c, &c->sigma, R * 8);
  hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(MAXR), 0, c->s, c->sigma,
                     (int64_t)R, 1.0);
  CPR_LAUNCH_CHECK();
}

// Workspaces of a mode solve for every rank up to Rws (shared by the
// contexts of one stream in a batch; each solve leaves them ready for the
// next one).  `own` holds the index (bucket regions are built there).
void init_workspace(cp_ctx *c, cp_ctx *own, int Rws) {
  const int N = c->N;
  const size_t ts = c->tsize();
  c->ws_R = Rws;
  if (c->sampler == CP_SAMPLER_STS) {
    int64_t mI = 0, mP2 = 1;
    for (int k = 0; k < N; ++k) {
      mI = std::max(mI, c->dims[k]);
      if (sts_tree_factor(N, k))
        mP2 = std::max(mP2, next_pow2((c->dims[k] + c->Fk[k] - 1) / c->Fk[k]));
    }
    dalloc(c, &c->sw.lev, sts_first_rows(mI) * 8);
    dalloc(c, &c->sw.sub, sts_first_sums(mI) * 8);
    const int64_t Js = std::max<int64_t>(c->max_J, 1);
    dalloc(c, &c->sw.h, (size_t)Js * sts_pad(Rws) * 8);
    for (int b = 0; b < 2; ++b) {
      dalloc(c, &c->sw.slot[b].s, Js * 4);
      dalloc(c, &c->sw.slot[b].v, Js * 4);
      dalloc(c, &c->sw.slot[b].t, Js * 8);
      dalloc(c, &c->sw.slot[b].m, Js * 8);
      dalloc(c, &c->sw.slot[b].z, Js * 8);
    }
    dalloc(c, &c->sw.lc, sts_counters(mP2) * 4);
    dalloc(c, &c->sw.rc, sts_counters(mP2) * 4);
    dalloc(c, &c->sw.sbeg, 2 * mP2 * 4);
    dalloc(c, &c->sw.send, 2 * mP2 * 4);
    dalloc(c, &c->sw.tcnt, (size_t)sts_top_counts(Js) * 4);
  }
  const size_t RR = (size_t)Rws * Rws * 8;
  dalloc(c, &c->Gfull, RR);
  dalloc(c, &c->Gp, RR);
  dalloc(c, &c->Gfull1, RR);
  dalloc(c, &c->Gp1, RR);
  dalloc(c, &c->pv_scratch, RR);
  dalloc(c, &c->ggt, (size_t)(N - 1) * RR);
  dalloc(c, &c->trace, 8);
  const int64_t J = std::max<int64_t>(c->max_J, 1);
  dalloc(c, &c->sidx, (size_t)J * (N - 1) * 4);
  dalloc(c, &c->prob, J * 8);
  dalloc(c, &c->h, (size_t)J * Rws * ts);
  dalloc(c, &c->w.col_id, J * 4);
  dalloc(c, &c->w.owner, own->max_cols * 4);
  dalloc(c, &c->w.dupcnt, J * 4);
  dalloc(c, &c->w.hc, (size_t)J * Rws * ts);
  dalloc(c, &c->w.uq_s, J * 4);
  dalloc(c, &c->w.uq_cid, J * 4);
  dalloc(c, &c->w.uq_cnt, J * 4);
  dalloc(c, &c->w.uq_w, J * 8);
  dalloc(c, &c->w.uq_off, (J + 1) * 8);
  dalloc(c, &c->w.uq_base, J * 8);
  c->w.max_u = J;
  dalloc(c, &c->w.counts, 16);
  dalloc(c, &c->w.stats, 4 * 8);
  dalloc(c, &c->w.scratch, (size_t)4 * J * 8);
  // output-row buckets of the sampled MTTKRP: the smallest bucket (most
  // buckets) and the largest B x R block over the ranks served
  int bb_min = 30;
  for (int r = 1; r <= Rws; ++r) bb_min = std::min(bb_min, c->bshift(r));
  const int64_t nbk = (c->max_I + (1 << bb_min) - 1) >> bb_min;
  dalloc(c, &c->w.scan_tmp, std::max(scan_temp_bytes(J),
                                     scan_temp_bytes(nbk + 1)));
  dalloc(c, &c->w.bk,
         (size_t)std::max<int64_t>(bucket_work_entries(nbk), nbk + 1) * 8);
  c->w.bk_max = nbk;
  // record capacity: at most J distinct columns are extracted, so the J
  // longest columns of a mode bound the extracted nonzeros of any solve
  int64_t cap = 1;
  if (c->sampler != CP_SAMPLER_EXACT) {
    for (int k = 0; k < N; ++k) {
      const int64_t top = top_columns_total(own->ix[k].col_ptr,
                                            own->ix[k].n_cols, own->nnz, J,
                                            c->s);
      require(top >= 0, CP_EHIP, "column length statistics failed");
      cap = std::max(cap, top);
    }
  }
  c->w.rec_cap = cap;
  if (c->sampler != CP_SAMPLER_EXACT) {
    // records sit in each bucket's fixed region: nnz of them at most
    dalloc(c, &c->w.rec, (size_t)c->nnz * bucket_record_bytes((int)ts));
    if (two_pass_placement(nbk)) {  // some mode places in two passes
      dalloc(c, &c->w.rec1, (size_t)c->nnz * super_record_bytes((int)ts));
      dalloc(c, &c->w.sb, (size_t)super_work_entries() * 8);
      zero_fill<int64_t>(c->w.sb, super_work_entries(), c->s);
    }
  }
  dalloc(c, &c->w.tile_first, (size_t)bucket_tiles(cap) * 8);
  dalloc(c, &c->w.item_bk, (size_t)bucket_max_items(cap, nbk) * 4);
  size_t blk = 0;  // largest B x R block of a split bucket
  for (int r = 1; r <= Rws; ++r)
    blk = std::max(blk, ((size_t)1 << c->bshift(r)) * r * ts);
  dalloc(c, &c->w.part, (size_t)bucket_max_items(cap, nbk) * blk);
  zero_fill<int64_t>(c->w.stats, 4, c->s);
  dalloc(c, &c->M, (size_t)c->max_I * Rws * ts);
  dalloc(c, &c->X, (size_t)c->max_I * Rws * 8);
  dalloc(c, &c->partial, (size_t)(1024 + 2) * Rws * 8);
  dalloc(c, &c->tmp, std::max(gram_temp_bytes(std::max(c->max_I, J), Rws),
                              256 + scan_temp_bytes(c->max_I)));
  if (c->sketched) {
    dalloc(c, &c->hs, (size_t)J * Rws * 8);
    dalloc(c, &c->Gs, RR);
  }
  dalloc(c, &c->d_fit, 4 * 8);
  dalloc(c, &c->fit_partial, fit_blocks(c->nnz) * 8);
  hipLaunchKernelGGL(k_fill_i32, dim3(ceil_div(own->max_cols, 256)), dim3(256),
                     0, c->s, c->w.owner, own->max_cols, INT_MAX);
  zero_fill<int32_t>(c->w.dupcnt, J, c->s);
  CPR_LAUNCH_CHECK();
}

// The index (and its bucket regions for this rank) of `own`, borrowed.
void borrow_index(cp_ctx *c, const cp_ctx *own) {
  c->nnz = own->nnz;
  c->normT2 = own->normT2;
  c->max_cols = own->max_cols;
  for (int k = 0; k < c->N; ++k) c->ix[k] = own->ix[k];
}

// Workspace pointers of `ws` (sized for ranks up to ws->ws_R), borrowed.
void borrow_workspace(cp_ctx *c, const cp_ctx *ws) {
  c->ws_R = ws->ws_R;
  c->sw = ws->sw;
  c->Gfull = ws->Gfull;
  c->Gp = ws->Gp;
  c->Gfull1 = ws->Gfull1;
  c->Gp1 = ws->Gp1;
  c->pv_scratch = ws->pv_scratch;
  c->ggt = ws->ggt;
  c->trace = ws->trace;
  c->sidx = ws->sidx;
  c->prob = ws->prob;
  c->h = ws->h;
  c->w = ws->w;
  c->M = ws->M;
  c->X = ws->X;
  c->partial = ws->partial;
  c->tmp = ws->tmp;
  c->d_fit = ws->d_fit;
  c->fit_partial = ws->fit_partial;
  c->hs = ws->hs;
  c->Gs = ws->Gs;
}

// The bucket regions matching this context's rank (built in `own`, the
// index holder, on first use of a bucket size; the workspace's bucket
// array serves as their scratch and is then cleared: the fill cursors start
// at zero, and the accumulation plan clears them after every sampled MTTKRP).
void select_bucket_regions(cp_ctx *c, cp_ctx *own) {
  const int bb = c->bshift(c->R);
  c->bb = bb;
  if (c->sampler != CP_SAMPLER_EXACT)
    ensure_bucket_regions(own, bb, c->w.bk, c->w.scan_tmp);
  zero_fill<int64_t>(c->w.bk,
                     (size_t)std::max<int64_t>(bucket_work_entries(c->w.bk_max),
                                               c->w.bk_max + 1),
                     c->s);
  for (int k = 0; k < c->N; ++k) c->ix[k].bk_start = own->bk_start_bb[bb][k];
}

void init_ctx(cp_ctx *c, const cp_tensor *t, const cp_config *cfg) {
  set_config(c, t->N, t->dims, cfg);
  init_index(c, t);
  init_state(c);
  init_workspace(c, c, c->R);
  select_bucket_regions(c, c);
  read_errors(c);
}

void destroy_ctx(cp_ctx *c) {
  if (!c) return;
  if (c->s) (void)hipStreamSynchronize(c->s);
  for (void *p : c->allocs) (void)hipFree(p);
  for (auto &e : c->evs) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  delete c;
}


// Batched restarts: B decompositions of one tensor share its per-mode
// indices (built once by `base`); restart b has its own factors, Grams,
// sigma and sampler structures.  Restarts are spread over `st` streams
// (decreasing rank, round-robin); the restarts of one stream run one after
// another and share one set of workspaces, sized for the stream's largest
// rank.  A sweep of all restarts is captured once into a HIP graph (fork
// from the caller's stream into the branch streams, join back) and replayed
// with one hipGraphLaunch per sweep.
struct BatchState {
  cp_ctx *base = nullptr;
  std::vector<cp_ctx *> r;
  std::vector<int> branch;
  std::vector<hipStream_t> st;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  hipStream_t s = nullptr;   // the caller's stream (may be the null stream)
  hipStream_t cs = nullptr;  // the batch's own stream the graph is captured on
  int B = 0, N = 0;
  int64_t J = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const double *cap_uni = nullptr;
};

template <typename T>
void restart_sweep(cp_ctx *c, int64_t J, const double *uni) {
  const int N = c->N;
  for (int j = 0; j < N; ++j) {
    do_sample<T>(c, j, J, uni + (int64_t)j * J * (N - 1));
    do_mttkrp<T>(c, j);
    do_solve<T>(c, j);
  }
}

void drop_graph(BatchState &b) {
  if (b.exec) (void)hipGraphExecDestroy(b.exec);
  if (b.graph) (void)hipGraphDestroy(b.graph);
  b.exec = nullptr;
  b.graph = nullptr;
  b.cap_uni = nullptr;
}

// Captured on the batch's own stream (capture is not possible on the null
// stream); the graph is then launched on the caller's stream.
void capture_sweep(BatchState &b, const double *uni) {
  drop_graph(b);
  hip_ok(hipStreamBeginCapture(b.cs, hipStreamCaptureModeThreadLocal),
         "hipStreamBeginCapture");
  try {
    hip_ok(hipEventRecord(b.fork, b.cs), "hipEventRecord");
    for (hipStream_t x : b.st)
      hip_ok(hipStreamWaitEvent(x, b.fork, 0), "hipStreamWaitEvent");
    const int64_t per = (int64_t)b.N * b.J * (b.N - 1);
    for (int i = 0; i < b.B; ++i) {
      cp_ctx *c = b.r[i];
      c->s = b.st[b.branch[i]];
      if (c->f64) restart_sweep<double>(c, b.J, uni + i * per);
      else restart_sweep<float>(c, b.J, uni + i * per);
      c->s = b.s;
    }
    for (size_t q = 0; q < b.st.size(); ++q) {
      hip_ok(hipEventRecord(b.join[q], b.st[q]), "hipEventRecord");
      hip_ok(hipStreamWaitEvent(b.cs, b.join[q], 0), "hipStreamWaitEvent");
    }
  } catch (...) {
    for (cp_ctx *c : b.r) c->s = b.s;
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(b.cs, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  hip_ok(hipStreamEndCapture(b.cs, &b.graph), "hipStreamEndCapture");
  hip_ok(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0),
         "hipGraphInstantiate");
  b.cap_uni = uni;
}

void destroy_batch(BatchState *b) {
  if (!b) return;
  if (b->s) (void)hipStreamSynchronize(b->s);
  drop_graph(*b);
  for (cp_ctx *c : b->r) destroy_ctx(c);
  destroy_ctx(b->base);
  for (hipStream_t x : b->st) (void)hipStreamDestroy(x);
  if (b->cs) (void)hipStreamDestroy(b->cs);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (hipEvent_t e : b->join) (void)hipEventDestroy(e);
}

}  // namespace

extern "C" {

cp_status cp_init(const cp_tensor *t, const cp_config *cfg, void *stream,
                  cp_ctx **out) {
  if (!out) return CP_EINVAL;
  *out = nullptr;
  if (!t || !cfg || !t->dims || !t->idx || !t->val) return CP_EINVAL;
  if (t->N < 3 || t->N > MAXN || t->nnz < 1 || t->nnz >= (int64_t(1) << 32))
    return CP_EINVAL;
  for (int k = 0; k < t->N; ++k)
    if (t->dims[k] < 1 || t->dims[k] >= (int64_t(1) << 31)) return CP_EINVAL;
  if (cfg->R < 1 || cfg->R > MAXR) return CP_EINVAL;
  if (cfg->sampler < 0 || cfg->sampler > 2) return CP_EINVAL;
  if (cfg->precision < 0 || cfg->precision > 2) return CP_EINVAL;
  if (cfg->sampler != CP_SAMPLER_EXACT &&
      (cfg->max_J < 1 || cfg->max_J > (int64_t(1) << 24)))
    return CP_EINVAL;
  if (cfg->sts_leaf != 0 && cfg->sts_leaf != 16 && cfg->sts_leaf != 32 &&
      cfg->sts_leaf != 64)
    return CP_EINVAL;
  if (!valid_bucket_rows(cfg->bucket_rows)) return CP_EINVAL;
  if (cfg->solve_gram < 0 || cfg->solve_gram > 1) return CP_EINVAL;
  if (cfg->solve_refine < 0 || cfg->solve_refine > 2) return CP_EINVAL;
  cp_ctx *c = new (std::nothrow) cp_ctx;
  if (!c) return CP_ENOMEM;
  c->s = static_cast<hipStream_t>(stream);
  cp_status st = guard(c, [&] { init_ctx(c, t, cfg); });
  if (st != CP_OK) {
    // keep the message reachable through a minimal context
    std::string m = c->msg;
    destroy_ctx(c);
    c = new (std::nothrow) cp_ctx;
    if (c) {
      c->msg = m;
      c->s = static_cast<hipStream_t>(stream);
      c->N = 0;
    }
    *out = c;
    return st;
  }
  *out = c;
  return CP_OK;
}

cp_status cp_set_factor(cp_ctx *c, int32_t mode, const double *U) {
  if (!c || !c->N) return CP_EINVAL;
  return guard(c, [&] {
    check_mode(c, mode);
    require(U != nullptr, CP_EINVAL, "null factor");
    if (c->f64) do_set_factor<double>(c, mode, U);
    else do_set_factor<float>(c, mode, U);
    c->factor_set[mode] = true;
    c->sampled_mode = c->mttkrp_mode = -1;
  });
}

cp_status cp_set_sigma(cp_ctx *c, const double *sigma) {
  if (!c || !c->N) return CP_EINVAL;
  return guard(c, [&] {
    require(sigma != nullptr, CP_EINVAL, "null sigma");
    hip_ok(hipMemcpyAsync(c->sigma, sigma, c->R * 8, hipMemcpyDeviceToDevice,
                          c->s), "hipMemcpyAsync");
  });
}

cp_status cp_sample(cp_ctx *c, int32_t mode, int64_t J, const double *uni,
                    int32_t *idx_out, double *prob_out) {
  if (!c || !c->N) return CP_EINVAL;
  return guard(c, [&] {
    check_mode(c, mode);
    check_factors(c);
    require(c->sampler != CP_SAMPLER_EXACT, CP_EINVAL,
            "the exact sampler draws nothing");
    require(J >= 1 && J <= c->max_J, CP_EINVAL, "J outside [1, max_J]");
    require(uni != nullptr, CP_EINVAL, "null uniforms");
    if (c->f64) do_sample<double>(c, mode, J, uni);
    else do_sample<float>(c, mode, J, uni);
    if (idx_out)
      hip_ok(hipMemcpyAsync(idx_out, c->sidx, J * (c->N - 1) * 4,
                            hipMemcpyDeviceToDevice, c->s), "hipMemcpyAsync");
    if (prob_out)
      hip_ok(hipMemcpyAsync(prob_out, c->prob, J * 8, hipMemcpyDeviceToDevice,
                            c->s), "hipMemcpyAsync");
  });
}

cp_status cp_set_samples(cp_ctx *c, int32_t mode, int64_t J, const int32_t *idx,
                         const double *prob) {
  if (!c || !c->N) return CP_EINVAL;
  return guard(c, [&] {
    check_mode(c, mode);
    check_factors(c);
    require(c->sampler != CP_SAMPLER_EXACT, CP_EINVAL,
            "the exact sampler takes no samples");
    require(J >= 1 && J <= c->max_J, CP_EINVAL, "J outside [1, max_J]");
    require(idx && prob, CP_EINVAL, "null samples");
    if (c->f64) do_set_samples<double>(c, mode, J, idx, prob);
    else do_set_samples<float>(c, mode, J, idx, prob);
  });
}

cp_status cp_sampled_mttkrp(cp_ctx *c, int32_t mode, void *M_out,
                            int64_t *nnz_extracted) {
  if (!c || !c->N) return CP_EINVAL;
  return guard(c, [&] {
    check_mode(c, mode);
    check_factors(c);
    if (c->sampler == CP_SAMPLER_EXACT) {
      pinv_for(c, make_ml(c, mode), false);
    } else {
      require(c->sampled_mode == mode, CP_ESTATE,
              "cp_sampled_mttkrp without samples for this mode");
    }
    if (c->f64) do_mttkrp<double>(c, mode);
    else do_mttkrp<float>(c, mode);
    if (M_out)
      hip_ok(hipMemcpyAsync(M_out, c->M, c->dims[mode] * c->R * c->tsize(),
                            hipMemcpyDeviceToDevice, c->s), "hipMemcpyAsync");
    if (nnz_extracted) {
      if (c->sampler == CP_SAMPLER_EXACT) {
        *nnz_extracted = c->nnz;
        read_errors(c);
      } else {
        int64_t cnt[2] = {0, 0};
        hip_ok(hipMemcpyAsync(cnt, c->w.counts, 16, hipMemcpyDeviceToHost,
                              c->s), "hipMemcpyAsync");
        read_errors(c);
        *nnz_extracted = cnt[1];
      }
    }
  });
}

cp_status cp_solve_factor(cp_ctx *c, int32_t mode) {
  if (!c || !c->N) return CP_EINVAL;
  return guard(c, [&] {
    check_mode(c, mode);
    require(c->mttkrp_mode == mode, CP_ESTATE,
            "cp_solve_factor without a sampled MTTKRP for this mode");
    if (c->f64) do_solve<double>(c, mode);
    else do_solve<float>(c, mode);
  });
}

cp_status cp_sweep(cp_ctx *c, int32_t nsweeps, int64_t J, const double *uni) {
  if (!c || !c->N) return CP_EINVAL;
  return guard(c, [&] {
    check_factors(c);
    require(nsweeps >= 0, CP_EINVAL, "negative sweep count");
    const bool exact = c->sampler == CP_SAMPLER_EXACT;
    if (!exact) {
      require(J >= 1 && J <= c->max_J, CP_EINVAL, "J outside [1, max_J]");
      require(uni != nullptr, CP_EINVAL, "null uniforms");
    }
    const int N = c->N;
    for (int t = 0; t < nsweeps; ++t)
      for (int j = 0; j < N; ++j) {
        if (exact) {
          pinv_for(c, make_ml(c, j), false);
        } else {
          const double *u = uni + ((int64_t)t * N + j) * J * (N - 1);
          if (c->f64) do_sample<double>(c, j, J, u);
          else do_sample<float>(c, j, J, u);
        }
        if (c->f64) {
          do_mttkrp<double>(c, j);
          do_solve<double>(c, j);
        } else {
          do_mttkrp<float>(c, j);
          do_solve<float>(c, j);
        }
      }
  });
}

cp_status cp_fit(cp_ctx *c, double *fit) {
  if (!c || !c->N || !fit) return CP_EINVAL;
  return guard(c, [&] {
    check_factors(c);
    if (c->f64) do_fit<double>(c, fit);
    else do_fit<float>(c, fit);
  });
}

cp_status cp_sync(cp_ctx *c) {
  if (!c || !c->N) return CP_EINVAL;
  return guard(c, [&] { read_errors(c); });
}

cp_status cp_get_factor(cp_ctx *c, int32_t mode, double *U_out) {
  if (!c || !c->N || !U_out) return CP_EINVAL;
  return guard(c, [&] {
    check_mode(c, mode);
    copy_to_f64(c->U[mode], c->f64, U_out, c->dims[mode] * c->R, c->s);
  });
}

cp_status cp_get_sigma(cp_ctx *c, double *sigma_out) {
  if (!c || !c->N || !sigma_out) return CP_EINVAL;
  return guard(c, [&] {
    hip_ok(hipMemcpyAsync(sigma_out, c->sigma, c->R * 8,
                          hipMemcpyDeviceToDevice, c->s), "hipMemcpyAsync");
  });
}

cp_status cp_get_gram(cp_ctx *c, int32_t mode, double *G_out) {
  if (!c || !c->N || !G_out) return CP_EINVAL;
  return guard(c, [&] {
    check_mode(c, mode);
    hip_ok(hipMemcpyAsync(G_out, c->G[mode], c->R * c->R * 8,
                          hipMemcpyDeviceToDevice, c->s), "hipMemcpyAsync");
  });
}

cp_status cp_get_unique(cp_ctx *c, uint64_t *col_key, int32_t *rep,
                        int32_t *count, double *weight, int64_t cap,
                        int64_t *n_out) {
  if (!c || !c->N) return CP_EINVAL;
  return guard(c, [&] {
    require(c->sampled_mode >= 0, CP_ESTATE, "no samples");
    int64_t cnt[2] = {0, 0};
    hip_ok(hipMemcpyAsync(cnt, c->w.counts, 16, hipMemcpyDeviceToHost, c->s),
           "hipMemcpyAsync");
    hip_ok(hipStreamSynchronize(c->s), "hipStreamSynchronize");
    debug_unique(c->w, cnt[0], c->ix[c->sampled_mode].col_key, col_key, rep,
                 count, weight, cap, c->s);
    if (n_out) *n_out = cnt[0];
    read_errors(c);
  });
}

cp_status cp_get_extracted(cp_ctx *c, uint64_t *col_key, int32_t *row,
                           int32_t *rep, int64_t cap, int64_t *n_out) {
  if (!c || !c->N) return CP_EINVAL;
  return guard(c, [&] {
    require(c->sampled_mode >= 0, CP_ESTATE, "no samples");
    const ModeIndex &ix = c->ix[c->sampled_mode];
    int64_t cnt[2] = {0, 0};
    hip_ok(hipMemcpyAsync(cnt, c->w.counts, 16, hipMemcpyDeviceToHost, c->s),
           "hipMemcpyAsync");
    hip_ok(hipStreamSynchronize(c->s), "hipStreamSynchronize");
    debug_extracted(c->w, cnt[1], ix.col_ptr, ix.col_key, ix.row, col_key, row,
                    rep, cap, c->s);
    if (n_out) *n_out = cnt[1];
    read_errors(c);
  });
}

cp_status cp_profile(cp_ctx *c, int32_t enable) {
  return cp_profile_phases(c, enable ? (1u << CP_NPHASE) - 1 : 0u);
}

cp_status cp_profile_phases(cp_ctx *c, uint32_t mask) {
  if (!c || !c->N) return CP_EINVAL;
  return guard(c, [&] {
    if (mask) c->ev_used = 0;
    c->prof = mask != 0;
    c->prof_mask = mask;
  });
}

cp_status cp_profile_read(cp_ctx *c, double *ms, int64_t *launches) {
  if (!c || !c->N) return CP_EINVAL;
  return guard(c, [&] {
    hip_ok(hipStreamSynchronize(c->s), "hipStreamSynchronize");
    for (int p = 0; p < CP_NPHASE; ++p) {
      if (ms) ms[p] = 0;
      if (launches) launches[p] = 0;
    }
    for (size_t i = 0; i < c->ev_used; ++i) {
      float t = 0;
      hip_ok(hipEventElapsedTime(&t, c->evs[i].a, c->evs[i].b),
             "hipEventElapsedTime");
      const int p = c->evs[i].phase;
      if (ms) ms[p] += t;
      if (launches) launches[p] += 1;
    }
  });
}

cp_status cp_pinv(const double *G, int32_t R, double *Gp, void *stream) {
  if (!G || !Gp || R < 1 || R > MAXR) return CP_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double *scratch = nullptr, *Gfull = nullptr;
  uint32_t *err = nullptr;
  cp_status st = CP_OK;
  if (hipMalloc(&scratch, (size_t)R * R * 8) != hipSuccess ||
      hipMalloc(&Gfull, (size_t)R * R * 8) != hipSuccess ||
      hipMalloc(&err, 4) != hipSuccess) {
    st = CP_ENOMEM;
  } else {
    try {
      ModeList ml;
      std::memset(&ml, 0, sizeof(ml));
      ml.n = 1;
      ml.G[0] = G;
      uint32_t e = 0;
      if (hipMemsetAsync(err, 0, 4, s) != hipSuccess) throw Fail{CP_EHIP, ""};
      hadamard_pinv(ml, R, Gfull, Gp, nullptr, nullptr, scratch, err, s);
      if (hipMemcpyAsync(&e, err, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        throw Fail{CP_EHIP, ""};
      if (e & ERR_NONFINITE) st = CP_ENUMERIC;
      else if (e & ERR_PINV) st = CP_ENUMERIC;
    } catch (const Fail &f) {
      st = f.st;
    } catch (const HipFail &) {
      st = CP_EHIP;
    }
  }
  if (scratch) (void)hipFree(scratch);
  if (Gfull) (void)hipFree(Gfull);
  if (err) (void)hipFree(err);
  return st;
}

// Allocation-free pseudo-inverse: the scratch lives in a file-scope device
// array (one copy per GPU, held until the process ends), resolved per device
// with hipGetSymbolAddress on the first call there.  Layout: Hadamard copy
// (MAXR^2 doubles), pseudo-inverse work (MAXR^2 doubles), error word.
}  // extern "C"

static __device__ __align__(256) double scratch[2 * MAXR * MAXR + 32];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
double *g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};
std::mutex g_noalloc_mu;

__global__ void k_clear_word(uint32_t *w) { *w = 0u; }

// Device address of `scratch` on the current device (resolved once).
cp_status noalloc_scratch(double **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 ||
      dev >= NOALLOC_MAX_DEVICES)
    return CP_EHIP;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
      return CP_EHIP;
    g_noalloc_ptr[dev] = static_cast<double *>(p);
  }
  *out = g_noalloc_ptr[dev];
  return CP_OK;
}
}  // namespace

extern "C" {

cp_status cp_pinv_noalloc(const double *G, int32_t R, double *Gp,
                          void *stream) {
  if (!G || !Gp || R < 1 || R > MAXR) return CP_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double *base = nullptr;
  const cp_status st0 = noalloc_scratch(&base);
  if (st0 != CP_OK) return st0;
  double *Gfull = base;
  double *work = base + MAXR * MAXR;
  uint32_t *err = reinterpret_cast<uint32_t *>(base + 2 * MAXR * MAXR);
  try {
    ModeList ml;
    std::memset(&ml, 0, sizeof(ml));
    ml.n = 1;
    ml.G[0] = G;
    hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(1), 0, s, err);
    CPR_LAUNCH_CHECK();
    hadamard_pinv(ml, R, Gfull, Gp, nullptr, nullptr, work, err, s);
    uint32_t e = 0;
    if (hipMemcpyAsync(&e, err, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return CP_EHIP;
    if (e & (ERR_NONFINITE | ERR_PINV)) return CP_ENUMERIC;
  } catch (const HipFail &) {
    return CP_EHIP;
  }
  return CP_OK;
}

cp_status cp_counters(cp_ctx *c, int64_t *out, int32_t reset) {
  if (!c || !c->N || !out) return CP_EINVAL;
  return guard(c, [&] {
    hip_ok(hipMemcpyAsync(out, c->w.stats, 4 * 8, hipMemcpyDeviceToHost, c->s),
           "hipMemcpyAsync");
    hip_ok(hipStreamSynchronize(c->s), "hipStreamSynchronize");
    if (reset) zero_fill<int64_t>(c->w.stats, 4, c->s);
  });
}

const char *cp_phase_name(int32_t phase) {
  static const char *names[CP_NPHASE] = {
      "pinv", "sample", "merge", "mttkrp", "solve", "gram", "sampler_build",
      "fit"};
  return (phase >= 0 && phase < CP_NPHASE) ? names[phase] : "?";
}

cp_status cp_index_stats(cp_ctx *c, int32_t mode, int64_t *n_cols,
                         int64_t *max_col) {
  if (!c || !c->N) return CP_EINVAL;
  return guard(c, [&] {
    check_mode(c, mode);
    if (n_cols) *n_cols = c->ix[mode].n_cols;
    if (max_col) *max_col = c->ix[mode].max_col;
  });
}

cp_status cp_sts_leaf(cp_ctx *c, int32_t mode, int32_t *leaf_rows,
                      int64_t *leaves) {
  if (!c || !c->N) return CP_EINVAL;
  return guard(c, [&] {
    check_mode(c, mode);
    const bool tree = c->sampler == CP_SAMPLER_STS &&
                      sts_tree_factor(c->N, mode);
    if (leaf_rows) *leaf_rows = tree ? c->Fk[mode] : 0;
    if (leaves) *leaves = tree ? c->P2[mode] : 0;
  });
}

void cp_destroy(cp_ctx *c) { destroy_ctx(c); }

const char *cp_last_error(const cp_ctx *c) {
  return c ? c->msg.c_str() : "null context";
}

const char *cp_status_string(cp_status s) {
  switch (s) {
    case CP_OK: return "CP_OK";
    case CP_EINVAL: return "CP_EINVAL";
    case CP_ENOMEM: return "CP_ENOMEM";
    case CP_EHIP: return "CP_EHIP";
    case CP_ESTATE: return "CP_ESTATE";
    case CP_EDEGENERATE: return "CP_EDEGENERATE";
    case CP_ENUMERIC: return "CP_ENUMERIC";
    case CP_EUNSUPPORTED: return "CP_EUNSUPPORTED";
  }
  return "unknown";
}


// ---------------------------------------------------------------- batches

}  // extern "C"

struct cp_batch {
  BatchState b;
  std::string msg;
};

namespace {
template <typename F>
cp_status bguard(cp_batch *bt, F &&fn) {
  try {
    fn();
    bt->msg.clear();
    return CP_OK;
  } catch (const Fail &f) {
    bt->msg = f.msg;
    return f.st;
  } catch (const HipFail &h) {
    bt->msg = std::string("HIP launch error: ") + hipGetErrorString(h.e) +
              " at " + h.file + ":" + std::to_string(h.line);
    return CP_EHIP;
  } catch (const std::bad_alloc &) {
    bt->msg = "host allocation failed";
    return CP_ENOMEM;
  }
}
}  // namespace

extern "C" {

cp_status cp_batch_init(const cp_tensor *t, int32_t B, const int32_t *ranks,
                        const cp_config *cfg, int32_t nstreams, void *stream,
                        cp_batch **out) {
  if (!out) return CP_EINVAL;
  *out = nullptr;
  if (!t || !cfg || !ranks || !t->dims || !t->idx || !t->val) return CP_EINVAL;
  if (B < 1 || B > 4096 || nstreams < 0 || nstreams > 32) return CP_EINVAL;
  if (t->N < 3 || t->N > MAXN || t->nnz < 1 || t->nnz >= (int64_t(1) << 32))
    return CP_EINVAL;
  for (int k = 0; k < t->N; ++k)
    if (t->dims[k] < 1 || t->dims[k] >= (int64_t(1) << 31)) return CP_EINVAL;
  int rmax = 0;
  for (int i = 0; i < B; ++i) {
    if (ranks[i] < 1 || ranks[i] > MAXR) return CP_EINVAL;
    rmax = std::max(rmax, (int)ranks[i]);
  }
  if (cfg->sampler < 0 || cfg->sampler > 1) return CP_EINVAL;
  if (cfg->precision < 0 || cfg->precision > 2) return CP_EINVAL;
  if (cfg->max_J < 1 || cfg->max_J > (int64_t(1) << 24)) return CP_EINVAL;
  if (cfg->sts_leaf != 0 && cfg->sts_leaf != 16 && cfg->sts_leaf != 32 &&
      cfg->sts_leaf != 64)
    return CP_EINVAL;
  if (!valid_bucket_rows(cfg->bucket_rows)) return CP_EINVAL;
  if (cfg->solve_gram < 0 || cfg->solve_gram > 1) return CP_EINVAL;
  if (cfg->solve_refine < 0 || cfg->solve_refine > 2) return CP_EINVAL;
  cp_batch *bt = new (std::nothrow) cp_batch;
  if (!bt) return CP_ENOMEM;
  *out = bt;
  BatchState &b = bt->b;
  b.s = static_cast<hipStream_t>(stream);
  b.B = B;
  b.N = t->N;
  b.J = cfg->max_J;
  return bguard(bt, [&] {
    cp_config c0 = *cfg;
    c0.R = rmax;
    b.base = new cp_ctx;
    b.base->s = b.s;
    set_config(b.base, t->N, t->dims, &c0);
    init_index(b.base, t);
    const int ns = std::min<int>(nstreams ? nstreams : 4, B);
    for (int q = 0; q < ns; ++q) {
      hipStream_t x = nullptr;
      hip_ok(hipStreamCreateWithFlags(&x, hipStreamNonBlocking),
             "hipStreamCreateWithFlags");
      b.st.push_back(x);
      hipEvent_t e = nullptr;
      hip_ok(hipEventCreateWithFlags(&e, hipEventDisableTiming),
             "hipEventCreate");
      b.join.push_back(e);
    }
    hip_ok(hipEventCreateWithFlags(&b.fork, hipEventDisableTiming),
           "hipEventCreate");
    hip_ok(hipStreamCreateWithFlags(&b.cs, hipStreamNonBlocking),
           "hipStreamCreateWithFlags");
    std::vector<int> order(B);
    for (int i = 0; i < B; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return ranks[x] > ranks[y]; });
    b.r.assign(B, nullptr);
    b.branch.assign(B, 0);
    std::vector<cp_ctx *> owner(ns, nullptr);
    for (int o = 0; o < B; ++o) {
      const int i = order[o], q = o % ns;
      cp_config ci = *cfg;
      ci.R = ranks[i];
      cp_ctx *c = new cp_ctx;
      b.r[i] = c;
      b.branch[i] = q;
      c->s = b.s;
      set_config(c, t->N, t->dims, &ci);
      borrow_index(c, b.base);
      init_state(c);
      if (!owner[q]) {  // the stream's largest rank: its workspaces
        init_workspace(c, b.base, c->R);
        owner[q] = c;
      } else {
        borrow_workspace(c, owner[q]);
      }
      select_bucket_regions(c, b.base);
    }
    read_errors(b.base);
  });
}

cp_status cp_batch_set_factors(cp_batch *bt, int32_t b, int32_t mode,
                               const double *U) {
  if (!bt || !bt->b.base) return CP_EINVAL;
  return bguard(bt, [&] {
    require(b >= 0 && b < bt->b.B, CP_EINVAL, "restart out of range");
    cp_ctx *c = bt->b.r[b];
    check_mode(c, mode);
    require(U != nullptr, CP_EINVAL, "null factor");
    if (c->f64) do_set_factor<double>(c, mode, U);
    else do_set_factor<float>(c, mode, U);
    c->factor_set[mode] = true;
    c->sampled_mode = c->mttkrp_mode = -1;
  });
}

cp_status cp_batch_sweep(cp_batch *bt, const double *uni) {
  if (!bt || !bt->b.base) return CP_EINVAL;
  return bguard(bt, [&] {
    BatchState &b = bt->b;
    require(uni != nullptr, CP_EINVAL, "null uniforms");
    for (cp_ctx *c : b.r) check_factors(c);
    if (!b.exec || uni != b.cap_uni) capture_sweep(b, uni);
    hip_ok(hipGraphLaunch(b.exec, b.s), "hipGraphLaunch");
  });
}

cp_status cp_batch_fit(cp_batch *bt, double *fits) {
  if (!bt || !bt->b.base || !fits) return CP_EINVAL;
  return bguard(bt, [&] {
    for (int i = 0; i < bt->b.B; ++i) {
      cp_ctx *c = bt->b.r[i];
      check_factors(c);
      if (c->f64) do_fit<double>(c, &fits[i]);
      else do_fit<float>(c, &fits[i]);
    }
  });
}

cp_status cp_batch_sync(cp_batch *bt) {
  if (!bt || !bt->b.base) return CP_EINVAL;
  return bguard(bt, [&] {
    for (cp_ctx *c : bt->b.r) read_errors(c);
    read_errors(bt->b.base);
  });
}

cp_status cp_batch_get_factor(cp_batch *bt, int32_t b, int32_t mode,
                              double *U_out) {
  if (!bt || !bt->b.base || !U_out) return CP_EINVAL;
  return bguard(bt, [&] {
    require(b >= 0 && b < bt->b.B, CP_EINVAL, "restart out of range");
    cp_ctx *c = bt->b.r[b];
    check_mode(c, mode);
    copy_to_f64(c->U[mode], c->f64, U_out, c->dims[mode] * c->R, c->s);
  });
}

cp_status cp_batch_get_sigma(cp_batch *bt, int32_t b, double *sigma_out) {
  if (!bt || !bt->b.base || !sigma_out) return CP_EINVAL;
  return bguard(bt, [&] {
    require(b >= 0 && b < bt->b.B, CP_EINVAL, "restart out of range");
    cp_ctx *c = bt->b.r[b];
    hip_ok(hipMemcpyAsync(sigma_out, c->sigma, c->R * 8,
                          hipMemcpyDeviceToDevice, c->s), "hipMemcpyAsync");
  });
}

int32_t cp_batch_stream_of(const cp_batch *bt, int32_t b) {
  if (!bt || b < 0 || b >= bt->b.B) return -1;
  return bt->b.branch[b];
}

void cp_batch_destroy(cp_batch *bt) {
  if (!bt) return;
  destroy_batch(&bt->b);
  delete bt;
}

const char *cp_batch_last_error(const cp_batch *bt) {
  return bt ? bt->msg.c_str() : "null batch";
}

}  // extern "C"
