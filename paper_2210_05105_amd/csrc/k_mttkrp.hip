// Sketch application and the sampled MTTKRP (Section 2.2, Eq. 7, Section 4.3).
//
// 1. lookup: column key of each drawn Khatri-Rao row, binary search in the
//    mode's sorted distinct column keys; the first draw of each column
//    claims it with atomicMin.
// 2. merge: draws of the same column are merged (count c, weight
//    c / (J p)); distinct columns are compacted in first-draw order and the
//    lengths of their nonzero ranges are prefix-summed.
// 3. MTTKRP: the extracted nonzeros are consumed in place from the mode's
//    index (no triple buffer): equal-size chunks of the concatenated ranges
//    are spread over all waves, each nonzero (i, v) of column x adding
//    w_x v h_x to M[i, :] with hardware float atomics.  Work is balanced by
//    nonzeros, not by sample, so a heavy column does not serialise.
#include "internal.h"

#include <algorithm>
#include <climits>

namespace cpr {
namespace {

constexpr int LK_THREADS = 256;

template <typename T>
__global__ void k_sample_rows(ModeList ml, int64_t J, int R,
                              const int32_t *sidx, T *h, uint32_t *err) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= J * R) return;
  const int64_t s = e / R;
  const int r = (int)(e - s * R);
  double v = 1.0;
  for (int q = 0; q < ml.n; ++q) {
    int32_t i = sidx[s * ml.n + q];
    if (i < 0 || i >= ml.I[q]) {
      atomicOr(err, ERR_INDEX);
      i = 0;
    }
    v *= (double)static_cast<const T *>(ml.U[q])[(int64_t)i * R + r];
  }
  h[e] = (T)v;
}

__global__ void __launch_bounds__(LK_THREADS)
k_lookup(ModeList ml, int64_t J, const int32_t *sidx, const uint64_t *col_key,
         int64_t n_cols, int32_t *col_id, int32_t *owner) {
  const int64_t s = (int64_t)blockIdx.x * LK_THREADS + threadIdx.x;
  if (s >= J) return;
  uint64_t key = 0;
  bool ok = true;
  for (int q = 0; q < ml.n; ++q) {
    int32_t i = sidx[s * ml.n + q];
    ok &= (i >= 0 && i < ml.I[q]);
    key += (uint64_t)i * ml.stride[q];
  }
  int64_t lo = 0, hi = n_cols;
  while (lo < hi) {  // first column key >= key
    int64_t mid = (lo + hi) >> 1;
    if (col_key[mid] < key) lo = mid + 1; else hi = mid;
  }
  int32_t cid = (ok && lo < n_cols && col_key[lo] == key) ? (int32_t)lo : -1;
  col_id[s] = cid;
  if (cid >= 0) atomicMin(&owner[cid], (int32_t)s);
}

__global__ void k_dup(int64_t J, const int32_t *col_id, const int32_t *owner,
                      int32_t *dupcnt) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= J) return;
  const int32_t cid = col_id[s];
  if (cid < 0) return;
  const int32_t o = owner[cid];
  if (o != (int32_t)s) atomicAdd(&dupcnt[o], 1);
}

// First draw of each column: flag and nonzero-range length (prefix-summed
// next, to number the distinct columns in draw order and place their
// nonzero ranges).
__global__ void k_first(int64_t J, const int32_t *col_id, const int32_t *owner,
                        const int64_t *col_ptr, int64_t *flag, int64_t *len) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= J) return;
  const int32_t cid = col_id[s];
  const bool first = cid >= 0 && owner[cid] == (int32_t)s;
  flag[s] = first ? 1 : 0;
  len[s] = first ? col_ptr[cid + 1] - col_ptr[cid] : 0;
}

// Compaction of the first draws (weights count / (J p)); restores owner and
// dupcnt for the next call (owner is not read after k_first).
__global__ void k_compact(int64_t J, const double *prob, const int32_t *col_id,
                          const int64_t *flag, const int64_t *len,
                          const int64_t *uidx, const int64_t *off,
                          int32_t *owner, int32_t *dupcnt, int32_t *uq_s,
                          int32_t *uq_cid, int32_t *uq_cnt, double *uq_w,
                          int64_t *uq_off, int64_t *counts, int64_t *stats) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= J) return;
  if (flag[s]) {
    const int64_t u = uidx[s];
    const int32_t cid = col_id[s];
    const int32_t cnt = 1 + dupcnt[s];
    uq_s[u] = (int32_t)s;
    uq_cid[u] = cid;
    uq_cnt[u] = cnt;
    uq_w[u] = (double)cnt / ((double)J * prob[s]);
    uq_off[u] = off[s];
    owner[cid] = INT_MAX;
  }
  dupcnt[s] = 0;
  if (s == J - 1) {
    const int64_t nu = uidx[s] + flag[s], nz = off[s] + len[s];
    uq_off[nu] = nz;
    counts[0] = nu;
    counts[1] = nz;
    if (stats) {  // cumulative: mode solves, distinct columns, nonzeros
      stats[0] += 1;
      stats[1] += nu;
      stats[2] += nz;
    }
  }
}

// Sampled MTTKRP.  Waves take chunks of MT_CHUNK consecutive extracted
// nonzeros round-robin (balance by nonzeros).  In each 64-nonzero batch,
// lane i first resolves nonzero i of the batch on its own (distinct column
// by a short binary search, position in the mode's index, row, w v, sampled
// row id), so the dependent loads of 64 nonzeros are in flight together;
// then groups of L lanes (L = smallest power of two >= R, at most 64) take
// the resolved nonzeros from their owners by shuffle and add w v h into
// M[i, :] with hardware float atomics.
constexpr int MT_THREADS = 256;
constexpr int MT_CHUNK = 256;

template <typename T, int L>
__global__ void __launch_bounds__(MT_THREADS)
k_mttkrp(const int64_t *counts, const int32_t *uq_s, const int32_t *uq_cid,
         const double *uq_w, const int64_t *uq_off, const int64_t *col_ptr,
         const int32_t *row, const T *val, const T *h, int R, T *M) {
  constexpr int GPW = WAVE / L;
  const int l = lane_id();
  const int gl = l % L, g = l / L;
  const int64_t nu = counts[0], nz = counts[1];
  const int64_t wave = (int64_t)blockIdx.x * (MT_THREADS / WAVE) + threadIdx.x / WAVE;
  const int64_t nwave = (int64_t)gridDim.x * (MT_THREADS / WAVE);
  const int64_t nchunk = (nz + MT_CHUNK - 1) / MT_CHUNK;
  for (int64_t c = wave; c < nchunk; c += nwave) {
    const int64_t e0 = c * MT_CHUNK;
    const int64_t e1 = e0 + MT_CHUNK < nz ? e0 + MT_CHUNK : nz;
    // first distinct column of the chunk: last u with uq_off[u] <= e0
    int64_t lo = 0, hi = nu;
    while (hi - lo > 1) {
      int64_t mid = (lo + hi) >> 1;
      if (uq_off[mid] <= e0) lo = mid; else hi = mid;
    }
    const int64_t ub = lo;
    // a chunk touches at most MT_CHUNK + 1 distinct columns
    const int64_t ue = ub + MT_CHUNK + 1 < nu ? ub + MT_CHUNK + 1 : nu;
    for (int64_t b0 = e0; b0 < e1; b0 += WAVE) {
      const int64_t e = b0 + l;
      int32_t my_row = 0, my_s = 0;
      T my_coef = 0;
      if (e < e1) {
        int64_t a = ub, z = ue;  // last u in [ub, ue) with uq_off[u] <= e
        while (z - a > 1) {
          int64_t m = (a + z) >> 1;
          if (uq_off[m] <= e) a = m; else z = m;
        }
        const int64_t p = col_ptr[uq_cid[a]] + (e - uq_off[a]);
        my_row = row[p];
        my_coef = (T)(uq_w[a] * (double)val[p]);
        my_s = uq_s[a];
      }
      const int nb = (int)(e1 - b0 < WAVE ? e1 - b0 : WAVE);
      for (int i = 0; i < nb; i += GPW) {
        const int k = i + g;
        const int32_t rr = __shfl(my_row, k, WAVE);
        const T cf = __shfl(my_coef, k, WAVE);
        const int32_t ss = __shfl(my_s, k, WAVE);
        if (k < nb) {
          const T *hr = h + (int64_t)ss * R;
          T *mr = M + (int64_t)rr * R;
          for (int r = gl; r < R; r += L) unsafeAtomicAdd(mr + r, cf * hr[r]);
        }
      }
    }
  }
}

// Exact MTTKRP (every nonempty column at weight 1): a wave per column,
// Khatri-Rao row decoded from the column key.
template <typename T, int L>
__global__ void __launch_bounds__(MT_THREADS)
k_exact_mttkrp(ModeList ml, int64_t n_cols, const uint64_t *col_key,
               const int64_t *col_ptr, const int32_t *row, const T *val, int R,
               T *M) {
  constexpr int GPW = WAVE / L;
  const int l = lane_id();
  const int gl = l % L, g = l / L;
  const int64_t wave = (int64_t)blockIdx.x * (MT_THREADS / WAVE) + threadIdx.x / WAVE;
  const int64_t nwave = (int64_t)gridDim.x * (MT_THREADS / WAVE);
  for (int64_t c = wave; c < n_cols; c += nwave) {
    uint64_t key = col_key[c];
    int32_t ii[MAXN];
    for (int q = 0; q < ml.n; ++q) {
      ii[q] = (int32_t)(key % (uint64_t)ml.I[q]);
      key /= (uint64_t)ml.I[q];
    }
    const int64_t p0 = col_ptr[c], p1 = col_ptr[c + 1];
    for (int r0 = 0; r0 < R; r0 += L) {
      const int r = r0 + gl;
      double hv = 1.0;
      if (r < R)
        for (int q = 0; q < ml.n; ++q)
          hv *= (double)static_cast<const T *>(ml.U[q])[(int64_t)ii[q] * R + r];
      for (int64_t p = p0 + g; p < p1; p += GPW) {
        if (r < R) unsafeAtomicAdd(M + (int64_t)row[p] * R + r, (T)((double)val[p] * hv));
      }
    }
  }
}

__global__ void k_debug_extracted(const int64_t *counts, const int32_t *uq_s,
                                  const int32_t *uq_cid, const int64_t *uq_off,
                                  const int64_t *col_ptr,
                                  const uint64_t *col_key, const int32_t *row,
                                  uint64_t *ck_out, int32_t *row_out,
                                  int32_t *rep_out, int64_t cap) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nu = counts[0], nz = counts[1];
  if (e >= nz || e >= cap) return;
  int64_t lo = 0, hi = nu;
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) >> 1;
    if (uq_off[mid] <= e) lo = mid; else hi = mid;
  }
  const int32_t cid = uq_cid[lo];
  const int64_t p = col_ptr[cid] + (e - uq_off[lo]);
  if (ck_out) ck_out[e] = col_key[cid];
  if (row_out) row_out[e] = row[p];
  if (rep_out) rep_out[e] = uq_s[lo];
}

__global__ void k_debug_unique(const int64_t *counts, const int32_t *uq_s,
                               const int32_t *uq_cid, const int32_t *uq_cnt,
                               const double *uq_w, const uint64_t *col_key,
                               uint64_t *ck_out, int32_t *rep_out,
                               int32_t *cnt_out, double *w_out, int64_t cap) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= counts[0] || u >= cap) return;
  if (ck_out) ck_out[u] = col_key[uq_cid[u]];
  if (rep_out) rep_out[u] = uq_s[u];
  if (cnt_out) cnt_out[u] = uq_cnt[u];
  if (w_out) w_out[u] = uq_w[u];
}

int mttkrp_grid() { return 256 * 8; }

}  // namespace

template <typename T>
void set_sample_rows(const ModeList &ml, int64_t J, int R, const int32_t *sidx,
                     T *h, uint32_t *err, hipStream_t s) {
  hipLaunchKernelGGL((k_sample_rows<T>), dim3(ceil_div(J * R, 256)), dim3(256),
                     0, s, ml, J, R, sidx, h, err);
  CPR_LAUNCH_CHECK();
}
template void set_sample_rows<float>(const ModeList &, int64_t, int,
                                     const int32_t *, float *, uint32_t *,
                                     hipStream_t);
template void set_sample_rows<double>(const ModeList &, int64_t, int,
                                      const int32_t *, double *, uint32_t *,
                                      hipStream_t);

void lookup_columns(const ModeList &ml, int64_t J, const int32_t *sidx,
                    const uint64_t *col_key, int64_t n_cols, SampleWork &w,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_lookup, dim3(ceil_div(J, LK_THREADS)), dim3(LK_THREADS),
                     0, s, ml, J, sidx, col_key, n_cols, w.col_id, w.owner);
  CPR_LAUNCH_CHECK();
}

void merge_samples(int64_t J, const double *prob, const int64_t *col_ptr,
                   SampleWork &w, hipStream_t s) {
  const dim3 g(ceil_div(J, 256)), b(256);
  int64_t *flag = w.scratch, *len = w.scratch + J, *uidx = w.scratch + 2 * J,
          *off = w.scratch + 3 * J;
  hipLaunchKernelGGL(k_dup, g, b, 0, s, J, w.col_id, w.owner, w.dupcnt);
  hipLaunchKernelGGL(k_first, g, b, 0, s, J, w.col_id, w.owner, col_ptr, flag,
                     len);
  CPR_LAUNCH_CHECK();
  exclusive_scan_i64(flag, uidx, J, w.scan_tmp, s);
  exclusive_scan_i64(len, off, J, w.scan_tmp, s);
  hipLaunchKernelGGL(k_compact, g, b, 0, s, J, prob, w.col_id, flag, len, uidx,
                     off, w.owner, w.dupcnt, w.uq_s, w.uq_cid, w.uq_cnt,
                     w.uq_w, w.uq_off, w.counts, w.stats);
  CPR_LAUNCH_CHECK();
}

template <typename T>
void sampled_mttkrp(const SampleWork &w, int64_t J, const int64_t *col_ptr,
                    const int32_t *row, const T *val, const T *h, int R, T *M,
                    hipStream_t s) {
  const dim3 g(mttkrp_grid()), b(MT_THREADS);
  if (R <= 8)
    hipLaunchKernelGGL((k_mttkrp<T, 8>), g, b, 0, s, w.counts, w.uq_s, w.uq_cid, w.uq_w, w.uq_off, col_ptr, row, val, h, R, M);
  else if (R <= 16)
    hipLaunchKernelGGL((k_mttkrp<T, 16>), g, b, 0, s, w.counts, w.uq_s, w.uq_cid, w.uq_w, w.uq_off, col_ptr, row, val, h, R, M);
  else if (R <= 32)
    hipLaunchKernelGGL((k_mttkrp<T, 32>), g, b, 0, s, w.counts, w.uq_s, w.uq_cid, w.uq_w, w.uq_off, col_ptr, row, val, h, R, M);
  else
    hipLaunchKernelGGL((k_mttkrp<T, 64>), g, b, 0, s, w.counts, w.uq_s, w.uq_cid, w.uq_w, w.uq_off, col_ptr, row, val, h, R, M);
  CPR_LAUNCH_CHECK();
  (void)J;
}
template void sampled_mttkrp<float>(const SampleWork &, int64_t,
                                    const int64_t *, const int32_t *,
                                    const float *, const float *, int, float *,
                                    hipStream_t);
template void sampled_mttkrp<double>(const SampleWork &, int64_t,
                                     const int64_t *, const int32_t *,
                                     const double *, const double *, int,
                                     double *, hipStream_t);

template <typename T>
void exact_mttkrp(const ModeList &ml, int64_t n_cols, const uint64_t *col_key,
                  const int64_t *col_ptr, const int32_t *row, const T *val,
                  int R, T *M, hipStream_t s) {
  const int nb = (int)std::min<int64_t>(mttkrp_grid(), std::max<int64_t>(1, (n_cols + 3) / 4));
  const dim3 g(nb), b(MT_THREADS);
  if (R <= 8)
    hipLaunchKernelGGL((k_exact_mttkrp<T, 8>), g, b, 0, s, ml, n_cols, col_key, col_ptr, row, val, R, M);
  else if (R <= 16)
    hipLaunchKernelGGL((k_exact_mttkrp<T, 16>), g, b, 0, s, ml, n_cols, col_key, col_ptr, row, val, R, M);
  else if (R <= 32)
    hipLaunchKernelGGL((k_exact_mttkrp<T, 32>), g, b, 0, s, ml, n_cols, col_key, col_ptr, row, val, R, M);
  else
    hipLaunchKernelGGL((k_exact_mttkrp<T, 64>), g, b, 0, s, ml, n_cols, col_key, col_ptr, row, val, R, M);
  CPR_LAUNCH_CHECK();
}
template void exact_mttkrp<float>(const ModeList &, int64_t, const uint64_t *,
                                  const int64_t *, const int32_t *,
                                  const float *, int, float *, hipStream_t);
template void exact_mttkrp<double>(const ModeList &, int64_t, const uint64_t *,
                                   const int64_t *, const int32_t *,
                                   const double *, int, double *, hipStream_t);

void debug_extracted(const SampleWork &w, int64_t nz_host,
                     const int64_t *col_ptr, const uint64_t *col_key,
                     const int32_t *row, uint64_t *ck_out, int32_t *row_out,
                     int32_t *rep_out, int64_t cap, hipStream_t s) {
  const int64_t n = nz_host < cap ? nz_host : cap;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_debug_extracted, dim3(ceil_div(n, 256)), dim3(256), 0,
                     s, w.counts, w.uq_s, w.uq_cid, w.uq_off, col_ptr, col_key,
                     row, ck_out, row_out, rep_out, cap);
  CPR_LAUNCH_CHECK();
}

void debug_unique(const SampleWork &w, int64_t nu_host, const uint64_t *col_key,
                  uint64_t *ck_out, int32_t *rep_out, int32_t *cnt_out,
                  double *w_out, int64_t cap, hipStream_t s) {
  const int64_t n = nu_host < cap ? nu_host : cap;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_debug_unique, dim3(ceil_div(n, 256)), dim3(256), 0, s,
                     w.counts, w.uq_s, w.uq_cid, w.uq_cnt, w.uq_w, col_key,
                     ck_out, rep_out, cnt_out, w_out, cap);
  CPR_LAUNCH_CHECK();
}

}  // namespace cpr
