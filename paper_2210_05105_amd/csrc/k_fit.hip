// Fit of Section 5.1: 1 - ||[sigma; U] - T||_F / ||T||_F with
// ||[sigma; U] - T||^2 = ||T||^2 - 2 <T, [sigma; U]> + sigma^T (*G_k) sigma.
// <T, [sigma; U]> streams mode 0's index once (FP64 accumulation,
// fixed-order block reduction).
#include "internal.h"

#include <algorithm>

namespace cpr {
namespace {

constexpr int FT_THREADS = 256;
constexpr int FT_MAXBLK = 2048;

// <T, [sigma; U]> from mode 0's column-sorted index (the nonzeros in
// (column, row) order), so that no coordinate list is kept.  A block takes
// ranges of FI_E consecutive positions: the offsets of the range's columns
// and their coordinates (decoded from the column keys, mode 1 fastest) are
// staged in LDS; each group of L lanes takes one nonzero, finds its column
// by bisection of the staged offsets and adds
// v * sum_r sigma_r U_0[i_0, r] prod_{k > 0} U_k[i_k, r], lane gl of the
// group holding the VW consecutive columns from gl VW (one 16-byte load per
// factor row when R is a multiple of VW).
constexpr int FI_E = 1024;

template <typename T, int VW>
__device__ __forceinline__ void fit_cols(const T *r, int cb, int R, bool vec,
                                         T (&x)[VW]) {
  if (vec) {
    typedef T vec_t __attribute__((ext_vector_type(VW)));
    const vec_t v = *reinterpret_cast<const vec_t *>(r + (cb <= R - VW ? cb : R - VW));
#pragma unroll
    for (int q = 0; q < VW; ++q) x[q] = v[q];
  } else {
#pragma unroll
    for (int q = 0; q < VW; ++q) x[q] = r[cb + q < R ? cb + q : R - 1];
  }
}

template <typename T, int L>
__global__ void __launch_bounds__(FT_THREADS)
k_fit_index(const int64_t *col_ptr, const uint64_t *col_key, int64_t n_cols,
            const int32_t *row, const T *val, int64_t nnz, const T *U0,
            ModeList ml, const double *sigma, int R, double *partial) {
  constexpr int VW = 16 / sizeof(T);
  constexpr int GPW = WAVE / L, GPB = GPW * (FT_THREADS / WAVE);
  __shared__ int64_t sptr[FI_E + 1];
  __shared__ int32_t scrd[FI_E][MAXN - 1];
  __shared__ int64_t scol[2];
  __shared__ double red[FT_THREADS / WAVE];
  const int l = lane_id(), w = threadIdx.x / WAVE;
  const int gl = l % L, grp = w * GPW + l / L;
  const int cb = gl * VW;
  const bool vec = R % VW == 0;
  double sg[VW];  // sigma of this lane's columns (zero past R)
#pragma unroll
  for (int q = 0; q < VW; ++q) sg[q] = cb + q < R ? sigma[cb + q] : 0.0;
  const int64_t nrange = (nnz + FI_E - 1) / FI_E;
  double acc = 0;
  for (int64_t rg = blockIdx.x; rg < nrange; rg += gridDim.x) {
    const int64_t e0 = rg * FI_E;
    const int64_t e1 = e0 + FI_E < nnz ? e0 + FI_E : nnz;
    if (threadIdx.x < 2) {  // last column starting at or before e0 / e1 - 1
      const int64_t e = threadIdx.x == 0 ? e0 : e1 - 1;
      int64_t lo = 0, hi = n_cols - 1;
      while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (col_ptr[mid] <= e) lo = mid; else hi = mid - 1;
      }
      scol[threadIdx.x] = lo;
    }
    __syncthreads();
    const int64_t c0 = scol[0];
    const int nc = (int)(scol[1] - c0 + 1);  // <= FI_E
    for (int i = threadIdx.x; i <= nc; i += FT_THREADS) sptr[i] = col_ptr[c0 + i];
    for (int i = threadIdx.x; i < nc; i += FT_THREADS) {
      const uint64_t key = col_key[c0 + i];
      for (int q = 0; q < ml.n; ++q)
        scrd[i][q] = (int32_t)((key / ml.stride[q]) % (uint64_t)ml.I[q]);
    }
    __syncthreads();
    for (int64_t e = e0 + grp; e < e1; e += GPB) {
      int lo = 0, hi = nc - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sptr[mid] <= e) lo = mid; else hi = mid - 1;
      }
      T x[VW];
      fit_cols<T, VW>(U0 + (int64_t)row[e] * R, cb, R, vec, x);
      double p[VW];
#pragma unroll
      for (int q = 0; q < VW; ++q) p[q] = sg[q] * (double)x[q];
      for (int k = 0; k < ml.n; ++k) {
        fit_cols<T, VW>(static_cast<const T *>(ml.U[k]) + (int64_t)scrd[lo][k] * R,
                        cb, R, vec, x);
#pragma unroll
        for (int q = 0; q < VW; ++q) p[q] *= (double)x[q];
      }
      double part = 0;
#pragma unroll
      for (int q = 0; q < VW; ++q) part += p[q];
      acc += part * (double)val[e];
    }
    __syncthreads();
  }
  acc = wave_sum(acc);
  if (l == 0) red[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0;
    for (int i = 0; i < FT_THREADS / WAVE; ++i) s += red[i];
    partial[blockIdx.x] = s;
  }
}

__global__ void k_fit_finish(ModeList ml, int N, int R, const double *sigma,
                             const double *partial, int nblk, double normT2,
                             double *out) {
  __shared__ double red[FT_THREADS / WAVE];
  double m2 = 0;
  for (int e = threadIdx.x; e < R * R; e += FT_THREADS) {
    double g = sigma[e / R] * sigma[e % R];
    for (int k = 0; k < N; ++k) g *= ml.G[k][e];
    m2 += g;
  }
  m2 = wave_sum(m2);
  if (lane_id() == 0) red[threadIdx.x / WAVE] = m2;
  __syncthreads();
  if (threadIdx.x == 0) {
    double model2 = 0;
    for (int i = 0; i < FT_THREADS / WAVE; ++i) model2 += red[i];
    double inner = 0;
    for (int b = 0; b < nblk; ++b) inner += partial[b];
    double res2 = normT2 - 2.0 * inner + model2;
    if (!(res2 > 0)) res2 = 0;
    out[0] = 1.0 - sqrt(res2) / sqrt(normT2);
    out[1] = inner;
    out[2] = model2;
  }
}

template <typename T>
__global__ void k_sumsq(const T *v, int64_t n, double *partial) {
  double acc = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    double x = (double)v[e];
    acc += x * x;
  }
  acc = wave_sum(acc);
  __shared__ double red[FT_THREADS / WAVE];
  if (lane_id() == 0) red[threadIdx.x / WAVE] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0;
    for (int i = 0; i < FT_THREADS / WAVE; ++i) s += red[i];
    partial[blockIdx.x] = s;
  }
}

}  // namespace

int fit_blocks(int64_t nnz) {
  return (int)std::min<int64_t>(FT_MAXBLK, std::max<int64_t>(1, (nnz + 1023) / 1024));
}

template <typename T>
void fit_inner_index(const int64_t *col_ptr, const uint64_t *col_key,
                     int64_t n_cols, const int32_t *row, const T *val,
                     int64_t nnz, const T *U0, const ModeList &ml,
                     const double *sigma, int R, double *partial, int nblk,
                     hipStream_t s) {
  const dim3 g(nblk), b(FT_THREADS);
#define CPR_FIT(L)                                                         \
  hipLaunchKernelGGL((k_fit_index<T, L>), g, b, 0, s, col_ptr, col_key,    \
                     n_cols, row, val, nnz, U0, ml, sigma, R, partial)
  // L lanes of VW columns cover the rank (L VW >= R, R <= 128)
  const int vw = 16 / (int)sizeof(T), need = (R + vw - 1) / vw;
  if (need <= 2) CPR_FIT(2);
  else if (need <= 4) CPR_FIT(4);
  else if (need <= 8) CPR_FIT(8);
  else if (need <= 16) CPR_FIT(16);
  else if (need <= 32) CPR_FIT(32);
  else CPR_FIT(64);
#undef CPR_FIT
  CPR_LAUNCH_CHECK();
}
template void fit_inner_index<float>(const int64_t *, const uint64_t *,
                                     int64_t, const int32_t *, const float *,
                                     int64_t, const float *, const ModeList &,
                                     const double *, int, double *, int,
                                     hipStream_t);
template void fit_inner_index<double>(const int64_t *, const uint64_t *,
                                      int64_t, const int32_t *,
                                      const double *, int64_t, const double *,
                                      const ModeList &, const double *, int,
                                      double *, int, hipStream_t);

void fit_finish(const ModeList &ml, int N, int R, const double *sigma,
                const double *partial, int nblk, double normT2, double *out,
                hipStream_t s) {
  hipLaunchKernelGGL(k_fit_finish, dim3(1), dim3(FT_THREADS), 0, s, ml, N, R,
                     sigma, partial, nblk, normT2, out);
  CPR_LAUNCH_CHECK();
}

double sum_squares(const void *val, int fp64, int64_t nnz, hipStream_t s) {
  const int nb = fit_blocks(nnz);
  double *partial = nullptr;
  if (hipMalloc(&partial, nb * sizeof(double)) != hipSuccess) return -1;
  if (fp64)
    hipLaunchKernelGGL((k_sumsq<double>), dim3(nb), dim3(FT_THREADS), 0, s,
                       static_cast<const double *>(val), nnz, partial);
  else
    hipLaunchKernelGGL((k_sumsq<float>), dim3(nb), dim3(FT_THREADS), 0, s,
                       static_cast<const float *>(val), nnz, partial);
  std::vector<double> h(nb);
  double tot = -1;
  if (hipMemcpyAsync(h.data(), partial, nb * sizeof(double),
                     hipMemcpyDeviceToHost, s) == hipSuccess &&
      hipStreamSynchronize(s) == hipSuccess) {
    tot = 0;
    for (double x : h) tot += x;
  }
  (void)hipFree(partial);
  return tot;
}

}  // namespace cpr
