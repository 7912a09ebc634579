// Fit of Section 5.1: 1 - ||[sigma; U] - T||_F / ||T||_F with
// ||[sigma; U] - T||^2 = ||T||^2 - 2 <T, [sigma; U]> + sigma^T (*G_k) sigma.
// <T, [sigma; U]> streams the nonzeros once (FP64 accumulation, fixed-order
// block reduction).
#include "internal.h"

#include <algorithm>

namespace cpr {
namespace {

constexpr int FT_THREADS = 256;
constexpr int FT_MAXBLK = 2048;

template <typename T, int L>
__global__ void __launch_bounds__(FT_THREADS)
k_fit_inner(const int32_t *idx, const T *val, int64_t nnz, int N, ModeList ml,
            const double *sigma, int R, double *partial) {
  constexpr int GPW = WAVE / L;
  const int l = lane_id(), w = threadIdx.x / WAVE;
  const int gl = l % L;
  const int64_t group = ((int64_t)blockIdx.x * (FT_THREADS / WAVE) + w) * GPW + l / L;
  const int64_t ng = (int64_t)gridDim.x * (FT_THREADS / WAVE) * GPW;
  double acc = 0;
  for (int64_t e = group; e < nnz; e += ng) {
    double part = 0;
    for (int r = gl; r < R; r += L) {
      double p = sigma[r];
      for (int k = 0; k < N; ++k)
        p *= (double)static_cast<const T *>(ml.U[k])[(int64_t)idx[e * N + k] * R + r];
      part += p;
    }
    acc += part * (double)val[e];
  }
  acc = wave_sum(acc);
  __shared__ double red[FT_THREADS / WAVE];
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
void fit_inner(const int32_t *idx, const T *val, int64_t nnz, int N,
               const ModeList &ml, const double *sigma, int R, double *partial,
               int nblk, hipStream_t s) {
  const dim3 g(nblk), b(FT_THREADS);
  if (R <= 8)
    hipLaunchKernelGGL((k_fit_inner<T, 8>), g, b, 0, s, idx, val, nnz, N, ml, sigma, R, partial);
  else if (R <= 16)
    hipLaunchKernelGGL((k_fit_inner<T, 16>), g, b, 0, s, idx, val, nnz, N, ml, sigma, R, partial);
  else if (R <= 32)
    hipLaunchKernelGGL((k_fit_inner<T, 32>), g, b, 0, s, idx, val, nnz, N, ml, sigma, R, partial);
  else
    hipLaunchKernelGGL((k_fit_inner<T, 64>), g, b, 0, s, idx, val, nnz, N, ml, sigma, R, partial);
  CPR_LAUNCH_CHECK();
}
template void fit_inner<float>(const int32_t *, const float *, int64_t, int,
                               const ModeList &, const double *, int, double *,
                               int, hipStream_t);
template void fit_inner<double>(const int32_t *, const double *, int64_t, int,
                                const ModeList &, const double *, int, double *,
                                int, hipStream_t);

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
