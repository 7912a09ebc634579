// CP-ARLS-LEV on one GPU (Appendix A).  Build (Alg. 2 without the
// all-reduce): leverage scores l_i = U[i] G_k^+ U[i]^T of every row, their
// inclusive prefix sums (the CDF) and total Z.  Draw (Alg. 3 without the
// multinomial split and gather): one inverse-CDF search per (sample, factor),
// index = min{ i : u Z < F(i) }.
#include <algorithm>

#include "internal.h"

namespace cpr {

typedef double double4_t __attribute__((ext_vector_type(4)));

namespace {

// l_i for 16 rows per wave and tile: C = U_tile (16 x R) G^+ (R x R) on
// FP64 MFMA, then l_i = sum_j C[i][j] U[i][j].  Waves stride over the row
// tiles; the last row of positive mass is reduced per block and published
// with one atomicMax.  Up to 64 columns the B operand (G^+, zero beyond R)
// is staged once per block in LDS in fragment order (k-step, column tile,
// lane: 32 KiB at most), so a tile reads it with one conflict-free 8-byte
// LDS load per product instead of from global memory.
constexpr int LV_LDS_NT = 4;  // column tiles staged in LDS at most

template <typename T, int NT>
__global__ void __launch_bounds__(256)
k_leverage(const T *U, int64_t I, int R, const double *Gp, double *lev,
           unsigned long long *last, uint32_t *err) {
  constexpr bool SB = NT <= LV_LDS_NT;
  constexpr int Rp = NT * 16;
  __shared__ unsigned long long smax[4];
  __shared__ double sB[SB ? (Rp / 4) * NT * WAVE : 1];
  const int l = lane_id(), w = threadIdx.x / WAVE;
  if constexpr (SB) {
    for (int e = threadIdx.x; e < (Rp / 4) * NT * WAVE; e += 256) {
      const int ln = e % WAVE, t = (e / WAVE) % NT, ks = e / (WAVE * NT);
      const int ka = 4 * ks + ln / 16, jb = t * 16 + ln % 16;
      sB[e] = (ka < R && jb < R) ? Gp[ka * R + jb] : 0.0;
    }
    __syncthreads();
  }
  const int64_t ntiles = (I + 15) / 16;
  unsigned long long mx = 0;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + w; tile < ntiles;
       tile += (int64_t)gridDim.x * 4) {
    const int64_t row0 = tile * 16;
    double4_t acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = double4_t{0, 0, 0, 0};
    const int64_t ra = row0 + (l % 16);  // A operand row
    const int64_t rac = ra < I ? ra : I - 1;
    // four k-steps per pass: a full unroll would hoist every load of the
    // tile (all registers at four column tiles, spills beyond six)
#pragma unroll 4
    for (int k0 = 0; k0 < Rp; k0 += 4) {
      const int ka = k0 + l / 16;
      const int kac = ka < R ? ka : R - 1;
      const double av = (double)U[rac * R + kac];
      const double a = (ra < I && ka < R) ? av : 0.0;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        double b;
        if constexpr (SB) {
          b = sB[((k0 / 4) * NT + t) * WAVE + l];
        } else {
          const int jb = t * 16 + (l % 16);
          const int jbc = jb < R ? jb : R - 1;
          const double bv = Gp[kac * R + jbc];
          b = (ka < R && jb < R) ? bv : 0.0;
        }
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
      }
    }
    // D[i][j] of v_mfma_f64_16x16x4f64: lane l, element v -> i = l / 16 + 4 v,
    // j = l % 16
    double s[4] = {0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int j = t * 16 + (l % 16);
      const int jc = j < R ? j : R - 1;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = row0 + (l / 16) + 4 * v;
        const int64_t rc = r < I ? r : I - 1;
        const double u = (double)U[rc * R + jc];
        s[v] += (r < I && j < R) ? acc[t][v] * u : 0.0;
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
      for (int o = 1; o < 16; o <<= 1) s[v] += __shfl_xor(s[v], o, WAVE);
    if ((l % 16) == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = row0 + (l / 16) + 4 * v;
        if (r < I) {
          double x = s[v];
          if (!isfinite(x)) atomicOr(err, ERR_NONFINITE);
          x = x > 0 ? x : 0.0;
          lev[r] = x;
          if (x > 0 && (unsigned long long)(r + 1) > mx)
            mx = (unsigned long long)(r + 1);
        }
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long y = __shfl_xor(mx, o, WAVE);
    mx = y > mx ? y : mx;
  }
  if (l == 0) smax[w] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = smax[0];
    for (int q = 1; q < 4; ++q) m = smax[q] > m ? smax[q] : m;
    if (m) atomicMax(last, m);
  }
}

__global__ void k_arls_tail(const double *cdf, int64_t I,
                            const unsigned long long *lastp1, double *Z,
                            int64_t *last, uint32_t *err) {
  const double z = cdf[I - 1];
  *Z = z;
  *last = (int64_t)*lastp1 - 1;
  if (!(z > 0) || *lastp1 == 0) atomicOr(err, ERR_ZERO_MASS);
}

constexpr int DR_THREADS = 256;

// Coarse CDF: the inclusive prefix sum at the end of every 64-row chunk
// (the last chunk ends at row I - 1).
__global__ void k_arls_coarse(const double *cdf, int64_t I, double *coarse) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nb = (I + ARLS_CHUNK - 1) / ARLS_CHUNK;
  if (b >= nb) return;
  const int64_t e = (b + 1) * ARLS_CHUNK - 1;
  coarse[b] = cdf[e < I ? e : I - 1];
}

// Draws: index = min{ i : u Z < F(i) } per (sample, factor).  Each lane
// bisects the coarse CDF for its sample's 64-row chunk (a table 64 times
// shorter than F, mostly cache resident); then the wave settles the 64
// chunks of its 64 samples one after another, each with one coalesced
// load of the chunk's 64 prefix sums and a ballot of u Z < F(i) (the first
// set lane is the row).  The result is the first row whose prefix sum
// exceeds the target, as a bisection of F would give.
template <typename T>
__global__ void __launch_bounds__(DR_THREADS)
k_arls_draw(ModeList ml, int64_t J, int R, const double *uni, int32_t *sidx,
            double *prob, T *h, uint32_t *err) {
  __shared__ int32_t sh_idx[DR_THREADS * (MAXN - 1)];
  const int nq = ml.n;
  const int l = lane_id();
  const int64_t s = (int64_t)blockIdx.x * DR_THREADS + threadIdx.x;
  const bool act = s < J;
  const int64_t sc = act ? s : J - 1;  // lanes past J follow sample J - 1
  double p = 1.0;
  for (int q = 0; q < nq; ++q) {
    double u = uni[sc * nq + q];
    if (!(u >= 0.0 && u < 1.0)) {
      if (act) atomicOr(err, ERR_UNIFORM);
      u = 0.0;
    }
    const double Z = *ml.Z[q];
    const double t = u * Z;
    const int64_t I = ml.I[q];
    const double *cdf = ml.cdf[q], *coarse = ml.coarse[q];
    const int64_t nb = (I + ARLS_CHUNK - 1) / ARLS_CHUNK;
    int64_t lo = 0, hi = nb - 1;  // first chunk whose end exceeds t
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (t < coarse[mid]) hi = mid; else lo = mid + 1;
    }
    const int64_t myb = lo;
    int off = ARLS_CHUNK - 1;
#pragma unroll 4
    for (int i = 0; i < WAVE; ++i) {
      const int64_t bi = __shfl(myb, i, WAVE);
      const double ti = __shfl(t, i, WAVE);
      const int64_t e = bi * ARLS_CHUNK + l;
      const double v = cdf[e < I ? e : I - 1];
      const uint64_t m = __ballot(e < I && ti < v);
      if (l == i && m) off = __ffsll((long long)m) - 1;
    }
    int64_t idx = myb * ARLS_CHUNK + off;
    const int64_t last = *ml.last[q];
    if (idx > last) idx = last;  // rounding past the end: last positive row
    if (idx < 0) idx = 0;
    if (act) sidx[s * nq + q] = (int32_t)idx;
    sh_idx[threadIdx.x * nq + q] = (int32_t)idx;
    p = p * (ml.lev[q][idx] / Z);
  }
  if (act) prob[s] = p;
  __syncthreads();
  // Khatri-Rao rows of the block's samples, lanes over columns
  const int64_t s0 = (int64_t)blockIdx.x * DR_THREADS;
  for (int e = threadIdx.x; e < DR_THREADS * R; e += DR_THREADS) {
    const int sl = e / R, r = e - sl * R;
    if (s0 + sl >= J) break;
    double v = 1.0;
    for (int q = 0; q < nq; ++q)
      v *= (double)static_cast<const T *>(ml.U[q])[(int64_t)sh_idx[sl * nq + q] * R + r];
    h[(s0 + sl) * R + r] = (T)v;
  }
}

}  // namespace

template <typename T>
void arls_build(const T *U, int64_t I, int R, const double *Gp, double *lev,
                double *cdf, double *coarse, double *Z, int64_t *last,
                void *tmp, uint32_t *err, hipStream_t s) {
  unsigned long long *lastp1 = static_cast<unsigned long long *>(tmp);
  void *scan_tmp = static_cast<char *>(tmp) + 256;
  zero_fill<int64_t>(reinterpret_cast<int64_t *>(lastp1), 1, s);
  const int nt = (R + 15) / 16;
  const int64_t ntiles = (I + 15) / 16;
  // one round of resident blocks: four per CU up to four column tiles
  // (G^+ in LDS, at most 91 registers), two beyond
  const int64_t gmax = nt <= LV_LDS_NT ? 1024 : 512;
  const dim3 g((unsigned)std::min<int64_t>(ceil_div(ntiles, 4), gmax)), b(256);
  switch (nt) {
    case 1: hipLaunchKernelGGL((k_leverage<T, 1>), g, b, 0, s, U, I, R, Gp, lev, lastp1, err); break;
    case 2: hipLaunchKernelGGL((k_leverage<T, 2>), g, b, 0, s, U, I, R, Gp, lev, lastp1, err); break;
    case 3: hipLaunchKernelGGL((k_leverage<T, 3>), g, b, 0, s, U, I, R, Gp, lev, lastp1, err); break;
    case 4: hipLaunchKernelGGL((k_leverage<T, 4>), g, b, 0, s, U, I, R, Gp, lev, lastp1, err); break;
    case 5: hipLaunchKernelGGL((k_leverage<T, 5>), g, b, 0, s, U, I, R, Gp, lev, lastp1, err); break;
    case 6: hipLaunchKernelGGL((k_leverage<T, 6>), g, b, 0, s, U, I, R, Gp, lev, lastp1, err); break;
    case 7: hipLaunchKernelGGL((k_leverage<T, 7>), g, b, 0, s, U, I, R, Gp, lev, lastp1, err); break;
    default: hipLaunchKernelGGL((k_leverage<T, 8>), g, b, 0, s, U, I, R, Gp, lev, lastp1, err); break;
  }
  CPR_LAUNCH_CHECK();
  inclusive_scan_f64(lev, cdf, I, scan_tmp, s);
  hipLaunchKernelGGL(k_arls_tail, dim3(1), dim3(1), 0, s, cdf, I, lastp1, Z,
                     last, err);
  const int64_t nb = (I + ARLS_CHUNK - 1) / ARLS_CHUNK;
  hipLaunchKernelGGL(k_arls_coarse, dim3(ceil_div(nb, 256)), dim3(256), 0, s,
                     cdf, I, coarse);
  CPR_LAUNCH_CHECK();
}
template void arls_build<float>(const float *, int64_t, int, const double *,
                                double *, double *, double *, double *,
                                int64_t *, void *, uint32_t *, hipStream_t);
template void arls_build<double>(const double *, int64_t, int, const double *,
                                 double *, double *, double *, double *,
                                 int64_t *, void *, uint32_t *, hipStream_t);

template <typename T>
void arls_draw(const ModeList &ml, int64_t J, int R, const double *uni,
               int32_t *sidx, double *prob, T *h, uint32_t *err,
               hipStream_t s) {
  hipLaunchKernelGGL((k_arls_draw<T>), dim3(ceil_div(J, DR_THREADS)),
                     dim3(DR_THREADS), 0, s, ml, J, R, uni, sidx, prob, h, err);
  CPR_LAUNCH_CHECK();
}
template void arls_draw<float>(const ModeList &, int64_t, int, const double *,
                               int32_t *, double *, float *, uint32_t *,
                               hipStream_t);
template void arls_draw<double>(const ModeList &, int64_t, int, const double *,
                                int32_t *, double *, double *, uint32_t *,
                                hipStream_t);

}  // namespace cpr
