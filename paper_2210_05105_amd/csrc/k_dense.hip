// Dense kernels: factor Grams on FP64 MFMA, the R x R Hadamard Gram and its
// pseudo-inverse (Eq. 4, Eq. 5), the row-wise solve U_j = M G^+ with one
// refinement step, and column renormalisation (Alg. 1).
#include "internal.h"

#include <algorithm>
#include <type_traits>

namespace cpr {

typedef double double4_t __attribute__((ext_vector_type(4)));

namespace {

// ---------------------------------------------------------------------------
// Gram U^T U.  Each block stages 64-row chunks of U in LDS (as FP64, columns
// padded to a multiple of 16) and its four waves accumulate the upper-
// triangular 16x16 output tiles with v_mfma_f64_16x16x4f64.  Per-block
// partial Grams are summed in a fixed order by a second kernel, so the
// result is deterministic.  SCALE: the staging reads the solve's FP64 rows
// X instead and writes the factor U = X / sigma (zero columns stay zero) in
// the factor's precision; the Gram is of the stored values.
// ---------------------------------------------------------------------------
constexpr int GR_THREADS = 256;
constexpr int GR_ROWS = 64;      // row granularity of the block ranges
constexpr int GR_ELEMS = 4096;   // staged entries per chunk (32 KiB of LDS)
constexpr int GR_MAXBLK = 512;

template <typename T, int TPW, bool SCALE>
__global__ void __launch_bounds__(GR_THREADS)
k_gram_partial(const T *U, const double *X, const double *sigma, T *Uout,
               int64_t I, int R, int Rp, int64_t rows_per_blk,
               double *partial) {
  extern __shared__ double lds[];  // RC x Rp <= GR_ELEMS
  const int w = threadIdx.x / WAVE, l = lane_id();
  const int nt = Rp / 16;
  const int ntri = nt * (nt + 1) / 2;
  int ta[TPW], tb[TPW];
  double4_t acc[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    int t = w + 4 * i;
    ta[i] = tb[i] = -1;
    acc[i] = double4_t{0, 0, 0, 0};
    if (t < ntri) {  // t -> (a, b), a <= b, row-major upper triangle
      int a = 0, rem = t;
      while (rem >= nt - a) { rem -= nt - a; ++a; }
      ta[i] = a;
      tb[i] = a + rem;
    }
  }
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t r1 = std::min<int64_t>(I, r0 + rows_per_blk);
  // chunks of RC rows (RC Rp <= GR_ELEMS, RC a multiple of 4), one batch
  // of PE clamped loads per thread each, masked when stored; the next
  // chunk's batch is issued before the current chunk's MFMAs
  const int RC = (GR_ELEMS / Rp) & ~3, NE = RC * Rp;
  constexpr int PE = GR_ELEMS / GR_THREADS;
  double v[PE];
  auto load = [&](int64_t c0) {
    const int nrow = (int)std::min<int64_t>(RC, r1 - c0);
#pragma unroll
    for (int q = 0; q < PE; ++q) {
      const int e = q * GR_THREADS + threadIdx.x;
      const int rr = e / Rp, cc = e - rr * Rp;
      const int rc = rr < nrow ? rr : nrow - 1, ccc = cc < R ? cc : R - 1;
      if constexpr (SCALE) v[q] = X[(c0 + rc) * R + ccc];
      else v[q] = (double)U[(c0 + rc) * R + ccc];
    }
  };
  __shared__ double ssg[SCALE ? MAXR : 1];  // 1 / sigma, read per entry
  if constexpr (SCALE)
    for (int c = threadIdx.x; c < R; c += GR_THREADS) ssg[c] = inv_or_zero(sigma[c]);
  if (r0 < r1) load(r0);
  for (int64_t c0 = r0; c0 < r1; c0 += RC) {
    const int nrow = (int)std::min<int64_t>(RC, r1 - c0);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PE; ++q) {
      const int e = q * GR_THREADS + threadIdx.x;
      const int rr = e / Rp, cc = e - rr * Rp;
      const bool in = rr < nrow && cc < R;
      double x = v[q];
      if constexpr (SCALE) {
        const T u = (T)(x * ssg[cc < R ? cc : R - 1]);
        if (in) Uout[(c0 + rr) * R + cc] = u;
        x = (double)u;
      }
      if (e < NE) lds[e] = in ? x : 0.0;
    }
    __syncthreads();
    if (c0 + RC < r1) load(c0 + RC);
    for (int k0 = 0; k0 < RC; k0 += 4) {
      const double *rowp = lds + (k0 + l / 16) * Rp + (l % 16);
#pragma unroll
      for (int i = 0; i < TPW; ++i) {
        if (ta[i] < 0) continue;
        double a = rowp[ta[i] * 16];
        double b = rowp[tb[i] * 16];
        acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[i], 0, 0, 0);
      }
    }
  }
  // D[i][j] of v_mfma_f64_16x16x4f64: lane l, element v -> i = l / 16 + 4 v,
  // j = l % 16
  double *out = partial + (int64_t)blockIdx.x * R * R;
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    if (ta[i] < 0) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int gi = ta[i] * 16 + (l / 16) + 4 * v;
      int gj = tb[i] * 16 + (l % 16);
      if (gi < R && gj < R) {
        out[gi * R + gj] = acc[i][v];
        out[gj * R + gi] = acc[i][v];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Gram U^T U in reduced precision (FP32 factors).  Blocks of 8 waves stage
// GL_RC-row chunks of U (read linearly, coalesced) in LDS; output tiles
// accumulate on FP32 MFMA in FP32, flushed into FP64 registers after every
// chunk (GL_RC rows of FP32 accumulation per flush), then per-block partials
// reduced in FP64 in a fixed order as for the FP64 Gram.
//   GRAM_F32:    v_mfma_f32_16x16x4f32 on the FP32 values (LDS row-major).
//   GRAM_BF16X3: each value split once, at staging, into u = hi + lo, two
//                BF16 numbers (round to nearest even), kept column-major in
//                LDS so that one 8-byte read gives a lane its 4 k-values;
//                u_a u_b is taken as hi_a hi_b + hi_a lo_b + lo_a hi_b on
//                v_mfma_f32_16x16x16bf16 (products exact in FP32, relative
//                error of the dropped lo_a lo_b term about 2^-16).
// D layout of both FP32 MFMAs: lane l, element v holds D[4 (l / 16) + v]
// [l % 16].
// ---------------------------------------------------------------------------
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef short short4_t __attribute__((ext_vector_type(4)));
constexpr int GL_THREADS = 512;
constexpr int GL_RC = 64;           // rows per staged chunk (multiple of 16)
constexpr int GL_CS = GL_RC + 4;    // BF16 column stride in LDS (shorts)
constexpr int GL_MAXBLK = 1024;
constexpr int GL_PE = GL_RC * MAXR / GL_THREADS;  // staged values per thread

__device__ __forceinline__ short bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}
__device__ __forceinline__ float bf16_val(short h) {
  return __uint_as_float(((uint32_t)(uint16_t)h) << 16);
}

int gram_lp_blocks(int64_t I, int64_t *rows_per_blk) {
  const int64_t chunks = std::max<int64_t>((I + GL_RC - 1) / GL_RC, 1);
  int nblk = (int)std::min<int64_t>(chunks, GL_MAXBLK);
  const int64_t cpb = (chunks + nblk - 1) / nblk;
  *rows_per_blk = cpb * GL_RC;
  return (int)std::max<int64_t>(1, (I + *rows_per_blk - 1) / *rows_per_blk);
}

// VEC: FP32 values moved four at a time (R a multiple of 4 and 16-byte
// aligned rows, so that four consecutive values of a chunk share a row)
template <int MODE, int TPW, bool SCALE, typename XT, bool VEC>
__global__ void __launch_bounds__(GL_THREADS)
__attribute__((amdgpu_waves_per_eu(VEC && SCALE && TPW <= 4 ? 4 : 1)))
k_gram_lp(const float *U, const XT *X, const double *sigma, float *Uout,
          int64_t I, int R, int Rp, int64_t rows_per_blk, double *partial) {
  constexpr int LDS_BYTES = MODE == GRAM_F32 ? GL_RC * (MAXR + 4) * 4
                                             : 2 * MAXR * GL_CS * 2;
  __shared__ __align__(16) char lds_raw[LDS_BYTES];
  __shared__ double ssg[SCALE ? MAXR : 1];  // 1 / sigma, read from LDS
  float *ldsf = reinterpret_cast<float *>(lds_raw);  // F32: GL_RC x RS
  short *hiT = reinterpret_cast<short *>(lds_raw);   // BF16: Rp x GL_CS
  short *loT = hiT + MAXR * GL_CS;
  const int RS = Rp + 4;  // F32 row stride
  const int w = threadIdx.x / WAVE, l = lane_id();
  const int nt = Rp / 16;
  const int ntri = nt * (nt + 1) / 2;
  int ta[TPW], tb[TPW];
  float4_t acc[TPW];
  double accd[TPW][4];
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int t = w + (GL_THREADS / WAVE) * i;
    ta[i] = tb[i] = -1;
    acc[i] = float4_t{0, 0, 0, 0};
#pragma unroll
    for (int v = 0; v < 4; ++v) accd[i][v] = 0.0;
    if (t < ntri) {
      int a = 0, rem = t;
      while (rem >= nt - a) { rem -= nt - a; ++a; }
      ta[i] = a;
      tb[i] = a + rem;
    }
  }
  // padding (columns R..Rp-1, rows past a short last chunk) stays zero
  for (int e = threadIdx.x; e < LDS_BYTES / 4; e += GL_THREADS)
    reinterpret_cast<uint32_t *>(lds_raw)[e] = 0u;
  if constexpr (SCALE)
    for (int c = threadIdx.x; c < R; c += GL_THREADS) ssg[c] = inv_or_zero(sigma[c]);
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t r1 = std::min<int64_t>(I, r0 + rows_per_blk);
  const float rinv = 1.0f / (float)R;
  // the chunk's nrow x R values are contiguous: value f of the chunk is
  // row f / R, column f % R (the float quotient is exact to well under the
  // 0.5 / R margin for f < GL_RC * MAXR)
  using V = typename std::conditional<SCALE, XT, float>::type;
  static_assert(!VEC || std::is_same<V, float>::value, "FP32 values only");
  constexpr int VW = VEC ? 4 : 1;      // values per load
  constexpr int NL = GL_PE / VW;       // loads per thread per chunk
  // DEPTH chunks of values in flight: while one is staged and multiplied,
  // the one DEPTH chunks ahead is being loaded (one for the 16-byte scaling
  // pass, whose 128-register bound lets two blocks share a CU)
  constexpr int DEPTH = VEC && SCALE && TPW <= 4 ? 1 : 2;
  V va[GL_PE], vb[GL_PE];
  auto load = [&](int64_t c0, V (&v)[GL_PE]) {
    const int nv = (int)std::min<int64_t>(GL_RC, r1 - c0) * R;
    const V *src;
    if constexpr (SCALE) src = X + c0 * R;
    else src = U + c0 * R;
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int f = (q * GL_THREADS + threadIdx.x) * VW;
      if (f < nv) {
        if constexpr (VEC) {
          const float4_t x = *reinterpret_cast<const float4_t *>(src + f);
#pragma unroll
          for (int j = 0; j < 4; ++j) v[4 * q + j] = x[j];
        } else {
          v[q] = src[f];
        }
      }
    }
  };
  auto step = [&](int64_t c0, V (&v)[GL_PE]) {
    const int nrow = (int)std::min<int64_t>(GL_RC, r1 - c0);
    const int nv = nrow * R;
    __syncthreads();  // the previous chunk's products are done
    if (nrow < GL_RC)  // short last chunk: clear the rows it leaves
      for (int e = threadIdx.x; e < (GL_RC - nrow) * R; e += GL_THREADS) {
        const int rr = nrow + e / R, cc = e % R;
        if constexpr (MODE == GRAM_F32) ldsf[rr * RS + cc] = 0.0f;
        else hiT[cc * GL_CS + rr] = loT[cc * GL_CS + rr] = 0;
      }
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      const int f = (q * GL_THREADS + threadIdx.x) * VW;
      if (f < nv) {
        const int rr = (int)(((float)f + 0.5f) * rinv), cc = f - rr * R;
        float x[VW];
#pragma unroll
        for (int j = 0; j < VW; ++j) {
          if constexpr (SCALE) x[j] = (float)((double)v[VW * q + j] * ssg[cc + j]);
          else x[j] = v[VW * q + j];
        }
        if constexpr (SCALE) {
          if constexpr (VEC)
            *reinterpret_cast<float4_t *>(Uout + c0 * R + f) =
                float4_t{x[0], x[1], x[2], x[3]};
          else
            Uout[c0 * R + f] = x[0];
        }
#pragma unroll
        for (int j = 0; j < VW; ++j) {
          if constexpr (MODE == GRAM_F32) {
            ldsf[rr * RS + cc + j] = x[j];
          } else {
            const short h = bf16_rne(x[j]);
            hiT[(cc + j) * GL_CS + rr] = h;
            loT[(cc + j) * GL_CS + rr] = bf16_rne(x[j] - bf16_val(h));
          }
        }
      }
    }
    __syncthreads();
    if (c0 + DEPTH * GL_RC < r1) load(c0 + DEPTH * GL_RC, v);
    if constexpr (MODE == GRAM_F32) {
#pragma unroll 2
      for (int k0 = 0; k0 < GL_RC; k0 += 4) {
        const float *rowp = ldsf + (k0 + l / 16) * RS + (l % 16);
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
          if (ta[i] < 0) continue;
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(
              rowp[ta[i] * 16], rowp[tb[i] * 16], acc[i], 0, 0, 0);
        }
      }
    } else {
#pragma unroll 1
      for (int k0 = 0; k0 < GL_RC; k0 += 16) {
        const int ko = k0 + 4 * (l / 16);
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
          if (ta[i] < 0) continue;
          const int ca = (ta[i] * 16 + (l % 16)) * GL_CS + ko;
          const int cb = (tb[i] * 16 + (l % 16)) * GL_CS + ko;
          const short4_t ah = *reinterpret_cast<const short4_t *>(hiT + ca);
          const short4_t al = *reinterpret_cast<const short4_t *>(loT + ca);
          const short4_t bh = *reinterpret_cast<const short4_t *>(hiT + cb);
          const short4_t bl = *reinterpret_cast<const short4_t *>(loT + cb);
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc[i], 0, 0, 0);
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc[i], 0, 0, 0);
          acc[i] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc[i], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < TPW; ++i) {  // flush the chunk's FP32 sums
#pragma unroll
      for (int vv = 0; vv < 4; ++vv) accd[i][vv] += (double)acc[i][vv];
      acc[i] = float4_t{0, 0, 0, 0};
    }
  };
  if (r0 < r1) load(r0, va);
  if constexpr (DEPTH == 1) {
    for (int64_t c0 = r0; c0 < r1; c0 += GL_RC) step(c0, va);
  } else {
    if (r0 + GL_RC < r1) load(r0 + GL_RC, vb);
    for (int64_t c0 = r0; c0 < r1; c0 += 2 * GL_RC) {
      step(c0, va);
      if (c0 + GL_RC < r1) step(c0 + GL_RC, vb);
    }
  }
  double *out = partial + (int64_t)blockIdx.x * R * R;
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    if (ta[i] < 0) continue;
#pragma unroll
    for (int vv = 0; vv < 4; ++vv) {
      const int gi = ta[i] * 16 + 4 * (l / 16) + vv;
      const int gj = tb[i] * 16 + (l % 16);
      // a diagonal tile holds both (a, b) and (b, a), rounded differently
      // (hi_a lo_b and lo_a hi_b enter in different MFMAs): its upper
      // triangle is written to both halves so that G is exactly symmetric
      if (gi < R && gj < R && gi <= gj) {
        out[gi * R + gj] = accd[i][vv];
        out[gj * R + gi] = accd[i][vv];
      }
    }
  }
}

// out[c] = sum over b of P[b][c] (P is nrows x n), in a fixed order: CB
// columns per block, 256 / CB row lanes per column striding over the rows
// with 8 independent partial sums (loads in flight), combined pairwise;
// then the lane sums are added in lane order.  Optionally out[c] =
// sqrt(sum).
template <int CB>
__global__ void __launch_bounds__(256)
k_colsum(const double *P, int nrows, int n, double *out, int take_sqrt,
         uint32_t *err) {
  constexpr int RL = 256 / CB;
  __shared__ double red[RL][CB + 1];
  const int cl = threadIdx.x % CB, rl = threadIdx.x / CB;
  const int c = blockIdx.x * CB + cl;
  double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (c < n) {
    int b = rl;
    for (; b + 7 * RL < nrows; b += 8 * RL) {
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] += P[(int64_t)(b + u * RL) * n + c];
    }
    for (; b < nrows; b += RL) a[0] += P[(int64_t)b * n + c];
  }
  red[rl][cl] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  __syncthreads();
  if (rl == 0 && c < n) {
    double t = 0;
    for (int i = 0; i < RL; ++i) t += red[i][cl];
    if (take_sqrt) {
      t = sqrt(t);
      if (!isfinite(t)) atomicOr(err, ERR_NONFINITE);
    }
    out[c] = t;
  }
}

// column sums with enough blocks to spread the rows' loads
void colsum(const double *P, int nrows, int n, double *out, int take_sqrt,
            uint32_t *err, hipStream_t s) {
  if (n <= 128)
    hipLaunchKernelGGL(k_colsum<4>, dim3(ceil_div(n, 4)), dim3(256), 0, s, P,
                       nrows, n, out, take_sqrt, err);
  else
    hipLaunchKernelGGL(k_colsum<16>, dim3(ceil_div(n, 16)), dim3(256), 0, s,
                       P, nrows, n, out, take_sqrt, err);
}

int gram_blocks(int64_t I, int64_t *rows_per_blk) {
  int64_t chunks = (I + GR_ROWS - 1) / GR_ROWS;
  int nblk = (int)std::min<int64_t>(std::max<int64_t>(chunks, 1), GR_MAXBLK);
  int64_t cpb = (chunks + nblk - 1) / nblk;
  *rows_per_blk = std::max<int64_t>(cpb, 1) * GR_ROWS;
  nblk = (int)std::max<int64_t>(1, (I + *rows_per_blk - 1) / *rows_per_blk);
  return nblk;
}

template <typename T, int TPW, bool SCALE>
void launch_gram(const T *U, const double *X, const double *sigma, T *Uout,
                 int64_t I, int R, int Rp, double *partial, int nblk,
                 int64_t rpb, hipStream_t s) {
  hipLaunchKernelGGL((k_gram_partial<T, TPW, SCALE>), dim3(nblk),
                     dim3(GR_THREADS), GR_ELEMS * sizeof(double), s, U, X,
                     sigma, Uout, I, R, Rp, rpb, partial);
}

// ---------------------------------------------------------------------------
// Hadamard Gram and pseudo-inverse in one workgroup.
// ---------------------------------------------------------------------------
constexpr int PV_THREADS = 256;

__device__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  const int w = threadIdx.x / WAVE;
  __syncthreads();
  if (lane_id() == 0) red[w] = v;
  __syncthreads();
  double t = 0;
  for (int i = 0; i < PV_THREADS / WAVE; ++i) t += red[i];
  __syncthreads();
  return t;
}

__device__ double block_max(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
  const int w = threadIdx.x / WAVE;
  __syncthreads();
  if (lane_id() == 0) red[w] = v;
  __syncthreads();
  double t = red[0];
  for (int i = 1; i < PV_THREADS / WAVE; ++i) t = fmax(t, red[i]);
  __syncthreads();
  return t;
}

// A (LDS) holds G.  On success Gp = (L L^T)^{-1}; returns false if some
// pivot is <= tol (then A is garbage).
__device__ bool chol_inverse(double *A, int R, double tol, double *W,
                             double *Gp, int *flag) {
  const int t = threadIdx.x;
  if (t == 0) *flag = 1;
  __syncthreads();
  for (int k = 0; k < R; ++k) {
    const double d = A[k * R + k];
    if (!(d > tol)) {
      if (t == 0) *flag = 0;
    }
    __syncthreads();
    if (!*flag) return false;
    const double lkk = sqrt(d);
    for (int i = k + 1 + t; i < R; i += PV_THREADS) A[i * R + k] /= lkk;
    __syncthreads();
    if (t == 0) A[k * R + k] = lkk;
    // trailing update of the lower triangle
    const int m = R - k - 1;
    for (int e = t; e < m * m; e += PV_THREADS) {
      int i = k + 1 + e / m, c = k + 1 + e % m;
      if (c <= i) A[i * R + c] -= A[i * R + k] * A[c * R + k];
    }
    __syncthreads();
  }
  // W = L^{-1} (column c by thread c), forward substitution
  for (int c = t; c < R; c += PV_THREADS) {
    for (int i = 0; i < R; ++i) {
      if (i < c) { W[i * R + c] = 0; continue; }
      double acc = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) acc -= A[i * R + k] * W[k * R + c];
      W[i * R + c] = acc / A[i * R + i];
    }
  }
  __threadfence_block();
  __syncthreads();
  // Gp = W^T W
  for (int e = t; e < R * R; e += PV_THREADS) {
    int a = e / R, b = e % R;
    int k0 = a > b ? a : b;
    double acc = 0;
    for (int k = k0; k < R; ++k) acc += W[k * R + a] * W[k * R + b];
    Gp[e] = acc;
  }
  return true;
}

// As chol_inverse, for R > 64, where A alone fills the LDS: L^{-1} is kept
// in the strict upper triangle of A, transposed (W[i][c] at A[c][i], i > c;
// L stays in the lower triangle), with its diagonal in wd (R doubles of
// LDS), so the substitution and the product W^T W read LDS only.  Thread c
// forms column c of W in order of rows.
__device__ bool chol_inverse_lds(double *A, int R, double tol, double *wd,
                                 double *Gp, int *flag) {
  const int t = threadIdx.x;
  const int tr = t / 16, tc = t % 16;  // 16 x 16 thread grid of the update
  if (t == 0) *flag = 1;
  __syncthreads();
  for (int k = 0; k < R; ++k) {
    const double d = A[k * R + k];
    if (!(d > tol)) {
      if (t == 0) *flag = 0;
    }
    __syncthreads();
    if (!*flag) return false;
    const double lkk = sqrt(d);
    for (int i = k + 1 + t; i < R; i += PV_THREADS) A[i * R + k] /= lkk;
    __syncthreads();
    if (t == 0) A[k * R + k] = lkk;
    // trailing update of the lower triangle
    for (int i = k + 1 + tr; i < R; i += 16) {
      const double aik = A[i * R + k];
      for (int c = k + 1 + tc; c <= i; c += 16) A[i * R + c] -= aik * A[c * R + k];
    }
    __syncthreads();
  }
  // W = L^{-1}: W[c][c] = 1 / L[c][c];
  // W[i][c] = -(sum_{k = c}^{i - 1} L[i][k] W[k][c]) / L[i][i], i > c
  // (four partial sums in flight: the LDS loads pipeline)
  for (int c = t; c < R; c += PV_THREADS) {
    const double wcc = 1.0 / A[c * R + c];
    wd[c] = wcc;
    const double *wc = A + c * R;  // W[k][c] at wc[k], k > c
    for (int i = c + 1; i < R; ++i) {
      const double *li = A + i * R;
      double s0 = li[c] * wcc, s1 = 0, s2 = 0, s3 = 0;
      int k = c + 1;
      for (; k + 3 < i; k += 4) {
        s0 += li[k] * wc[k];
        s1 += li[k + 1] * wc[k + 1];
        s2 += li[k + 2] * wc[k + 2];
        s3 += li[k + 3] * wc[k + 3];
      }
      for (; k < i; ++k) s0 += li[k] * wc[k];
      A[c * R + i] = -((s0 + s1) + (s2 + s3)) / li[i];
    }
  }
  __syncthreads();
  // Gp = W^T W: Gp[a][b] = sum_{k >= max(a, b)} W[k][a] W[k][b]
  for (int e = t; e < R * R; e += PV_THREADS) {
    const int a = e / R, b = e % R;
    const int k0 = a > b ? a : b;
    const double wa = k0 == a ? wd[a] : A[a * R + k0];
    const double wb = k0 == b ? wd[b] : A[b * R + k0];
    const double *ra = A + a * R, *rb = A + b * R;
    double s0 = wa * wb, s1 = 0, s2 = 0, s3 = 0;
    int k = k0 + 1;
    for (; k + 3 < R; k += 4) {
      s0 += ra[k] * rb[k];
      s1 += ra[k + 1] * rb[k + 1];
      s2 += ra[k + 2] * rb[k + 2];
      s3 += ra[k + 3] * rb[k + 3];
    }
    for (; k < R; ++k) s0 += ra[k] * rb[k];
    Gp[e] = (s0 + s1) + (s2 + s3);
  }
  return true;
}

// Inverse of the symmetric A (LDS, R <= 32) by Gauss-Jordan elimination
// without row exchanges, in one wave: lane c < R holds column c of A and
// lane R + c column c of the identity, R values each in registers.  Step k
// scales row k by 1 / pivot and removes column k from every other row; the
// multipliers (column k) are written to LDS by lane k and read back by all
// lanes as broadcast loads.  The pivots are those of the LDL^T
// factorisation, all above tol for a clearly positive definite A; the
// first one at or below tol stops it (returns false, Gp untouched).
// Afterwards lane R + c holds column c of A^{-1}, written to Gp (global)
// and sGp (LDS).  col: 32 doubles of LDS.
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ bool gj_inverse_wave(const double *A, int R,
                                                double tol, double *Gp,
                                                double *sGp, double *col) {
  const int l = lane_id();
  double c[32];
#pragma unroll
  for (int i = 0; i < 32; ++i)
    c[i] = i >= R ? 0.0 : l < R ? A[i * R + l] : (l - R == i ? 1.0 : 0.0);
  // rows i >= R stay zero: their multipliers are zero
  double2 *col2 = reinterpret_cast<double2 *>(col);
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    if (k < R && ok) {
      if (l == k)
#pragma unroll
        for (int i = 0; i < 16; ++i) col2[i] = double2{c[2 * i], c[2 * i + 1]};
      wave_lds_fence();
      double m[32];
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const double2 x = col2[i];
        m[2 * i] = x.x;
        m[2 * i + 1] = x.y;
      }
      const double piv = m[k];
      if (piv > tol) {
        const double r = c[k] / piv;
#pragma unroll
        for (int i = 0; i < 32; ++i)
          if (i != k) c[i] = fma(-m[i], r, c[i]);
        c[k] = r;
      } else {
        ok = false;
      }
      wave_lds_fence();  // every lane has read col before the next write
    }
  }
  if (!ok) return false;
  if (l >= R && l < 2 * R)
#pragma unroll
    for (int i = 0; i < 32; ++i)
      if (i < R) {
        Gp[i * R + (l - R)] = c[i];
        sGp[i * R + (l - R)] = c[i];
      }
  return true;
}

// Cyclic Jacobi eigendecomposition of the symmetric A (LDS); V in global.
// Gp = V diag(1/lambda, lambda > R 2^-52 lambda_max) V^T.
__device__ bool jacobi_pinv(double *A, int R, double *V, double *Gp,
                            double *red, double *rot) {
  const int t = threadIdx.x;
  const int m = R + (R & 1);  // players, one dummy when R is odd
  for (int e = t; e < R * R; e += PV_THREADS)
    V[e] = (e / R == e % R) ? 1.0 : 0.0;
  __threadfence_block();
  __syncthreads();
  bool conv = false;
  double off = 0, dia = 0;
  for (int sweep = 0; sweep < 40 && !conv; ++sweep) {
    off = 0;
    dia = 0;
    for (int e = t; e < R * R; e += PV_THREADS) {
      double v = A[e] * A[e];
      if (e / R == e % R) dia += v; else off += v;
    }
    off = block_sum(off, red);
    dia = block_sum(dia, red);
    if (off <= 1e-26 * dia || off == 0) { conv = true; break; }
    for (int r = 0; r < m - 1; ++r) {
      // pair i: (arr[i], arr[m-1-i]) with arr[0] = 0, arr[x] = 1 + (x-1+r)%(m-1)
      for (int i = t; i < m / 2; i += PV_THREADS) {
        int x = i, y = m - 1 - i;
        int p = x == 0 ? 0 : 1 + (x - 1 + r) % (m - 1);
        int q = 1 + (y - 1 + r) % (m - 1);
        if (p > q) { int tmp = p; p = q; q = tmp; }
        double c = 1, s = 0;
        if (q < R) {
          double apq = A[p * R + q];
          if (fabs(apq) > 1e-300) {
            double tau = (A[q * R + q] - A[p * R + p]) / (2 * apq);
            double tt = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1 + tau * tau));
            c = 1 / sqrt(1 + tt * tt);
            s = tt * c;
          }
        }
        rot[4 * i + 0] = p; rot[4 * i + 1] = q;
        rot[4 * i + 2] = c; rot[4 * i + 3] = s;
      }
      __syncthreads();
      // columns: A J and V J
      for (int e = t; e < (m / 2) * R; e += PV_THREADS) {
        int i = e / R, row = e % R;
        int p = (int)rot[4 * i], q = (int)rot[4 * i + 1];
        if (q >= R) continue;
        double c = rot[4 * i + 2], s = rot[4 * i + 3];
        double ap = A[row * R + p], aq = A[row * R + q];
        A[row * R + p] = c * ap - s * aq;
        A[row * R + q] = s * ap + c * aq;
        double vp = V[row * R + p], vq = V[row * R + q];
        V[row * R + p] = c * vp - s * vq;
        V[row * R + q] = s * vp + c * vq;
      }
      __threadfence_block();
      __syncthreads();
      // rows: J^T (A J)
      for (int e = t; e < (m / 2) * R; e += PV_THREADS) {
        int i = e / R, col = e % R;
        int p = (int)rot[4 * i], q = (int)rot[4 * i + 1];
        if (q >= R) continue;
        double c = rot[4 * i + 2], s = rot[4 * i + 3];
        double ap = A[p * R + col], aq = A[q * R + col];
        A[p * R + col] = c * ap - s * aq;
        A[q * R + col] = s * ap + c * aq;
      }
      __syncthreads();
    }
  }
  double lmax = 0;
  for (int i = t; i < R; i += PV_THREADS) lmax = fmax(lmax, A[i * R + i]);
  lmax = block_max(lmax, red);
  const double cut = R * 0x1p-52 * fmax(lmax, 0.0);
  for (int e = t; e < R * R; e += PV_THREADS) {
    int a = e / R, b = e % R;
    double acc = 0;
    for (int k = 0; k < R; ++k) {
      double lam = A[k * R + k];
      if (lam > cut) acc += V[a * R + k] * V[b * R + k] / lam;
    }
    Gp[e] = acc;
  }
  return conv || off <= 1e-20 * dia;
}

__global__ void __launch_bounds__(PV_THREADS)
k_hadamard_pinv(ModeList ml, int R, double *Gfull, double *Gp, double *ggt,
                double *trace_out, double *scratch, uint32_t *err) {
  extern __shared__ double A[];  // R x R
  __shared__ double red[PV_THREADS / WAVE];
  __shared__ __align__(16) double gjcol[32];  // pivot column of the one-wave inverse
  __shared__ double rot[4 * (MAXR / 2 + 1)];
  __shared__ double wdiag[MAXR];  // diagonal of L^{-1} (R > 64)
  __shared__ int flag;
  const int t = threadIdx.x;
  double tr = 0, dmax = 0;
  bool bad = false;
  // Hadamard product of the other modes' Grams, 4 entries per thread at a
  // time, the loads of all Grams issued together (clamped, then masked)
  const int RR = R * R;
  constexpr int QM = MAXN - 1;  // at most N - 1 Grams
  for (int e0 = 0; e0 < RR; e0 += 4 * PV_THREADS) {
    double x[QM][4];
#pragma unroll
    for (int i = 0; i < QM; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = e0 + t + q * PV_THREADS;
        x[i][q] = ml.G[i < ml.n ? i : 0][e < RR ? e : RR - 1];
      }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = e0 + t + q * PV_THREADS;
      double v = 1.0;
#pragma unroll
      for (int i = QM - 1; i >= 0; --i)
        if (i < ml.n) v *= x[i][q];
      if (e < RR) {
        A[e] = v;
        Gfull[e] = v;
        if (!isfinite(v)) bad = true;
        if (e / R == e % R) {
          tr += v;
          dmax = fmax(dmax, v);
        }
      }
    }
  }
  if (bad) atomicOr(err, ERR_NONFINITE);
  tr = block_sum(tr, red);
  dmax = block_max(dmax, red);
  // Cholesky only for clearly positive definite G (every pivot above
  // 1e-9 of the largest diagonal entry); anything closer to singular takes
  // the eigendecomposition, whose cutoff defines the pseudo-inverse.
  const double tol = fmax(R * 0x1p-52 * tr, 1e-9 * dmax);
  __syncthreads();
  // L^{-1} next to A in LDS when both fit (R <= 64), else in scratch
  double *W = R <= 64 ? A + R * R : scratch;
  bool ok;
  if (R <= 32) {
    if (t < WAVE) {
      const bool g = gj_inverse_wave(A, R, tol, Gp, A + RR, gjcol);
      if (t == 0) flag = g ? 1 : 0;
    }
    __threadfence_block();
    __syncthreads();
    ok = flag != 0;
  } else if (R <= 64) {
    ok = chol_inverse(A, R, tol, W, Gp, &flag);
  } else {
    ok = chol_inverse_lds(A, R, tol, wdiag, Gp, &flag);
  }
  if (!ok) {
    __syncthreads();
    for (int e = t; e < R * R; e += PV_THREADS) A[e] = Gfull[e];
    __syncthreads();
    if (!jacobi_pinv(A, R, scratch, Gp, red, rot) && t == 0)
      atomicOr(err, ERR_PINV);
  }
  // G^+ (global) was written by other threads of this workgroup
  __threadfence_block();
  __syncthreads();
  // G^+ in LDS beside G when both fit (the one-wave inverse put it there)
  const double *gps = Gp;
  if (R <= 64) {
    if (!(R <= 32 && ok)) {
      for (int e = t; e < RR; e += PV_THREADS) A[RR + e] = Gp[e];
      __syncthreads();
    }
    gps = A + RR;
  }
  // <G^+, G> and, for STS, G_{>k} = G^+ (*) Hadamard of the Grams after
  // position k (the suffix products of the same Gram loads, issued together)
  double ip = 0;
  for (int e0 = 0; e0 < RR; e0 += 4 * PV_THREADS) {
    double x[QM][4], gp[4], gf[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = e0 + t + q * PV_THREADS, ec = e < RR ? e : RR - 1;
      gp[q] = gps[ec];
      gf[q] = Gfull[ec];
#pragma unroll
      for (int i = 0; i < QM; ++i)
        x[i][q] = ggt ? ml.G[i < ml.n ? i : 0][ec] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = e0 + t + q * PV_THREADS;
      if (e >= RR) continue;
      ip += gp[q] * gf[q];
      if (ggt) {
        double h = 1.0;
#pragma unroll
        for (int i = QM - 1; i >= 0; --i)
          if (i < ml.n) {
            ggt[(int64_t)i * RR + e] = h * gp[q];
            h *= x[i][q];
          }
      }
    }
  }
  ip = block_sum(ip, red);
  if (trace_out && t == 0) *trace_out = ip;
}

// ---------------------------------------------------------------------------
// Row solve: X[i] = m G^+ + (m - (m G^+) G) G^+  (FP64), column sums of X^2.
// REFINE = false drops the refinement term: X[i] = m G^+, a third of the
// MFMA work.  (FP32 factors without refinement take k_solve_f32 below.)
// One wave per 16-row tile of M, on FP64 MFMA in transposed form:
// X^T = (G^+)^T M^T.  With A = (G^+)^T (or G^T) and B = M^T, the accumulator
// of tile t holds X[row0 + l % 16][16 t + l / 16 + 4 v] in lane l, element v,
// which is also the B-operand layout of k-step 4 t + v of the next product,
// so the residual R^T = M^T - G^T X^T and the correction
// X^T += (G^+)^T R^T chain in registers.  A zero row of M gives an exactly
// zero row of X.
// ---------------------------------------------------------------------------
constexpr int SV_THREADS = 256;
constexpr int SV_RESBLK = 512;  // blocks resident at once (2 waves per SIMD)

template <int NT>
__device__ __forceinline__ double afrag(const double *A, int R, int t, int ks,
                                        int l) {
  // (A^T)[i][k] of tile t, k-step ks: i = 16 t + l % 16, k = 4 ks + l / 16
  const int i = 16 * t + (l % 16), k = 4 * ks + l / 16;
  const int ic = i < R ? i : R - 1, kc = k < R ? k : R - 1;
  const double v = A[kc * R + ic];
  return (i < R && k < R) ? v : 0.0;
}

template <typename T, int NT, bool REFINE>
__global__ void __launch_bounds__(SV_THREADS)
__attribute__((amdgpu_waves_per_eu((NT <= 2 || !REFINE) ? 2 : 1)))
k_solve(const T *M, int64_t I, int R, const double *G, const double *Gp,
        double *X, double *partial, int64_t *rows_out) {
  constexpr int KS = 4 * NT;          // k-steps
  constexpr int RP = 16 * NT;
  constexpr int NM = REFINE ? 2 : 1;  // matrices staged: G^+ (and G)
  constexpr bool LDS = NT <= 4;       // staged square (zero padded)
  // wider ranks: their upper triangles, packed
  // (RP (RP + 1) / 2 doubles each: 51 KiB at RP = 112, 66 KiB at RP = 128)
  constexpr int PT = RP * (RP + 1) / 2;
  const int l = lane_id(), w = threadIdx.x / WAVE;
  __shared__ double sG[LDS ? NM * RP * RP : NM * PT];
  if (!LDS) {
    for (int e = threadIdx.x; e < RP * RP; e += SV_THREADS) {
      const int a = e / RP, b = e % RP;
      if (a <= b) {
        const bool in = a < R && b < R;
        const int ec = in ? a * R + b : 0;
        const int pi = a * (2 * RP - a + 1) / 2 + (b - a);
        sG[pi] = in ? Gp[ec] : 0.0;
        if constexpr (REFINE) sG[PT + pi] = in ? G[ec] : 0.0;
      }
    }
    __syncthreads();
  }
  if (LDS) {
    constexpr int NS = (RP * RP + SV_THREADS - 1) / SV_THREADS;
    double gp[NS], g[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) {  // loads first, clamped
      const int e = q * SV_THREADS + threadIdx.x;
      const int a = e / RP, b = e % RP;
      const int ec = (e < RP * RP && a < R && b < R) ? a * R + b : 0;
      gp[q] = Gp[ec];
      if constexpr (REFINE) g[q] = G[ec];
    }
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      const int e = q * SV_THREADS + threadIdx.x;
      const int a = e / RP, b = e % RP;
      const double m = (e < RP * RP && a < R && b < R) ? 1.0 : 0.0;
      if (e < RP * RP) {
        sG[e] = gp[q] * m;
        if constexpr (REFINE) sG[RP * RP + e] = g[q] * m;
      }
    }
    __syncthreads();
  }
  // (A^T)[i][k] fragments, i = 16 t + l % 16, k = 4 ks + l / 16
  int lz = l;  // the tile loop re-derives it opaquely (see opaque_lane)
  auto pk = [&](int t, int ks) -> int {  // packed index of a symmetric pair
    const int i = 16 * t + (lz % 16), k = 4 * ks + lz / 16;
    const int a = k < i ? k : i, b = k < i ? i : k;
    return a * (2 * RP - a + 1) / 2 + (b - a);
  };
  auto fp = [&](int t, int ks) -> double {
    return LDS ? sG[(4 * ks + l / 16) * RP + 16 * t + (l % 16)]
               : sG[pk(t, ks)];
  };
  auto fg = [&](int t, int ks) -> double {
    return LDS ? sG[RP * RP + (4 * ks + l / 16) * RP + 16 * t + (l % 16)]
               : sG[PT + pk(t, ks)];
  };
  // Column sums of X^2: in registers for NT <= 4; wider ranks add each
  // tile's sums (a shuffle tree over its 16 rows) to the wave's row of
  // `red` in LDS, in tile order, to leave registers to the products (and
  // do not prefetch the next tile: one tile's MFMA work hides its loads).
  constexpr bool WIDE = NT > 4;
  __shared__ double red[SV_THREADS / WAVE][MAXR];
  if constexpr (WIDE) {
    for (int c = l; c < MAXR; c += WAVE) red[w][c] = 0.0;
  }
  double ss[WIDE ? 1 : NT][4];
#pragma unroll
  for (int t = 0; t < (WIDE ? 1 : NT); ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) ss[t][v] = 0.0;
  int nrows = 0;
  const int64_t ntiles = (I + 15) / 16;
  const int64_t tstep = (int64_t)gridDim.x * (SV_THREADS / WAVE);
  // B fragments of M^T: M[row][4 ks + l / 16], all loads of a tile issued
  // together (clamped), the next tile's before the current tile's products;
  // masked by a product, not a select, so that no load is moved into a
  // branch (branch-guarded loads wait one by one)
  T raw[KS];
  auto load_tile = [&](int64_t tl) {
    const int64_t rr = tl * 16 + (l % 16);
    const T *mrow = M + (rr < I ? rr : I - 1) * R;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k = 4 * ks + l / 16;
      raw[ks] = mrow[k < R ? k : R - 1];
    }
  };
  int64_t tile = (int64_t)blockIdx.x * (SV_THREADS / WAVE) + w;
  if (!WIDE && tile < ntiles) load_tile(tile);
  for (; tile < ntiles; tile += tstep) {
    const int64_t row = tile * 16 + (l % 16);
    if constexpr (WIDE) load_tile(tile);
    T cur[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) cur[ks] = raw[ks];
    if (!WIDE && tile + tstep < ntiles) load_tile(tile + tstep);
    // G, G^+ fragments are read from LDS in every tile rather than held in
    // registers
    asm volatile("" ::: "memory");
    if constexpr (WIDE) lz = opaque_lane();
    double mf[KS];
    bool nz = false;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k = 4 * ks + l / 16;
      mf[ks] = (double)cur[ks] * ((row < I && k < R) ? 1.0 : 0.0);
      nz |= (mf[ks] != 0.0);
    }
    const uint64_t b = __ballot(nz);
    nrows += __popcll((b | (b >> 16) | (b >> 32) | (b >> 48)) & 0xffffull);
    // X^T = G^+ M^T (wide ranks: a scheduling barrier per output tile
    // keeps each tile's fragment loads next to its MFMAs)
    double4_t ax[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      ax[t] = double4_t{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        ax[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(fp(t, ks), mf[ks], ax[t],
                                                     0, 0, 0);
      }
      if constexpr (WIDE) __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (REFINE) {
    // R^T = M^T - G X^T
    double rf[KS];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      double4_t ar = double4_t{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        ar = __builtin_amdgcn_mfma_f64_16x16x4f64(fg(t, ks), ax[ks / 4][ks % 4],
                                                  ar, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) rf[4 * t + v] = mf[4 * t + v] - ar[v];
      if constexpr (WIDE) __builtin_amdgcn_sched_barrier(0);
    }
    // X^T += G^+ R^T
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        ax[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(fp(t, ks), rf[ks], ax[t],
                                                     0, 0, 0);
      }
      if constexpr (WIDE) __builtin_amdgcn_sched_barrier(0);
    }
    }
    if (row < I) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int c = 16 * t + l / 16 + 4 * v;
          if (c < R) {
            X[row * R + c] = ax[t][v];
            if constexpr (!WIDE) ss[t][v] += ax[t][v] * ax[t][v];
          }
        }
    }
    if constexpr (WIDE) {
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int c = 16 * t + l / 16 + 4 * v;
          double q = (row < I) ? ax[t][v] * ax[t][v] : 0.0;
          for (int o = 1; o < 16; o <<= 1) q += __shfl_xor(q, o, WAVE);
          if ((l % 16) == 0 && c < R) red[w][c] += q;
        }
    }
  }
  if (rows_out) {
    __shared__ int cnt[SV_THREADS / WAVE];
    if (l == 0) cnt[w] = nrows;
    __syncthreads();
    if (threadIdx.x == 0) {
      int n = 0;
      for (int q = 0; q < SV_THREADS / WAVE; ++q) n += cnt[q];
      if (n) atomicAdd((unsigned long long *)rows_out, (unsigned long long)n);
    }
  }
  // fixed-order reduction of the column sums: the 16 row lanes of a column
  // (shuffle tree), then waves (LDS, in wave order)
  if constexpr (!WIDE) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double s = ss[t][v];
        for (int o = 1; o < 16; o <<= 1) s += __shfl_xor(s, o, WAVE);
        const int c = 16 * t + l / 16 + 4 * v;
        if ((l % 16) == 0 && c < R) red[w][c] = s;
      }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < R; c += SV_THREADS) {
    double v = 0;
    for (int q = 0; q < SV_THREADS / WAVE; ++q) v += red[q][c];
    partial[(int64_t)blockIdx.x * R + c] = v;
  }
}

// Row solve of the FP32 forms without refinement: X^T = (G^+)^T M^T on
// v_mfma_f32_16x16x4f32 (G^+ rounded to FP32 once, staged in LDS; M is
// FP32 already; FP32 accumulation over the R terms of an entry), X written
// in FP32, column sums of X^2 in FP64.  Twice the FP32 MFMA rate of the FP64
// MFMA, and a relative error of the order of M's own FP32 rounding.  The D
// layout puts X[row0 + l % 16][16 t + 4 (l / 16) + v] in lane l, element v.
// Eight waves share the staged G^+.  Only the KS - D = (R + 3) / 4 k-steps
// that hold columns below R are multiplied.  Each wave stages its 16 X rows in LDS and
// writes them as one contiguous span (16 R floats, 16-byte stores when R is a
// multiple of 4), so every output line is written whole.  Each lane keeps the
// FP64 sums of squares of its 4 NT columns over the tiles it computed; they
// are reduced over the 16 rows of a wave and the block's waves once, at the
// end (a fixed order for a given grid).
constexpr int SF_THREADS = 512;

template <int NT, int D>
__global__ void __launch_bounds__(SF_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
k_solve_f32(const float *M, int64_t I, int R, const double *Gp, float *X,
            double *partial, int64_t *rows_out) {
  constexpr int KS = 4 * NT - D;  // k-steps with a column below R
  constexpr int RP = 16 * NT;
  constexpr int RS = RP + 4;  // LDS row stride of G^+ and of the X tiles
  constexpr int NW = SF_THREADS / WAVE;
  __shared__ float sG[RP * RS];
  __shared__ float sX[NW][16 * RS];
  __shared__ double red[NW][MAXR];
  const int l = lane_id(), w = threadIdx.x / WAVE;
  for (int e = threadIdx.x; e < RP * RP; e += SF_THREADS) {
    const int a = e / RP, b = e % RP;
    sG[a * RS + b] = (a < R && b < R) ? (float)Gp[a * R + b] : 0.0f;
  }
  __syncthreads();
  const bool vec = (R & 3) == 0;
  float *xs = sX[w];
  double sq[NT][4];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) sq[t][v] = 0.0;
  int nrows = 0;
  const int64_t ntiles = (I + 15) / 16;
  const int64_t tstep = (int64_t)gridDim.x * NW;
  float raw[KS];
  auto load_tile = [&](int64_t tl) {
    const int64_t rr = tl * 16 + (l % 16);
    const float *mrow = M + (rr < I ? rr : I - 1) * R;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k = 4 * ks + l / 16;
      raw[ks] = mrow[k < R ? k : R - 1];
    }
  };
  int64_t tile = (int64_t)blockIdx.x * NW + w;
  if (tile < ntiles) load_tile(tile);
  for (; tile < ntiles; tile += tstep) {
    const int64_t row0 = tile * 16;
    const int64_t row = row0 + (l % 16);
    float mf[KS];
    bool nz = false;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k = 4 * ks + l / 16;
      mf[ks] = (row < I && k < R) ? raw[ks] : 0.0f;
      nz |= (mf[ks] != 0.0f);
    }
    if (tile + tstep < ntiles) load_tile(tile + tstep);
    const uint64_t b = __ballot(nz);
    nrows += __popcll((b | (b >> 16) | (b >> 32) | (b >> 48)) & 0xffffull);
    // the G^+ fragments are read from LDS in every tile (an opaque lane
    // index keeps them from being hoisted out of the tile loop into
    // registers), one output tile at a time
    asm volatile("" ::: "memory");
    const int lz = opaque_lane();
    const float *gA = sG + (lz / 16) * RS + (lz % 16);
    const bool live = row < I;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      float4_t acc = float4_t{0, 0, 0, 0};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(
            gA[4 * ks * RS + 16 * t], mf[ks], acc, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double x = (double)acc[v];
        sq[t][v] += live ? x * x : 0.0;
      }
      *reinterpret_cast<float4_t *>(xs + (l % 16) * RS + 16 * t + 4 * (l / 16)) = acc;
      __builtin_amdgcn_sched_barrier(0);
    }
    wave_lds_sync();  // the tile's X rows are in LDS
    const int nv = I - row0 < 16 ? (int)(I - row0) : 16;
    float *dst = X + row0 * R;
    if (vec) {  // nv R / 4 chunks of 4 floats, each inside one row
      const int nch = nv * R / 4;
      for (int q = l; q < nch; q += WAVE) {
        const int e = 4 * q, r = e / R, c = e - r * R;
        *reinterpret_cast<float4_t *>(dst + e) =
            *reinterpret_cast<const float4_t *>(xs + r * RS + c);
      }
    } else {
      const int ne = nv * R;
      for (int e = l; e < ne; e += WAVE) {
        const int r = e / R, c = e - r * R;
        dst[e] = xs[r * RS + c];
      }
    }
    wave_lds_sync();  // reads done before the next tile's LDS stores
  }
  // column sums: lane l holds columns 16 t + 4 (l / 16) + v for the rows
  // l % 16 of its tiles; sum over the 16 row lanes, then over the waves
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double q = sq[t][v];
      for (int o = 1; o < 16; o <<= 1) q += __shfl_xor(q, o, WAVE);
      const int c = 16 * t + 4 * (l / 16) + v;
      if ((l % 16) == 0 && c < MAXR) red[w][c] = q;
    }
  if (rows_out) {
    __shared__ int cnt[NW];
    if (l == 0) cnt[w] = nrows;
    __syncthreads();
    if (threadIdx.x == 0) {
      int n = 0;
      for (int q = 0; q < NW; ++q) n += cnt[q];
      if (n) atomicAdd((unsigned long long *)rows_out, (unsigned long long)n);
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < R; c += SF_THREADS) {
    double v = 0;
    for (int q = 0; q < NW; ++q) v += red[q][c];
    partial[(int64_t)blockIdx.x * R + c] = v;
  }
}

template <typename T>
__global__ void k_colsumsq(const T *X, int64_t I, int R, double *partial) {
  // block b sums rows b, b + grid, ... ; thread c owns column c
  __shared__ double red[256];
  for (int c0 = 0; c0 < R; c0 += 256) {
    int c = c0 + threadIdx.x;
    double s = 0;
    if (c < R)
      for (int64_t i = blockIdx.x; i < I; i += gridDim.x) {
        double v = (double)X[i * R + c];
        s += v * v;
      }
    red[threadIdx.x] = s;
    __syncthreads();
    if (c < R) partial[(int64_t)blockIdx.x * R + c] = red[threadIdx.x];
    __syncthreads();
  }
}

template <typename T>
__global__ void k_scale_cols(const double *X, int64_t n, int R,
                             const double *sigma, T *U) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  U[e] = (T)(X[e] * inv_or_zero(sigma[e % R]));
}

template <typename T>
__global__ void k_zero(T *p, int64_t n) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (; e < n; e += st) p[e] = T(0);
}

__global__ void k_to_f64(const void *src, int fp64, double *dst, int64_t n) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  dst[e] = fp64 ? static_cast<const double *>(src)[e]
                : (double)static_cast<const float *>(src)[e];
}

__global__ void k_convert(const void *src, int sf, void *dst, int df,
                          int64_t n) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double v = sf ? static_cast<const double *>(src)[e]
                : (double)static_cast<const float *>(src)[e];
  if (df) static_cast<double *>(dst)[e] = v;
  else static_cast<float *>(dst)[e] = (float)v;
}

}  // namespace

void convert_values(const void *src, int src_fp64, void *dst, int dst_fp64,
                    int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_convert, dim3(ceil_div(n, 256)), dim3(256), 0, s, src,
                     src_fp64, dst, dst_fp64, n);
  CPR_LAUNCH_CHECK();
}

size_t gram_temp_bytes(int64_t I, int R) {
  int64_t rpb;
  const int nblk = std::max(gram_blocks(I, &rpb), gram_lp_blocks(I, &rpb));
  return (size_t)nblk * R * R * sizeof(double) + 256;
}

// XT: the type of the solve's rows X when SCALE (FP32 only for FP32
// factors, which take the reduced-precision Gram)
template <typename T, bool SCALE, typename XT = double>
void gram_any(const T *U, const XT *X, const double *sigma, T *Uout,
              int64_t I, int R, double *G, void *tmp, int mode,
              hipStream_t s) {
  int64_t rpb;
  const int nblk = gram_blocks(I, &rpb);
  const int Rp = (R + 15) / 16 * 16;
  const int nt = Rp / 16, ntri = nt * (nt + 1) / 2;
  const int tpw = (ntri + 3) / 4;
  double *partial = static_cast<double *>(tmp);
  if constexpr (std::is_same<T, float>::value) {
    if (mode != GRAM_F64) {
      const int nbl = gram_lp_blocks(I, &rpb);
      const int tpl = (ntri + GL_THREADS / WAVE - 1) / (GL_THREADS / WAVE);
      // four values per load: FP32 values, R a multiple of 4, 16-byte
      // aligned arrays (rows then start on 16-byte boundaries)
      constexpr bool V32 = !SCALE || std::is_same<XT, float>::value;
      const bool vec = V32 && R % 4 == 0 &&
                       ((uintptr_t)(SCALE ? (const void *)X : (const void *)U) |
                        (uintptr_t)(SCALE ? (void *)Uout : nullptr)) % 16 == 0;
#define CPR_GRAM_LP(M, K)                                                     \
  if constexpr (V32) {                                                        \
    if (vec)                                                                  \
      hipLaunchKernelGGL((k_gram_lp<M, K, SCALE, XT, V32>), dim3(nbl),       \
                         dim3(GL_THREADS), 0, s, U, X, sigma, Uout, I, R, Rp, \
                         rpb, partial);                                       \
    else                                                                      \
      hipLaunchKernelGGL((k_gram_lp<M, K, SCALE, XT, false>), dim3(nbl),     \
                         dim3(GL_THREADS), 0, s, U, X, sigma, Uout, I, R, Rp, \
                         rpb, partial);                                       \
  } else                                                                      \
    hipLaunchKernelGGL((k_gram_lp<M, K, SCALE, XT, false>), dim3(nbl),       \
                       dim3(GL_THREADS), 0, s, U, X, sigma, Uout, I, R, Rp,   \
                       rpb, partial)
#define CPR_GRAM_LP_T(M)              \
  switch (tpl) {                      \
    case 1: CPR_GRAM_LP(M, 1); break; \
    case 2: CPR_GRAM_LP(M, 2); break; \
    case 3: CPR_GRAM_LP(M, 3); break; \
    case 4: CPR_GRAM_LP(M, 4); break; \
    default: CPR_GRAM_LP(M, 5); break; \
  }
      if (mode == GRAM_F32) {
        CPR_GRAM_LP_T(GRAM_F32)
      } else {
        CPR_GRAM_LP_T(GRAM_BF16X3)
      }
#undef CPR_GRAM_LP_T
#undef CPR_GRAM_LP
      CPR_LAUNCH_CHECK();
      colsum(partial, nbl, R * R, G, 0, nullptr, s);
      CPR_LAUNCH_CHECK();
      return;
    }
  }
  if constexpr (!std::is_same<XT, double>::value) {
    // FP32 rows X come only with the FP32 forms' reduced-precision Grams
    throw HipFail(hipErrorInvalidValue, __FILE__, __LINE__);
  } else {
#define CPR_GRAM(K) \
  launch_gram<T, K, SCALE>(U, X, sigma, Uout, I, R, Rp, partial, nblk, rpb, s)
  switch (tpw) {
    case 1: CPR_GRAM(1); break;
    case 2: CPR_GRAM(2); break;
    case 3: CPR_GRAM(3); break;
    case 4: CPR_GRAM(4); break;
    case 6: case 5: CPR_GRAM(6); break;
    default: CPR_GRAM(9); break;
  }
#undef CPR_GRAM
  colsum(partial, nblk, R * R, G, 0, nullptr, s);
  CPR_LAUNCH_CHECK();
  }
}

template <typename T>
void gram(const T *U, int64_t I, int R, double *G, void *tmp, int mode,
          hipStream_t s) {
  gram_any<T, false, double>(U, nullptr, nullptr, nullptr, I, R, G, tmp, mode,
                            s);
}
template void gram<float>(const float *, int64_t, int, double *, void *, int,
                          hipStream_t);
template void gram<double>(const double *, int64_t, int, double *, void *,
                           int, hipStream_t);

template <typename T>
void gram_scaled(const void *X, bool x32, const double *sigma, int64_t I,
                 int R, T *U, double *G, void *tmp, int mode, hipStream_t s) {
  if constexpr (std::is_same<T, float>::value) {
    if (x32) {
      gram_any<T, true, float>(nullptr, static_cast<const float *>(X), sigma,
                               U, I, R, G, tmp, mode, s);
      return;
    }
  }
  gram_any<T, true, double>(nullptr, static_cast<const double *>(X), sigma, U,
                            I, R, G, tmp, mode, s);
}
template void gram_scaled<float>(const void *, bool, const double *, int64_t,
                                 int, float *, double *, void *, int,
                                 hipStream_t);
template void gram_scaled<double>(const void *, bool, const double *, int64_t,
                                  int, double *, double *, void *, int,
                                  hipStream_t);

namespace {
template <typename T>
__global__ void k_scale_draws(const T *h, const double *prob, int64_t J,
                              int R, double *hs) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= J * R) return;
  const int64_t s = e / R;
  hs[e] = (double)h[e] * sqrt(1.0 / ((double)J * prob[s]));
}
}  // namespace

template <typename T>
void sketched_gram(const T *h, const double *prob, int64_t J, int R,
                   double *hs, double *Gs, void *tmp, hipStream_t s) {
  hipLaunchKernelGGL((k_scale_draws<T>), dim3(ceil_div(J * R, 256)),
                     dim3(256), 0, s, h, prob, J, R, hs);
  CPR_LAUNCH_CHECK();
  gram_any<double, false, double>(hs, nullptr, nullptr, nullptr, J, R, Gs, tmp,
                          GRAM_F64, s);
}
template void sketched_gram<float>(const float *, const double *, int64_t,
                                   int, double *, double *, void *,
                                   hipStream_t);
template void sketched_gram<double>(const double *, const double *, int64_t,
                                    int, double *, double *, void *,
                                    hipStream_t);

void column_norms(const double *partial, int nblk, int R, double *sigma,
                  uint32_t *err, hipStream_t s) {
  colsum(partial, nblk, R, sigma, 1, err, s);
  CPR_LAUNCH_CHECK();
}

void hadamard_pinv(const ModeList &ml, int R, double *Gfull, double *Gp,
                   double *ggt_out, double *trace_out, double *scratch,
                   uint32_t *err, hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {  // up to 2 R^2 (R <= 64) or R^2 doubles: beyond 64 KiB
    hipError_t e = hipFuncSetAttribute(
        reinterpret_cast<const void *>(&k_hadamard_pinv),
        hipFuncAttributeMaxDynamicSharedMemorySize, MAXR * MAXR * 8);
    if (e != hipSuccess) throw HipFail(e, __FILE__, __LINE__);
    attr_set = true;
  }
  const size_t lds = (size_t)(R <= 64 ? 2 : 1) * R * R * sizeof(double);
  hipLaunchKernelGGL(k_hadamard_pinv, dim3(1), dim3(PV_THREADS), lds, s, ml,
                     R, Gfull, Gp, ggt_out, trace_out, scratch, err);
  CPR_LAUNCH_CHECK();
}

int solve_blocks(int64_t I) {
  // four 16-row tiles per block (one per wave) or more: every block is
  // resident, and a wave prefetches its next tile
  return (int)std::min<int64_t>(SV_RESBLK, std::max<int64_t>(1, (I + 63) / 64));
}

template <typename T, bool RF>
void solve_rows_nt(const T *M, int64_t I, int R, const double *Gfull,
                   const double *Gp, void *Xv, double *partial, int nblk,
                   int64_t *rows_out, hipStream_t s) {
  const dim3 g(nblk), b(SV_THREADS), bf(SF_THREADS);
  constexpr bool F32 = std::is_same<T, float>::value && !RF;
  const int dk = 4 * ((R + 15) / 16) - (R + 3) / 4;  // all-zero k-steps
#define CPR_SOLVE_F32(NT, D)                                                 \
  hipLaunchKernelGGL((k_solve_f32<NT, D>), g, bf, 0, s,                      \
                     reinterpret_cast<const float *>(M), I, R, Gp,           \
                     static_cast<float *>(Xv), partial, rows_out)
#define CPR_SOLVE(NT)                                                        \
  if constexpr (F32) {                                                       \
    switch (dk) {                                                            \
      case 0: CPR_SOLVE_F32(NT, 0); break;                                   \
      case 1: CPR_SOLVE_F32(NT, 1); break;                                   \
      case 2: CPR_SOLVE_F32(NT, 2); break;                                   \
      default: CPR_SOLVE_F32(NT, 3); break;                                  \
    }                                                                        \
  } else                                                                     \
    hipLaunchKernelGGL((k_solve<T, NT, RF>), g, b, 0, s, M, I, R, Gfull, Gp, \
                       static_cast<double *>(Xv), partial, rows_out)
  switch ((R + 15) / 16) {
    case 1: CPR_SOLVE(1); break;
    case 2: CPR_SOLVE(2); break;
    case 3: CPR_SOLVE(3); break;
    case 4: CPR_SOLVE(4); break;
    case 5: CPR_SOLVE(5); break;
    case 6: CPR_SOLVE(6); break;
    case 7: CPR_SOLVE(7); break;
    default: CPR_SOLVE(8); break;
  }
#undef CPR_SOLVE
#undef CPR_SOLVE_F32
  CPR_LAUNCH_CHECK();
}

template <typename T>
void solve_rows(const T *M, int64_t I, int R, const double *Gfull,
                const double *Gp, void *X, double *partial, int nblk,
                int64_t *rows_out, bool refine, hipStream_t s) {
  if (refine)
    solve_rows_nt<T, true>(M, I, R, Gfull, Gp, X, partial, nblk, rows_out, s);
  else
    solve_rows_nt<T, false>(M, I, R, Gfull, Gp, X, partial, nblk, rows_out, s);
}
template void solve_rows<float>(const float *, int64_t, int, const double *,
                                const double *, void *, double *, int,
                                int64_t *, bool, hipStream_t);
template void solve_rows<double>(const double *, int64_t, int, const double *,
                                 const double *, void *, double *, int,
                                 int64_t *, bool, hipStream_t);

template <typename T>
void finish_normalize(const double *X, int64_t I, int R, const double *partial,
                      int nblk, double *sigma, T *U, uint32_t *err,
                      hipStream_t s) {
  colsum(partial, nblk, R, sigma, 1, err, s);
  hipLaunchKernelGGL((k_scale_cols<T>), dim3(ceil_div(I * R, 256)), dim3(256),
                     0, s, X, I * R, R, sigma, U);
  CPR_LAUNCH_CHECK();
}
template void finish_normalize<float>(const double *, int64_t, int,
                                      const double *, int, double *, float *,
                                      uint32_t *, hipStream_t);
template void finish_normalize<double>(const double *, int64_t, int,
                                       const double *, int, double *, double *,
                                       uint32_t *, hipStream_t);

template <typename T>
void normalize_in_place(const double *Uin, int64_t I, int R, T *U,
                        double *partial, uint32_t *err, hipStream_t s) {
  const int nblk = (int)std::min<int64_t>(256, std::max<int64_t>(1, I));
  hipLaunchKernelGGL((k_colsumsq<double>), dim3(nblk), dim3(256), 0, s, Uin, I,
                     R, partial);
  CPR_LAUNCH_CHECK();
  // sigma of the input is not kept: Alg. 1 starts from sigma = 1
  double *sig = partial + (int64_t)nblk * R;
  finish_normalize<T>(Uin, I, R, partial, nblk, sig, U, err, s);
}
template void normalize_in_place<float>(const double *, int64_t, int, float *,
                                        double *, uint32_t *, hipStream_t);
template void normalize_in_place<double>(const double *, int64_t, int,
                                         double *, double *, uint32_t *,
                                         hipStream_t);

template <typename T>
void zero_fill(T *p, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int nb = (int)std::min<int64_t>(4096, (n + 255) / 256);
  hipLaunchKernelGGL((k_zero<T>), dim3(nb), dim3(256), 0, s, p, n);
  CPR_LAUNCH_CHECK();
}
template void zero_fill<float>(float *, int64_t, hipStream_t);
template void zero_fill<double>(double *, int64_t, hipStream_t);
template void zero_fill<int32_t>(int32_t *, int64_t, hipStream_t);
template void zero_fill<int64_t>(int64_t *, int64_t, hipStream_t);

void copy_to_f64(const void *src, int src_fp64, double *dst, int64_t n,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_to_f64, dim3(ceil_div(n, 256)), dim3(256), 0, s, src,
                     src_fp64, dst, n);
  CPR_LAUNCH_CHECK();
}

}  // namespace cpr
