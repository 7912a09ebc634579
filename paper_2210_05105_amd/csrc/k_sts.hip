// STS-CP on one GPU (Section 4.1, Appendix B).
//
// Tree (Alg. 4 without the exchange): leaf b holds the Gram of rows
// [bF, bF + F) of U_k; an internal node holds the sum of its children.
// Nodes are stored in heap order (root 1, children 2v and 2v+1, leaves
// P2 .. 2 P2 - 1 with P2 a power of two) as packed upper triangles in FP64.
//
// Draw (Alg. 5 without routing): for the factors != j in ascending order,
// the first factor (h = 1, a law shared by all samples) is drawn from a flat
// CDF of row masses; every later factor walks its tree.
// with h the Hadamard product of the rows drawn so far and
// G_{>k} = G^+ (*) (Grams of the factors drawn later), the mass of a node is
// <(h h^T) (*) G_{>k}, G^node>.  A wave carries the absolute target
// t = u * Z down the tree (go right iff t >= mass(left child), subtracting
// that mass), which is the paper's rescaled-threshold walk without the
// repeated division.  In the leaf, the row masses (U[i] (*) h)^T G_{>k}
// (U[i] (*) h) come from one FP64 MFMA product U_leaf W (W = (h h^T) (*)
// G_{>k}) and a wave prefix scan picks min{ i : t < F(i) }.
#include "internal.h"

namespace cpr {

typedef double double4_t __attribute__((ext_vector_type(4)));

int sts_packed(int R) { return R * (R + 1) / 2; }

namespace {

// Order LDS writes of one wave before its later reads by other lanes.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int packed_index(int a, int b, int R) {
  // a <= b; row-major upper triangle
  return a * (2 * R - a + 1) / 2 + (b - a);
}

// ---------------------------------------------------------------------------
// Build: leaf Grams on FP64 MFMA (one wave per leaf), then the subtree of
// LB consecutive leaves of the block; upper levels by k_tree_level.
// ---------------------------------------------------------------------------
template <typename T, int NT>
__global__ void __launch_bounds__(256)
k_tree_leaves(const T *U, int64_t I, int R, int F, int64_t P2, int LB,
              double *tree) {
  constexpr int NTRI = NT * (NT + 1) / 2;
  const int P = R * (R + 1) / 2;
  const int w = threadIdx.x / WAVE, l = lane_id();
  const int64_t leaf0 = (int64_t)blockIdx.x * LB;
  for (int lf = w; lf < LB; lf += 4) {
    const int64_t leaf = leaf0 + lf;
    double *node = tree + (P2 + leaf) * (int64_t)P;
    const int64_t rbase = leaf * F;
    double4_t acc[NTRI];
#pragma unroll
    for (int i = 0; i < NTRI; ++i) acc[i] = double4_t{0, 0, 0, 0};
    if (rbase < I) {
      for (int k0 = 0; k0 < F; k0 += 4) {
        const int64_t r = rbase + k0 + l / 16;
        const bool rv = r < I;
        double col[NT];
#pragma unroll
        for (int ta = 0; ta < NT; ++ta) {
          const int ca = ta * 16 + (l % 16);
          col[ta] = (rv && ca < R) ? (double)U[r * R + ca] : 0.0;
        }
#pragma unroll
        for (int ta = 0; ta < NT; ++ta)
#pragma unroll
          for (int tb = ta; tb < NT; ++tb) {
            const int i = ta * NT - ta * (ta - 1) / 2 + (tb - ta);
            acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(col[ta], col[tb],
                                                          acc[i], 0, 0, 0);
          }
      }
    }
    // tile (ta, tb), lane l, element v -> (ta*16 + l/16 + 4v, tb*16 + l%16)
#pragma unroll
    for (int ta = 0; ta < NT; ++ta)
#pragma unroll
      for (int tb = ta; tb < NT; ++tb) {
        const int i = ta * NT - ta * (ta - 1) / 2 + (tb - ta);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ga = ta * 16 + (l / 16) + 4 * v;
          const int gb = tb * 16 + (l % 16);
          if (ga < R && gb < R && ga <= gb)
            node[packed_index(ga, gb, R)] = acc[i][v];
        }
      }
  }
  __threadfence_block();
  __syncthreads();
  // in-block subtree: parents of the block's leaves up to the block root
  int64_t first = (P2 + leaf0) / 2;  // first node of the level above
  for (int cnt = LB / 2; cnt >= 1; cnt /= 2, first /= 2) {
    for (int64_t e = threadIdx.x; e < (int64_t)cnt * P; e += 256) {
      const int64_t v = first + e / P;
      const int c = (int)(e % P);
      tree[v * P + c] = tree[(2 * v) * P + c] + tree[(2 * v + 1) * P + c];
    }
    __threadfence_block();
    __syncthreads();
  }
}

__global__ void k_tree_level(double *tree, int64_t first, int64_t cnt, int P) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cnt * P) return;
  const int64_t v = first + e / P;
  const int c = (int)(e % P);
  tree[v * P + c] = tree[(2 * v) * P + c] + tree[(2 * v + 1) * P + c];
}

// ---------------------------------------------------------------------------
// Draw: one wave per sample.  E = packed entries per lane (ceil(P / 64)),
// NT = 16-column tiles of R.
// ---------------------------------------------------------------------------
constexpr int SD_THREADS = 256;
constexpr int SD_WAVES = SD_THREADS / WAVE;

template <typename T, int E, int NT>
__global__ void __launch_bounds__(SD_THREADS)
k_sts_draw(ModeList ml, int64_t J, int R, int F, const double *uni,
           const double *Gp, const double *trace, int32_t *sidx, double *prob,
           T *h_out, uint32_t *err) {
  __shared__ double sh_h[SD_WAVES][MAXR];
  __shared__ double sh_m[SD_WAVES][64];
  const int w = threadIdx.x / WAVE, l = lane_id();
  const int64_t s = (int64_t)blockIdx.x * SD_WAVES + w;
  if (s >= J) return;
  const int P = R * (R + 1) / 2;
  const int nq = ml.n;
  double *h = sh_h[w];
  for (int r = l; r < R; r += WAVE) h[r] = 1.0;
  wave_sync();
  // (a, b) of this lane's packed entries e = l + 64 c
  int ea[E], eb[E];
#pragma unroll
  for (int c = 0; c < E; ++c) {
    int e = l + 64 * c, a = 0;
    if (e < P) {
      while (e >= R - a) { e -= R - a; ++a; }
      ea[c] = a;
      eb[c] = a + e;
    } else {
      ea[c] = eb[c] = -1;
    }
  }
  for (int q = 0; q < nq; ++q) {
    const T *U = static_cast<const T *>(ml.U[q]);
    const int64_t I = ml.I[q];
    const int64_t P2 = ml.P2[q];
    const double *tree = ml.tree[q];
    const double *Gg = ml.Ggt[q];
    double u = uni[s * nq + q];
    if (!(u >= 0.0 && u < 1.0)) {
      if (l == 0) atomicOr(err, ERR_UNIFORM);
      u = 0.0;
    }
    if (q == 0) {
      // h = 1: every sample shares this conditional law, held as a flat
      // CDF of the row masses U[i] G_{>k} U[i]^T; index = min{i : uZ < F(i)}
      const double Z0 = *ml.Z[0];
      const double t0 = u * Z0;
      const double *cdf = ml.cdf[0];
      int64_t lo = 0, hi = I;
      while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (t0 < cdf[mid]) hi = mid; else lo = mid + 1;
      }
      const int64_t last = *ml.last[0];
      if (lo > last) lo = last;
      if (lo < 0) lo = 0;
      if (l == 0) sidx[s * nq + q] = (int32_t)lo;
      for (int r = l; r < R; r += WAVE) h[r] = (double)U[lo * R + r];
      wave_sync();
      continue;
    }
    // W entries (packed, off-diagonal doubled)
    double W[E];
#pragma unroll
    for (int c = 0; c < E; ++c) {
      W[c] = 0;
      if (ea[c] >= 0) {
        const int a = ea[c], b = eb[c];
        W[c] = h[a] * h[b] * Gg[a * R + b] * (a == b ? 1.0 : 2.0);
      }
    }
    auto node_mass = [&](int64_t v) {
      const double *nd = tree + v * (int64_t)P;
      double acc = 0;
#pragma unroll
      for (int c = 0; c < E; ++c)
        if (ea[c] >= 0) acc += W[c] * nd[l + 64 * c];
      return wave_sum(acc);
    };
    const double Z = node_mass(1);
    if (!(Z > 0)) {
      if (l == 0) atomicOr(err, ERR_ZERO_MASS);
    }
    double t = u * Z, mv = Z;
    int64_t v = 1;
    while (v < P2) {
      const double mL = node_mass(2 * v);
      if (mL <= 0 || (t >= mL && mv - mL > 0)) {
        t -= (mL > 0 ? mL : 0.0);
        mv -= mL;
        v = 2 * v + 1;
      } else {
        mv = mL;
        v = 2 * v;
      }
    }
    // leaf rows: masses m_i = U[i] W' U[i]^T, W' = (h h^T) (*) G_{>k}
    const int64_t row0 = (v - P2) * F;
    for (int tile = 0; tile < F / 16; ++tile) {
      double4_t acc[NT];
#pragma unroll
      for (int x = 0; x < NT; ++x) acc[x] = double4_t{0, 0, 0, 0};
      const int64_t ra = row0 + tile * 16 + (l % 16);
      const bool rav = ra < I;
      for (int k0 = 0; k0 < NT * 16; k0 += 4) {
        const int ka = k0 + l / 16;
        const bool kv = ka < R;
        const double a = (rav && kv) ? (double)U[ra * R + ka] : 0.0;
        const double hk = kv ? h[ka] : 0.0;
#pragma unroll
        for (int x = 0; x < NT; ++x) {
          const int jb = x * 16 + (l % 16);
          const double b = (kv && jb < R) ? hk * h[jb] * Gg[ka * R + jb] : 0.0;
          acc[x] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[x], 0, 0, 0);
        }
      }
      double sm[4] = {0, 0, 0, 0};
#pragma unroll
      for (int x = 0; x < NT; ++x) {
        const int j = x * 16 + (l % 16);
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) {
          const int64_t r = row0 + tile * 16 + (l / 16) + 4 * vv;
          if (r < I && j < R) sm[vv] += acc[x][vv] * (double)U[r * R + j];
        }
      }
#pragma unroll
      for (int vv = 0; vv < 4; ++vv)
        for (int o = 1; o < 16; o <<= 1) sm[vv] += __shfl_xor(sm[vv], o, WAVE);
      if ((l % 16) == 0)
        for (int vv = 0; vv < 4; ++vv) sh_m[w][tile * 16 + (l / 16) + 4 * vv] = sm[vv];
    }
    wave_sync();
    // prefix over the leaf's rows (lane i = row row0 + i)
    double mi = (l < F && row0 + l < I) ? sh_m[w][l] : 0.0;
    if (!(mi > 0)) mi = 0.0;
    double pre = mi;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      double y = __shfl_up(pre, o, WAVE);
      if (l >= o) pre += y;
    }
    const uint64_t pos = __ballot(mi > 0);
    const uint64_t hit = __ballot(mi > 0 && t < pre);
    int pick;
    if (hit) pick = __ffsll((long long)hit) - 1;
    else if (pos) pick = 63 - __clzll((long long)pos);
    else {
      pick = 0;
      if (l == 0) atomicOr(err, ERR_ZERO_MASS);
    }
    int64_t idx = row0 + pick;
    if (idx >= I) idx = I - 1;
    if (l == 0) sidx[s * nq + q] = (int32_t)idx;
    wave_sync();  // every lane has read h for this factor
    for (int r = l; r < R; r += WAVE) h[r] = h[r] * (double)U[idx * R + r];
    wave_sync();
  }
  // probability of the drawn Khatri-Rao row: (h^T G^+ h) / <G^+, G>
  double acc = 0;
  for (int e = l; e < R * R; e += WAVE) acc += h[e / R] * Gp[e] * h[e % R];
  acc = wave_sum(acc);
  if (l == 0) prob[s] = acc / *trace;
  for (int r = l; r < R; r += WAVE) h_out[s * R + r] = (T)h[r];
}

template <typename T, int E, int NT>
void launch_draw(const ModeList &ml, int64_t J, int R, int F, const double *uni,
                 const double *Gp, const double *trace, int32_t *sidx,
                 double *prob, T *h, uint32_t *err, hipStream_t s) {
  hipLaunchKernelGGL((k_sts_draw<T, E, NT>), dim3(ceil_div(J, SD_WAVES)),
                     dim3(SD_THREADS), 0, s, ml, J, R, F, uni, Gp, trace, sidx,
                     prob, h, err);
}

}  // namespace

template <typename T>
void sts_build(const T *U, int64_t I, int R, int F, int64_t P2, double *tree,
               hipStream_t s) {
  const int P = sts_packed(R);
  const int LB = (int)(P2 < 64 ? P2 : 64);
  const int nt = (R + 15) / 16;
  const dim3 g((unsigned)(P2 / LB)), b(256);
  switch (nt) {
    case 1: hipLaunchKernelGGL((k_tree_leaves<T, 1>), g, b, 0, s, U, I, R, F, P2, LB, tree); break;
    case 2: hipLaunchKernelGGL((k_tree_leaves<T, 2>), g, b, 0, s, U, I, R, F, P2, LB, tree); break;
    case 3: hipLaunchKernelGGL((k_tree_leaves<T, 3>), g, b, 0, s, U, I, R, F, P2, LB, tree); break;
    case 4: hipLaunchKernelGGL((k_tree_leaves<T, 4>), g, b, 0, s, U, I, R, F, P2, LB, tree); break;
    case 5: hipLaunchKernelGGL((k_tree_leaves<T, 5>), g, b, 0, s, U, I, R, F, P2, LB, tree); break;
    case 6: hipLaunchKernelGGL((k_tree_leaves<T, 6>), g, b, 0, s, U, I, R, F, P2, LB, tree); break;
    case 7: hipLaunchKernelGGL((k_tree_leaves<T, 7>), g, b, 0, s, U, I, R, F, P2, LB, tree); break;
    default: hipLaunchKernelGGL((k_tree_leaves<T, 8>), g, b, 0, s, U, I, R, F, P2, LB, tree); break;
  }
  CPR_LAUNCH_CHECK();
  for (int64_t cnt = P2 / LB / 2; cnt >= 1; cnt /= 2) {
    hipLaunchKernelGGL(k_tree_level, dim3(ceil_div(cnt * P, 256)), dim3(256),
                       0, s, tree, cnt, cnt, P);
    CPR_LAUNCH_CHECK();
  }
}
template void sts_build<float>(const float *, int64_t, int, int, int64_t,
                               double *, hipStream_t);
template void sts_build<double>(const double *, int64_t, int, int, int64_t,
                                double *, hipStream_t);

template <typename T>
void sts_draw(const ModeList &ml, int64_t J, int R, int F, const double *uni,
              const double *Gp, const double *trace, int32_t *sidx,
              double *prob, T *h, uint32_t *err, hipStream_t s) {
  if (R <= 8)
    launch_draw<T, 1, 1>(ml, J, R, F, uni, Gp, trace, sidx, prob, h, err, s);
  else if (R <= 16)
    launch_draw<T, 3, 1>(ml, J, R, F, uni, Gp, trace, sidx, prob, h, err, s);
  else if (R <= 32)
    launch_draw<T, 9, 2>(ml, J, R, F, uni, Gp, trace, sidx, prob, h, err, s);
  else if (R <= 48)
    launch_draw<T, 19, 3>(ml, J, R, F, uni, Gp, trace, sidx, prob, h, err, s);
  else
    launch_draw<T, 33, 4>(ml, J, R, F, uni, Gp, trace, sidx, prob, h, err, s);
  CPR_LAUNCH_CHECK();
}
template void sts_draw<float>(const ModeList &, int64_t, int, int,
                              const double *, const double *, const double *,
                              int32_t *, double *, float *, uint32_t *,
                              hipStream_t);
template void sts_draw<double>(const ModeList &, int64_t, int, int,
                               const double *, const double *, const double *,
                               int32_t *, double *, double *, uint32_t *,
                               hipStream_t);

}  // namespace cpr
