// STS-CP on one GPU (Section 4.1, Appendix B).
//
// Tree (Alg. 4 without the exchange): leaf b holds the Gram of rows
// [bF, bF + F) of U_k; an internal node holds the sum of its children.
// Nodes are stored in heap order (root 1, children 2v and 2v+1, leaves
// P2 .. 2 P2 - 1 with P2 a power of two) as packed upper triangles in FP64.
//
// Draw (Alg. 5 without routing): the factors != j are drawn in ascending
// order.  With h the Hadamard product of the rows drawn so far and
// G_{>k} = G^+ (*) (Grams of the factors drawn later), the mass of a node
// is <(h h^T) (*) G_{>k}, G^node>.  The first factor has h = 1, a law shared
// by all samples, and is drawn from a flat CDF of row masses.  Every later
// factor walks its tree carrying the absolute target t = u Z (go right iff
// t >= mass(left child), subtracting that mass): the paper's
// rescaled-threshold walk without the repeated division.  In the leaf the
// row masses (U[i] (*) h)^T G_{>k} (U[i] (*) h) are accumulated in row order
// and the index is min{ i : t < F(i) }.
#include "internal.h"

namespace cpr {

typedef double double4_t __attribute__((ext_vector_type(4)));

// Rank padded to a multiple of 16 (the MFMA tile); tree nodes and h rows use
// it with exact zeros beyond R.
int sts_pad(int R) { return 16 * ((R + 15) / 16); }

int sts_packed(int R) {
  const int RP = sts_pad(R);
  return RP * (RP + 1) / 2;
}

namespace {

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
k_tree_leaves(const T *U, int64_t I, int R, int RP, int F, int64_t P2, int LB,
              double *tree) {
  constexpr int NTRI = NT * (NT + 1) / 2;
  const int P = RP * (RP + 1) / 2;
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
          // entries beyond R are exact zeros (zero columns)
          if (ga < RP && gb < RP && ga <= gb)
            node[packed_index(ga, gb, RP)] = acc[i][v];
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
// Draw.  The samples of a tree factor descend level by level; a slot array
// keeps them grouped by their current node (a node owns a contiguous range
// of slots: samples sent left fill it from the front, samples sent right
// from the back), so consecutive slots share node Grams.  h, the Hadamard
// product of the rows drawn so far, is kept in FP64 in the work buffer.
//
// Every mass is a quadratic form x^T Q x in FP64.  16 of them are computed
// at a time on FP64 MFMA: with the 16 vectors as the rows of A (16 x RP),
// D = A Q, and x_i^T Q x_i = sum_j D[i][j] A[i][j].  Fragment layouts of
// v_mfma_f64_16x16x4f64 (lane l, k-step ks, 16-column tile t):
//   A: A[l % 16][4 ks + l / 16]      B: Q[4 ks + l / 16][16 t + l % 16]
//   D: element v of lane l holds D[l / 16 + 4 v][16 t + l % 16]
// ---------------------------------------------------------------------------
constexpr int ST = 256;

// B fragments of an R x R row-major matrix, zeros beyond R
template <int NT>
__device__ __forceinline__ void load_bfrag(const double *A, int R,
                                           double (&f)[NT][4 * NT]) {
  const int l = lane_id();
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int ks = 0; ks < 4 * NT; ++ks) {
      const int k = 4 * ks + l / 16, j = 16 * t + (l % 16);
      const int kc = k < R ? k : R - 1, jc = j < R ? j : R - 1;
      const double v = A[kc * R + jc];
      f[t][ks] = (k < R && j < R) ? v : 0.0;
    }
}

// packed-node offsets of the B fragments (node symmetric, upper triangle)
template <int NT>
__device__ __forceinline__ void node_offsets(int (&off)[NT][4 * NT]) {
  constexpr int RP = 16 * NT;
  const int l = lane_id();
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int ks = 0; ks < 4 * NT; ++ks) {
      const int k = 4 * ks + l / 16, j = 16 * t + (l % 16);
      off[t][ks] = k <= j ? packed_index(k, j, RP) : packed_index(j, k, RP);
    }
}

// masses of the 16 rows: lanes of group l / 16 get row l / 16 + 4 v in ms[v]
template <int NT>
__device__ __forceinline__ void tile_mass(const double (&xA)[4 * NT],
                                          const double (&xD)[NT][4],
                                          const double (&qB)[NT][4 * NT],
                                          double (&ms)[4]) {
#pragma unroll
  for (int v = 0; v < 4; ++v) ms[v] = 0.0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    double4_t acc = double4_t{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < 4 * NT; ++ks)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xA[ks], qB[t][ks], acc, 0, 0,
                                                 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) ms[v] = fma(acc[v], xD[t][v], ms[v]);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v)
    for (int o = 1; o < 16; o <<= 1) ms[v] += __shfl_xor(ms[v], o, WAVE);
}

// A and D-layout fragments of the h rows of the 16 samples held by lanes
// 16 tau .. 16 tau + 15 (rows of stride 16 NT, zeros beyond R)
template <int NT>
__device__ __forceinline__ void load_hfrag(const double *hb, int32_t s,
                                           int tau, double (&xA)[4 * NT],
                                           double (&xD)[NT][4]) {
  constexpr int RP = 16 * NT;
  const int l = lane_id();
  const int32_t sa = __shfl(s, 16 * tau + (l % 16), WAVE);
#pragma unroll
  for (int ks = 0; ks < 4 * NT; ++ks)
    xA[ks] = hb[(int64_t)sa * RP + 4 * ks + l / 16];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int32_t sd = __shfl(s, 16 * tau + l / 16 + 4 * v, WAVE);
#pragma unroll
    for (int t = 0; t < NT; ++t)
      xD[t][v] = hb[(int64_t)sd * RP + 16 * t + (l % 16)];
  }
}

// mass of the tile row held by this lane (lane 16 tau + i gets row i)
__device__ __forceinline__ double lane_mass(const double (&ms)[4]) {
  const int l = lane_id(), src = (l & 3) * 16, vv = (l >> 2) & 3;
  const double x0 = __shfl(ms[0], src, WAVE), x1 = __shfl(ms[1], src, WAVE);
  const double x2 = __shfl(ms[2], src, WAVE), x3 = __shfl(ms[3], src, WAVE);
  return vv == 0 ? x0 : vv == 1 ? x1 : vv == 2 ? x2 : x3;
}

// First factor (h = 1): every sample shares one conditional law, held as a
// flat CDF of the row masses U[i] G_{>k} U[i]^T; index = min{i : uZ < F(i)}.
template <typename T>
__global__ void __launch_bounds__(ST)
k_sts_first(const T *U, int64_t I, int R, const double *cdf, const double *Zp,
            const int64_t *lastp, const double *uni, int nq, int64_t J,
            int32_t *sidx, double *hbuf, int HS, uint32_t *err) {
  const int64_t s = (int64_t)blockIdx.x * ST + threadIdx.x;
  if (s >= J) return;
  double u = uni[s * nq];
  if (!(u >= 0.0 && u < 1.0)) {
    atomicOr(err, ERR_UNIFORM);
    u = 0.0;
  }
  const double t = u * *Zp;
  int64_t lo = 0, hi = I;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (t < cdf[mid]) hi = mid; else lo = mid + 1;
  }
  const int64_t last = *lastp;
  if (lo > last) lo = last;
  if (lo < 0) lo = 0;
  sidx[s * nq] = (int32_t)lo;
  for (int a = 0; a < HS; ++a)
    hbuf[s * HS + a] = (a < R) ? (double)U[lo * R + a] : 0.0;
}

// Root of a tree factor: node mass Z(h) and target t = u Z; clears the
// per-node placement counters of this factor's tree.
template <int NT>
__global__ void __launch_bounds__(ST)
k_sts_root(const double *tree, const double *Gg, int64_t P2, int R,
           const double *uni, int q, int nq, int64_t J, StsWork w,
           uint32_t *err) {
  constexpr int RP = 16 * NT, P = RP * (RP + 1) / 2;
  const int64_t g = (int64_t)blockIdx.x * ST + threadIdx.x;
  for (int64_t i = g; i < 2 * P2; i += (int64_t)gridDim.x * ST) {
    w.lc[i] = 0;
    w.rc[i] = 0;
  }
  if (g == 0) {
    w.sbeg[1] = 0;
    w.send[1] = (int32_t)J;
  }
  if ((int64_t)blockIdx.x * ST + (threadIdx.x & ~(WAVE - 1)) >= J) return;
  const bool act = g < J;
  const int32_t s = act ? (int32_t)g : 0;
  double qB[NT][4 * NT];
  int off[NT][4 * NT];
  load_bfrag<NT>(Gg, R, qB);
  node_offsets<NT>(off);
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int ks = 0; ks < 4 * NT; ++ks) qB[t][ks] *= tree[P + off[t][ks]];
  double Z = 0.0;
  for (int tau = 0; tau < 4; ++tau) {
    double xA[4 * NT], xD[NT][4], ms[4];
    load_hfrag<NT>(w.h, s, tau, xA, xD);
    tile_mass<NT>(xA, xD, qB, ms);
    const double m = lane_mass(ms);
    if ((lane_id() >> 4) == tau) Z = m;
  }
  if (!act) return;
  double u = uni[g * nq + q];
  if (!(u >= 0.0 && u < 1.0)) {
    atomicOr(err, ERR_UNIFORM);
    u = 0.0;
  }
  if (!(Z > 0)) atomicOr(err, ERR_ZERO_MASS);
  w.tgt[g] = u * Z;
  w.mv[g] = Z;
  w.node[g] = 1;
  w.perm[0][g] = (int32_t)g;
}

// One level: lane p takes the sample in slot p; per 16-slot tile and per
// distinct node v among its slots, the masses of the left child 2v.  Go
// right iff that mass is not positive, or the target is at or past it and
// the right child has mass; then place the sample in its child's range.
template <int NT>
__global__ void __launch_bounds__(ST)
k_sts_level(const double *tree, const double *Gg, int R, int64_t J,
            StsWork w, const int32_t *pin, int32_t *pout, int level) {
  constexpr int RP = 16 * NT, P = RP * (RP + 1) / 2;
  const int64_t p = (int64_t)blockIdx.x * ST + threadIdx.x;
  if ((int64_t)blockIdx.x * ST + (threadIdx.x & ~(WAVE - 1)) >= J) return;
  const int l = lane_id();
  const bool act = p < J;
  const int32_t s = act ? pin[p] : 0;
  const int32_t v = act ? w.node[s] : (int32_t)(1 << level);
  int32_t beg, end;  // slot range of node v
  if (v == 1) {
    beg = w.sbeg[1];
    end = w.send[1];
  } else {
    const int32_t par = v >> 1, pb = w.sbeg[par], nl = w.lc[par];
    if (v & 1) {
      beg = pb + nl;
      end = w.send[par];
    } else {
      beg = pb;
      end = pb + nl;
    }
  }
  if (act && p == beg) {
    w.sbeg[v] = beg;
    w.send[v] = end;
  }
  double gB[NT][4 * NT];
  int off[NT][4 * NT];
  load_bfrag<NT>(Gg, R, gB);
  node_offsets<NT>(off);
  const uint64_t actm = __ballot(act);
  double mL = 0.0;
  for (int tau = 0; tau < 4; ++tau) {
    uint64_t rem = actm & (0xffffull << (16 * tau));
    if (!rem) continue;
    double xA[4 * NT], xD[NT][4];
    load_hfrag<NT>(w.h, s, tau, xA, xD);
    while (rem) {
      const int ld = __ffsll((long long)rem) - 1;
      const int32_t v0 = __shfl(v, ld, WAVE);
      const uint64_t grp = __ballot(v == v0) & rem;
      const double *nd = tree + (int64_t)(2 * v0) * P;
      double qB[NT][4 * NT], ms[4];
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int ks = 0; ks < 4 * NT; ++ks)
          qB[t][ks] = gB[t][ks] * nd[off[t][ks]];
      tile_mass<NT>(xA, xD, qB, ms);
      const double m = lane_mass(ms);
      if ((grp >> l) & 1ull) mL = m;
      rem &= ~grp;
    }
  }
  double t = act ? w.tgt[s] : 0.0, m = act ? w.mv[s] : 0.0;
  const bool right = mL <= 0 || (t >= mL && m - mL > 0);
  if (right) {
    t -= (mL > 0 ? mL : 0.0);
    m -= mL;
  } else {
    m = mL;
  }
  if (act) {
    w.tgt[s] = t;
    w.mv[s] = m;
    w.node[s] = 2 * v + (right ? 1 : 0);
  }
  // one atomic per (wave, node, side)
  uint64_t todo = actm;
  const uint64_t rm = __ballot(act && right);
  const uint64_t below = (l == 0) ? 0ull : (~0ull >> (64 - l));
  int32_t pos = 0;
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int32_t v0 = __shfl(v, leader, WAVE);
    const uint64_t grp = __ballot(act && v == v0) & todo;
    const uint64_t gl = grp & ~rm, gr = grp & rm;
    int32_t bl = 0, br = 0;
    if (l == leader) {
      if (gl) bl = atomicAdd(&w.lc[v0], (int32_t)__popcll(gl));
      if (gr) br = atomicAdd(&w.rc[v0], (int32_t)__popcll(gr));
    }
    bl = __shfl(bl, leader, WAVE);
    br = __shfl(br, leader, WAVE);
    if ((grp >> l) & 1ull)
      pos = right ? end - 1 - (br + (int32_t)__popcll(gr & below))
                  : beg + bl + (int32_t)__popcll(gl & below);
    todo &= ~grp;
  }
  if (act) pout[pos] = s;
}

// Leaf: one wave per 16 slots, one sample at a time.  Row masses
// (U[i] (*) h)^T G_{>k} (U[i] (*) h) for 16 rows per MFMA tile, accumulated
// in row order; index = min{i : t < F(i)} over rows of positive mass, then
// h *= U[index].
template <typename T, int NT>
__global__ void __launch_bounds__(ST)
k_sts_leaf(const T *U, int64_t I, int R, int F, int64_t P2, const double *Gg,
           int64_t J, StsWork w, const int32_t *pin, int q, int nq,
           int32_t *sidx, uint32_t *err) {
  constexpr int RP = 16 * NT, KS = 4 * NT;
  const int l = lane_id();
  const int64_t p0 = ((int64_t)blockIdx.x * (ST / WAVE) + threadIdx.x / WAVE) * 16;
  if (p0 >= J) return;
  double gB[NT][KS];
  load_bfrag<NT>(Gg, R, gB);
  const int64_t pend = p0 + 16 < J ? p0 + 16 : J;
  for (int64_t p = p0; p < pend; ++p) {
    const int32_t s = pin[p];
    const int64_t row0 = (int64_t)(w.node[s] - P2) * F;
    const double *hrow = w.h + (int64_t)s * RP;
    const double t = w.tgt[s];
    double hk[KS], hj[NT];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) hk[ks] = hrow[4 * ks + l / 16];
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) hj[tt] = hrow[16 * tt + (l % 16)];
    double pre = 0.0;
    int pick = -1, lastpos = -1;
    for (int sub = 0; sub < F && pick < 0; sub += 16) {
      const int64_t rb = row0 + sub;
      if (rb >= I) break;
      double xA[KS], xD[NT][4], ms[4];
      {
        const int64_t r = rb + (l % 16);
        const int64_t rc = r < I ? r : I - 1;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const int k = 4 * ks + l / 16, kc = k < R ? k : R - 1;
          const double x = (double)U[rc * R + kc] * hk[ks];
          xA[ks] = r < I ? x : 0.0;
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = rb + l / 16 + 4 * v;
        const int64_t rc = r < I ? r : I - 1;
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) {
          const int j = 16 * tt + (l % 16), jc = j < R ? j : R - 1;
          const double x = (double)U[rc * R + jc] * hj[tt];
          xD[tt][v] = r < I ? x : 0.0;
        }
      }
      tile_mass<NT>(xA, xD, gB, ms);
      // row order over the 16 rows (every lane runs the same scan)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const double mi = __shfl(ms[i / 4], (i % 4) * 16, WAVE);
        if (pick < 0 && rb + i < I && mi > 0) {
          pre += mi;
          lastpos = sub + i;
          if (t < pre) pick = sub + i;
        }
      }
    }
    if (pick < 0) {
      pick = lastpos;
      if (pick < 0) {
        pick = 0;
        if (l == 0) atomicOr(err, ERR_ZERO_MASS);
      }
    }
    int64_t idx = row0 + pick;
    if (idx >= I) idx = I - 1;
    if (l == 0) sidx[(int64_t)s * nq + q] = (int32_t)idx;
    if (l < RP) {
      const int lc = l < R ? l : R - 1;
      const double x = hrow[l] * (double)U[idx * R + lc];
      w.h[(int64_t)s * RP + l] = l < R ? x : 0.0;
    }
  }
}

// Probability of the drawn Khatri-Rao row, (h^T G^+ h) / <G^+, G>, and the
// row itself in the path precision.
template <typename T, int NT>
__global__ void __launch_bounds__(ST)
k_sts_final(int R, int64_t J, const double *hbuf, const double *Gp,
            const double *trace, double *prob, T *h_out) {
  constexpr int RP = 16 * NT;
  const int64_t g = (int64_t)blockIdx.x * ST + threadIdx.x;
  if ((int64_t)blockIdx.x * ST + (threadIdx.x & ~(WAVE - 1)) >= J) return;
  const bool act = g < J;
  const int32_t s = act ? (int32_t)g : 0;
  double qB[NT][4 * NT];
  load_bfrag<NT>(Gp, R, qB);
  double mass = 0.0;
  for (int tau = 0; tau < 4; ++tau) {
    double xA[4 * NT], xD[NT][4], ms[4];
    load_hfrag<NT>(hbuf, s, tau, xA, xD);
    tile_mass<NT>(xA, xD, qB, ms);
    const double m = lane_mass(ms);
    if ((lane_id() >> 4) == tau) mass = m;
  }
  if (!act) return;
  prob[g] = mass / *trace;
  for (int a = 0; a < R; ++a) h_out[g * R + a] = (T)hbuf[g * RP + a];
}

template <typename T, int NT>
void draw_nt(const ModeList &ml, int64_t J, int R, int F, const double *uni,
             const double *Gp, const double *trace, int32_t *sidx,
             double *prob, T *h, const StsWork &w, uint32_t *err,
             hipStream_t st) {
  const int nq = ml.n;
  const dim3 g(ceil_div(J, ST)), b(ST), gl(ceil_div(J, 16 * (ST / WAVE)));
  hipLaunchKernelGGL((k_sts_first<T>), g, b, 0, st,
                     static_cast<const T *>(ml.U[0]), ml.I[0], R, ml.cdf[0],
                     ml.Z[0], ml.last[0], uni, nq, J, sidx, w.h, 16 * NT, err);
  CPR_LAUNCH_CHECK();
  for (int q = 1; q < nq; ++q) {
    const double *tree = ml.tree[q], *Gg = ml.Ggt[q];
    const int64_t P2 = ml.P2[q];
    hipLaunchKernelGGL((k_sts_root<NT>), g, b, 0, st, tree, Gg, P2, R, uni,
                       q, nq, J, w, err);
    CPR_LAUNCH_CHECK();
    int cur = 0, level = 0;
    for (int64_t n = 1; n < P2; n <<= 1, ++level) {
      hipLaunchKernelGGL((k_sts_level<NT>), g, b, 0, st, tree, Gg, R, J, w,
                         w.perm[cur], w.perm[cur ^ 1], level);
      CPR_LAUNCH_CHECK();
      cur ^= 1;
    }
    hipLaunchKernelGGL((k_sts_leaf<T, NT>), gl, b, 0, st,
                       static_cast<const T *>(ml.U[q]), ml.I[q], R, F, P2, Gg,
                       J, w, w.perm[cur], q, nq, sidx, err);
    CPR_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL((k_sts_final<T, NT>), g, b, 0, st, R, J, w.h, Gp, trace,
                     prob, h);
  CPR_LAUNCH_CHECK();
}

}  // namespace

template <typename T>
void sts_build(const T *U, int64_t I, int R, int F, int64_t P2, double *tree,
               hipStream_t s) {
  const int P = sts_packed(R), RP = sts_pad(R);
  const int LB = (int)(P2 < 64 ? P2 : 64);
  const int nt = (R + 15) / 16;
  const dim3 g((unsigned)(P2 / LB)), b(256);
  switch (nt) {
    case 1: hipLaunchKernelGGL((k_tree_leaves<T, 1>), g, b, 0, s, U, I, R, RP, F, P2, LB, tree); break;
    case 2: hipLaunchKernelGGL((k_tree_leaves<T, 2>), g, b, 0, s, U, I, R, RP, F, P2, LB, tree); break;
    case 3: hipLaunchKernelGGL((k_tree_leaves<T, 3>), g, b, 0, s, U, I, R, RP, F, P2, LB, tree); break;
    case 4: hipLaunchKernelGGL((k_tree_leaves<T, 4>), g, b, 0, s, U, I, R, RP, F, P2, LB, tree); break;
    case 5: hipLaunchKernelGGL((k_tree_leaves<T, 5>), g, b, 0, s, U, I, R, RP, F, P2, LB, tree); break;
    case 6: hipLaunchKernelGGL((k_tree_leaves<T, 6>), g, b, 0, s, U, I, R, RP, F, P2, LB, tree); break;
    case 7: hipLaunchKernelGGL((k_tree_leaves<T, 7>), g, b, 0, s, U, I, R, RP, F, P2, LB, tree); break;
    default: hipLaunchKernelGGL((k_tree_leaves<T, 8>), g, b, 0, s, U, I, R, RP, F, P2, LB, tree); break;
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
              double *prob, T *h, const StsWork &w, uint32_t *err,
              hipStream_t s) {
  switch ((R + 15) / 16) {
    case 1: draw_nt<T, 1>(ml, J, R, F, uni, Gp, trace, sidx, prob, h, w, err, s); break;
    case 2: draw_nt<T, 2>(ml, J, R, F, uni, Gp, trace, sidx, prob, h, w, err, s); break;
    case 3: draw_nt<T, 3>(ml, J, R, F, uni, Gp, trace, sidx, prob, h, w, err, s); break;
    default: draw_nt<T, 4>(ml, J, R, F, uni, Gp, trace, sidx, prob, h, w, err, s); break;
  }
}
template void sts_draw<float>(const ModeList &, int64_t, int, int,
                              const double *, const double *, const double *,
                              int32_t *, double *, float *, const StsWork &,
                              uint32_t *, hipStream_t);
template void sts_draw<double>(const ModeList &, int64_t, int, int,
                               const double *, const double *, const double *,
                               int32_t *, double *, double *,
                               const StsWork &, uint32_t *, hipStream_t);

}  // namespace cpr
