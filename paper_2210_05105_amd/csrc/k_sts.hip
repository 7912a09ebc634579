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

#include <type_traits>

namespace cpr {

typedef double double4_t __attribute__((ext_vector_type(4)));

// Rank padded to a multiple of 16 (the MFMA tile); tree nodes and h rows use
// it with exact zeros beyond R.
int sts_pad(int R) { return 16 * ((R + 15) / 16); }

// Placement counter of node v.  Every block updates the counters of the top
// nodes, so those get a 128-byte line each; deeper nodes are packed.
constexpr int64_t CTOP = 1024, CLINE = 32;
__host__ __device__ __forceinline__ int64_t cslot(int64_t v) {
  return v < CTOP ? v * CLINE : CTOP * CLINE + (v - CTOP);
}

int64_t sts_counters(int64_t P2) { return CTOP * CLINE + 2 * P2; }

int sts_packed(int R) {
  const int RP = sts_pad(R);
  return RP * (RP + 1) / 2;
}

// First factor: row masses in groups of FIRST_SUB rows (one block pass),
// 2^gshift such groups per top-level group, at most FIRST_GROUPS top-level
// groups (their prefix sums are built in LDS by every draw block).
constexpr int FIRST_SUB = 64, FIRST_GROUPS = 4096;
static int64_t first_nsub(int64_t I) { return (I + FIRST_SUB - 1) / FIRST_SUB; }
static int first_gshift(int64_t I) {
  int g = 0;
  while (((first_nsub(I) + (int64_t(1) << g) - 1) >> g) > FIRST_GROUPS) ++g;
  return g;
}
static int64_t first_ngroups(int64_t I) {
  const int g = first_gshift(I);
  return (first_nsub(I) + (int64_t(1) << g) - 1) >> g;
}
int64_t sts_first_rows(int64_t I) { return first_nsub(I) * FIRST_SUB; }
int64_t sts_first_sums(int64_t I) { return first_nsub(I) + first_ngroups(I); }

namespace {

__device__ __forceinline__ int packed_index(int a, int b, int R) {
  // a <= b; row-major upper triangle
  return a * (2 * R - a + 1) / 2 + (b - a);
}


// ---------------------------------------------------------------------------
// Build.  Block b computes the Grams of leaves [b LB, (b + 1) LB) on FP64
// MFMA (one wave per leaf, 16 x 16 tiles), keeps them in LDS and writes the
// internal nodes of its LB-leaf subtree (one thread per packed entry,
// pairwise sums in registers).  Upper levels: k_tree_up sums groups of up to
// TU_MAX = 16 sibling subtree roots, four levels per launch.
// ---------------------------------------------------------------------------
template <int LBMAX>
__device__ __forceinline__ void sum_up(double (&x)[LBMAX], int n, double *tree,
                                       int64_t first, int P, int c, double *G,
                                       int R, int RP) {
  // x[0..n) are entry c of consecutive nodes first .. first + n - 1 of one
  // level; write entry c of every ancestor up to their common root
  for (int m = n / 2; m >= 1; m /= 2) {
    first /= 2;
#pragma unroll
    for (int i = 0; i < LBMAX / 2; ++i)
      if (i < m) {
        x[i] = x[2 * i] + x[2 * i + 1];
        tree[(first + i) * P + c] = x[i];
      }
  }
  // the root is the Gram U^T U: entry c is (a, b) of the packed upper
  // triangle, written to both halves of the R x R matrix
  if (G && first == 1 && n > 1) {
    int a = 0, rem = c;
    while (rem >= RP - a) {
      rem -= RP - a;
      ++a;
    }
    const int b = a + rem;
    if (b < R) {
      G[a * R + b] = x[0];
      G[b * R + a] = x[0];
    }
  }
}

constexpr int TB_LBMAX = 16;

// SCALE: the leaf pass reads the solve's FP64 rows X and writes the factor
// U = X / sigma (zero columns stay zero) in the factor's precision; the
// Grams are of the stored values.  G (or null) receives the root as an
// R x R matrix when this launch writes the root.
template <typename T, int NT, bool SCALE, typename XT>
__global__ void __launch_bounds__(256)
k_tree_build(const T *U, const XT *X, const double *sigma, T *Uout,
             int64_t I, int R, int F, int64_t P2, int lb, double *tree,
             double *G) {
  constexpr int NTRI = NT * (NT + 1) / 2, RP = 16 * NT;
  constexpr int P = RP * (RP + 1) / 2;
  extern __shared__ double leaves[];  // LB x P
  const int LB = 1 << lb;
  const int w = threadIdx.x / WAVE, l = lane_id();
  const int64_t leaf0 = (int64_t)blockIdx.x * LB;
  double sg[NT];
  if constexpr (SCALE) {
#pragma unroll
    for (int ta = 0; ta < NT; ++ta) {
      const int ca = ta * 16 + (l % 16);
      sg[ta] = inv_or_zero(sigma[ca < R ? ca : R - 1]);  // 1 / sigma
    }
  }
  for (int lf = w; lf < LB; lf += 4) {
    const int64_t leaf = leaf0 + lf;
    const int64_t rbase = leaf * F;
    double4_t acc[NTRI];
#pragma unroll
    for (int i = 0; i < NTRI; ++i) acc[i] = double4_t{0, 0, 0, 0};
    // 16 rows (four k-steps) at a time: their loads issued together, then
    // the renormalised values stored (F is a multiple of 16)
    for (int k0 = 0; k0 < F; k0 += 16) {
      double col[4][NT];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = rbase + k0 + 4 * q + l / 16;
        const int64_t ro = (r < I ? r : I - 1) * R;
#pragma unroll
        for (int ta = 0; ta < NT; ++ta) {
          const int ca = ta * 16 + (l % 16);
          const int cc = ca < R ? ca : R - 1;
          if constexpr (SCALE) col[q][ta] = (double)X[ro + cc];
          else col[q][ta] = (double)U[ro + cc];
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = rbase + k0 + 4 * q + l / 16;
        const double rm = r < I ? 1.0 : 0.0;
#pragma unroll
        for (int ta = 0; ta < NT; ++ta) {
          const int ca = ta * 16 + (l % 16);
          double x = col[q][ta];
          if constexpr (SCALE) {
            const T u = (T)(x * sg[ta]);
            if (r < I && ca < R) Uout[r * R + ca] = u;
            x = (double)u;
          }
          col[q][ta] = x * (ca < R ? rm : 0.0);
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int ta = 0; ta < NT; ++ta)
#pragma unroll
          for (int tb = ta; tb < NT; ++tb) {
            const int i = ta * NT - ta * (ta - 1) / 2 + (tb - ta);
            acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                col[q][ta], col[q][tb], acc[i], 0, 0, 0);
          }
    }
    // tile (ta, tb), lane l, element v -> (ta*16 + l/16 + 4v, tb*16 + l%16);
    // entries beyond R are exact zeros (zero columns)
    double *node = tree + (P2 + leaf) * (int64_t)P;
    double *ln = leaves + lf * P;
#pragma unroll
    for (int ta = 0; ta < NT; ++ta)
#pragma unroll
      for (int tb = ta; tb < NT; ++tb) {
        const int i = ta * NT - ta * (ta - 1) / 2 + (tb - ta);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ga = ta * 16 + (l / 16) + 4 * v;
          const int gb = tb * 16 + (l % 16);
          if (ga <= gb) {
            const int o = packed_index(ga, gb, RP);
            node[o] = acc[i][v];
            ln[o] = acc[i][v];
          }
        }
      }
  }
  __syncthreads();
  // internal nodes of the block's subtree
  for (int c = threadIdx.x; c < P; c += 256) {
    double x[TB_LBMAX];
#pragma unroll
    for (int i = 0; i < TB_LBMAX; ++i) x[i] = i < LB ? leaves[i * P + c] : 0.0;
    sum_up<TB_LBMAX>(x, LB, tree, P2 + leaf0, P, c, G, R, RP);
  }
}

// group g of G consecutive nodes from `first` (one level): entry c of every
// ancestor up to the group's common root
constexpr int TU_MAX = 16;
__global__ void __launch_bounds__(256)
k_tree_up(double *tree, int64_t first, int G, int P, double *Gm, int R,
          int RP) {
  const int64_t f = first + (int64_t)blockIdx.x * G;
  for (int c = threadIdx.x; c < P; c += 256) {
    double x[TU_MAX];
#pragma unroll
    for (int i = 0; i < TU_MAX; ++i) {  // clamped loads, then masked
      const double y = tree[(f + (i < G ? i : G - 1)) * P + c];
      x[i] = i < G ? y : 0.0;
    }
    sum_up<TU_MAX>(x, G, tree, f, P, c, Gm, R, RP);
  }
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
// (tile_mass_t forms the product transposed, see there).
// ---------------------------------------------------------------------------
constexpr int ST = 256;

// Descent: a sample goes right when its target t lies beyond the left
// child's mass mL and the right child's mass m - mL is positive.  That
// difference is formed, not computed from the right child's Gram, so where
// the right subtree is empty it is only the rounding of the masses above
// (a few ulps of the root mass z).  A right child below STS_RTOL z counts
// as empty: the law moves by less than that fraction of the total.
constexpr double STS_RTOL = 1e-13;
__device__ __forceinline__ bool goes_right(double t, double m, double mL,
                                           double z) {
  return mL <= 0 || (t >= mL && m - mL > STS_RTOL * z);
}

// R x R row-major matrix into LDS as RP x RP with zeros beyond R (block-wide;
// a barrier must follow)
template <int RP>
__device__ __forceinline__ void stage_pad(double *dst, const double *A, int R) {
  constexpr int NS = (RP * RP + ST - 1) / ST;
  double x[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) {  // all loads first (clamped), then masked
    const int e = q * ST + threadIdx.x;
    const int a = e / RP, b = e % RP;
    x[q] = A[(a < R ? a : R - 1) * R + (b < R ? b : R - 1)];
  }
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    const int e = q * ST + threadIdx.x;
    const int a = e / RP, b = e % RP;
    if (e < RP * RP) dst[e] = x[q] * ((a < R && b < R) ? 1.0 : 0.0);
  }
}

// B fragments of a symmetric R x R matrix for tile_mass_t, staged in LDS in
// fragment order: entry f WAVE + lane holds fragment f = 2 t (t + 1) + ks
// (tile t, k-step ks <= 4 t + 3) of that lane, the off-diagonal blocks
// doubled, zeros beyond R.  Each wave then reads a fragment with one
// conflict-free LDS load.  Block-wide; a barrier must follow.
template <int NT>
constexpr int bfrag_count() { return 2 * NT * (NT + 1); }

template <int NT>
__device__ __forceinline__ void bfrag_entry(int f, int ln, int &k, int &c,
                                            bool &off) {
  int t = 0;
  while (f >= 2 * (t + 1) * (t + 2)) ++t;
  const int ks = f - 2 * t * (t + 1);
  k = 4 * ks + ln / 16;
  c = 16 * t + (ln % 16);
  off = ks / 4 < t;
}

template <int NT, int NTH = ST>
__device__ __forceinline__ void stage_bfrag(double *dst, const double *A,
                                            int R) {
  constexpr int NE = bfrag_count<NT>() * WAVE, NS = (NE + NTH - 1) / NTH;
  double x[NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) {  // all loads first (clamped), then masked
    const int e = q * NTH + threadIdx.x;
    int k, c;
    bool off;
    bfrag_entry<NT>((e < NE ? e : NE - 1) / WAVE, e % WAVE, k, c, off);
    x[q] = A[(k < R ? k : R - 1) * R + (c < R ? c : R - 1)];
  }
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    const int e = q * NTH + threadIdx.x;
    int k, c;
    bool off;
    bfrag_entry<NT>((e < NE ? e : NE - 1) / WAVE, e % WAVE, k, c, off);
    if (e < NE)
      dst[e] = (off ? 2.0 : 1.0) * x[q] * ((k < R && c < R) ? 1.0 : 0.0);
  }
}

template <int NT>
__device__ __forceinline__ void lds_bfrag_f(const double *sF,
                                            double (&f)[NT][4 * NT]) {
  const int l = lane_id();
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int ks = 0; ks < 4 * (t + 1); ++ks)
      f[t][ks] = sF[(2 * t * (t + 1) + ks) * WAVE + l];
}

// Fragments of a zero-padded symmetric RP x RP matrix held in LDS, for
// tile_mass_t: block (tile t, k-tile) is used only for k-tile <= t, the
// blocks off the diagonal doubled
template <int NT>
__device__ __forceinline__ void lds_bfrag(const double *sA,
                                          double (&f)[NT][4 * NT]) {
  constexpr int RP = 16 * NT;
  const int l = lane_id();
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int ks = 0; ks < 4 * (t + 1); ++ks)
      f[t][ks] = (ks / 4 < t ? 2.0 : 1.0) *
                 sA[(4 * ks + l / 16) * RP + 16 * t + (l % 16)];
}

// Masses x_i^T Q x_i of the 16 rows of X for a symmetric Q.  With X_t the
// 16-column tiles of X and Q_tu the blocks of Q,
//   x^T Q x = sum_t x_t^T (Q_tt x_t + 2 sum_{u<t} Q_tu x_u),
// so tile t needs (X Q')_t^T = sum_{u<=t} c_tu Q_tu X_u^T (c = 2 off the
// diagonal): NT (NT + 1) / 2 blocks of 4 MFMA k-steps instead of NT^2.  The
// product is formed transposed (A = Q fragments, which for symmetric Q are
// the B-layout values of lds_bfrag; B = X^T, which are the A-layout values
// xA of X): lane l, element v of tile t then holds (X Q')[l % 16][16 t +
// l / 16 + 4 v], whose matching X entry is the lane's own xA[4 t + v].  The
// row-dot is a local sum over the lane's 4 NT products and two shuffles
// over the four lanes of one row.  Every lane returns the mass of row
// l % 16.
template <int NT>
__device__ __forceinline__ double tile_mass_t(const double (&xA)[4 * NT],
                                              const double (&qB)[NT][4 * NT]) {
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    double4_t acc = double4_t{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < 4 * (t + 1); ++ks)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(qB[t][ks], xA[ks], acc, 0, 0,
                                                 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) s = fma(acc[v], xA[4 * t + v], s);
  }
  s += __shfl_xor(s, 16, WAVE);
  s += __shfl_xor(s, 32, WAVE);
  return s;
}


// LDS row stride of a staged 16-row tile: RP + 1 doubles, so the 16 rows
// of a fragment read fall in different banks
template <int NT>
constexpr int tile_stride() { return 16 * NT + 1; }

// The h rows (stride RP, 16-byte aligned) of the 16 samples held by lanes
// 0..15, staged in the wave's LDS buffer (16 x (RP + 1) doubles) with
// 16-byte loads, then read in A and D fragment layouts.
template <int NT>
__device__ __forceinline__ void load_hfrag_lds(const double *hb, int32_t s,
                                               double *buf,
                                               double (&xA)[4 * NT],
                                               double (&xD)[NT][4]) {
  constexpr int RP = 16 * NT, RS = tile_stride<NT>(), CH = RP / 2;
  const int l = lane_id();
#pragma unroll
  for (int i = 0; i < (16 * CH) / WAVE; ++i) {
    const int e = i * WAVE + l, r = e / CH, c = e % CH;
    const int32_t sr = __shfl(s, r, WAVE);
    const double2 v = *reinterpret_cast<const double2 *>(hb + (int64_t)sr * RP + 2 * c);
    buf[r * RS + 2 * c] = v.x;
    buf[r * RS + 2 * c + 1] = v.y;
  }
  wave_lds_sync();
#pragma unroll
  for (int ks = 0; ks < 4 * NT; ++ks) xA[ks] = buf[(l % 16) * RS + 4 * ks + l / 16];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int t = 0; t < NT; ++t) xD[t][v] = buf[(l / 16 + 4 * v) * RS + 16 * t + (l % 16)];
}


// First factor (h = 1): every sample shares one conditional law, the row
// masses U[i] G_{>k} U[i]^T; index = min{i : uZ < F(i)} with F their
// inclusive prefix sums.  No flat CDF is built: k_sts_mass writes the masses
// (zero beyond I) with their sums per FIRST_SUB rows and per top-level
// group, k_sts_first scans the group sums in LDS and, per sample, walks the
// FIRST_SUB-row sums of its group and then the row masses.

// Masses of FIRST_SUB rows per pass (16 per wave, one MFMA tile with the
// symmetric G_{>k}); block b takes the 2^gshift passes of top-level group b.
// Sums are formed in a fixed order.
template <typename T, int NT>
__global__ void __launch_bounds__(ST) __attribute__((amdgpu_waves_per_eu(4)))
k_sts_mass(const T *U, int64_t I, int R, const double *Gg, int gshift,
           double *lev, double *sub, double *grp, uint32_t *err) {
  constexpr int RP = 16 * NT, KS = 4 * NT, RS = tile_stride<NT>();
  static_assert(FIRST_SUB == 16 * (ST / WAVE), "one row tile per wave");
  __shared__ double sG[bfrag_count<NT>() * WAVE];
  __shared__ double sH[ST / WAVE][16 * RS];
  __shared__ double wsum[ST / WAVE];
  stage_bfrag<NT>(sG, Gg, R);
  __syncthreads();
  const int l = lane_id(), wv = threadIdx.x / WAVE;
  double *buf = sH[wv];
  const int lc = l < R ? l : R - 1;
  const int64_t nsub = (I + FIRST_SUB - 1) / FIRST_SUB;
  const int64_t sb0 = (int64_t)blockIdx.x << gshift;
  const int64_t sb1 = sb0 + (int64_t(1) << gshift) < nsub
                          ? sb0 + (int64_t(1) << gshift) : nsub;
  double gs = 0.0;
  for (int64_t sb = sb0; sb < sb1; ++sb) {
    const int64_t row0 = sb * FIRST_SUB + 16 * wv;
    T raw[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int64_t row = row0 + i;
      raw[i] = U[(row < I ? row : I - 1) * R + lc];
    }
    wave_lds_sync();
    if (l < RP) {
#pragma unroll
      for (int i = 0; i < 16; ++i)
        buf[i * RS + l] = (row0 + i < I && l < R) ? (double)raw[i] : 0.0;
    }
    wave_lds_sync();
    asm volatile("" ::: "memory");
    double gB[NT][KS], xA[KS];
    lds_bfrag_f<NT>(sG, gB);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) xA[ks] = buf[(l % 16) * RS + 4 * ks + l / 16];
    double m = tile_mass_t<NT>(xA, gB);  // lanes 0..15: row row0 + l
    const int64_t r = row0 + l;
    if (l < 16 && r < I && !isfinite(m)) atomicOr(err, ERR_NONFINITE);
    m = (l < 16 && r < I && m > 0) ? m : 0.0;
    if (l < 16) lev[r] = m;  // rows past I (up to the allocation) get 0
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) m += __shfl_xor(m, o, WAVE);
    if (l == 0) wsum[wv] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      double x = 0.0;
#pragma unroll
      for (int q = 0; q < ST / WAVE; ++q) x += wsum[q];
      sub[sb] = x;
      gs += x;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) grp[blockIdx.x] = gs;
}

// One sample per thread.  Every block builds the inclusive prefix sums of
// the group masses in LDS (contiguous runs per thread, then a block scan of
// the run totals).  A target past every prefix (rounding) falls back to the
// last row of positive mass, as do the walks inside a group.
template <typename T, int NT>
__global__ void __launch_bounds__(ST)
k_sts_first(const T *U, int64_t I, int R, const double *lev, const double *sub,
            const double *grp, int gshift, const double *uni, int nq,
            int64_t J, int32_t *sidx, double *hbuf, uint32_t *err) {
  constexpr int RP = 16 * NT;
  __shared__ double gc[FIRST_GROUPS];
  __shared__ double wtot[ST / WAVE];
  const int l = lane_id(), wv = threadIdx.x / WAVE;
  const int64_t nsub = (I + FIRST_SUB - 1) / FIRST_SUB;
  const int ng = (int)((nsub + (int64_t(1) << gshift) - 1) >> gshift);
  const int per = (ng + ST - 1) / ST;
  const int k0 = threadIdx.x * per, k1 = k0 + per < ng ? k0 + per : ng;
  // this thread's uniform, issued before the scan
  const int64_t s = (int64_t)blockIdx.x * ST + threadIdx.x;
  const bool act = s < J;
  double u = uni[(act ? s : J - 1) * nq];
  // the run's group sums, loaded together (clamped, then masked)
  constexpr int GPT = FIRST_GROUPS / ST;
  double gv[GPT];
#pragma unroll
  for (int j = 0; j < GPT; ++j) gv[j] = grp[k0 + j < ng ? k0 + j : ng - 1];
  double run = 0.0;
#pragma unroll
  for (int j = 0; j < GPT; ++j)
    if (k0 + j < k1) {
      run += gv[j];
      gc[k0 + j] = run;
    }
  double x = run;  // inclusive scan of the run totals within the wave
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const double y = __shfl_up(x, o, WAVE);
    if (l >= o) x += y;
  }
  if (l == WAVE - 1) wtot[wv] = x;
  __syncthreads();
  double off = x - run;
  for (int q = 0; q < wv; ++q) off += wtot[q];
  for (int k = k0; k < k1; ++k) gc[k] += off;
  __syncthreads();
  const double Z = gc[ng - 1];
  const int64_t sw0 = s - l;  // first sample of the wave
  if (sw0 >= J) return;
  // lanes past J draw for sample J - 1 and store nothing
  if (!(u >= 0.0 && u < 1.0)) {
    if (act) atomicOr(err, ERR_UNIFORM);
    u = 0.0;
  }
  if (!(Z > 0) && act) atomicOr(err, ERR_ZERO_MASS);
  double t = u * Z;
  int glo = 0, ghi = ng;  // first group with t < prefix
  while (glo < ghi) {
    const int mid = (glo + ghi) >> 1;
    if (t < gc[mid]) ghi = mid; else glo = mid + 1;
  }
  bool clamp = glo >= ng;
  if (clamp) {  // last group of positive mass: first with prefix >= Z
    int a = 0, b = ng - 1;
    while (a < b) {
      const int mid = (a + b) >> 1;
      if (gc[mid] >= Z) b = mid; else a = mid + 1;
    }
    glo = a;
  }
  t -= glo > 0 ? gc[glo - 1] : 0.0;
  // FIRST_SUB-row sums of the group (a group of one block is that block)
  const int64_t sb0 = (int64_t)glo << gshift;
  const int64_t sb1 = sb0 + (int64_t(1) << gshift) < nsub
                          ? sb0 + (int64_t(1) << gshift) : nsub;
  int64_t sb = gshift == 0 ? sb0 : -1, lastsb = sb0;
  for (int64_t k = sb0; k < sb1 && gshift > 0; ++k) {
    const double y = sub[k];
    if (y > 0) {
      lastsb = k;
      if (!clamp && t < y) { sb = k; break; }
      t -= y;
    }
  }
  if (sb < 0) {
    sb = lastsb;
    clamp = true;
  }
  // row masses of the FIRST_SUB rows (zero past I), 16 bytes per load
  const double2 *lv = reinterpret_cast<const double2 *>(lev + sb * FIRST_SUB);
  double2 mv[FIRST_SUB / 2];
#pragma unroll
  for (int i = 0; i < FIRST_SUB / 2; ++i) mv[i] = lv[i];
  int pick = -1, lastpos = -1;
#pragma unroll
  for (int i = 0; i < FIRST_SUB; ++i) {
    const double m = (i & 1) ? mv[i / 2].y : mv[i / 2].x;
    if (pick < 0 && m > 0) {
      lastpos = i;
      if (!clamp && t < m) pick = i; else t -= m;
    }
  }
  if (pick < 0) pick = lastpos < 0 ? 0 : lastpos;
  int64_t lo = sb * FIRST_SUB + pick;
  if (lo >= I) lo = I - 1;
  if (act) sidx[s * nq] = (int32_t)lo;
  // h = U[lo] for the wave's samples, the rows read and written coalesced
  // (WAVE samples x RP entries, WAVE per pass, eight passes' loads issued
  // together; a full wave stores without a condition, so that no load is
  // moved into a branch)
  const int nw = J - sw0 < WAVE ? (int)(J - sw0) : WAVE;
#pragma unroll
  for (int it0 = 0; it0 < RP; it0 += 8) {
    double x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = (it0 + j) * WAVE + l, k = e / RP, a = e % RP;
      const int64_t ik = __shfl(lo, k, WAVE);
      x[j] = (double)U[ik * R + (a < R ? a : R - 1)] * (a < R ? 1.0 : 0.0);
    }
    if (nw == WAVE) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int e = (it0 + j) * WAVE + l;
        hbuf[(sw0 + e / RP) * RP + e % RP] = x[j];
      }
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int e = (it0 + j) * WAVE + l;
        if (e / RP < nw) hbuf[(sw0 + e / RP) * RP + e % RP] = x[j];
      }
    }
  }
}

// Root of a tree factor: node mass Z(h) and target t = u Z; slot s holds
// sample s; clears the per-node placement counters of this factor's tree.
// 16 samples per wave (lanes 0..15), one MFMA tile.
template <int NT>
__global__ void __launch_bounds__(ST)
k_sts_root(const double *tree, const double *Gg, int64_t P2, int R,
           const double *uni, int q, int nq, int64_t J, StsWork w,
           SlotBuf out, uint32_t *err) {
  constexpr int RP = 16 * NT, P = RP * (RP + 1) / 2;
  __shared__ double sQ[RP * RP];  // G_{>k} (*) G^root, zeros beyond R
  __shared__ double sH[ST / WAVE][16 * tile_stride<NT>()];
  const int64_t g0 = (int64_t)blockIdx.x * ST + threadIdx.x;
  for (int64_t i = g0; i < CTOP * CLINE + 2 * P2; i += (int64_t)gridDim.x * ST) {
    w.lc[i] = 0;
    w.rc[i] = 0;
  }
  if (g0 == 0) {
    w.sbeg[1] = 0;
    w.send[1] = (int32_t)J;
  }
  stage_pad<RP>(sQ, Gg, R);
  __syncthreads();
  for (int e = threadIdx.x; e < RP * RP; e += ST) {
    const int a = e / RP, b = e % RP;
    sQ[e] *= tree[P + (a <= b ? packed_index(a, b, RP) : packed_index(b, a, RP))];
  }
  __syncthreads();
  const int l = lane_id();
  const int64_t p0 = ((int64_t)blockIdx.x * (ST / WAVE) + threadIdx.x / WAVE) * 16;
  if (p0 >= J) return;
  const int64_t g = p0 + l;
  const bool act = l < 16 && g < J;
  const int32_t s = (int32_t)(p0 + ((l % 16) < J - p0 ? (l % 16) : 0));
  double qB[NT][4 * NT], xA[4 * NT], xD[NT][4];
  lds_bfrag<NT>(sQ, qB);
  load_hfrag_lds<NT>(w.h, s, sH[threadIdx.x / WAVE], xA, xD);
  const double Z = tile_mass_t<NT>(xA, qB);
  if (!act) return;
  double u = uni[g * nq + q];
  if (!(u >= 0.0 && u < 1.0)) {
    atomicOr(err, ERR_UNIFORM);
    u = 0.0;
  }
  if (!(Z > 0)) atomicOr(err, ERR_ZERO_MASS);
  out.s[g] = (int32_t)g;
  out.v[g] = 1;
  out.t[g] = u * Z;
  out.m[g] = Z;
  out.z[g] = Z;
}

// Top of a tree factor (trees of at least 2 TOP_N leaves): instead of the
// root and TOP_D levels, each sample takes a depth-TOP_D node directly by
// inverse CDF over the TOP_N node masses <(h h^T) (*) G_{>k}, G^v> in node
// order (their sum is the root mass Z; t = u Z).  16 samples per wave, one
// MFMA tile per node, the TOP_N products G_{>k} (*) G^v packed in LDS.
// Writes (node, t - mass before it, node mass) per sample in sample order,
// counts per node (one atomic per block and node) and clears the placement
// counters of the levels below.
constexpr int TOP_D = 3, TOP_N = 1 << TOP_D;
constexpr int TOP_ST = 512;  // 8 waves per block share the staged nodes

template <int NT>
__global__ void __launch_bounds__(TOP_ST)
k_sts_top(const double *tree, const double *Gg, int64_t P2, int R,
          const double *uni, int q, int nq, int64_t J, StsWork w,
          SlotBuf out, int32_t *tcnt, uint32_t *err) {
  constexpr int RP = 16 * NT, P = RP * (RP + 1) / 2, KS = 4 * NT;
  // B fragments of the TOP_N products 2^[off-diagonal block] G_{>k} (*) G^v,
  // fragment f = 2 t (t + 1) + ks of tile t, k-step ks, one double per lane:
  // built once per block, then read by every wave without bank conflicts.
  // The same LDS first holds each wave's 16 h rows.
  constexpr int NQ = 2 * NT * (NT + 1);
  constexpr int QE = TOP_N * NQ * WAVE;
  constexpr int HE = (TOP_ST / WAVE) * 16 * tile_stride<NT>();
  static_assert(QE == NQ * TOP_ST, "fragment entries per thread");
  __shared__ double sQ[QE > HE ? QE : HE];
  __shared__ double sG[RP * RP];    // G_{>k}, zeros beyond R
  __shared__ int32_t scnt[TOP_N];
  const int l = lane_id();
  const int64_t g0 = (int64_t)blockIdx.x * TOP_ST + threadIdx.x;
  // this lane's uniform (if it has a sample), issued before the staging
  const int64_t gu = ((int64_t)blockIdx.x * (TOP_ST / WAVE) + threadIdx.x / WAVE) * 16 +
                     l % 16;
  const double u0 = uni[(gu < J ? gu : J - 1) * nq + q];
  for (int64_t i = g0; i < CTOP * CLINE + 2 * P2; i += (int64_t)gridDim.x * TOP_ST) {
    w.lc[i] = 0;
    w.rc[i] = 0;
  }
  if (threadIdx.x < TOP_N) scnt[threadIdx.x] = 0;
  // every staging load first: G_{>k} (clamped, masked when stored) and this
  // thread's NQ node entries (nodes TOP_N .. 2 TOP_N - 1)
  constexpr int NG = (RP * RP + TOP_ST - 1) / TOP_ST;
  double z[NG], y[NQ];
#pragma unroll
  for (int j = 0; j < NG; ++j) {
    const int e = j * TOP_ST + threadIdx.x, a = e / RP, b = e % RP;
    z[j] = Gg[(a < R ? a : R - 1) * R + (b < R ? b : R - 1)];
  }
  auto entry = [&](int j, int &v, int &k, int &c, bool &off) {
    const int idx = j * TOP_ST + threadIdx.x;  // lane of the entry: l
    v = idx / (NQ * WAVE);
    const int f = (idx / WAVE) % NQ;
    int tt = 0;
    while (f >= 2 * (tt + 1) * (tt + 2)) ++tt;
    const int ks = f - 2 * tt * (tt + 1);
    k = 4 * ks + l / 16;
    c = 16 * tt + (l % 16);
    off = ks / 4 < tt;
  };
#pragma unroll
  for (int j = 0; j < NQ; ++j) {
    int v, k, c;
    bool off;
    entry(j, v, k, c, off);
    y[j] = tree[(int64_t)(TOP_N + v) * P +
                (k <= c ? packed_index(k, c, RP) : packed_index(c, k, RP))];
  }
  const int64_t p0 = ((int64_t)blockIdx.x * (TOP_ST / WAVE) + threadIdx.x / WAVE) * 16;
  const int64_t g = p0 + l;
  const bool act = p0 < J && l < 16 && g < J;
  double xA[KS], xD[NT][4];
  if (p0 < J) {
    const int32_t s = (int32_t)(p0 + ((l % 16) < J - p0 ? (l % 16) : 0));
    load_hfrag_lds<NT>(w.h, s, sQ + (threadIdx.x / WAVE) * 16 * tile_stride<NT>(),
                       xA, xD);
  }
#pragma unroll
  for (int j = 0; j < NG; ++j) {
    const int e = j * TOP_ST + threadIdx.x, a = e / RP, b = e % RP;
    if (e < RP * RP) sG[e] = z[j] * ((a < R && b < R) ? 1.0 : 0.0);
  }
  __syncthreads();  // h tiles read, G_{>k} staged
#pragma unroll
  for (int j = 0; j < NQ; ++j) {
    int v, k, c;
    bool off;
    entry(j, v, k, c, off);
    sQ[j * TOP_ST + threadIdx.x] = (off ? 2.0 : 1.0) * sG[k * RP + c] * y[j];
  }
  __syncthreads();
  if (p0 < J) {
    double mm[TOP_N];
#pragma unroll 2
    for (int v = 0; v < TOP_N; ++v) {  // two nodes' MFMA chains interleaved
      double qB[NT][KS];
#pragma unroll
      for (int tt = 0; tt < NT; ++tt)
#pragma unroll
        for (int ks = 0; ks < 4 * (tt + 1); ++ks)
          qB[tt][ks] = sQ[(v * NQ + 2 * tt * (tt + 1) + ks) * WAVE + l];
      const double x = tile_mass_t<NT>(xA, qB);  // lanes 0..15: sample l
#pragma unroll
      for (int i = 0; i < TOP_N; ++i)
        if (i == v) mm[i] = x;
    }
    double Z = 0.0;
#pragma unroll
    for (int i = 0; i < TOP_N; ++i) Z += mm[i] > 0 ? mm[i] : 0.0;
    if (act) {
      double u = u0;  // g == gu for active lanes
      if (!(u >= 0.0 && u < 1.0)) {
        atomicOr(err, ERR_UNIFORM);
        u = 0.0;
      }
      if (!(Z > 0)) atomicOr(err, ERR_ZERO_MASS);
      // first node with t < cumulative mass (t then relative to it); past
      // the end (rounding): the last node of positive mass with t at its
      // mass, so that the levels below end in its last row of positive mass
      double t = u * Z, mv = 0.0, lastm = 0.0;
      int pick = -1, lastpos = -1;
#pragma unroll
      for (int i = 0; i < TOP_N; ++i) {
        const double x = mm[i];
        if (pick < 0 && x > 0) {
          lastpos = i;
          lastm = x;
          if (t < x) {
            pick = i;
            mv = x;
          } else {
            t -= x;
          }
        }
      }
      if (pick < 0) {
        pick = lastpos < 0 ? 0 : lastpos;
        mv = lastm;
        t = mv;
      }
      out.s[g] = (int32_t)g;
      out.v[g] = TOP_N + pick;
      out.t[g] = t;
      out.m[g] = mv;
      out.z[g] = Z;
      atomicAdd(&scnt[pick], 1);
    }
  }
  __syncthreads();
  if (threadIdx.x < TOP_N)  // this block's count per node (no atomics)
    tcnt[(int64_t)blockIdx.x * TOP_N + threadIdx.x] = scnt[threadIdx.x];
}

// Place the samples of the top stage in their node's slot range (nodes in
// order, ranges contiguous); sets the ranges and left counts of the nodes
// one level up so that the next level finds them as it does below a level.
// A block places ST consecutive samples, which are those of top-stage blocks
// 2b and 2b + 1: from the per-block counts it forms the node totals (range
// starts) and its own offsets inside each range (the samples of the
// earlier blocks), with no global atomics; ranks inside the block come from
// LDS counters.
constexpr int TOP_SPB = 16 * (TOP_ST / WAVE);  // samples per top-stage block
static_assert(ST == 2 * TOP_SPB, "two top-stage blocks per placement block");

__global__ void __launch_bounds__(ST)
k_sts_top_place(int64_t J, StsWork w, SlotBuf in, SlotBuf out,
                const int32_t *tcnt, int ntb) {
  __shared__ int32_t start[TOP_N + 1], bcnt[TOP_N], bbase[TOP_N];
  __shared__ int32_t red[ST / WAVE][2 * TOP_N];
  const int l = lane_id(), wv = threadIdx.x / WAVE;
  // this thread's record first (clamped; its loads overlap the count sums)
  const int64_t g = (int64_t)blockIdx.x * ST + threadIdx.x;
  const bool a = g < J;
  const int64_t gc = a ? g : J - 1;
  const int32_t s = in.s[gc], v = in.v[gc];
  const double t = in.t[gc], m = in.m[gc], z = in.z[gc];
  int32_t tot[TOP_N], pre[TOP_N];
#pragma unroll
  for (int i = 0; i < TOP_N; ++i) tot[i] = pre[i] = 0;
  for (int tb = threadIdx.x; tb < ntb; tb += ST) {
    const int4 *row = reinterpret_cast<const int4 *>(tcnt + (int64_t)tb * TOP_N);
    const int4 c0 = row[0], c1 = row[1];
    const int32_t c[TOP_N] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
    const bool before = tb < 2 * (int)blockIdx.x;
#pragma unroll
    for (int i = 0; i < TOP_N; ++i) {
      tot[i] += c[i];
      pre[i] += before ? c[i] : 0;
    }
  }
#pragma unroll
  for (int i = 0; i < TOP_N; ++i)
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
      tot[i] += __shfl_xor(tot[i], o, WAVE);
      pre[i] += __shfl_xor(pre[i], o, WAVE);
    }
  if (l == 0)
#pragma unroll
    for (int i = 0; i < TOP_N; ++i) {
      red[wv][i] = tot[i];
      red[wv][TOP_N + i] = pre[i];
    }
  if (threadIdx.x < TOP_N) bcnt[threadIdx.x] = 0;
  __syncthreads();
  if (threadIdx.x < 2 * TOP_N) {
    int32_t x = 0;
    for (int q = 0; q < ST / WAVE; ++q) x += red[q][threadIdx.x];
    if (threadIdx.x >= TOP_N) bbase[threadIdx.x - TOP_N] = x;
    else red[0][threadIdx.x] = x;  // read back by thread 0 after a barrier
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t a = 0;
    for (int i = 0; i < TOP_N; ++i) {
      start[i] = a;
      a += red[0][i];
    }
    start[TOP_N] = a;
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x < TOP_N / 2) {  // parents TOP_N/2 ..
    const int p = TOP_N / 2 + threadIdx.x, i = 2 * threadIdx.x;
    w.sbeg[p] = start[i];
    w.send[p] = start[i + 2];
    w.lc[cslot(p)] = start[i + 1] - start[i];
  }
  int32_t rank = 0;
  if (a) rank = atomicAdd(&bcnt[v - TOP_N], 1);
  __syncthreads();
  if (a) {
    const int32_t pos = start[v - TOP_N] + bbase[v - TOP_N] + rank;
    out.s[pos] = s;
    out.v[pos] = v;
    out.t[pos] = t;
    out.m[pos] = m;
    out.z[pos] = z;
  }
}

// One level.  A block owns 64 consecutive slots; wave i takes slots
// 16 i .. 16 i + 15 in lanes 0..15 and, per distinct node v among them, the
// masses of the left child 2v on MFMA.  Go right iff that mass is not
// positive, or the target is at or past it and the right child has mass.
// Wave 0 then places the block's 64 samples in their children's slot
// ranges with one atomic per (node, side).
template <int NT>
__global__ void __launch_bounds__(ST) __attribute__((amdgpu_waves_per_eu(4)))
k_sts_level(const double *tree, const double *Gg, int R, int64_t J,
            StsWork w, SlotBuf in, SlotBuf out) {
  constexpr int RP = 16 * NT, P = RP * (RP + 1) / 2;
  __shared__ int32_t sh_s[64], sh_v[64], sh_beg[64], sh_end[64];
  __shared__ double sh_t[64], sh_m[64], sh_z[64];
  __shared__ int32_t sh_r[64];
  __shared__ double sG[bfrag_count<NT>() * WAVE];  // G_{>k}, zeros beyond R
  __shared__ double sH[ST / WAVE][16 * tile_stride<NT>()];
  const int64_t pb = (int64_t)blockIdx.x * 64;
  if (pb >= J) return;
  const int l = lane_id(), wv = threadIdx.x / WAVE;
  const int64_t p = pb + 16 * wv + l;
  const bool act = l < 16 && p < J;
  // slot record (clamped slot; inactive lanes are ignored), issued before
  // the staging barrier
  const int64_t pc = p < J ? p : J - 1;
  const int32_t s = in.s[pc];
  const int32_t v = in.v[pc];
  double t = in.t[pc], m = in.m[pc];
  const double z = in.z[pc];
  stage_bfrag<NT>(sG, Gg, R);
  // slot range of node v: the root's, or the parent's split at its left count
  const int32_t par = v > 1 ? v >> 1 : 1;
  const int32_t pbg = w.sbeg[par], pen = w.send[par], nl = w.lc[cslot(par)];
  // h fragments of the 16 slots and the node of slot 0, loaded together
  double xA[4 * NT], xD[NT][4];
  load_hfrag_lds<NT>(w.h, s, sH[wv], xA, xD);
  const uint64_t actm = __ballot(act);
  const int ld0 = actm ? __ffsll((long long)actm) - 1 : 0;
  int32_t v0 = __shfl(v, ld0, WAVE);
  double nv[NT][4 * NT];  // node blocks used by tile_mass_t (k-tile <= tile)
  auto load_node = [&](int32_t vn) {
    const double *nd = tree + (int64_t)(2 * vn) * P;
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
      for (int ks = 0; ks < 4 * (tt + 1); ++ks) {
        const int k = 4 * ks + l / 16, j = 16 * tt + (l % 16);
        nv[tt][ks] = nd[k <= j ? packed_index(k, j, RP) : packed_index(j, k, RP)];
      }
  };
  load_node(v0);
  __syncthreads();
  const int32_t beg = v == 1 ? pbg : (v & 1) ? pbg + nl : pbg;
  const int32_t end = v == 1 ? pen : (v & 1) ? pen : pbg + nl;
  if (act && p == beg) {
    w.sbeg[v] = beg;
    w.send[v] = end;
  }
  double mL = 0.0;
  uint64_t rem = actm;
  while (rem) {
    const uint64_t grp = __ballot(v == v0) & rem;
    // nv becomes the B fragments of G_{>k} (*) node in place; G_{>k} is
    // read from LDS again in every pass rather than held in registers
    asm volatile("" ::: "memory");
#pragma unroll
    for (int tt = 0; tt < NT; ++tt)
#pragma unroll
      for (int ks = 0; ks < 4 * (tt + 1); ++ks)
        nv[tt][ks] *= sG[(2 * tt * (tt + 1) + ks) * WAVE + l];
    const double x = tile_mass_t<NT>(xA, nv);
    if ((grp >> l) & 1ull) mL = x;
    rem &= ~grp;
    if (rem) {
      v0 = __shfl(v, __ffsll((long long)rem) - 1, WAVE);
      load_node(v0);
    }
  }
  const bool right = goes_right(t, m, mL, z);
  if (right) {
    t -= (mL > 0 ? mL : 0.0);
    m -= mL;
  } else {
    m = mL;
  }
  if (l < 16) {
    const int i = 16 * wv + l;
    sh_s[i] = s;
    sh_v[i] = v;
    sh_beg[i] = beg;
    sh_end[i] = end;
    sh_t[i] = t;
    sh_m[i] = m;
    sh_z[i] = z;
    sh_r[i] = right ? 1 : 0;
  }
  __syncthreads();
  if (wv != 0) return;
  // placement of the block's 64 slots (lane i = slot pb + i): left children
  // fill a node's range from the front, right children from the back.  The
  // slots of one node are consecutive, so each node's first lane leads its
  // group, and all groups reserve their slots with one atomic instruction
  // per side (the leaders' lanes), waited for once.
  const bool a2 = pb + l < J;  // the active lanes are a prefix
  const int32_t v2 = sh_v[l], b2 = sh_beg[l], e2 = sh_end[l];
  const bool r2 = sh_r[l] != 0;
  const int32_t vp = __shfl_up(v2, 1, WAVE);
  const bool lead = a2 && (l == 0 || vp != v2);
  const uint64_t leads = __ballot(lead), am = __ballot(a2);
  const uint64_t rm = __ballot(a2 && r2);
  const uint64_t upto = (2ull << l) - 1;  // lanes 0 .. l
  const uint64_t below = upto >> 1;       // lanes 0 .. l - 1
  const uint64_t ldb = leads & upto;
  const int myld = ldb ? 63 - __clzll((long long)ldb) : 0;
  const uint64_t nxt = leads & ~upto;
  const uint64_t gend = nxt ? ((1ull << __ffsll((long long)nxt) - 1) - 1) : ~0ull;
  const uint64_t grp = am & gend & ~((1ull << myld) - 1);
  const uint64_t gL = grp & ~rm, gR = grp & rm;
  int32_t bl = 0, br = 0;
  if (lead && gL) bl = atomicAdd(&w.lc[cslot(v2)], (int32_t)__popcll(gL));
  if (lead && gR) br = atomicAdd(&w.rc[cslot(v2)], (int32_t)__popcll(gR));
  bl = __shfl(bl, myld, WAVE);
  br = __shfl(br, myld, WAVE);
  const int32_t pos = r2 ? e2 - 1 - (br + (int32_t)__popcll(gR & below))
                         : b2 + bl + (int32_t)__popcll(gL & below);
  if (a2) {
    out.s[pos] = sh_s[l];
    out.v[pos] = 2 * v2 + (r2 ? 1 : 0);
    out.t[pos] = sh_t[l];
    out.m[pos] = sh_m[l];
    out.z[pos] = sh_z[l];
  }
}

// Leaf: one wave per 16 slots, the 16 samples side by side (lane i and the
// rows i of the MFMA tiles belong to slot i).  Pass r computes the masses
// (U[row0 + r] (*) h)^T G_{>k} (U[row0 + r] (*) h) of row r of every
// sample's leaf; each sample accumulates its rows in order and takes
// index = min{i : t < F(i)} over rows of positive mass.  Then h *= U[index].
// A sample's leaf is F consecutive rows of U: they are read PB rows at a
// time as 16-byte chunks spread over all 64 lanes, staged in LDS in the
// factor's precision, and the next batch is in flight while the current
// one's PB passes run on the MFMA.
template <typename T, int NT>
constexpr int leaf_pb() {  // rows per batch (F is a multiple)
  return 2;
}

template <typename T, int NT, bool VEC>
__global__ void __launch_bounds__(ST)
__attribute__((amdgpu_waves_per_eu(VEC ? 4 : 2)))
k_sts_leaf(const T *U, int64_t I, int R, int F, int64_t P2, const double *Gg,
           int64_t J, StsWork w, SlotBuf in, int q, int nq, int32_t *sidx,
           uint32_t *err) {
  constexpr int RP = 16 * NT, KS = 4 * NT, PB = leaf_pb<T, NT>();
  constexpr int CE = VEC ? 16 / (int)sizeof(T) : 1;  // elements per chunk
  constexpr int RSU = RP + 16 / (int)sizeof(T);      // staged row stride
  constexpr int NCH = (16 * PB * RP / CE + WAVE - 1) / WAVE;
  constexpr int HB = 16 * tile_stride<NT>() * 8;     // h staging bytes
  constexpr int UB = PB * 16 * RSU * (int)sizeof(T);
  constexpr int WB = (HB > UB ? HB : UB) / 8;        // doubles per wave
  __shared__ double sG[bfrag_count<NT>() * WAVE];
  __shared__ double sW[ST / WAVE][WB];
  __shared__ int64_t sR0[ST / WAVE][16];  // first leaf row of each slot
  stage_bfrag<NT>(sG, Gg, R);
  __syncthreads();
  const int l = lane_id();
  const int64_t p0 = ((int64_t)blockIdx.x * (ST / WAVE) + threadIdx.x / WAVE) * 16;
  if (p0 >= J) return;
  const int n = J - p0 < 16 ? (int)(J - p0) : 16;
  // lane l holds slot l % 16 (slot 0 stands in beyond n)
  const int64_t ps = p0 + ((l % 16) < n ? (l % 16) : 0);
  const int32_t s = in.s[ps];
  const int64_t row0 = (int64_t)(in.v[ps] - P2) * F;
  const double t = in.t[ps];
  double hA[KS], hD[NT][4];
  double *buf = sW[threadIdx.x / WAVE];
  load_hfrag_lds<NT>(w.h, s, buf, hA, hD);
  T *stg = reinterpret_cast<T *>(buf);  // [PB][16][RSU], after h
  int64_t *r0s = sR0[threadIdx.x / WAVE];
  if (l < 16) r0s[l] = row0;
  // chunk j of this lane: sample i, row r of the batch, column c, packed
  // as (i << 24) | (r << 16) | c (i = 16: no chunk); rows past I are read
  // clamped and staged as zeros
  const int cps = PB * R / CE;  // chunks per sample and batch
  int cm[NCH];
#pragma unroll
  for (int j = 0; j < NCH; ++j) {
    const int qq = l + WAVE * j;
    if (qq < 16 * cps) {
      const int i = qq / cps, e = (qq - i * cps) * CE;
      cm[j] = (i << 24) | ((e / R) << 16) | (e % R);
    } else {
      cm[j] = 16 << 24;
    }
  }
  typedef T chunk_t __attribute__((ext_vector_type(CE)));
  chunk_t ch[NCH];
  wave_lds_sync();  // h fragments read, r0s written
  auto chunk_row = [&](int j, int bt) -> int64_t {
    const int i = cm[j] >> 24;
    return r0s[i < 16 ? i : 0] + (int64_t)bt * PB + ((cm[j] >> 16) & 255);
  };
  auto load_batch = [&](int bt) {
#pragma unroll
    for (int j = 0; j < NCH; ++j) {
      int64_t row = chunk_row(j, bt);
      row = row < I ? row : I - 1;
      ch[j] = *reinterpret_cast<const chunk_t *>(U + row * R + (cm[j] & 65535));
    }
  };
  if (R < RP)  // columns R .. RP - 1 stay zero
    for (int e = l; e < PB * 16 * (RP - R); e += WAVE) {
      const int pr = e / (RP - R), c = R + e % (RP - R);
      stg[pr * RSU + c] = T(0);
    }
  double pre = 0.0;
  int pick = -1, lastpos = -1;
  const int nb = F / PB;
  load_batch(0);
  for (int bt = 0; bt < nb; ++bt) {
    wave_lds_sync();  // the previous batch's fragment reads are done
#pragma unroll
    for (int j = 0; j < NCH; ++j) {
      const int i = cm[j] >> 24;
      if (i < 16) {
        const bool ok = chunk_row(j, bt) < I;
        T *d = stg + (((cm[j] >> 16) & 255) * 16 + i) * RSU + (cm[j] & 65535);
#pragma unroll
        for (int c = 0; c < CE; ++c) d[c] = ok ? ch[j][c] : T(0);
      }
    }
    load_batch(bt + 1 < nb ? bt + 1 : bt);
    wave_lds_sync();
    // the PB rows' masses as independent MFMA chains; G_{>k} fragments are
    // read from LDS again in every batch rather than held in registers
    asm volatile("" ::: "memory");
    double mr[PB];
    {
      double gB[NT][KS], xA[PB][KS];
      lds_bfrag_f<NT>(sG, gB);
#pragma unroll
      for (int pp = 0; pp < PB; ++pp)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
          xA[pp][ks] = (double)stg[(pp * 16 + l % 16) * RSU + 4 * ks + l / 16] *
                       hA[ks];
#pragma unroll
      for (int pp = 0; pp < PB; ++pp)
        mr[pp] = tile_mass_t<NT>(xA[pp], gB);  // lanes 0..15: row of slot l
    }
#pragma unroll
    for (int pp = 0; pp < PB; ++pp) {
      const int r = bt * PB + pp;
      const double m = mr[pp];
      if (pick < 0 && row0 + r < I && m > 0) {
        pre += m;
        lastpos = r;
        if (t < pre) pick = r;
      }
    }
    // the wave's 16 slots have all found their row: later rows change nothing
    if (__ballot(pick < 0) == 0) break;
  }
  const bool act = l < n;
  if (pick < 0) {
    pick = lastpos;
    if (pick < 0) {
      pick = 0;
      if (act) atomicOr(err, ERR_ZERO_MASS);
    }
  }
  int64_t idx = row0 + pick;
  if (idx >= I) idx = I - 1;
  if (act) sidx[(int64_t)s * nq + q] = (int32_t)idx;
#pragma unroll
  for (int it = 0; it < RP / 4; ++it) {  // 16 RP entries, 64 per pass
    const int e = it * WAVE + l, k = e / RP, a = e % RP;
    const int64_t sk = __shfl(s, k, WAVE), ik = __shfl(idx, k, WAVE);
    if (k < n) {
      const int ac = a < R ? a : R - 1;
      const double x = w.h[sk * RP + a] * (double)U[ik * R + ac];
      w.h[sk * RP + a] = a < R ? x : 0.0;
    }
  }
}

// Probability of the drawn Khatri-Rao row, (h^T G^+ h) / <G^+, G>, and the
// row itself in the path precision.  16 samples per wave (lanes 0..15).
template <typename T, int NT>
__global__ void __launch_bounds__(ST)
k_sts_final(int R, int64_t J, const double *hbuf, const double *Gp,
            const double *trace, double *prob, T *h_out) {
  constexpr int RP = 16 * NT;
  __shared__ double sP[bfrag_count<NT>() * WAVE];
  __shared__ double sH[ST / WAVE][16 * tile_stride<NT>()];
  stage_bfrag<NT>(sP, Gp, R);
  __syncthreads();
  const int l = lane_id();
  const int64_t p0 = ((int64_t)blockIdx.x * (ST / WAVE) + threadIdx.x / WAVE) * 16;
  if (p0 >= J) return;
  const int n = J - p0 < 16 ? (int)(J - p0) : 16;
  const int32_t s = (int32_t)(p0 + ((l % 16) < n ? (l % 16) : 0));
  double qB[NT][4 * NT], xA[4 * NT], xD[NT][4];
  lds_bfrag_f<NT>(sP, qB);
  load_hfrag_lds<NT>(hbuf, s, sH[threadIdx.x / WAVE], xA, xD);
  const double mass = tile_mass_t<NT>(xA, qB);
  if (l < n) prob[p0 + l] = mass / *trace;
  // the 16 rows of h in the path precision, coalesced
  const int ne = n * R;
  double hv[RP / 4];  // ne <= 16 R <= 64 (RP / 4); loads first (clamped)
#pragma unroll
  for (int it = 0; it < RP / 4; ++it) {
    const int e = it * WAVE + l < ne ? it * WAVE + l : ne - 1;
    hv[it] = hbuf[(p0 + e / R) * RP + e % R];
  }
#pragma unroll
  for (int it = 0; it < RP / 4; ++it) {
    const int e = it * WAVE + l;
    if (e < ne) h_out[(p0 + e / R) * R + e % R] = (T)hv[it];
  }
}

// ---------------------------------------------------------------------------
// Wide ranks (NT >= 5, R > 64).  The kernels above hold a whole symmetric
// Q in MFMA fragments (NT (NT + 1) / 2 blocks of 4 k-steps per lane), which
// past NT = 4 exceeds the register file.  Here the fragments are streamed
// tile by tile: G_{>k} (or G^+) from LDS in fragment order, a node product
// G_{>k} (*) G^node formed on the way from the tree's packed node and the
// LDS fragment.  The 16-row X tiles (h rows, factor rows) are read from
// global memory directly in A-fragment layout, so LDS holds only the
// fragments (57 KiB at NT = 7, 74 KiB at NT = 8).
// ---------------------------------------------------------------------------
constexpr int WNT_MIN = 5;

// x^T Q x of the 16 rows of X (lane l: row l % 16) for Q given by its
// fragments in LDS (stage_bfrag layout): as tile_mass_t, one tile at a time.
template <int NT>
__device__ __forceinline__ double tile_mass_s(const double (&xA)[4 * NT],
                                              const double *sF) {
  const int l = lane_id();
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    double4_t acc = double4_t{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < 4 * (t + 1); ++ks)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(
          sF[(2 * t * (t + 1) + ks) * WAVE + l], xA[ks], acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) s = fma(acc[v], xA[4 * t + v], s);
    // keep each tile's fragment loads next to its MFMAs (bounded registers)
    __builtin_amdgcn_sched_barrier(0);
  }
  s += __shfl_xor(s, 16, WAVE);
  s += __shfl_xor(s, 32, WAVE);
  return s;
}

// The same for Q = G_{>k} (*) G^node with the node's packed upper triangle
// nd (global) and the G_{>k} fragments sG (LDS, off-diagonal blocks doubled).
template <int NT>
__device__ __forceinline__ double tile_mass_node(const double (&xA)[4 * NT],
                                                 const double *nd,
                                                 const double *sG) {
  constexpr int RP = 16 * NT;
  const int l = opaque_lane();
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    double q[4 * NT];
#pragma unroll
    for (int ks = 0; ks < 4 * (t + 1); ++ks) {  // tile t's loads together
      const int k = 4 * ks + l / 16, j = 16 * t + (l % 16);
      q[ks] = nd[k <= j ? packed_index(k, j, RP) : packed_index(j, k, RP)];
    }
    double4_t acc = double4_t{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < 4 * (t + 1); ++ks)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(
          q[ks] * sG[(2 * t * (t + 1) + ks) * WAVE + l], xA[ks], acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) s = fma(acc[v], xA[4 * t + v], s);
    __builtin_amdgcn_sched_barrier(0);  // one tile's node loads at a time
  }
  s += __shfl_xor(s, 16, WAVE);
  s += __shfl_xor(s, 32, WAVE);
  return s;
}

// A-fragment of the 16 h rows (FP64, row stride RP, zeros beyond R) of the
// samples held by lanes 0..15 (s: this lane's sample; lane l takes row
// l % 16): xA[ks] = h[sample of row l % 16][4 ks + l / 16].
template <int NT>
__device__ __forceinline__ void load_hfrag_direct(const double *hb, int32_t s,
                                                  double (&xA)[4 * NT]) {
  constexpr int RP = 16 * NT;
  const int l = lane_id();
  const int32_t sr = __shfl(s, l % 16, WAVE);
  const double *row = hb + (int64_t)sr * RP + l / 16;
#pragma unroll
  for (int ks = 0; ks < 4 * NT; ++ks) xA[ks] = row[4 * ks];
}

// First factor, wide ranks: as k_sts_mass, but each wave takes whole
// FIRST_SUB-row blocks (four 16-row tiles in order) and writes their sums,
// so the block's waves meet only once, for the group sum; every sum is
// formed in the same order as in k_sts_mass.
template <typename T, int NT>
__global__ void __launch_bounds__(ST) __attribute__((amdgpu_waves_per_eu(2)))
k_sts_mass_w(const T *U, int64_t I, int R, const double *Gg, int gshift,
             double *lev, double *sub, double *grp, uint32_t *err) {
  constexpr int KS = 4 * NT, NTILE = FIRST_SUB / 16;
  __shared__ double sG[bfrag_count<NT>() * WAVE];
  stage_bfrag<NT>(sG, Gg, R);
  __syncthreads();
  const int l = lane_id(), wv = threadIdx.x / WAVE;
  const int64_t nsub = (I + FIRST_SUB - 1) / FIRST_SUB;
  const int64_t sb0 = (int64_t)blockIdx.x << gshift;
  const int64_t sb1 = sb0 + (int64_t(1) << gshift) < nsub
                          ? sb0 + (int64_t(1) << gshift) : nsub;
  // this wave's tiles: block sb0 + wv + 4 i, tile tt; rows clamped, masked
  T raw[KS];
  auto load_tile = [&](int64_t sb, int tt) {
    const int64_t r = sb * FIRST_SUB + 16 * tt + (l % 16);
    const T *src = U + (r < I ? r : I - 1) * R;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int c = 4 * ks + l / 16;
      raw[ks] = src[c < R ? c : R - 1];
    }
  };
  // FP32 rows: the next tile is loaded while this one is multiplied (FP64
  // rows would take twice the registers: loaded at the tile's start)
  constexpr bool PF = sizeof(T) == 4 && NT <= 7;
  const int64_t wsb0 = sb0 + wv;
  if (PF && wsb0 < sb1) load_tile(wsb0, 0);
  for (int64_t sb = wsb0; sb < sb1; sb += ST / WAVE) {
    double x = 0.0;  // the block's sum, tile by tile
#pragma unroll 1
    for (int tt = 0; tt < NTILE; ++tt) {
      const int64_t row0 = sb * FIRST_SUB + 16 * tt;
      const int64_t r = row0 + (l % 16);
      const double rm = r < I ? 1.0 : 0.0;
      if (!PF) load_tile(sb, tt);
      double xA[KS];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
        xA[ks] = (4 * ks + l / 16 < R) ? (double)raw[ks] * rm : 0.0;
      if (PF) {
        if (tt + 1 < NTILE) load_tile(sb, tt + 1);
        else if (sb + ST / WAVE < sb1) load_tile(sb + ST / WAVE, 0);
      }
      double m = tile_mass_s<NT>(xA, sG);  // lanes 0..15: row row0 + l
      if (l < 16 && r < I && !isfinite(m)) atomicOr(err, ERR_NONFINITE);
      m = (l < 16 && r < I && m > 0) ? m : 0.0;
      if (l < 16) lev[row0 + l] = m;  // rows past I (up to the allocation) get 0
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) m += __shfl_xor(m, o, WAVE);
      x += m;
    }
    if (l == 0) sub[sb] = x;
  }
  __threadfence_block();  // the waves' block sums, read back by thread 0
  __syncthreads();
  if (threadIdx.x == 0) {
    double gs = 0.0;
    for (int64_t sb = sb0; sb < sb1; ++sb) gs += sub[sb];
    grp[blockIdx.x] = gs;
  }
}

// sQ = G_{>k} (*) G^node in the fragment order of stage_bfrag (off-diagonal
// blocks doubled, zeros beyond R), in chunks of CH entries per thread: the
// chunk's loads first, then its products.  Block-wide; a barrier must follow.
template <int NT, int NTH>
__device__ __forceinline__ void form_q(double *sQ, const double *Gg,
                                       const double *nd, int R) {
  constexpr int RP = 16 * NT;
  constexpr int NE = bfrag_count<NT>() * WAVE, NS = (NE + NTH - 1) / NTH;
  constexpr int CH = 8;
#pragma unroll
  for (int q0 = 0; q0 < NS; q0 += CH) {
    double g[CH], x[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int e = (q0 + j) * NTH + threadIdx.x;
      int k, c;
      bool off;
      bfrag_entry<NT>((e < NE ? e : NE - 1) / WAVE, e % WAVE, k, c, off);
      g[j] = Gg[(k < R ? k : R - 1) * R + (c < R ? c : R - 1)];
      x[j] = nd[k <= c ? packed_index(k, c, RP) : packed_index(c, k, RP)];
    }
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int e = (q0 + j) * NTH + threadIdx.x;
      int k, c;
      bool off;
      bfrag_entry<NT>((e < NE ? e : NE - 1) / WAVE, e % WAVE, k, c, off);
      const double gv = (off ? 2.0 : 1.0) * g[j] * ((k < R && c < R) ? 1.0 : 0.0);
      if (q0 + j < NS && e < NE) sQ[e] = x[j] * gv;
    }
    __builtin_amdgcn_sched_barrier(0);  // one chunk's loads at a time
  }
}

// Root of a tree factor, wide ranks (as k_sts_root).
template <int NT>
__global__ void __launch_bounds__(ST) __attribute__((amdgpu_waves_per_eu(2)))
k_sts_root_w(const double *tree, const double *Gg, int64_t P2, int R,
             const double *uni, int q, int nq, int64_t J, StsWork w,
             SlotBuf out, uint32_t *err) {
  __shared__ double sQ[bfrag_count<NT>() * WAVE];  // G_{>k} (*) G^root
  const int64_t g0 = (int64_t)blockIdx.x * ST + threadIdx.x;
  for (int64_t i = g0; i < CTOP * CLINE + 2 * P2; i += (int64_t)gridDim.x * ST) {
    w.lc[i] = 0;
    w.rc[i] = 0;
  }
  if (g0 == 0) {
    w.sbeg[1] = 0;
    w.send[1] = (int32_t)J;
  }
  constexpr int RP = 16 * NT, P = RP * (RP + 1) / 2;
  form_q<NT, ST>(sQ, Gg, tree + P, R);  // the product k_sts_level_q forms
  __syncthreads();
  const int l = lane_id();
  // every block stages the product once and its waves take 16-slot tiles
  const int64_t ntile = (J + 15) / 16;
  for (int64_t tile = (int64_t)blockIdx.x * (ST / WAVE) + threadIdx.x / WAVE;
       tile < ntile; tile += (int64_t)gridDim.x * (ST / WAVE)) {
    const int64_t p0 = tile * 16;
    const int64_t g = p0 + l;
    const bool act = l < 16 && g < J;
    const int32_t s = (int32_t)(p0 + ((l % 16) < J - p0 ? (l % 16) : 0));
    double xA[4 * NT];
    load_hfrag_direct<NT>(w.h, s, xA);
    const double Z = tile_mass_s<NT>(xA, sQ);
    if (act) {
      double u = uni[g * nq + q];
      if (!(u >= 0.0 && u < 1.0)) {
        atomicOr(err, ERR_UNIFORM);
        u = 0.0;
      }
      if (!(Z > 0)) atomicOr(err, ERR_ZERO_MASS);
      out.s[g] = (int32_t)g;
      out.v[g] = 1;
      out.t[g] = u * Z;
      out.m[g] = Z;
      out.z[g] = Z;
    }
  }
}

// One level, wide ranks (as k_sts_level; the mass of each distinct node's
// left child streamed from the tree).
template <int NT>
__global__ void __launch_bounds__(ST) __attribute__((amdgpu_waves_per_eu(2)))
k_sts_level_w(const double *tree, const double *Gg, int R, int64_t J,
              StsWork w, SlotBuf in, SlotBuf out) {
  constexpr int RP = 16 * NT, P = RP * (RP + 1) / 2;
  __shared__ int32_t sh_s[64], sh_v[64], sh_beg[64], sh_end[64];
  __shared__ double sh_t[64], sh_m[64], sh_z[64];
  __shared__ int32_t sh_r[64];
  __shared__ double sG[bfrag_count<NT>() * WAVE];  // G_{>k}, zeros beyond R
  const int64_t pb = (int64_t)blockIdx.x * 64;
  if (pb >= J) return;
  const int l = lane_id(), wv = threadIdx.x / WAVE;
  const int64_t p = pb + 16 * wv + l;
  const bool act = l < 16 && p < J;
  const int64_t pc = p < J ? p : J - 1;
  const int32_t s = in.s[pc];
  const int32_t v = in.v[pc];
  double t = in.t[pc], m = in.m[pc];
  const double z = in.z[pc];
  stage_bfrag<NT>(sG, Gg, R);
  const int32_t par = v > 1 ? v >> 1 : 1;
  const int32_t pbg = w.sbeg[par], pen = w.send[par], nl = w.lc[cslot(par)];
  double xA[4 * NT];
  load_hfrag_direct<NT>(w.h, s, xA);
  __syncthreads();
  const uint64_t actm = __ballot(act);
  const int32_t beg = v == 1 ? pbg : (v & 1) ? pbg + nl : pbg;
  const int32_t end = v == 1 ? pen : (v & 1) ? pen : pbg + nl;
  if (act && p == beg) {
    w.sbeg[v] = beg;
    w.send[v] = end;
  }
  double mL = 0.0;
  uint64_t rem = actm;
  while (rem) {
    const int32_t v0 = __shfl(v, __ffsll((long long)rem) - 1, WAVE);
    const uint64_t grp = __ballot(v == v0) & rem;
    // G_{>k} fragments are read from LDS in every pass, not hoisted into
    // registers
    asm volatile("" ::: "memory");
    const double x = tile_mass_node<NT>(xA, tree + (int64_t)(2 * v0) * P, sG);
    if ((grp >> l) & 1ull) mL = x;
    rem &= ~grp;
  }
  const bool right = goes_right(t, m, mL, z);
  if (right) {
    t -= (mL > 0 ? mL : 0.0);
    m -= mL;
  } else {
    m = mL;
  }
  if (l < 16) {
    const int i = 16 * wv + l;
    sh_s[i] = s;
    sh_v[i] = v;
    sh_beg[i] = beg;
    sh_end[i] = end;
    sh_t[i] = t;
    sh_m[i] = m;
    sh_z[i] = z;
    sh_r[i] = right ? 1 : 0;
  }
  __syncthreads();
  if (wv != 0) return;
  // placement of the block's 64 slots, as in k_sts_level
  const bool a2 = pb + l < J;
  const int32_t v2 = sh_v[l], b2 = sh_beg[l], e2 = sh_end[l];
  const bool r2 = sh_r[l] != 0;
  const int32_t vp = __shfl_up(v2, 1, WAVE);
  const bool lead = a2 && (l == 0 || vp != v2);
  const uint64_t leads = __ballot(lead), am = __ballot(a2);
  const uint64_t rm = __ballot(a2 && r2);
  const uint64_t upto = (2ull << l) - 1;
  const uint64_t below = upto >> 1;
  const uint64_t ldb = leads & upto;
  const int myld = ldb ? 63 - __clzll((long long)ldb) : 0;
  const uint64_t nxt = leads & ~upto;
  const uint64_t gend = nxt ? ((1ull << __ffsll((long long)nxt) - 1) - 1) : ~0ull;
  const uint64_t grp = am & gend & ~((1ull << myld) - 1);
  const uint64_t gL = grp & ~rm, gR = grp & rm;
  int32_t bl = 0, br = 0;
  if (lead && gL) bl = atomicAdd(&w.lc[cslot(v2)], (int32_t)__popcll(gL));
  if (lead && gR) br = atomicAdd(&w.rc[cslot(v2)], (int32_t)__popcll(gR));
  bl = __shfl(bl, myld, WAVE);
  br = __shfl(br, myld, WAVE);
  const int32_t pos = r2 ? e2 - 1 - (br + (int32_t)__popcll(gR & below))
                         : b2 + bl + (int32_t)__popcll(gL & below);
  if (a2) {
    out.s[pos] = sh_s[l];
    out.v[pos] = 2 * v2 + (r2 ? 1 : 0);
    out.t[pos] = sh_t[l];
    out.m[pos] = sh_m[l];
    out.z[pos] = sh_z[l];
  }
}

// One level, wide ranks, at depths where each node holds many slots: a
// block takes a run of consecutive groups of LQ_GROUP slots (16 per wave).
// Slots are ordered by node, so a group meets few distinct nodes, and
// consecutive groups mostly continue the previous group's node.  For each node the
// product G_{>k} (*) G^{left child} is formed once in LDS, in fragment order
// (kept while the next group stays on that node), and the waves holding
// slots at that node take their masses from LDS: the same FP64 products and
// MFMA sums as k_sts_level_w, so the same masses, without every wave
// streaming the node from global memory tile by tile.  Placement as in
// k_sts_level_w.
constexpr int LQ_THREADS = 256;
constexpr int LQ_GROUP = 16 * (LQ_THREADS / WAVE);
constexpr int LQ_BLOCKS = 512;    // two blocks per CU
constexpr int64_t LQ_MIN = 512;   // slots per node on average to use it
constexpr int LP_BLOCKS = 512;    // persistent per-sample kernels: two per CU

template <int NT>
__global__ void __launch_bounds__(LQ_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
k_sts_level_q(const double *tree, const double *Gg, int R, int64_t J,
              StsWork w, SlotBuf in, SlotBuf out) {
  constexpr int RP = 16 * NT, P = RP * (RP + 1) / 2;
  constexpr int NE = bfrag_count<NT>() * WAVE;
  __shared__ double sQ[NE];  // G_{>k} (*) G^qnode, fragment order
  __shared__ int32_t sh_s[LQ_GROUP], sh_v[LQ_GROUP], sh_beg[LQ_GROUP],
      sh_end[LQ_GROUP], sh_r[LQ_GROUP];
  __shared__ double sh_t[LQ_GROUP], sh_m[LQ_GROUP], sh_z[LQ_GROUP];
  const int l = lane_id(), wv = threadIdx.x / WAVE;
  // a contiguous run of groups per block, so consecutive groups share nodes
  const int64_t ngrp = (J + LQ_GROUP - 1) / LQ_GROUP;
  const int64_t gpb = (ngrp + gridDim.x - 1) / gridDim.x;
  const int64_t g0 = (int64_t)blockIdx.x * gpb;
  const int64_t g1 = g0 + gpb < ngrp ? g0 + gpb : ngrp;
  int32_t qnode = -1;  // the node whose product sQ holds (block-uniform)
  for (int64_t grp = g0; grp < g1; ++grp) {
    const int64_t pb = grp * LQ_GROUP;
    const int64_t p = pb + 16 * wv + l;
    const bool act = l < 16 && p < J;
    const int64_t pc = p < J ? p : J - 1;
    const int32_t s = in.s[pc];
    const int32_t v = in.v[pc];
    double t = in.t[pc], m = in.m[pc];
    const double z = in.z[pc];
    const int32_t par = v > 1 ? v >> 1 : 1;
    const int32_t pbg = w.sbeg[par], pen = w.send[par], nl = w.lc[cslot(par)];
    double xA[4 * NT];
    load_hfrag_direct<NT>(w.h, s, xA);
    const int32_t beg = v == 1 ? pbg : (v & 1) ? pbg + nl : pbg;
    const int32_t end = v == 1 ? pen : (v & 1) ? pen : pbg + nl;
    if (act && p == beg) {
      w.sbeg[v] = beg;
      w.send[v] = end;
    }
    if (l < 16) sh_v[16 * wv + l] = act ? v : INT32_MAX;  // ascending
    __syncthreads();
    double mL = 0.0;
    int32_t cur = sh_v[0];
    while (cur != INT32_MAX) {  // the group's distinct nodes, in order
      // first slot past cur's run
      int lo = 0, hi = LQ_GROUP;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sh_v[mid] <= cur) lo = mid + 1; else hi = mid;
      }
      const int32_t nxt = lo < LQ_GROUP ? sh_v[lo] : INT32_MAX;
      if (cur != qnode) {
        form_q<NT, LQ_THREADS>(sQ, Gg, tree + (int64_t)(2 * cur) * P, R);
        qnode = cur;
        __syncthreads();  // sQ formed
      }
      const uint64_t here = __ballot(act && v == cur);
      if (here) {
        const double x = tile_mass_s<NT>(xA, sQ);
        if ((here >> l) & 1ull) mL = x;
      }
      if (nxt != INT32_MAX) __syncthreads();  // sQ read before it changes
      cur = nxt;
    }
    const bool right = goes_right(t, m, mL, z);
    if (right) {
      t -= (mL > 0 ? mL : 0.0);
      m -= mL;
    } else {
      m = mL;
    }
    if (l < 16) {
      const int i = 16 * wv + l;
      sh_s[i] = s;
      sh_beg[i] = beg;
      sh_end[i] = end;
      sh_t[i] = t;
      sh_m[i] = m;
      sh_z[i] = z;
      sh_r[i] = right ? 1 : 0;
    }
    __syncthreads();  // also: every wave's sQ reads are done
    if (wv == 0) {  // placement of the group's 64 slots
      const bool a2 = pb + l < J;
      const int32_t v2 = sh_v[l], b2 = sh_beg[l], e2 = sh_end[l];
      const bool r2 = sh_r[l] != 0;
      const int32_t vp = __shfl_up(v2, 1, WAVE);
      const bool lead = a2 && (l == 0 || vp != v2);
      const uint64_t leads = __ballot(lead), am = __ballot(a2);
      const uint64_t rm = __ballot(a2 && r2);
      const uint64_t upto = (2ull << l) - 1;
      const uint64_t below = upto >> 1;
      const uint64_t ldb = leads & upto;
      const int myld = ldb ? 63 - __clzll((long long)ldb) : 0;
      const uint64_t nxl = leads & ~upto;
      const uint64_t gend = nxl ? ((1ull << __ffsll((long long)nxl) - 1) - 1) : ~0ull;
      const uint64_t grpm = am & gend & ~((1ull << myld) - 1);
      const uint64_t gL = grpm & ~rm, gR = grpm & rm;
      int32_t bl = 0, br = 0;
      if (lead && gL) bl = atomicAdd(&w.lc[cslot(v2)], (int32_t)__popcll(gL));
      if (lead && gR) br = atomicAdd(&w.rc[cslot(v2)], (int32_t)__popcll(gR));
      bl = __shfl(bl, myld, WAVE);
      br = __shfl(br, myld, WAVE);
      const int32_t pos = r2 ? e2 - 1 - (br + (int32_t)__popcll(gR & below))
                             : b2 + bl + (int32_t)__popcll(gL & below);
      if (a2) {
        out.s[pos] = sh_s[l];
        out.v[pos] = 2 * v2 + (r2 ? 1 : 0);
        out.t[pos] = sh_t[l];
        out.m[pos] = sh_m[l];
        out.z[pos] = sh_z[l];
      }
    }
    __syncthreads();  // sh_* read before the next group writes them
  }
}

// Leaf, wide ranks (as k_sts_leaf): one wave per 16 slots, one leaf row of
// every slot per pass, the next row's values in flight during the pass.
template <typename T, int NT>
__global__ void __launch_bounds__(ST) __attribute__((amdgpu_waves_per_eu(2)))
k_sts_leaf_w(const T *U, int64_t I, int R, int F, int64_t P2, const double *Gg,
             int64_t J, StsWork w, SlotBuf in, int q, int nq, int32_t *sidx,
             uint32_t *err) {
  constexpr int RP = 16 * NT, KS = 4 * NT;
  __shared__ double sG[bfrag_count<NT>() * WAVE];
  stage_bfrag<NT>(sG, Gg, R);
  __syncthreads();
  const int l = lane_id();
  const int64_t p0 = ((int64_t)blockIdx.x * (ST / WAVE) + threadIdx.x / WAVE) * 16;
  if (p0 >= J) return;
  const int n = J - p0 < 16 ? (int)(J - p0) : 16;
  const int64_t ps = p0 + ((l % 16) < n ? (l % 16) : 0);
  const int32_t s = in.s[ps];
  const int64_t row0 = (int64_t)(in.v[ps] - P2) * F;
  const double t = in.t[ps];
  double hA[KS];
  load_hfrag_direct<NT>(w.h, s, hA);
  // lane l reads row row0 + r of slot l % 16, columns 4 ks + l / 16
  auto load_row = [&](int r, T (&x)[KS]) {
    const int64_t row = row0 + r;
    const T *src = U + (row < I ? row : I - 1) * R;
    const int lz = opaque_lane();
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int c = 4 * ks + lz / 16;
      x[ks] = src[c < R ? c : R - 1];
    }
  };
  double pre = 0.0;
  int pick = -1, lastpos = -1;
  T nx[KS];
  load_row(0, nx);
  for (int r = 0; r < F; ++r) {
    double xA[KS];
    const double rm = row0 + r < I ? 1.0 : 0.0;
    const int lz = opaque_lane();
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      xA[ks] = (4 * ks + lz / 16 < R) ? (double)nx[ks] * hA[ks] * rm : 0.0;
    load_row(r + 1 < F ? r + 1 : r, nx);
    asm volatile("" ::: "memory");  // G_{>k} fragments re-read per row
    const double mm = tile_mass_s<NT>(xA, sG);  // lanes 0..15: slot l
    if (pick < 0 && row0 + r < I && mm > 0) {
      pre += mm;
      lastpos = r;
      if (t < pre) pick = r;
    }
    // the wave's 16 slots have all found their row: later rows change nothing
    if (__ballot(pick < 0) == 0) break;
  }
  const bool act = l < n;
  if (pick < 0) {
    pick = lastpos;
    if (pick < 0) {
      pick = 0;
      if (act) atomicOr(err, ERR_ZERO_MASS);
    }
  }
  int64_t idx = row0 + pick;
  if (idx >= I) idx = I - 1;
  if (act) sidx[(int64_t)s * nq + q] = (int32_t)idx;
#pragma unroll
  for (int it = 0; it < RP / 4; ++it) {  // 16 RP entries, 64 per pass
    const int e = it * WAVE + l, k = e / RP, a = e % RP;
    const int64_t sk = __shfl(s, k, WAVE), ik = __shfl(idx, k, WAVE);
    if (k < n) {
      const int ac = a < R ? a : R - 1;
      const double x = w.h[sk * RP + a] * (double)U[ik * R + ac];
      w.h[sk * RP + a] = a < R ? x : 0.0;
    }
  }
}

// Probabilities and h rows in the path precision, wide ranks (as k_sts_final).
template <typename T, int NT>
__global__ void __launch_bounds__(ST) __attribute__((amdgpu_waves_per_eu(2)))
k_sts_final_w(int R, int64_t J, const double *hbuf, const double *Gp,
              const double *trace, double *prob, T *h_out) {
  constexpr int RP = 16 * NT;
  __shared__ double sP[bfrag_count<NT>() * WAVE];
  stage_bfrag<NT>(sP, Gp, R);
  __syncthreads();
  const int l = lane_id();
  // G^+ staged once per block; its waves take 16-sample tiles
  const int64_t ntile = (J + 15) / 16;
  for (int64_t tile = (int64_t)blockIdx.x * (ST / WAVE) + threadIdx.x / WAVE;
       tile < ntile; tile += (int64_t)gridDim.x * (ST / WAVE)) {
    const int64_t p0 = tile * 16;
    const int n = J - p0 < 16 ? (int)(J - p0) : 16;
    const int32_t s = (int32_t)(p0 + ((l % 16) < n ? (l % 16) : 0));
    double xA[4 * NT];
    load_hfrag_direct<NT>(hbuf, s, xA);
    const double mass = tile_mass_s<NT>(xA, sP);
    if (l < n) prob[p0 + l] = mass / *trace;
    const int ne = n * R;
    double hv[RP / 4];
#pragma unroll
    for (int it = 0; it < RP / 4; ++it) {
      const int e = it * WAVE + l < ne ? it * WAVE + l : ne - 1;
      hv[it] = hbuf[(p0 + e / R) * RP + e % R];
    }
#pragma unroll
    for (int it = 0; it < RP / 4; ++it) {
      const int e = it * WAVE + l;
      if (e < ne) h_out[(p0 + e / R) * R + e % R] = (T)hv[it];
    }
  }
}

// Tree leaves, wide ranks: one block per pair of sibling leaves (two leaf
// Grams, then their parent as the sum of the two, kept in registers: the
// upper levels then start one level up), the NT (NT + 1) / 2 tiles of a
// Gram split over the 4 waves (tile i to wave i % 4); every wave reads the
// leaves' rows, wave 0 writes the renormalised factor (SCALE).  Nodes above
// the parents come from k_tree_up.
// Rows of U staged by wave 0 of the build (SCALE): 16 rows, stride RP + one
// 16-byte chunk, so each k-block's rows go out as one contiguous span.
template <typename T, int NT>
constexpr int ustage_stride() { return 16 * NT + 16 / (int)sizeof(T); }
// staged only where two blocks (the leaf stash and the rows) still fit a CU
template <typename T, int NT, bool PAIR>
constexpr bool ustage_fits() {
  return 2 * ((PAIR ? 4 * ((NT * (NT + 1) / 2 + 3) / 4) * WAVE * 32 : 32) +
              16 * ustage_stride<T, NT>() * (int)sizeof(T)) <= 160 * 1024;
}

template <typename T, int NT, bool SCALE, int W, typename XT, bool STAGE>
__device__ __forceinline__ void leaf_acc(const T *U, const XT *X,
                                         const double (&sg)[NT], T *Uout,
                                         T *ubuf,
                                         int64_t I, int R, int F, int64_t leaf,
                                         double4_t (&acc)[(NT * (NT + 1) / 2 - W + 3) / 4 > 0
                                                              ? (NT * (NT + 1) / 2 - W + 3) / 4
                                                              : 1]) {
  constexpr int NTRI = NT * (NT + 1) / 2;
  constexpr int NMY = (NTRI - W + 3) / 4;  // tiles of this wave
  constexpr int QH = 2;  // k-steps whose rows are read together
  const int l = lane_id();
#pragma unroll
  for (int i = 0; i < (NMY > 0 ? NMY : 1); ++i) acc[i] = double4_t{0, 0, 0, 0};
  const int64_t rbase = leaf * F;
  for (int k0 = 0; k0 < F; k0 += 16) {
#pragma unroll
    for (int q0 = 0; q0 < 4; q0 += QH) {
      double col[QH][NT];
#pragma unroll
      for (int qq = 0; qq < QH; ++qq) {
        const int64_t r = rbase + k0 + 4 * (q0 + qq) + l / 16;
        const int64_t ro = (r < I ? r : I - 1) * R;
#pragma unroll
        for (int ta = 0; ta < NT; ++ta) {
          const int ca = ta * 16 + (l % 16);
          const int cc = ca < R ? ca : R - 1;
          if constexpr (SCALE) col[qq][ta] = (double)X[ro + cc];
          else col[qq][ta] = (double)U[ro + cc];
        }
      }
#pragma unroll
      for (int qq = 0; qq < QH; ++qq) {
        const int64_t r = rbase + k0 + 4 * (q0 + qq) + l / 16;
        const double rm = r < I ? 1.0 : 0.0;
#pragma unroll
        for (int ta = 0; ta < NT; ++ta) {
          const int ca = ta * 16 + (l % 16);
          double x = col[qq][ta];
          if constexpr (SCALE) {
            const T u = (T)(x * sg[ta]);
            if constexpr (STAGE) {
              if (W == 0 && ca < R)
                ubuf[(4 * (q0 + qq) + l / 16) * ustage_stride<T, NT>() + ca] = u;
            } else {
              if (W == 0 && r < I && ca < R) Uout[r * R + ca] = u;
            }
            x = (double)u;
          }
          col[qq][ta] = x * (ca < R ? rm : 0.0);
        }
      }
#pragma unroll
      for (int qq = 0; qq < QH; ++qq)
#pragma unroll
        for (int ta = 0; ta < NT; ++ta)
#pragma unroll
          for (int tb = ta; tb < NT; ++tb) {
            const int i = ta * NT - ta * (ta - 1) / 2 + (tb - ta);
            if (i % 4 == W)
              acc[i / 4] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                  col[qq][ta], col[qq][tb], acc[i / 4], 0, 0, 0);
          }
      __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (SCALE && STAGE && W == 0) {  // the 16 staged rows, contiguous
      constexpr int US = ustage_stride<T, NT>(), VW = 16 / (int)sizeof(T);
      wave_lds_sync();
      const int64_t r0 = rbase + k0;
      const int nv = I - r0 < 16 ? (int)(I - r0) : 16;
      T *dst = Uout + r0 * R;
      if (nv > 0 && R % VW == 0) {
        typedef T vec_t __attribute__((ext_vector_type(VW)));
        for (int q = l; q < nv * R / VW; q += WAVE) {
          const int e = VW * q, rr = e / R, c = e - rr * R;
          *reinterpret_cast<vec_t *>(dst + e) =
              *reinterpret_cast<const vec_t *>(ubuf + rr * US + c);
        }
      } else if (nv > 0) {
        for (int e = l; e < nv * R; e += WAVE) {
          const int rr = e / R;
          dst[e] = ubuf[rr * US + (e - rr * R)];
        }
      }
      wave_lds_sync();  // read before the next k-block's rows are staged
    }
  }
}

template <int NT, int W, int NA>
__device__ __forceinline__ void write_tiles(const double4_t (&acc)[NA],
                                            double *node) {
  constexpr int RP = 16 * NT;
  const int l = lane_id();
#pragma unroll
  for (int ta = 0; ta < NT; ++ta)
#pragma unroll
    for (int tb = ta; tb < NT; ++tb) {
      const int i = ta * NT - ta * (ta - 1) / 2 + (tb - ta);
      if (i % 4 == W) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ga = ta * 16 + (l / 16) + 4 * v;
          const int gb = tb * 16 + (l % 16);
          if (ga <= gb) node[packed_index(ga, gb, RP)] = acc[i / 4][v];
        }
      }
    }
}

// The tile entries as the full R x R matrix G (both halves), for a node
// that is the tree's root.
template <int NT, int W, int NA>
__device__ __forceinline__ void write_full(const double4_t (&acc)[NA],
                                           double *G, int R) {
  const int l = lane_id();
#pragma unroll
  for (int ta = 0; ta < NT; ++ta)
#pragma unroll
    for (int tb = ta; tb < NT; ++tb) {
      const int i = ta * NT - ta * (ta - 1) / 2 + (tb - ta);
      if (i % 4 == W) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ga = ta * 16 + (l / 16) + 4 * v;
          const int gb = tb * 16 + (l % 16);
          if (ga <= gb && gb < R) {
            G[ga * R + gb] = acc[i / 4][v];
            G[gb * R + ga] = acc[i / 4][v];
          }
        }
      }
    }
}

// PAIR: leaves 2b and 2b + 1 and their parent; else leaf b alone.  G (or
// null) receives the root when this block writes it (P2 = 2 with pairs).
// The first leaf's tiles wait in LDS (each lane its own entries, so no
// barrier) while the second leaf is formed in the same registers.
template <typename T, int NT, bool SCALE, bool PAIR, int W, typename XT>
__device__ __forceinline__ void leaf_block(const T *U, const XT *X,
                                           const double (&sg)[NT], T *Uout,
                                           T *ubuf,
                                           int64_t I, int R, int F, int64_t P2,
                                           int64_t b, double *tree, double *G,
                                           double4_t *stash) {
  constexpr int RP = 16 * NT, P = RP * (RP + 1) / 2;
  constexpr int NTRI = NT * (NT + 1) / 2;
  constexpr int NA = (NTRI - W + 3) / 4 > 0 ? (NTRI - W + 3) / 4 : 1;
  const int l = lane_id();
  double4_t a0[NA];
  if constexpr (!PAIR) {
    leaf_acc<T, NT, SCALE, W, XT, ustage_fits<T, NT, PAIR>()>(U, X, sg, Uout, ubuf, I, R, F, b, a0);
    write_tiles<NT, W>(a0, tree + (P2 + b) * (int64_t)P);
  } else {
    leaf_acc<T, NT, SCALE, W, XT, ustage_fits<T, NT, PAIR>()>(U, X, sg, Uout, ubuf, I, R, F, 2 * b, a0);
    write_tiles<NT, W>(a0, tree + (P2 + 2 * b) * (int64_t)P);
#pragma unroll
    for (int i = 0; i < NA; ++i) stash[i * WAVE + l] = a0[i];
    leaf_acc<T, NT, SCALE, W, XT, ustage_fits<T, NT, PAIR>()>(U, X, sg, Uout, ubuf, I, R, F, 2 * b + 1, a0);
    write_tiles<NT, W>(a0, tree + (P2 + 2 * b + 1) * (int64_t)P);
#pragma unroll
    for (int i = 0; i < NA; ++i) a0[i] += stash[i * WAVE + l];
    write_tiles<NT, W>(a0, tree + (P2 / 2 + b) * (int64_t)P);
    if (G && P2 == 2) write_full<NT, W>(a0, G, R);
  }
}

template <typename T, int NT, bool SCALE, bool PAIR, typename XT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_tree_build_w(const T *U, const XT *X, const double *sigma, T *Uout,
               int64_t I, int R, int F, int64_t P2, double *tree, double *G) {
  const int l = lane_id();
  double sg[NT];
#pragma unroll
  for (int ta = 0; ta < NT; ++ta) {
    const int ca = ta * 16 + (l % 16);
    sg[ta] = SCALE ? inv_or_zero(sigma[ca < R ? ca : R - 1]) : 1.0;  // 1 / sigma
  }
  constexpr int NAMAX = (NT * (NT + 1) / 2 + 3) / 4;
  __shared__ double4_t stash[PAIR ? 4 * NAMAX * WAVE : 1];
  __shared__ __align__(16)
      T ubuf[SCALE && ustage_fits<T, NT, PAIR>() ? 16 * ustage_stride<T, NT>() : 1];
  const int64_t b = blockIdx.x;
  const int w = threadIdx.x / WAVE;
  double4_t *st = stash + (PAIR ? w * NAMAX * WAVE : 0);
  switch (w) {
    case 0: leaf_block<T, NT, SCALE, PAIR, 0, XT>(U, X, sg, Uout, ubuf, I, R, F, P2, b, tree, G, st); break;
    case 1: leaf_block<T, NT, SCALE, PAIR, 1, XT>(U, X, sg, Uout, ubuf, I, R, F, P2, b, tree, G, st); break;
    case 2: leaf_block<T, NT, SCALE, PAIR, 2, XT>(U, X, sg, Uout, ubuf, I, R, F, P2, b, tree, G, st); break;
    default: leaf_block<T, NT, SCALE, PAIR, 3, XT>(U, X, sg, Uout, ubuf, I, R, F, P2, b, tree, G, st); break;
  }
}

template <typename T, int NT>
void draw_nt(const ModeList &ml, int64_t J, int R, const double *uni,
             const double *Gp, const double *trace, int32_t *sidx,
             double *prob, T *h, const StsWork &w, uint32_t *err,
             hipStream_t st) {
  constexpr bool WIDE = NT >= WNT_MIN;
  const int nq = ml.n;
  const dim3 g(ceil_div(J, ST)), b(ST), gl(ceil_div(J, 16 * (ST / WAVE)));
  // the kernels that stage one matrix per block and loop over sample tiles
  const dim3 glp((unsigned)std::min<int64_t>(gl.x, LP_BLOCKS));
  const int64_t I0 = ml.I[0];
  const int gs = first_gshift(I0);
  double *grp = w.sub + first_nsub(I0);
  const dim3 gm((unsigned)first_ngroups(I0));
  if constexpr (WIDE)
    hipLaunchKernelGGL((k_sts_mass_w<T, NT>), gm, b, 0, st,
                       static_cast<const T *>(ml.U[0]), I0, R, ml.Ggt[0], gs,
                       w.lev, w.sub, grp, err);
  else
    hipLaunchKernelGGL((k_sts_mass<T, NT>), gm, b, 0, st,
                       static_cast<const T *>(ml.U[0]), I0, R, ml.Ggt[0], gs,
                       w.lev, w.sub, grp, err);
  CPR_LAUNCH_CHECK();
  hipLaunchKernelGGL((k_sts_first<T, NT>), g, b, 0, st,
                     static_cast<const T *>(ml.U[0]), I0, R, w.lev, w.sub, grp,
                     gs, uni, nq, J, sidx, w.h, err);
  CPR_LAUNCH_CHECK();
  for (int q = 1; q < nq; ++q) {
    const double *tree = ml.tree[q], *Gg = ml.Ggt[q];
    const int64_t P2 = ml.P2[q];
    int cur = 0;
    int64_t n0 = 1;
    bool top = false;
    if constexpr (NT <= 3) {  // the packed node products fit LDS
      if (P2 >= 2 * TOP_N) {  // top stage: nodes TOP_N .. 2 TOP_N - 1
        const int ntb = (int)ceil_div(J, TOP_SPB);
        hipLaunchKernelGGL((k_sts_top<NT>), dim3(ntb), dim3(TOP_ST), 0, st,
                           tree, Gg, P2, R, uni, q, nq, J, w, w.slot[1],
                           w.tcnt, err);
        CPR_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_sts_top_place, g, b, 0, st, J, w, w.slot[1],
                           w.slot[0], w.tcnt, ntb);
        CPR_LAUNCH_CHECK();
        n0 = TOP_N;
        top = true;
      }
    }
    if (!top) {
      if constexpr (WIDE)
        hipLaunchKernelGGL((k_sts_root_w<NT>), glp, b, 0, st, tree, Gg, P2, R,
                           uni, q, nq, J, w, w.slot[0], err);
      else
        hipLaunchKernelGGL((k_sts_root<NT>), gl, b, 0, st, tree, Gg, P2, R,
                           uni, q, nq, J, w, w.slot[0], err);
      CPR_LAUNCH_CHECK();
    }
    for (int64_t n = n0; n < P2; n <<= 1) {
      if constexpr (WIDE) {
        // n nodes at this depth: with LQ_MIN slots per node on average, a
        // slot group meets about two nodes and the LDS-staged form is used
        if (n * LQ_MIN <= J) {
          const int64_t ng = (J + LQ_GROUP - 1) / LQ_GROUP;
          hipLaunchKernelGGL((k_sts_level_q<NT>),
                             dim3((unsigned)std::min<int64_t>(ng, LQ_BLOCKS)),
                             dim3(LQ_THREADS), 0, st, tree, Gg, R, J, w,
                             w.slot[cur], w.slot[cur ^ 1]);
        } else {
          hipLaunchKernelGGL((k_sts_level_w<NT>), gl, b, 0, st, tree, Gg, R,
                             J, w, w.slot[cur], w.slot[cur ^ 1]);
        }
      } else
        hipLaunchKernelGGL((k_sts_level<NT>), gl, b, 0, st, tree, Gg, R, J, w,
                           w.slot[cur], w.slot[cur ^ 1]);
      CPR_LAUNCH_CHECK();
      cur ^= 1;
    }
    const T *Uq = static_cast<const T *>(ml.U[q]);
    const int F = ml.F[q];
    if constexpr (WIDE) {
      hipLaunchKernelGGL((k_sts_leaf_w<T, NT>), gl, b, 0, st, Uq, ml.I[q], R,
                         F, P2, Gg, J, w, w.slot[cur], q, nq, sidx, err);
    } else {
      if (R % (16 / (int)sizeof(T)) == 0)
        hipLaunchKernelGGL((k_sts_leaf<T, NT, true>), gl, b, 0, st, Uq,
                           ml.I[q], R, F, P2, Gg, J, w, w.slot[cur], q, nq,
                           sidx, err);
      else
        hipLaunchKernelGGL((k_sts_leaf<T, NT, false>), gl, b, 0, st, Uq,
                           ml.I[q], R, F, P2, Gg, J, w, w.slot[cur], q, nq,
                           sidx, err);
    }
    CPR_LAUNCH_CHECK();
  }
  if constexpr (WIDE)
    hipLaunchKernelGGL((k_sts_final_w<T, NT>), glp, b, 0, st, R, J, w.h, Gp,
                       trace, prob, h);
  else
    hipLaunchKernelGGL((k_sts_final<T, NT>), gl, b, 0, st, R, J, w.h, Gp,
                       trace, prob, h);
  CPR_LAUNCH_CHECK();
}

}  // namespace

int64_t sts_top_counts(int64_t J) {
  return (J + TOP_SPB - 1) / TOP_SPB * TOP_N;
}

// leaves per block of the build: LB x P doubles in at most 48 KiB of LDS
int tree_leaf_shift(int R, int64_t P2) {
  const int64_t bytes = (int64_t)sts_packed(R) * 8;
  int lb = 0;
  while ((2 << lb) <= TB_LBMAX && (2 << lb) * bytes <= 49152 &&
         (int64_t(2) << lb) <= P2)
    ++lb;
  return lb;
}

template <typename T, bool SCALE, typename XT = double>
void tree_build(const T *U, const XT *X, const double *sigma, T *Uout,
                int64_t I, int R, int F, int64_t P2, double *tree, double *G,
                hipStream_t s) {
  const int nt = (R + 15) / 16;
  // wide ranks: one block per pair of leaves (their parents written too)
  const int lb = nt >= WNT_MIN ? (P2 >= 2 ? 1 : 0) : tree_leaf_shift(R, P2);
  const size_t lds = ((size_t)1 << lb) * sts_packed(R) * 8;
  const dim3 g((unsigned)(P2 >> lb)), b(256);
  switch (nt) {
    case 1: hipLaunchKernelGGL((k_tree_build<T, 1, SCALE, XT>), g, b, lds, s, U, X, sigma, Uout, I, R, F, P2, lb, tree, G); break;
    case 2: hipLaunchKernelGGL((k_tree_build<T, 2, SCALE, XT>), g, b, lds, s, U, X, sigma, Uout, I, R, F, P2, lb, tree, G); break;
    case 3: hipLaunchKernelGGL((k_tree_build<T, 3, SCALE, XT>), g, b, lds, s, U, X, sigma, Uout, I, R, F, P2, lb, tree, G); break;
    case 4: hipLaunchKernelGGL((k_tree_build<T, 4, SCALE, XT>), g, b, lds, s, U, X, sigma, Uout, I, R, F, P2, lb, tree, G); break;
#define CPR_TBW(NT)                                                         \
  if (lb)                                                                   \
    hipLaunchKernelGGL((k_tree_build_w<T, NT, SCALE, true, XT>), g, b, 0, s, \
                       U, X, sigma, Uout, I, R, F, P2, tree, G);            \
  else                                                                      \
    hipLaunchKernelGGL((k_tree_build_w<T, NT, SCALE, false, XT>), g, b, 0,  \
                       s, U, X, sigma, Uout, I, R, F, P2, tree, G)
    case 5: CPR_TBW(5); break;
    case 6: CPR_TBW(6); break;
    case 7: CPR_TBW(7); break;
    default: CPR_TBW(8); break;
#undef CPR_TBW
  }
  CPR_LAUNCH_CHECK();
  // subtree roots: nodes P2 >> lb .. 2 (P2 >> lb) - 1
  const int P = sts_packed(R), RP = sts_pad(R);
  for (int64_t n = P2 >> lb; n > 1;) {
    int gs = 0;  // up to four levels (TU_MAX nodes) per launch
    while ((2 << gs) <= TU_MAX && (int64_t(2) << gs) <= n) ++gs;
    const int G1 = 1 << gs;
    hipLaunchKernelGGL(k_tree_up, dim3((unsigned)(n / G1)), dim3(256), 0, s,
                       tree, n, G1, P, G, R, RP);
    CPR_LAUNCH_CHECK();
    n /= G1;
  }
}

template <typename T>
void sts_build(const T *U, int64_t I, int R, int F, int64_t P2, double *tree,
               hipStream_t s) {
  tree_build<T, false>(U, static_cast<const double *>(nullptr), nullptr,
                       nullptr, I, R, F, P2, tree, nullptr, s);
}

template <typename T>
void sts_build_scaled(const void *X, bool x32, const double *sigma, T *U,
                      int64_t I, int R, int F, int64_t P2, double *tree,
                      double *G, hipStream_t s) {
  double *Gr = P2 >= 2 ? G : nullptr;
  if constexpr (std::is_same<T, float>::value) {
    if (x32) {
      tree_build<T, true, float>(nullptr, static_cast<const float *>(X), sigma,
                                 U, I, R, F, P2, tree, Gr, s);
      return;
    }
  }
  tree_build<T, true, double>(nullptr, static_cast<const double *>(X), sigma,
                              U, I, R, F, P2, tree, Gr, s);
}
template void sts_build_scaled<float>(const void *, bool, const double *,
                                      float *, int64_t, int, int, int64_t,
                                      double *, double *, hipStream_t);
template void sts_build_scaled<double>(const void *, bool, const double *,
                                       double *, int64_t, int, int, int64_t,
                                       double *, double *, hipStream_t);
template void sts_build<float>(const float *, int64_t, int, int, int64_t,
                               double *, hipStream_t);
template void sts_build<double>(const double *, int64_t, int, int, int64_t,
                                double *, hipStream_t);

template <typename T>
void sts_draw(const ModeList &ml, int64_t J, int R, const double *uni,
              const double *Gp, const double *trace, int32_t *sidx,
              double *prob, T *h, const StsWork &w, uint32_t *err,
              hipStream_t s) {
  switch ((R + 15) / 16) {
    case 1: draw_nt<T, 1>(ml, J, R, uni, Gp, trace, sidx, prob, h, w, err, s); break;
    case 2: draw_nt<T, 2>(ml, J, R, uni, Gp, trace, sidx, prob, h, w, err, s); break;
    case 3: draw_nt<T, 3>(ml, J, R, uni, Gp, trace, sidx, prob, h, w, err, s); break;
    case 4: draw_nt<T, 4>(ml, J, R, uni, Gp, trace, sidx, prob, h, w, err, s); break;
    case 5: draw_nt<T, 5>(ml, J, R, uni, Gp, trace, sidx, prob, h, w, err, s); break;
    case 6: draw_nt<T, 6>(ml, J, R, uni, Gp, trace, sidx, prob, h, w, err, s); break;
    case 7: draw_nt<T, 7>(ml, J, R, uni, Gp, trace, sidx, prob, h, w, err, s); break;
    default: draw_nt<T, 8>(ml, J, R, uni, Gp, trace, sidx, prob, h, w, err, s); break;
  }
}
template void sts_draw<float>(const ModeList &, int64_t, int,
                              const double *, const double *, const double *,
                              int32_t *, double *, float *, const StsWork &,
                              uint32_t *, hipStream_t);
template void sts_draw<double>(const ModeList &, int64_t, int,
                               const double *, const double *, const double *,
                               int32_t *, double *, double *,
                               const StsWork &, uint32_t *, hipStream_t);

}  // namespace cpr
