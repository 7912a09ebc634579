// Sketch application and the sampled MTTKRP (Section 2.2, Eq. 7, Section 4.3).
//
// 1. lookup: column key of each drawn Khatri-Rao row, probed in the mode's
//    open-addressing hash of its distinct column keys; per block, the draws
//    of one column are pre-merged in an LDS hash (smallest draw index) and
//    the block's first draw of each column is published with one atomicMin.
// 2. merge: draws of the same column are merged (count c, weight
//    w = c / (J p)); distinct columns u are compacted in first-draw order,
//    the lengths of their nonzero ranges are prefix-summed, and
//    hc[u] = w h[first draw] holds the column's weighted Khatri-Rao row.
// 3. MTTKRP by blocks of B output rows (the paper's transposition of the
//    extracted nonzeros to row order, Section 4.3, as one counting-sort
//    pass): each block's records sit in a fixed region (sized once from the
//    mode's row histogram); the scatter places compact records
//    (u, row % B, v) in their block's region, one atomic per run of one
//    block in a wave (positions of one column are row-sorted), then each
//    block's records are accumulated into its B rows of M.  Record order
//    inside a region follows the atomics, so FP32 sums are not bitwise
//    reproducible run to run (their order of addition varies).
#include "internal.h"

#include <algorithm>
#include <climits>

namespace cpr {
namespace {

constexpr int LK_THREADS = 256;
constexpr int BK_TILE = 4096;  // positions per scatter tile

template <typename T>
__global__ void k_sample_rows(ModeList ml, int64_t J, int R,
                              const int32_t *sidx, const double *prob, T *h,
                              uint32_t *err) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= J * R) return;
  const int64_t s = e / R;
  const int r = (int)(e - s * R);
  if (r == 0) {  // a draw's weight is count / (J p): p must be finite, > 0
    const double p = prob[s];
    if (!(p > 0.0 && p <= 1.7976931348623157e308)) atomicOr(err, ERR_PROB);
  }
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

// Column of each draw: its key, probed in the mode's hash table from the
// key's home entry (a column id per entry, its key read from col_key) until
// the key or an empty entry.  The first draw of a column claims it with atomicMin on its owner
// word, once per block and column: the block's draws of a column meet in an
// LDS table first (a heavily drawn column would otherwise take one global
// atomic per draw, all on one address).
constexpr int LK_HASH = 2 * LK_THREADS;

__global__ void __launch_bounds__(LK_THREADS)
k_lookup(ModeList ml, int64_t J, const int32_t *sidx, const uint32_t *tab,
         const uint64_t *col_key, int hbits, int32_t *col_id,
         int32_t *owner) {
  __shared__ int32_t hk[LK_HASH], hm[LK_HASH];
  for (int e = threadIdx.x; e < LK_HASH; e += LK_THREADS) {
    hk[e] = -1;
    hm[e] = INT32_MAX;
  }
  const int64_t s = (int64_t)blockIdx.x * LK_THREADS + threadIdx.x;
  int32_t cid = -1;
  if (s < J) {
    uint64_t key = 0;
    bool ok = true;
    for (int q = 0; q < ml.n; ++q) {
      int32_t i = sidx[s * ml.n + q];
      ok &= (i >= 0 && i < ml.I[q]);
      key += (uint64_t)i * ml.stride[q];
    }
    if (ok) {
      const uint64_t mask = (1ull << hbits) - 1;
      uint64_t p = col_hash(key, hbits);
      for (uint64_t n = 0; n <= mask; ++n) {
        const uint32_t c = tab[p];
        if (c == ~0u) break;
        if (col_key[c] == key) {
          cid = (int32_t)c;
          break;
        }
        p = (p + 1) & mask;
      }
    }
    col_id[s] = cid;
  }
  __syncthreads();
  if (cid >= 0) {  // at most LK_THREADS keys in 2 LK_THREADS entries
    uint32_t e = ((uint32_t)cid * 2654435761u) % LK_HASH;
    for (int probe = 0; probe < LK_HASH; ++probe) {
      const int32_t prev = atomicCAS(&hk[e], -1, cid);
      if (prev == -1 || prev == cid) {
        atomicMin(&hm[e], (int32_t)s);
        break;
      }
      e = (e + 1) % LK_HASH;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < LK_HASH; e += LK_THREADS) {
    const int32_t c = hk[e];
    if (c >= 0 && owner[c] > hm[e]) atomicMin(&owner[c], hm[e]);
  }
}

// Merge in two launches.  Block b owns the contiguous draws
// [b chunk, (b + 1) chunk), taken in passes of LK_THREADS.
//   k_dup_first: extra draws per first draw, aggregated per pass in an LDS
//     hash table (one global atomic per distinct first draw and pass); the
//     first-draw flag and nonzero-range length of every draw, and the
//     block's totals of both.
//   k_compact: the block's offsets (sum of the earlier blocks' totals), a
//     block scan per pass, and the compaction of the first draws in draw
//     order (weight count / (J p)); restores owner and dupcnt for the next
//     call (owner is not read after k_dup_first).
constexpr int DUP_HASH = 2 * LK_THREADS;
constexpr int MG_MAXBLK = 1024;

__device__ __forceinline__ int64_t wave_incl_scan_i64(int64_t x) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int64_t y = __shfl_up(x, o, WAVE);
    if (l >= o) x += y;
  }
  return x;
}

// Block-wide exclusive scan of (a, b) per thread; totals through ta, tb.
__device__ __forceinline__ void block_excl_scan2(int64_t &a, int64_t &b,
                                                 int64_t &ta, int64_t &tb) {
  __shared__ int64_t wa[LK_THREADS / WAVE], wb[LK_THREADS / WAVE];
  const int w = threadIdx.x / WAVE, l = lane_id();
  const int64_t ia = wave_incl_scan_i64(a), ib = wave_incl_scan_i64(b);
  if (l == WAVE - 1) {
    wa[w] = ia;
    wb[w] = ib;
  }
  __syncthreads();
  int64_t oa = 0, ob = 0;
  ta = 0;
  tb = 0;
#pragma unroll
  for (int i = 0; i < LK_THREADS / WAVE; ++i) {
    if (i < w) {
      oa += wa[i];
      ob += wb[i];
    }
    ta += wa[i];
    tb += wb[i];
  }
  __syncthreads();
  a = oa + ia - a;
  b = ob + ib - b;
}

__global__ void __launch_bounds__(LK_THREADS)
k_dup_first(int64_t J, int64_t chunk, const int32_t *col_id,
            const int32_t *owner, const int64_t *col_ptr, int32_t *dupcnt,
            int64_t *first, int64_t *len, int64_t *part) {
  __shared__ int32_t hkey[DUP_HASH], hcnt[DUP_HASH];
  const int64_t c0 = (int64_t)blockIdx.x * chunk;
  const int64_t c1 = c0 + chunk < J ? c0 + chunk : J;
  int64_t nf = 0, nl = 0;
  for (int64_t p0 = c0; p0 < c1; p0 += LK_THREADS) {
    for (int e = threadIdx.x; e < DUP_HASH; e += LK_THREADS) {
      hkey[e] = -1;
      hcnt[e] = 0;
    }
    __syncthreads();
    const int64_t s = p0 + threadIdx.x;
    if (s < c1) {
      const int32_t cid = col_id[s];
      const int32_t o = cid >= 0 ? owner[cid] : (int32_t)s;
      const bool f = cid >= 0 && o == (int32_t)s;
      const int64_t ln = f ? col_ptr[cid + 1] - col_ptr[cid] : 0;
      first[s] = f ? 1 : 0;
      len[s] = ln;
      nf += f ? 1 : 0;
      nl += ln;
      if (o != (int32_t)s) {  // at most LK_THREADS keys: a slot is found
        uint32_t hsh = ((uint32_t)o * 2654435761u) % DUP_HASH;
        for (int probe = 0; probe < DUP_HASH; ++probe) {
          const int32_t prev = atomicCAS(&hkey[hsh], -1, o);
          if (prev == -1 || prev == o) {
            atomicAdd(&hcnt[hsh], 1);
            break;
          }
          hsh = (hsh + 1) % DUP_HASH;
        }
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < DUP_HASH; e += LK_THREADS)
      if (hkey[e] >= 0) atomicAdd(&dupcnt[hkey[e]], hcnt[e]);
    __syncthreads();
  }
  int64_t ta, tb;
  block_excl_scan2(nf, nl, ta, tb);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = ta;
    part[2 * blockIdx.x + 1] = tb;
  }
}

template <typename T>
__global__ void __launch_bounds__(LK_THREADS)
k_compact(int64_t J, int64_t chunk, const double *prob, const int32_t *col_id,
          const int64_t *first, const int64_t *len, const int64_t *part,
          const int64_t *col_ptr, const T *h, int R, int32_t *owner,
          int32_t *dupcnt, int32_t *uq_s, int32_t *uq_cid, int32_t *uq_cnt,
          double *uq_w, int64_t *uq_off, int64_t *uq_base, T *hc,
          int64_t *tile_first, int64_t *counts, int64_t *stats) {
  // offsets of this block: totals of the blocks before it
  int64_t bu = 0, bo = 0;
  for (int k = threadIdx.x; k < (int)blockIdx.x; k += LK_THREADS) {
    bu += part[2 * k];
    bo += part[2 * k + 1];
  }
  {
    int64_t ta, tb;
    block_excl_scan2(bu, bo, ta, tb);
    bu = ta;
    bo = tb;
  }
  const int64_t c0 = (int64_t)blockIdx.x * chunk;
  const int64_t c1 = c0 + chunk < J ? c0 + chunk : J;
  for (int64_t p0 = c0; p0 < c1; p0 += LK_THREADS) {
    const int64_t s = p0 + threadIdx.x;
    const bool in = s < c1;
    const int64_t f = in ? first[s] : 0, ln = in ? len[s] : 0;
    int64_t u = f, off = ln, ta, tb;
    block_excl_scan2(u, off, ta, tb);
    u += bu;
    off += bo;
    if (f) {
      const int32_t cid = col_id[s];
      const int32_t cnt = 1 + dupcnt[s];
      const double wu = (double)cnt / ((double)J * prob[s]);
      uq_s[u] = (int32_t)s;
      uq_cid[u] = cid;
      uq_cnt[u] = cnt;
      uq_w[u] = wu;
      uq_off[u] = off;
      uq_base[u] = col_ptr[cid] - off;  // index position = uq_base + e
      owner[cid] = INT_MAX;
      // tile_first[t] = the distinct column holding extracted position
      // t BK_TILE
      for (int64_t tt = (off + BK_TILE - 1) / BK_TILE; tt * BK_TILE < off + ln;
           ++tt)
        tile_first[tt] = u;
      const T *hs = h + s * R;
      T *hu = hc + u * R;
      for (int c0 = 0; c0 < R; c0 += 16) {  // 16 loads in flight
        T x[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) x[j] = hs[c0 + j < R ? c0 + j : R - 1];
#pragma unroll
        for (int j = 0; j < 16; ++j)
          if (c0 + j < R) hu[c0 + j] = (T)(wu * (double)x[j]);
      }
    }
    if (in) dupcnt[s] = 0;
    if (s == J - 1) {
      const int64_t nu = u + f, nz = off + ln;
      uq_off[nu] = nz;
      counts[0] = nu;
      counts[1] = nz;
      if (stats) {  // cumulative: mode solves, distinct columns, nonzeros
        stats[0] += 1;
        stats[1] += nu;
        stats[2] += nz;
      }
    }
    bu += ta;
    bo += tb;
  }
}

// Sampled MTTKRP, output-row-block form (the paper's transposition of the
// extracted nonzeros to row order, Section 4.3, done as one counting-sort
// pass by blocks of B output rows):
//   count   : bucket (= row / B) histogram of the extracted nonzeros;
//   scatter : compact records (u, row % B, v) grouped by bucket;
//   accum   : one workgroup per (bucket, slice of <= BK_SLICE records)
//             adds v hc[u] into the bucket's B rows (sorted by row in LDS,
//             runs summed in registers), then writes the rows once: to M
//             when the bucket is one slice, else to a per-slice block that
//             k_bk_combine adds in slice order.
// Extracted nonzeros are never materialised: position e of the
// concatenated sampled-column ranges is resolved to (distinct column,
// position in the mode's index) by a binary search over uq_off.
constexpr int MT_THREADS = 256;
constexpr int BK_ITEMS = BK_TILE / MT_THREADS;
constexpr int BK_LDS_MAX = 4096;  // buckets histogrammed in LDS
constexpr int BK_SLICE = 4096;    // records per accumulation workgroup

// The distinct columns overlapping tile [e0, e1): [ub, ue).  Their start
// positions relative to e0 go to LDS (cst); a position's column is then a
// binary search in LDS.
__device__ __forceinline__ void tile_columns(const int64_t *counts,
                                             const int64_t *uq_off,
                                             const int64_t *tile_first,
                                             int64_t tile, int64_t ntile,
                                             int64_t e0, int32_t *cst,
                                             int64_t &ub, int &ncol) {
  const int64_t nu = counts[0];
  ub = tile_first[tile];
  const int64_t ue = tile + 1 < ntile ? tile_first[tile + 1] + 1 : nu;
  ncol = (int)(ue - ub);
  for (int k = threadIdx.x; k < ncol; k += MT_THREADS)
    cst[k] = (int32_t)(uq_off[ub + k] - e0);  // cst[0] <= 0
}

__device__ __forceinline__ int find_local(const int32_t *cst, int ncol,
                                          int pos) {
  int lo = 0, hi = ncol;  // last k with cst[k] <= pos
  while (hi - lo > 1) {
    const int m = (lo + hi) >> 1;
    if (cst[m] <= pos) lo = m; else hi = m;
  }
  return lo;
}

// Runs of equal bucket among the valid lanes of a wave (valid lanes are a
// prefix, holding consecutive positions): the run's first lane and, for
// that lane, the run length.
__device__ __forceinline__ void bucket_runs(int bk, bool valid, int &leader,
                                            int &len) {
  const int l = lane_id();
  const int prev = __shfl_up(bk, 1, WAVE);
  const uint64_t sm = __ballot(valid && (l == 0 || bk != prev));
  const uint64_t vm = __ballot(valid);
  const uint64_t upto = sm & ((2ull << l) - 1);  // starts at or below l
  leader = upto ? 63 - __clzll((long long)upto) : l;
  const uint64_t above = sm & ~((2ull << l) - 1);
  const int nxt = above ? __ffsll((long long)above) - 1
                        : (vm ? 64 - __clzll((long long)vm) : 0);
  len = nxt - l;
}

// Accumulation plan: bucket b's records occupy [bk_start[b], bk_start[b] +
// bk_fill[b]) of its fixed region; bk_end is that end, item_start the
// exclusive prefix sums of the slices per bucket (nbk + 1 entries) and
// item_bk[i] the bucket of slice i; split lists the buckets of more than
// one slice (nsplit of them), for k_bk_combine.  Every bucket gets at least
// one slice (an empty one writes zero rows), so the accumulation writes
// every row of M.  Two launches over blocks of PL_THREADS consecutive
// buckets (coalesced): per-block totals, then offsets (the sum of the
// earlier blocks' totals) and the block's scans.
constexpr int PL_THREADS = 1024;

__device__ __forceinline__ int64_t plan_slices(const int64_t *bk_fill, int nbk,
                                               int64_t b) {
  if (b >= nbk) return 0;
  const int64_t n = bk_fill[b];
  return n > BK_SLICE ? (n + BK_SLICE - 1) / BK_SLICE : 1;
}

// block-wide exclusive scan of (a, c) per thread, totals in ta, tc
__device__ __forceinline__ void plan_scan2(int64_t &a, int64_t &c, int64_t &ta,
                                           int64_t &tc) {
  __shared__ int64_t wa[PL_THREADS / WAVE], wc[PL_THREADS / WAVE];
  const int l = lane_id(), w = threadIdx.x / WAVE;
  int64_t ia = a, ic = c;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int64_t ya = __shfl_up(ia, o, WAVE), yc = __shfl_up(ic, o, WAVE);
    if (l >= o) {
      ia += ya;
      ic += yc;
    }
  }
  if (l == WAVE - 1) {
    wa[w] = ia;
    wc[w] = ic;
  }
  __syncthreads();
  int64_t oa = 0, oc = 0;
  ta = tc = 0;
  for (int i = 0; i < PL_THREADS / WAVE; ++i) {
    if (i < w) {
      oa += wa[i];
      oc += wc[i];
    }
    ta += wa[i];
    tc += wc[i];
  }
  a = oa + ia - a;
  c = oc + ic - c;
  __syncthreads();
}

__global__ void __launch_bounds__(PL_THREADS)
k_bk_plan_count(const int64_t *bk_fill, int nbk, int64_t *btot) {
  const int64_t b = (int64_t)blockIdx.x * PL_THREADS + threadIdx.x;
  int64_t sl = plan_slices(bk_fill, nbk, b);
  int64_t sp = sl > 1 ? 1 : 0;
  int64_t ts, tp;
  plan_scan2(sl, sp, ts, tp);
  if (threadIdx.x == 0) {
    btot[2 * blockIdx.x] = ts;
    btot[2 * blockIdx.x + 1] = tp;
  }
}

__global__ void __launch_bounds__(PL_THREADS)
k_bk_plan(const int64_t *bk_start, int64_t *bk_fill, int nbk,
          const int64_t *btot, int64_t *bk_end, int64_t *item_start,
          int32_t *item_bk, int64_t *split, int64_t *nsplit) {
  __shared__ int64_t red[2][PL_THREADS / WAVE];
  const int t = threadIdx.x, l = lane_id(), w = t / WAVE;
  // offsets of this block: the earlier blocks' totals
  int64_t os = 0, op = 0;
  for (int i = t; i < (int)blockIdx.x; i += PL_THREADS) {
    os += btot[2 * i];
    op += btot[2 * i + 1];
  }
#pragma unroll
  for (int o = WAVE / 2; o >= 1; o >>= 1) {
    os += __shfl_xor(os, o, WAVE);
    op += __shfl_xor(op, o, WAVE);
  }
  if (l == 0) {
    red[0][w] = os;
    red[1][w] = op;
  }
  __syncthreads();
  os = op = 0;
  for (int i = 0; i < PL_THREADS / WAVE; ++i) {
    os += red[0][i];
    op += red[1][i];
  }
  const int64_t b = (int64_t)blockIdx.x * PL_THREADS + t;
  const int64_t fill = b < nbk ? bk_fill[b] : 0;
  const int64_t ni = plan_slices(bk_fill, nbk, b);
  int64_t es = ni, ep = ni > 1 ? 1 : 0;
  int64_t ts, tp;
  plan_scan2(es, ep, ts, tp);
  if (b < nbk) {
    bk_end[b] = bk_start[b] + fill;
    bk_fill[b] = 0;  // read: clear it for the next call
  }
  if (b <= nbk) item_start[b] = os + es;
  for (int64_t i = 0; i < ni; ++i) item_bk[os + es + i] = (int32_t)b;
  if (ni > 1) split[op + ep] = b;
  if (blockIdx.x == gridDim.x - 1 && t == 0) *nsplit = op + tp;
}

// Fixed record regions of the output-row buckets of one mode (built once):
// the bucket's nonzeros in the whole mode bound the nonzeros any solve can
// extract into it (extracted positions are distinct).  starts = exclusive
// prefix sums of the row-bucket histogram (nbk + 1 entries).
//
// Power-law rows put a large share of the nonzeros in a few buckets, and
// global atomics on one address serialise; so each workgroup counts one
// window of BH_WIN buckets in LDS over one chunk of the nonzeros (grid.x =
// chunks, grid.y = windows) and flushes its window with one atomic per
// bucket.  Every window re-reads the row array: (nbk / BH_WIN) passes.
constexpr int BH_THREADS = 1024;
constexpr int BH_WIN = 32768;  // 128 KiB of u32 counters
__global__ void __launch_bounds__(BH_THREADS)
k_bucket_hist(const int32_t *row, int64_t nnz, int nbk, int bb, int64_t *cnt) {
  extern __shared__ uint32_t bh[];
  const int b0 = blockIdx.y * BH_WIN;
  const int nw = nbk - b0 < BH_WIN ? nbk - b0 : BH_WIN;
  for (int b = threadIdx.x; b < nw; b += BH_THREADS) bh[b] = 0;
  __syncthreads();
  // chunk of whole int4 groups (the row array is 16-byte aligned)
  const int64_t nq = nnz >> 2;
  const int64_t per = (nq + gridDim.x - 1) / gridDim.x;
  const int64_t q0 = (int64_t)blockIdx.x * per;
  const int64_t q1 = q0 + per < nq ? q0 + per : nq;
  const int4 *row4 = reinterpret_cast<const int4 *>(row);
  for (int64_t q = q0 + threadIdx.x; q < q1; q += BH_THREADS) {
    const int4 r = row4[q];
    const unsigned a = (unsigned)((r.x >> bb) - b0), b = (unsigned)((r.y >> bb) - b0),
                   c = (unsigned)((r.z >> bb) - b0), d = (unsigned)((r.w >> bb) - b0);
    if (a < (unsigned)nw) atomicAdd(&bh[a], 1u);
    if (b < (unsigned)nw) atomicAdd(&bh[b], 1u);
    if (c < (unsigned)nw) atomicAdd(&bh[c], 1u);
    if (d < (unsigned)nw) atomicAdd(&bh[d], 1u);
  }
  if (blockIdx.x == 0)  // the last nnz % 4 nonzeros
    for (int64_t e = (nq << 2) + threadIdx.x; e < nnz; e += BH_THREADS) {
      const unsigned a = (unsigned)((row[e] >> bb) - b0);
      if (a < (unsigned)nw) atomicAdd(&bh[a], 1u);
    }
  __syncthreads();
  for (int b = threadIdx.x; b < nw; b += BH_THREADS)
    if (bh[b])
      atomicAdd((unsigned long long *)&cnt[b0 + b], (unsigned long long)bh[b]);
}

// One extracted nonzero in bucket order: key = (distinct column u << 8) |
// row % B, coef = its value (the column's weight is folded into hc[u]).
template <typename T>
struct BkRec {
  uint32_t key;
  T coef;
};

// The same nonzero in the first of two placement passes (grouped by super
// bucket: 2^sh consecutive buckets), with its whole row.
template <typename T>
struct BkRec1 {
  uint32_t u;
  int32_t row;
  T coef;
};

// SUPER: the first of two placement passes.  Groups are then super buckets
// (nbk of them, <= SB_MAX: 2^sh buckets each, so that a 4096-position tile
// puts runs of about 16 records in each group it touches), whose regions
// are the unions of their buckets' regions; records are BkRec1.
template <typename T, bool SUPER>
__global__ void __launch_bounds__(MT_THREADS)
k_bk_scatter(const int64_t *counts, const int64_t *uq_off,
             const int64_t *tile_first,
             const int64_t *uq_base, const int32_t *row, const T *val, int nbk,
             int bb, int sh, const int64_t *bk_start, int64_t *bk_fill,
             void *rec_out) {
  extern __shared__ int64_t sc_lds[];  // base, cnt: nbk each (<= BK_LDS_MAX)
  int64_t *base = sc_lds;  // record position of the tile's first record
  uint32_t *cnt = reinterpret_cast<uint32_t *>(sc_lds + nbk);
  __shared__ int32_t cst[BK_TILE + 1];
  const int64_t nz = counts[1];
  const bool use_lds = SUPER || nbk <= BK_LDS_MAX;
  const int gshift = SUPER ? bb + sh : bb;  // row -> group
  const int64_t ntile = (nz + BK_TILE - 1) / BK_TILE;
  const uint32_t bmask = (1u << bb) - 1;
  const int l = lane_id();
  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int64_t e0 = tile * BK_TILE;
    const int64_t e1 = e0 + BK_TILE < nz ? e0 + BK_TILE : nz;
    if (use_lds)
      for (int b = threadIdx.x; b < nbk; b += MT_THREADS) cnt[b] = 0;
    int64_t ub;
    int ncol;
    tile_columns(counts, uq_off, tile_first, tile, ntile, e0, cst, ub, ncol);
    __syncthreads();
    int64_t p[BK_ITEMS];
    int my_bk[BK_ITEMS];
    uint32_t my_u[BK_ITEMS];
    int32_t my_rw[BK_ITEMS];
    T my_cf[BK_ITEMS];
#pragma unroll
    for (int i = 0; i < BK_ITEMS; ++i) {
      const int pos = i * MT_THREADS + threadIdx.x;
      const int64_t e = e0 + pos < e1 ? e0 + pos : e1 - 1;
      const int64_t u = ub + find_local(cst, ncol, (int)(e - e0));
      my_u[i] = (uint32_t)u;
      p[i] = uq_base[u] + e;
    }
#pragma unroll
    for (int i = 0; i < BK_ITEMS; ++i) {
      my_rw[i] = row[p[i]];
      my_cf[i] = val[p[i]];
      my_bk[i] = my_rw[i] >> gshift;
    }
#pragma unroll
    for (int i = 0; i < BK_ITEMS; ++i) {
      const bool valid = e0 + i * MT_THREADS + threadIdx.x < e1;
      if (!valid) my_bk[i] = -1;
      int lead, len;
      bucket_runs(my_bk[i], valid, lead, len);
      if (use_lds && valid && lead == l)
        atomicAdd(&cnt[my_bk[i]], (uint32_t)len);
    }
    __syncthreads();
    if (use_lds)
      for (int b = threadIdx.x; b < nbk; b += MT_THREADS) {
        const uint32_t c = cnt[b];
        if (c)
          base[b] = bk_start[SUPER ? (int64_t)b << sh : b] +
                    (int64_t)atomicAdd((unsigned long long *)&bk_fill[b],
                                       (unsigned long long)c);
        cnt[b] = 0;
      }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < BK_ITEMS; ++i) {
      const int bk = my_bk[i];
      // the run's first lane reserves the run's slots; members follow it
      int lead, len;
      bucket_runs(bk, bk >= 0, lead, len);
      int64_t off = 0;
      if (bk >= 0 && lead == l)
        off = use_lds ? base[bk] + (int64_t)atomicAdd(&cnt[bk], (uint32_t)len)
                      : bk_start[bk] + (int64_t)atomicAdd(
                            (unsigned long long *)&bk_fill[bk],
                            (unsigned long long)len);
      off = __shfl(off, lead, WAVE);
      if (bk >= 0) {
        if constexpr (SUPER)
          static_cast<BkRec1<T> *>(rec_out)[off + (l - lead)] =
              BkRec1<T>{my_u[i], my_rw[i], my_cf[i]};
        else
          static_cast<BkRec<T> *>(rec_out)[off + (l - lead)] = BkRec<T>{
              (my_u[i] << 8) | ((uint32_t)my_rw[i] & bmask), my_cf[i]};
      }
    }
    __syncthreads();
  }
}

// Second placement pass: the records of each super bucket, in chunks of
// DS_CHUNK, counted per bucket in LDS; one global atomic per (chunk,
// bucket) reserves the chunk's run in the bucket's region, so runs of about
// DS_CHUNK / 2^sh records are written together.  k_ds_plan first lists the
// chunks (ds_start: exclusive prefix sums of the chunks per super bucket),
// takes the fill counts of pass 1 (ds_fill) and clears them for the next
// call.
constexpr int SB_MAX = 256;      // super buckets at most
constexpr int DS_THREADS = 512;
constexpr int DS_ITEMS = 16;
constexpr int DS_CHUNK = DS_THREADS * DS_ITEMS;
constexpr int DS_LDS_MAX = 4096;  // buckets per super bucket at most

__global__ void __launch_bounds__(SB_MAX)
k_ds_plan(int64_t *sfill, int nsb, int64_t *ds_fill, int64_t *ds_start) {
  __shared__ int64_t wsum[SB_MAX / WAVE];
  const int t = threadIdx.x, l = lane_id(), w = t / WAVE;
  const int64_t f = t < nsb ? sfill[t] : 0;
  const int64_t n = (f + DS_CHUNK - 1) / DS_CHUNK;
  int64_t inc = n;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    const int64_t y = __shfl_up(inc, o, WAVE);
    if (l >= o) inc += y;
  }
  if (l == WAVE - 1) wsum[w] = inc;
  __syncthreads();
  int64_t off = 0;
  for (int i = 0; i < w; ++i) off += wsum[i];
  if (t < nsb) {
    ds_fill[t] = f;
    ds_start[t] = off + inc - n;
    sfill[t] = 0;
  }
  if (t == SB_MAX - 1) ds_start[nsb] = off + inc;
}

template <typename T>
__global__ void __launch_bounds__(DS_THREADS)
k_bk_distribute(const int64_t *ds_start, const int64_t *ds_fill, int nsb,
                int sh, int nbk, int bb, const int64_t *bk_start,
                int64_t *bk_fill, const BkRec1<T> *rec1, BkRec<T> *rec) {
  __shared__ int64_t base[DS_LDS_MAX];
  __shared__ uint32_t cnt[DS_LDS_MAX];
  const int l = lane_id();
  const uint32_t bmask = (1u << bb) - 1;
  const int64_t nitems = ds_start[nsb];
  for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    int lo = 0, hi = nsb;  // last super bucket with ds_start <= it
    while (hi - lo > 1) {
      const int m = (lo + hi) >> 1;
      if (ds_start[m] <= it) lo = m; else hi = m;
    }
    const int sb = lo;
    const int64_t b0 = (int64_t)sb << sh;
    const int nb = (int)(nbk - b0 < (1 << sh) ? nbk - b0 : (1 << sh));
    const int64_t reg = bk_start[b0];
    const int64_t r0 = reg + (it - ds_start[sb]) * DS_CHUNK;
    const int64_t r1 = r0 + DS_CHUNK < reg + ds_fill[sb] ? r0 + DS_CHUNK
                                                          : reg + ds_fill[sb];
    for (int b = threadIdx.x; b < nb; b += DS_THREADS) cnt[b] = 0;
    __syncthreads();
    BkRec1<T> my[DS_ITEMS];
    int lb[DS_ITEMS];
#pragma unroll
    for (int i = 0; i < DS_ITEMS; ++i) {
      const int64_t r = r0 + i * DS_THREADS + threadIdx.x;
      my[i] = rec1[r < r1 ? r : r1 - 1];
    }
#pragma unroll
    for (int i = 0; i < DS_ITEMS; ++i) {
      const bool valid = r0 + i * DS_THREADS + threadIdx.x < r1;
      lb[i] = valid ? (int)((my[i].row >> bb) - b0) : -1;
      int lead, len;
      bucket_runs(lb[i], valid, lead, len);
      if (valid && lead == l) atomicAdd(&cnt[lb[i]], (uint32_t)len);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += DS_THREADS) {
      const uint32_t c = cnt[b];
      if (c)
        base[b] = bk_start[b0 + b] +
                  (int64_t)atomicAdd((unsigned long long *)&bk_fill[b0 + b],
                                     (unsigned long long)c);
      cnt[b] = 0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < DS_ITEMS; ++i) {
      int lead, len;
      bucket_runs(lb[i], lb[i] >= 0, lead, len);
      int64_t off = 0;
      if (lb[i] >= 0 && lead == l)
        off = base[lb[i]] + (int64_t)atomicAdd(&cnt[lb[i]], (uint32_t)len);
      off = __shfl(off, lead, WAVE);
      if (lb[i] >= 0)
        rec[off + (l - lead)] = BkRec<T>{
            (my[i].u << 8) | ((uint32_t)my[i].row & bmask), my[i].coef};
    }
    __syncthreads();
  }
}

// Super-bucket shift of a mode with nbk buckets for the two-pass placement
// (-1: one pass).  One pass when the buckets are few enough that a tile's
// runs are already long, or too many for one super bucket's LDS counts.
int super_shift(int64_t nbk) {
  if (nbk <= SB_MAX) return -1;
  int sh = 0;
  while (((nbk + (int64_t(1) << sh) - 1) >> sh) > SB_MAX) ++sh;
  return (1 << sh) <= DS_LDS_MAX ? sh : -1;
}

// Accumulation without floating-point LDS atomics (they run at a small
// fraction of LDS speed): the slice's records (read once into registers)
// are counting-sorted by row of the bucket in LDS with integer atomics;
// each group of L lanes, VW consecutive columns per lane, then walks a
// contiguous chunk of the sorted records, 16 records (and their h rows) in
// flight at a time, accumulating runs of one row in registers.  A row inside
// the chunk belongs to the group alone and is stored; only rows cut by a
// chunk boundary are added with atomics.
constexpr int AC_ITEMS = BK_SLICE / MT_THREADS;  // records per thread
constexpr int AC_BATCH = 6;  // records per batch (two batches in flight)

// VW consecutive columns of an h row as one 16-byte load (R a multiple of
// VW; rows are then 16-byte aligned) or VW clamped loads
template <typename T, int VW, bool VEC>
__device__ __forceinline__ void load_cols(const T *hr, int cb, int R,
                                          T (&out)[VW]) {
  if constexpr (VEC) {
    const int c = cb <= R - VW ? cb : R - VW;
    typedef T vec_t __attribute__((ext_vector_type(VW)));
    const vec_t v = *reinterpret_cast<const vec_t *>(hr + c);
#pragma unroll
    for (int q = 0; q < VW; ++q) out[q] = v[q];
  } else {
#pragma unroll
    for (int q = 0; q < VW; ++q) out[q] = hr[cb + q < R ? cb + q : R - 1];
  }
}

template <typename T, int L, int VW, bool VEC>
__global__ void __launch_bounds__(MT_THREADS)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 2)))
k_bk_accum(const int64_t *item_start, const int32_t *item_bk,
           const int64_t *bk_start, const int64_t *bk_end, int nbk, int bb,
           const BkRec<T> *rec,
           const T *hc, int R, int64_t I, T *M, T *part) {
  constexpr int G = MT_THREADS / L;  // lane groups per block
  extern __shared__ unsigned char bk_lds_raw[];
  const int B = 1 << bb;
  T *lc = reinterpret_cast<T *>(bk_lds_raw);                   // coefs
  uint32_t *lk = reinterpret_cast<uint32_t *>(lc + BK_SLICE);  // keys
  // partial sums of the runs cut by chunk boundaries: [group][first, last]
  T *pr = reinterpret_cast<T *>(lk + BK_SLICE);
  __shared__ int32_t cnt[256 + 1];
  __shared__ int32_t wsum[MT_THREADS / WAVE];
  __shared__ int32_t s_fa[G], s_fb[G];
  const int t = threadIdx.x, l = lane_id();
  const int gl = t % L, g = t / L;
  const int cb = gl * VW;
  const int64_t nitems = item_start[nbk];
  for (int64_t item = blockIdx.x; item < nitems; item += gridDim.x) {
    const int bk = item_bk[item];
    const int64_t k = item - item_start[bk];
    const int64_t r0 = bk_start[bk] + k * BK_SLICE;
    const int64_t r1 = r0 + BK_SLICE < bk_end[bk] ? r0 + BK_SLICE : bk_end[bk];
    const int n = (int)(r1 - r0);
    const bool single = item_start[bk + 1] - item_start[bk] == 1;
    const int64_t row0 = (int64_t)bk * B;
    const int nrows = (int)(I - row0 < B ? I - row0 : B);
    // a bucket held by one slice goes straight to M; the slices of a split
    // bucket write their block to their own scratch slot for k_bk_combine
    T *mo = single ? M + row0 * R : part + item * (int64_t)B * R;
    // this thread's records: positions t, t + 256, ...
    BkRec<T> my[AC_ITEMS];
    if (n > 0) {
#pragma unroll
      for (int i = 0; i < AC_ITEMS; ++i) {
        const int e = i * MT_THREADS + t;
        my[i] = rec[r0 + (e < n ? e : n - 1)];
      }
    }
    for (int e = t; e <= 256; e += MT_THREADS) cnt[e] = 0;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < AC_ITEMS; ++i)
      if (i * MT_THREADS + t < n) atomicAdd(&cnt[my[i].key & 255u], 1);
    __syncthreads();
    bool empty_row;  // row t of the bucket has no record in this slice
    {  // exclusive scan of the 256 row counts (thread t owns row t)
      const int w = t / WAVE;
      const int v = t < 256 ? cnt[t] : 0;
      empty_row = v == 0;
      int inc = v;
      for (int o = 1; o < WAVE; o <<= 1) {
        int y = __shfl_up(inc, o, WAVE);
        if (l >= o) inc += y;
      }
      if (l == WAVE - 1) wsum[w] = inc;
      __syncthreads();
      int off = 0;
      for (int i = 0; i < w; ++i) off += wsum[i];
      if (t < 256) cnt[t] = off + inc - v;  // becomes the fill cursor
      __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < AC_ITEMS; ++i)
      if (i * MT_THREADS + t < n) {
        const int pos = atomicAdd(&cnt[my[i].key & 255u], 1);
        lk[pos] = my[i].key;
        lc[pos] = my[i].coef;
      }
    __syncthreads();
    // rows without records are zero
    if (t < nrows && empty_row) {
      T *zr = mo + (int64_t)t * R;
      for (int c = 0; c < R; ++c) zr[c] = T(0);
    }
    // group g: sorted records [c0, c1); lane gl owns columns cb .. cb+VW-1
    const int per = (n + G - 1) / G;
    const int c0 = g * per < n ? g * per : n;
    const int c1 = c0 + per < n ? c0 + per : n;
    // the chunk's first run continues the previous chunk's row (fa) and its
    // last run goes on in the next chunk (fb); those two partial sums go to
    // LDS, every other run is a whole row of this chunk and is stored
    const int fa = (c0 < c1 && c0 > 0 && ((lk[c0 - 1] ^ lk[c0]) & 255u) == 0)
                       ? (int)(lk[c0] & 255u) : -1;
    const int fb = (c0 < c1 && c1 < n && ((lk[c1] ^ lk[c1 - 1]) & 255u) == 0)
                       ? (int)(lk[c1 - 1] & 255u) : -1;
    if (gl == 0) {
      s_fa[g] = fa;
      s_fb[g] = fb;
    }
    typedef T vec_t __attribute__((ext_vector_type(VW)));
    auto put = [&](T *dst, const T (&v)[VW]) {
      if constexpr (VEC) {
        if (cb < R) {
          vec_t x;
#pragma unroll
          for (int q = 0; q < VW; ++q) x[q] = v[q];
          *reinterpret_cast<vec_t *>(dst) = x;
        }
      } else {
#pragma unroll
        for (int q = 0; q < VW; ++q)
          if (cb + q < R) dst[q] = v[q];
      }
    };
    T acc[VW];
#pragma unroll
    for (int q = 0; q < VW; ++q) acc[q] = T(0);
    auto flush = [&](int row) {
      if (row == fa)
        put(pr + (2 * g) * (L * VW) + cb, acc);
      else if (row == fb)
        put(pr + (2 * g + 1) * (L * VW) + cb, acc);
      else
        put(mo + (int64_t)row * R + cb, acc);
#pragma unroll
      for (int q = 0; q < VW; ++q) acc[q] = T(0);
    };
    // batches of AC_BATCH records (indices clamped to the chunk, so every
    // load is issued unconditionally); the next batch is in flight while
    // the current one is accumulated.  A run of one row ends where the next
    // record's row differs or the chunk ends.
    struct Batch {
      T hv[AC_BATCH][VW];
      T cf[AC_BATCH];
      int rw[AC_BATCH];
    };
    auto load_batch = [&](int kk, Batch &bt) {
#pragma unroll
      for (int u = 0; u < AC_BATCH; ++u) {
        const int kc = kk + u < c1 ? kk + u : c1 - 1;
        const uint32_t key = lk[kc];
        bt.rw[u] = (int)(key & 255u);
        bt.cf[u] = kk + u < c1 ? lc[kc] : T(0);
        load_cols<T, VW, VEC>(hc + (int64_t)(key >> 8) * R, cb, R, bt.hv[u]);
      }
    };
    auto run_batch = [&](int kk, const Batch &bt, int next_row) {
#pragma unroll
      for (int u = 0; u < AC_BATCH; ++u) {
#pragma unroll
        for (int q = 0; q < VW; ++q) acc[q] = fma(bt.cf[u], bt.hv[u][q], acc[q]);
        const int nr = u + 1 < AC_BATCH ? bt.rw[u + 1] : next_row;
        const bool last = kk + u + 1 >= c1;
        if (kk + u < c1 && (last || nr != bt.rw[u])) flush(bt.rw[u]);
      }
    };
    if (c0 < c1) {
      Batch b0, b1;
      load_batch(c0, b0);
      for (int kk = c0; kk < c1; kk += 2 * AC_BATCH) {
        load_batch(kk + AC_BATCH, b1);
        run_batch(kk, b0, b1.rw[0]);
        load_batch(kk + 2 * AC_BATCH, b0);
        run_batch(kk + AC_BATCH, b1, b0.rw[0]);
      }
    }
    __syncthreads();
    // a row cut by chunk boundaries is summed by the group where it starts:
    // its last-run partial, then the first-run partials of the following
    // groups in order
    if (fb >= 0 && fb != fa) {
      T sum[VW];
      const T *p0 = pr + (2 * g + 1) * (L * VW) + cb;
#pragma unroll
      for (int q = 0; q < VW; ++q) sum[q] = p0[q];
      for (int h2 = g + 1; h2 < G && s_fa[h2] == fb; ++h2) {
        const T *p1 = pr + (2 * h2) * (L * VW) + cb;
#pragma unroll
        for (int q = 0; q < VW; ++q) sum[q] += p1[q];
        if (s_fb[h2] != fb) break;
      }
      put(mo + (int64_t)fb * R + cb, sum);
    }
    __syncthreads();
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

// Rows of a split bucket: sum of its slices' blocks, in slice order.
// Split buckets only: entry e of bucket split[i]'s B x R block is the sum
// of its slices' blocks, in slice order.
template <typename T>
__global__ void k_bk_combine(const int64_t *item_start, const int64_t *split,
                             const int64_t *nsplit, int bb, int R, int64_t I,
                             const T *part, T *M) {
  const int B = 1 << bb;
  const int64_t per = (int64_t)B * R;
  const int64_t total = *nsplit * per;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t si = g / per;
    const int e = (int)(g - si * per);
    const int64_t bk = split[si];
    const int64_t k0 = item_start[bk], k1 = item_start[bk + 1];
    const int64_t row0 = bk * B;
    if (row0 + e / R >= I) continue;
    T acc = 0;
    for (int64_t k = k0; k < k1; ++k) acc += part[k * per + e];
    M[row0 * R + e] = acc;
  }
}

int mttkrp_grid() { return 256 * 8; }


}  // namespace

template <typename T>
void set_sample_rows(const ModeList &ml, int64_t J, int R, const int32_t *sidx,
                     const double *prob, T *h, uint32_t *err, hipStream_t s) {
  hipLaunchKernelGGL((k_sample_rows<T>), dim3(ceil_div(J * R, 256)), dim3(256),
                     0, s, ml, J, R, sidx, prob, h, err);
  CPR_LAUNCH_CHECK();
}
template void set_sample_rows<float>(const ModeList &, int64_t, int,
                                     const int32_t *, const double *, float *,
                                     uint32_t *, hipStream_t);
template void set_sample_rows<double>(const ModeList &, int64_t, int,
                                      const int32_t *, const double *,
                                      double *, uint32_t *, hipStream_t);

void lookup_columns(const ModeList &ml, int64_t J, const int32_t *sidx,
                    const ModeIndex &ix, SampleWork &w, hipStream_t s) {
  hipLaunchKernelGGL(k_lookup, dim3(ceil_div(J, LK_THREADS)), dim3(LK_THREADS),
                     0, s, ml, J, sidx, ix.hash, ix.col_key, ix.hbits,
                     w.col_id, w.owner);
  CPR_LAUNCH_CHECK();
}

void merge_samples(int64_t J, const double *prob, const int64_t *col_ptr,
                   const void *h, int R, int tsize, SampleWork &w,
                   hipStream_t s) {
  const int nb = (int)std::min<int64_t>(ceil_div(J, LK_THREADS), MG_MAXBLK);
  const int64_t chunk = ceil_div(ceil_div(J, nb), LK_THREADS) * LK_THREADS;
  int64_t *first = w.scratch, *len = w.scratch + J, *part = w.scratch + 2 * J;
  hipLaunchKernelGGL(k_dup_first, dim3(nb), dim3(LK_THREADS), 0, s, J, chunk,
                     w.col_id, w.owner, col_ptr, w.dupcnt, first, len, part);
  CPR_LAUNCH_CHECK();
  if (tsize == 4)
    hipLaunchKernelGGL((k_compact<float>), dim3(nb), dim3(LK_THREADS), 0, s, J,
                       chunk, prob, w.col_id, first, len, part, col_ptr,
                       static_cast<const float *>(h), R, w.owner, w.dupcnt,
                       w.uq_s, w.uq_cid, w.uq_cnt, w.uq_w, w.uq_off, w.uq_base,
                       static_cast<float *>(w.hc), w.tile_first, w.counts,
                       w.stats);
  else
    hipLaunchKernelGGL((k_compact<double>), dim3(nb), dim3(LK_THREADS), 0, s, J,
                       chunk, prob, w.col_id, first, len, part, col_ptr,
                       static_cast<const double *>(h), R, w.owner, w.dupcnt,
                       w.uq_s, w.uq_cid, w.uq_cnt, w.uq_w, w.uq_off, w.uq_base,
                       static_cast<double *>(w.hc), w.tile_first, w.counts,
                       w.stats);
  CPR_LAUNCH_CHECK();
}

int bucket_shift(int R, int tsize) {
  // B rows of M per bucket: 128 (measured best at R = 32: larger buckets
  // split into more slices that k_bk_combine must add, smaller ones take
  // more scatter atomics), fewer when a B x R block exceeds 32 KiB
  int bb = 7;
  while (bb > 0 && ((1 << bb) * R * tsize) > 32768) --bb;
  return bb;
}

size_t lds_cap() { return 160 * 1024 - 8 * 1024; }

template <typename T>
void sampled_mttkrp(const SampleWork &w, int64_t I, const int64_t *col_ptr,
                    const int32_t *row, const T *val, const int64_t *bk_start,
                    int R, int bb, T *M, hipStream_t s) {
  const T *hc = static_cast<const T *>(w.hc);
  const int nbk = (int)((I + (1 << bb) - 1) >> bb);
  // fixed offsets: the fill cursors of every mode stay zero between calls
  // (each plan clears the ones it read), whatever the mode's bucket count
  int64_t *bk_fill = w.bk, *bk_end = w.bk + (w.bk_max + 1),
          *item_start = w.bk + 2 * (w.bk_max + 1),
          *split = w.bk + 3 * (w.bk_max + 1),
          *btot = w.bk + 4 * (w.bk_max + 1),
          *nsplit = btot + 2 * ((w.bk_max + 1 + PL_THREADS - 1) / PL_THREADS);
  const dim3 b(MT_THREADS), gt(mttkrp_grid());
  BkRec<T> *rec = static_cast<BkRec<T> *>(w.rec);
  T *part = static_cast<T *>(w.part);
  const int sh = w.rec1 ? super_shift(nbk) : -1;
  if (sh >= 0) {  // two passes: super buckets, then buckets
    const int nsb = (int)((nbk + (1 << sh) - 1) >> sh);
    int64_t *sfill = w.sb, *ds_fill = w.sb + (SB_MAX + 1),
            *ds_start = w.sb + 2 * (SB_MAX + 1);
    hipLaunchKernelGGL((k_bk_scatter<T, true>), gt, b, 3 * (size_t)nsb * 4, s,
                       w.counts, w.uq_off, w.tile_first, w.uq_base, row, val,
                       nsb, bb, sh, bk_start, sfill, w.rec1);
    CPR_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_ds_plan, dim3(1), dim3(SB_MAX), 0, s, sfill, nsb,
                       ds_fill, ds_start);
    CPR_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_bk_distribute<T>), gt, dim3(DS_THREADS), 0, s,
                       ds_start, ds_fill, nsb, sh, nbk, bb, bk_start, bk_fill,
                       static_cast<const BkRec1<T> *>(w.rec1), rec);
    CPR_LAUNCH_CHECK();
  } else {
    const size_t hl = nbk <= BK_LDS_MAX ? (size_t)nbk * 4 : 0;
    hipLaunchKernelGGL((k_bk_scatter<T, false>), gt, b, 3 * hl, s, w.counts,
                       w.uq_off, w.tile_first, w.uq_base, row, val, nbk, bb, 0,
                       bk_start, bk_fill, static_cast<void *>(rec));
    CPR_LAUNCH_CHECK();
  }
  const int nplan = (int)((nbk + 1 + PL_THREADS - 1) / PL_THREADS);
  hipLaunchKernelGGL(k_bk_plan_count, dim3(nplan), dim3(PL_THREADS), 0, s,
                     bk_fill, nbk, btot);
  CPR_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_bk_plan, dim3(nplan), dim3(PL_THREADS), 0, s, bk_start,
                     bk_fill, nbk, btot, bk_end, item_start, w.item_bk, split,
                     nsplit);
  CPR_LAUNCH_CHECK();
  constexpr int VW = 16 / sizeof(T);  // columns per lane
  // records, then the boundary partials: 2 per lane group, L VW columns
  const int lanes_r = (R + VW - 1) / VW;
  int lanes_p = 1;
  while (lanes_p < lanes_r) lanes_p *= 2;
  const size_t lds = (size_t)BK_SLICE * (sizeof(T) + 4) +
                     (size_t)2 * (MT_THREADS / lanes_p) * lanes_p * VW * sizeof(T);
  static bool attr_set[2][14] = {};
  auto launch = [&](auto kern, int li) {
    if (!attr_set[sizeof(T) == 8][li]) {
      hipError_t e = hipFuncSetAttribute(
          reinterpret_cast<const void *>(kern),
          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_cap());
      if (e != hipSuccess) throw HipFail(e, __FILE__, __LINE__);
      attr_set[sizeof(T) == 8][li] = true;
    }
    hipLaunchKernelGGL(kern, gt, b, lds, s, item_start, w.item_bk, bk_start,
                       bk_end,
                       nbk, bb, rec, hc, R, I, M, part);
  };
  const int lanes = (R + VW - 1) / VW;  // lanes per record
  if (R % VW == 0) {
    if (lanes <= 1) launch(k_bk_accum<T, 1, VW, true>, 0);
    else if (lanes <= 2) launch(k_bk_accum<T, 2, VW, true>, 1);
    else if (lanes <= 4) launch(k_bk_accum<T, 4, VW, true>, 2);
    else if (lanes <= 8) launch(k_bk_accum<T, 8, VW, true>, 3);
    else if (lanes <= 16) launch(k_bk_accum<T, 16, VW, true>, 4);
    else if (lanes <= 32) launch(k_bk_accum<T, 32, VW, true>, 5);
    else launch(k_bk_accum<T, 64, VW, true>, 6);
  } else {
    if (lanes <= 1) launch(k_bk_accum<T, 1, VW, false>, 7);
    else if (lanes <= 2) launch(k_bk_accum<T, 2, VW, false>, 8);
    else if (lanes <= 4) launch(k_bk_accum<T, 4, VW, false>, 9);
    else if (lanes <= 8) launch(k_bk_accum<T, 8, VW, false>, 10);
    else if (lanes <= 16) launch(k_bk_accum<T, 16, VW, false>, 11);
    else if (lanes <= 32) launch(k_bk_accum<T, 32, VW, false>, 12);
    else launch(k_bk_accum<T, 64, VW, false>, 13);
  }
  CPR_LAUNCH_CHECK();
  hipLaunchKernelGGL((k_bk_combine<T>), gt, b, 0, s, item_start, split,
                     nsplit, bb, R, I, part, M);
  CPR_LAUNCH_CHECK();
}
int64_t bucket_tiles(int64_t rec_cap) { return rec_cap / BK_TILE + 2; }

int64_t bucket_work_entries(int64_t bk_max) {
  // fill cursors, ends, slice starts, split buckets (bk_max + 1 each), the
  // plan's per-block totals and the split count
  return 4 * (bk_max + 1) + 2 * ((bk_max + 1 + PL_THREADS - 1) / PL_THREADS) +
         1;
}

int64_t bucket_max_items(int64_t rec_cap, int64_t nbk) {
  return rec_cap / BK_SLICE + nbk + 1;
}

size_t bucket_record_bytes(int tsize) {
  return tsize == 4 ? sizeof(BkRec<float>) : sizeof(BkRec<double>);
}

size_t super_record_bytes(int tsize) {
  return tsize == 4 ? sizeof(BkRec1<float>) : sizeof(BkRec1<double>);
}

bool two_pass_placement(int64_t nbk) { return super_shift(nbk) >= 0; }

int64_t super_work_entries() { return 3 * (SB_MAX + 1); }
template void sampled_mttkrp<float>(const SampleWork &, int64_t,
                                    const int64_t *, const int32_t *,
                                    const float *, const int64_t *, int, int,
                                    float *, hipStream_t);
template void sampled_mttkrp<double>(const SampleWork &, int64_t,
                                     const int64_t *, const int32_t *,
                                     const double *, const int64_t *, int,
                                     int, double *, hipStream_t);

void bucket_regions(const int32_t *row, int64_t nnz, int64_t I, int bb,
                    int64_t *starts, int64_t *cnt, void *scan_tmp,
                    hipStream_t s) {
  const int nbk = (int)((I + (1 << bb) - 1) >> bb);
  zero_fill<int64_t>(cnt, nbk + 1, s);
  const int nwin = (nbk + BH_WIN - 1) / BH_WIN;
  const size_t hl = (size_t)std::min(nbk, BH_WIN) * 4;
  // about one workgroup per CU and window, fewer for small inputs
  const int64_t chunks = std::min<int64_t>(
      std::max<int64_t>(ceil_div(nnz, (int64_t)BH_THREADS * 16), 1), 256);
  hipLaunchKernelGGL(k_bucket_hist, dim3((unsigned)chunks, (unsigned)nwin),
                     dim3(BH_THREADS), hl, s, row, nnz, nbk, bb, cnt);
  CPR_LAUNCH_CHECK();
  exclusive_scan_i64(cnt, starts, nbk + 1, scan_tmp, s);
}

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
