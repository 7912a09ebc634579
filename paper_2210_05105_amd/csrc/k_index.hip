// Per-mode column-sorted index of the nonzeros (Section 4.3: one copy of the
// tensor per matricization, coordinates sorted by the column of mat(T, j)).
//
// Each mode's copy is produced by a stable LSD radix sort (8-bit digits,
// wave-ballot ranking) of the key (column of mat(T, j), i_j); the distinct
// columns and their offsets are then extracted with a scan.  Built once at
// init; the hot path only reads the result.
#include "internal.h"

#include <functional>

#include <algorithm>

namespace cpr {
namespace {

constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;
constexpr int RS_WAVES = RS_THREADS / WAVE;

int bits_for(uint64_t n) {  // bits to represent values in [0, n)
  int b = 0;
  while (b < 64 && (n - 1) >> b) ++b;
  return std::max(b, 1);
}

__global__ void k_validate(const int32_t *idx, const void *val, int val_fp64,
                           int64_t nnz, int N, const int64_t *dims,
                           uint32_t *err) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  uint32_t bad = 0;
  for (int k = 0; k < N; ++k) {
    int32_t i = idx[e * N + k];
    if (i < 0 || (int64_t)i >= dims[k]) bad |= ERR_INDEX;
  }
  double v = val_fp64 ? static_cast<const double *>(val)[e]
                      : (double)static_cast<const float *>(val)[e];
  if (!isfinite(v)) bad |= ERR_NONFINITE;
  if (bad) atomicOr(err, bad);
}

// key = (column of mat(T, j)) << lo_bits | i_j  when it fits in 64 bits,
// otherwise hi = column and lo = i_j separately.
__global__ void k_make_keys(const int32_t *idx, int64_t nnz, int N, int j,
                            const uint64_t *stride, int lo_bits, int combined,
                            uint64_t *hi, uint32_t *lo, uint32_t *payload) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  uint64_t c = 0;
  for (int k = 0; k < N; ++k)
    if (k != j) c += (uint64_t)idx[e * N + k] * stride[k];
  uint32_t r = (uint32_t)idx[e * N + j];
  if (combined) {
    hi[e] = (c << lo_bits) | r;
  } else {
    hi[e] = c;
    lo[e] = r;
  }
  payload[e] = (uint32_t)e;
}

__device__ __forceinline__ uint32_t digit_of(const uint64_t *hi,
                                             const uint32_t *lo, int64_t p,
                                             int shift, int from_lo) {
  return from_lo ? (lo[p] >> shift) & 255u
                 : (uint32_t)((hi[p] >> shift) & 255u);
}

__global__ void __launch_bounds__(RS_THREADS)
k_rs_hist(const uint64_t *hi, const uint32_t *lo, int64_t n, int shift,
          int from_lo, uint32_t *hist, int64_t ntiles) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int i = 0; i < RS_ITEMS; ++i) {
    int64_t p = base + (int64_t)i * RS_THREADS + threadIdx.x;
    if (p < n) atomicAdd(&h[digit_of(hi, lo, p, shift, from_lo)], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: elements of a tile are visited in 16 rounds of 256
// consecutive elements; within a round, equal digits are ranked by lane
// order (ballot match) and by wave order (per-wave digit counts in LDS).
__global__ void __launch_bounds__(RS_THREADS)
k_rs_scatter(const uint64_t *hi, const uint32_t *lo, const uint32_t *pay,
             int64_t n, int shift, int from_lo, const uint32_t *offs,
             int64_t ntiles, uint64_t *hi_o, uint32_t *lo_o, uint32_t *pay_o) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[RS_WAVES][256];
  const int t = threadIdx.x, w = t / WAVE, l = lane_id();
  base[t] = offs[(int64_t)t * ntiles + blockIdx.x];
  const uint64_t lt = (l == 0) ? 0ull : (~0ull >> (64 - l));
  const int64_t tb = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ITEMS; ++r) {
    for (int q = 0; q < RS_WAVES; ++q) wcnt[q][t] = 0;
    __syncthreads();
    const int64_t p = tb + (int64_t)r * RS_THREADS + t;
    const bool valid = p < n;
    uint32_t d = valid ? digit_of(hi, lo, p, shift, from_lo) : 0u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t dst = base[d] + rank;
      for (int q = 0; q < w; ++q) dst += wcnt[q][d];
      hi_o[dst] = hi[p];
      if (lo) lo_o[dst] = lo[p];
      pay_o[dst] = pay[p];
    }
    __syncthreads();
    uint32_t add = 0;
    for (int q = 0; q < RS_WAVES; ++q) add += wcnt[q][t];
    base[t] += add;
    __syncthreads();
  }
}

template <typename VO>
__global__ void k_finish(const uint64_t *hi, const uint32_t *lo,
                         const uint32_t *pay, int64_t n, int lo_bits,
                         int combined, const void *val_in, int in_fp64,
                         int32_t *row, VO *val, uint32_t *flag, uint32_t *err) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint64_t mask = (lo_bits >= 64) ? ~0ull : ((1ull << lo_bits) - 1);
  auto col_of = [&](int64_t q) { return combined ? hi[q] >> lo_bits : hi[q]; };
  auto row_of = [&](int64_t q) {
    return combined ? (uint32_t)(hi[q] & mask) : lo[q];
  };
  const uint64_t c = col_of(p);
  const uint32_t rr = row_of(p);
  row[p] = (int32_t)rr;
  const uint32_t e = pay[p];
  double v = in_fp64 ? static_cast<const double *>(val_in)[e]
                     : (double)static_cast<const float *>(val_in)[e];
  val[p] = (VO)v;
  uint32_t f = 1;
  if (p > 0) {
    const uint64_t cp = col_of(p - 1);
    if (cp == c) {
      f = 0;
      if (row_of(p - 1) == rr) atomicOr(err, ERR_DUP);
    }
  }
  flag[p] = f;
}

__global__ void k_cols(const uint64_t *hi, int64_t n, int lo_bits,
                       int combined, const uint32_t *flag, const uint32_t *cid,
                       uint64_t *col_key, int64_t *col_ptr) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n || !flag[p]) return;
  const uint64_t c = combined ? hi[p] >> lo_bits : hi[p];
  col_key[cid[p]] = c;
  col_ptr[cid[p]] = p;
}

// column lookup table: each column claims the first empty entry from its
// key's home entry on (keys are distinct, so a claim never meets its own key)
__global__ void k_hash_insert(const uint64_t *col_key, int64_t n_cols,
                              int hbits, uint32_t *tab) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_cols) return;
  const uint64_t key = col_key[c], mask = (1ull << hbits) - 1;
  uint64_t p = col_hash(key, hbits);
  for (uint64_t n = 0; n <= mask; ++n) {
    if (atomicCAS(tab + p, ~0u, (uint32_t)c) == ~0u) return;
    p = (p + 1) & mask;
  }
}

// longest column: grid-stride per thread, then wave and block maxima and
// one atomicMax per block (same-address atomics serialise)
__global__ void __launch_bounds__(256)
k_max_col(const int64_t *col_ptr, int64_t n_cols, unsigned long long *mx) {
  __shared__ unsigned long long sm[4];
  unsigned long long m = 0;
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n_cols;
       c += (int64_t)gridDim.x * 256) {
    const unsigned long long len =
        (unsigned long long)(col_ptr[c + 1] - col_ptr[c]);
    m = len > m ? len : m;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long y = __shfl_xor(m, o, WAVE);
    m = y > m ? y : m;
  }
  if (lane_id() == 0) sm[threadIdx.x / WAVE] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < 4; ++q) m = sm[q] > m ? sm[q] : m;
    m = sm[0] > m ? sm[0] : m;
    if (m) atomicMax(mx, m);
  }
}

// Column lengths for the sum of the J longest columns: lengths below
// LH_SMALL counted in an LDS histogram per block (added to the global one
// at the end), longer ones appended to a list (at most nnz / LH_SMALL).
constexpr int LH_SMALL = 4096;
__global__ void __launch_bounds__(256)
k_len_hist(const int64_t *col_ptr, int64_t n_cols, unsigned long long *hist,
           int64_t *big, unsigned long long *nbig, int64_t big_cap) {
  __shared__ uint32_t h[LH_SMALL];
  for (int i = threadIdx.x; i < LH_SMALL; i += 256) h[i] = 0;
  __syncthreads();
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n_cols;
       c += (int64_t)gridDim.x * 256) {
    const int64_t len = col_ptr[c + 1] - col_ptr[c];
    if (len < LH_SMALL) {
      atomicAdd(&h[len], 1u);
    } else {
      const unsigned long long at = atomicAdd(nbig, 1ull);
      if ((int64_t)at < big_cap) big[at] = len;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < LH_SMALL; i += 256)
    if (h[i]) atomicAdd(&hist[i], (unsigned long long)h[i]);
}

struct DevBuf {
  void *p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  template <typename T>
  T *get() { return static_cast<T *>(p); }
};

bool dalloc(DevBuf &b, size_t bytes) {
  return hipMalloc(&b.p, std::max<size_t>(bytes, 16)) == hipSuccess;
}

}  // namespace

uint32_t *validate_coo(const int32_t *idx, const void *val, int val_fp64,
                       int64_t nnz, int N, const int64_t *dims, uint32_t *err,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_validate, dim3(ceil_div(nnz, 256)), dim3(256), 0, s,
                     idx, val, val_fp64, nnz, N, dims, err);
  CPR_LAUNCH_CHECK();
  return err;
}

std::string build_mode_index(const int32_t *idx, const void *val, int val_fp64,
                             int64_t nnz, int N, const int64_t *dims_h, int j,
                             int out_fp64, ModeIndex &out, uint32_t *err,
                             hipStream_t s) {
  // column strides of mat(T, j): mode 1 fastest among the modes != j
  uint64_t stride[MAXN] = {0};
  unsigned __int128 ncols = 1;
  for (int k = 0; k < N; ++k) {
    if (k == j) continue;
    stride[k] = (uint64_t)ncols;
    ncols *= (unsigned __int128)dims_h[k];
  }
  if (ncols >= ((unsigned __int128)1 << 63))
    return "column keys of mat(T, j) need more than 63 bits";
  const int lo_bits = bits_for((uint64_t)dims_h[j]);
  const int hi_bits = bits_for((uint64_t)ncols);
  const int combined = (lo_bits + hi_bits <= 64);
  out.I = dims_h[j];

  DevBuf d_stride, hiA, hiB, loA, loB, payA, payB, hist, scan_tmp, flag, cid;
  const int64_t ntiles = (nnz + RS_TILE - 1) / RS_TILE;
  if (!dalloc(d_stride, sizeof(stride)) || !dalloc(hiA, nnz * 8) ||
      !dalloc(hiB, nnz * 8) || !dalloc(payA, nnz * 4) ||
      !dalloc(payB, nnz * 4) || !dalloc(hist, 256 * ntiles * 4) ||
      !dalloc(scan_tmp, std::max(scan_temp_bytes(256 * ntiles),
                                 scan_temp_bytes(nnz))))
    return "out of device memory building the mode index";
  if (!combined && (!dalloc(loA, nnz * 4) || !dalloc(loB, nnz * 4)))
    return "out of device memory building the mode index";
  if (hipMemcpyAsync(d_stride.p, stride, sizeof(stride), hipMemcpyHostToDevice,
                     s) != hipSuccess)
    return "hipMemcpyAsync failed";
  const dim3 g1(ceil_div(nnz, 256)), b1(256);
  hipLaunchKernelGGL(k_make_keys, g1, b1, 0, s, idx, nnz, N, j,
                     d_stride.get<uint64_t>(), lo_bits, combined,
                     hiA.get<uint64_t>(), loA.get<uint32_t>(),
                     payA.get<uint32_t>());
  CPR_LAUNCH_CHECK();

  // digit passes: least significant first (row bits, then column bits)
  struct Pass { int shift, from_lo; };
  std::vector<Pass> passes;
  if (combined) {
    for (int sh = 0; sh < lo_bits + hi_bits; sh += 8) passes.push_back({sh, 0});
  } else {
    for (int sh = 0; sh < lo_bits; sh += 8) passes.push_back({sh, 1});
    for (int sh = 0; sh < hi_bits; sh += 8) passes.push_back({sh, 0});
  }
  uint64_t *hi_in = hiA.get<uint64_t>(), *hi_out = hiB.get<uint64_t>();
  uint32_t *lo_in = loA.get<uint32_t>(), *lo_out = loB.get<uint32_t>();
  uint32_t *pay_in = payA.get<uint32_t>(), *pay_out = payB.get<uint32_t>();
  for (const Pass &ps : passes) {
    hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)ntiles), dim3(RS_THREADS), 0,
                       s, hi_in, lo_in, nnz, ps.shift, ps.from_lo,
                       hist.get<uint32_t>(), ntiles);
    exclusive_scan_u32(hist.get<uint32_t>(), hist.get<uint32_t>(), 256 * ntiles,
                       scan_tmp.p, s);
    hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)ntiles), dim3(RS_THREADS),
                       0, s, hi_in, lo_in, pay_in, nnz, ps.shift, ps.from_lo,
                       hist.get<uint32_t>(), ntiles, hi_out, lo_out, pay_out);
    CPR_LAUNCH_CHECK();
    std::swap(hi_in, hi_out);
    std::swap(lo_in, lo_out);
    std::swap(pay_in, pay_out);
  }

  if (hipMalloc((void **)&out.row, nnz * 4) != hipSuccess ||
      hipMalloc(&out.val, nnz * (out_fp64 ? 8 : 4)) != hipSuccess)
    return "out of device memory for the mode index";
  if (!dalloc(flag, nnz * 4) || !dalloc(cid, nnz * 4))
    return "out of device memory building the mode index";
  if (out_fp64)
    hipLaunchKernelGGL(k_finish<double>, g1, b1, 0, s, hi_in, lo_in, pay_in,
                       nnz, lo_bits, combined, val, val_fp64, out.row,
                       static_cast<double *>(out.val), flag.get<uint32_t>(),
                       err);
  else
    hipLaunchKernelGGL(k_finish<float>, g1, b1, 0, s, hi_in, lo_in, pay_in,
                       nnz, lo_bits, combined, val, val_fp64, out.row,
                       static_cast<float *>(out.val), flag.get<uint32_t>(),
                       err);
  CPR_LAUNCH_CHECK();
  exclusive_scan_u32(flag.get<uint32_t>(), cid.get<uint32_t>(), nnz,
                     scan_tmp.p, s);
  uint32_t last_cid = 0, last_flag = 0;
  if (hipMemcpyAsync(&last_cid, cid.get<uint32_t>() + nnz - 1, 4,
                     hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&last_flag, flag.get<uint32_t>() + nnz - 1, 4,
                     hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return "hip error while building the mode index";
  out.n_cols = (int64_t)last_cid + last_flag;
  if (hipMalloc((void **)&out.col_key, out.n_cols * 8) != hipSuccess ||
      hipMalloc((void **)&out.col_ptr, (out.n_cols + 1) * 8) != hipSuccess)
    return "out of device memory for the mode index";
  hipLaunchKernelGGL(k_cols, g1, b1, 0, s, hi_in, nnz, lo_bits, combined,
                     flag.get<uint32_t>(), cid.get<uint32_t>(), out.col_key,
                     out.col_ptr);
  CPR_LAUNCH_CHECK();
  const int64_t nnz_h = nnz;
  DevBuf mx;
  if (!dalloc(mx, 8)) return "out of device memory";
  if (hipMemcpyAsync(out.col_ptr + out.n_cols, &nnz_h, 8,
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemsetAsync(mx.p, 0, 8, s) != hipSuccess)
    return "hip error while building the mode index";
  hipLaunchKernelGGL(k_max_col,
                     dim3((unsigned)std::min<int64_t>(ceil_div(out.n_cols, 256), 512)),
                     dim3(256), 0, s,
                     out.col_ptr, out.n_cols,
                     mx.get<unsigned long long>());
  CPR_LAUNCH_CHECK();
  unsigned long long mxh = 0;
  if (hipMemcpyAsync(&mxh, mx.p, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return "hip error while building the mode index";
  out.max_col = (int64_t)mxh;
  // column lookup table, at least twice as many entries as columns
  int hbits = 4;
  while (((int64_t)1 << hbits) < 2 * out.n_cols) ++hbits;
  out.hbits = hbits;
  const size_t hbytes = ((size_t)1 << hbits) * 4;
  if (hipMalloc((void **)&out.hash, hbytes) != hipSuccess)
    return "out of device memory for the mode index";
  if (hipMemsetAsync(out.hash, 0xff, hbytes, s) != hipSuccess)
    return "hip error while building the mode index";
  hipLaunchKernelGGL(k_hash_insert, dim3(ceil_div(out.n_cols, 256)), dim3(256),
                     0, s, out.col_key, out.n_cols, hbits, out.hash);
  CPR_LAUNCH_CHECK();
  return "";
}

// Sum of the lengths of the J longest columns of a mode (all nonzeros when
// J >= n_cols): a bound on the nonzeros any solve extracts, since it takes
// at most J distinct columns.  Returns -1 on a HIP failure.
int64_t top_columns_total(const int64_t *col_ptr, int64_t n_cols, int64_t nnz,
                          int64_t J, hipStream_t s) {
  if (J >= n_cols) return nnz;
  const int64_t big_cap = nnz / LH_SMALL + 1;
  DevBuf hist, big, nbig;
  if (!dalloc(hist, LH_SMALL * 8) || !dalloc(big, big_cap * 8) ||
      !dalloc(nbig, 8))
    return -1;
  if (hipMemsetAsync(hist.p, 0, LH_SMALL * 8, s) != hipSuccess ||
      hipMemsetAsync(nbig.p, 0, 8, s) != hipSuccess)
    return -1;
  const unsigned nb = (unsigned)std::min<int64_t>(ceil_div(n_cols, 256), 2048);
  hipLaunchKernelGGL(k_len_hist, dim3(nb), dim3(256), 0, s, col_ptr, n_cols,
                     hist.get<unsigned long long>(), big.get<int64_t>(),
                     nbig.get<unsigned long long>(), big_cap);
  if (hipGetLastError() != hipSuccess) return -1;
  std::vector<unsigned long long> hh(LH_SMALL);
  unsigned long long nb_h = 0;
  if (hipMemcpyAsync(hh.data(), hist.p, LH_SMALL * 8, hipMemcpyDeviceToHost,
                     s) != hipSuccess ||
      hipMemcpyAsync(&nb_h, nbig.p, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return -1;
  const int64_t n_big = std::min<int64_t>((int64_t)nb_h, big_cap);
  std::vector<int64_t> bl(n_big);
  if (n_big > 0 &&
      (hipMemcpyAsync(bl.data(), big.p, n_big * 8, hipMemcpyDeviceToHost, s) !=
           hipSuccess ||
       hipStreamSynchronize(s) != hipSuccess))
    return -1;
  std::sort(bl.begin(), bl.end(), std::greater<int64_t>());
  int64_t left = J, tot = 0;
  for (int64_t i = 0; i < n_big && left > 0; ++i, --left) tot += bl[i];
  for (int len = LH_SMALL - 1; len >= 1 && left > 0; --len) {
    const int64_t take = std::min<int64_t>(left, (int64_t)hh[len]);
    tot += take * len;
    left -= take;
  }
  return std::min(tot, nnz);
}

}  // namespace cpr
