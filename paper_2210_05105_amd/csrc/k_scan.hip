// Deterministic device-wide prefix sums (reduce, scan of tile totals, then
// per-tile scan).  The summation order is fixed by the tile shape, so the
// FP64 result is bitwise reproducible; its rounding error is about
// (ITEMS + log2(THREADS) + log2(tiles)) ulps of the running total.
#include "internal.h"

namespace cpr {
namespace {

constexpr int SC_THREADS = 256;
constexpr int SC_ITEMS = 16;
constexpr int SC_TILE = SC_THREADS * SC_ITEMS;

template <typename T>
__device__ T wave_incl_scan(T x) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    T y = __shfl_up(x, o, WAVE);
    if (l >= o) x += y;
  }
  return x;
}

// Exclusive scan of one value per thread across the block; returns the
// block total through *total.
template <typename T>
__device__ T block_excl_scan(T x, T *total) {
  __shared__ T wsum[SC_THREADS / WAVE];
  const int w = threadIdx.x / WAVE, l = lane_id();
  T inc = wave_incl_scan(x);
  if (l == WAVE - 1) wsum[w] = inc;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < SC_THREADS / WAVE; ++i) {
    if (i < w) off += wsum[i];
    tot += wsum[i];
  }
  __syncthreads();
  *total = tot;
  return off + inc - x;
}

template <typename T>
__global__ void __launch_bounds__(SC_THREADS)
k_tile_reduce(const T *in, int64_t n, T *partial) {
  const int64_t base = (int64_t)blockIdx.x * SC_TILE;
  T acc = 0;
#pragma unroll
  for (int i = 0; i < SC_ITEMS; ++i) {
    int64_t p = base + (int64_t)threadIdx.x * SC_ITEMS + i;
    if (p < n) acc += in[p];
  }
  T tot;
  block_excl_scan(acc, &tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// One block scans the tile totals in chunks, carrying the running sum.
template <typename T>
__global__ void __launch_bounds__(SC_THREADS)
k_scan_partials(T *partial, int64_t nb) {
  T carry = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += SC_TILE) {
    T v[SC_ITEMS];
    T acc = 0;
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i) {
      int64_t p = c0 + (int64_t)threadIdx.x * SC_ITEMS + i;
      v[i] = p < nb ? partial[p] : T(0);
      acc += v[i];
    }
    T tot;
    T off = block_excl_scan(acc, &tot) + carry;
#pragma unroll
    for (int i = 0; i < SC_ITEMS; ++i) {
      int64_t p = c0 + (int64_t)threadIdx.x * SC_ITEMS + i;
      if (p < nb) partial[p] = off;
      off += v[i];
    }
    carry += tot;
    __syncthreads();
  }
}

template <typename T, bool INCLUSIVE>
__global__ void __launch_bounds__(SC_THREADS)
k_tile_scan(const T *in, T *out, int64_t n, const T *partial) {
  const int64_t base = (int64_t)blockIdx.x * SC_TILE;
  T v[SC_ITEMS];
  T acc = 0;
#pragma unroll
  for (int i = 0; i < SC_ITEMS; ++i) {
    int64_t p = base + (int64_t)threadIdx.x * SC_ITEMS + i;
    v[i] = p < n ? in[p] : T(0);
    acc += v[i];
  }
  T tot;
  T off = block_excl_scan(acc, &tot) + partial[blockIdx.x];
#pragma unroll
  for (int i = 0; i < SC_ITEMS; ++i) {
    int64_t p = base + (int64_t)threadIdx.x * SC_ITEMS + i;
    T inc = off + v[i];
    if (p < n) out[p] = INCLUSIVE ? inc : off;
    off = inc;
  }
}

template <typename T, bool INCLUSIVE>
void run_scan(const T *in, T *out, int64_t n, void *tmp, hipStream_t s) {
  if (n <= 0) return;
  const int64_t nb = (n + SC_TILE - 1) / SC_TILE;
  T *partial = static_cast<T *>(tmp);
  hipLaunchKernelGGL(k_tile_reduce<T>, dim3((unsigned)nb), dim3(SC_THREADS), 0,
                     s, in, n, partial);
  hipLaunchKernelGGL(k_scan_partials<T>, dim3(1), dim3(SC_THREADS), 0, s,
                     partial, nb);
  hipLaunchKernelGGL((k_tile_scan<T, INCLUSIVE>), dim3((unsigned)nb),
                     dim3(SC_THREADS), 0, s, in, out, n, partial);
  CPR_LAUNCH_CHECK();
}

}  // namespace

size_t scan_temp_bytes(int64_t n) {
  return (size_t)((n + SC_TILE - 1) / SC_TILE + 1) * 8 + 256;
}

void inclusive_scan_f64(const double *in, double *out, int64_t n, void *tmp,
                        hipStream_t s) {
  run_scan<double, true>(in, out, n, tmp, s);
}
void exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, void *tmp,
                        hipStream_t s) {
  run_scan<int64_t, false>(in, out, n, tmp, s);
}
void exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n,
                        void *tmp, hipStream_t s) {
  run_scan<uint32_t, false>(in, out, n, tmp, s);
}

}  // namespace cpr
