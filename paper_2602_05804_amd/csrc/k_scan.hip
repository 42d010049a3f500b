// k_scan.hip -- exclusive prefix sums (u32, u64) used to size and place the
// tree's nodes, the radix-sort digits and the per-leaf interaction lists.
// Two passes: tile totals, then the tile scan, each block first adding up the
// totals of the tiles before its own (a few hundred at most for the sizes
// here, so this costs less than a launch of its own).  Deterministic (integer
// arithmetic, fixed order).
#include "sfmm_internal.h"

namespace sfmm {
namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

template <typename T>
__device__ T block_exclusive(T v, T* sh, T* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < SCAN_THREADS; off <<= 1) {
    T x = t >= off ? sh[t - off] : T(0);
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  T incl = sh[t];
  *total = sh[SCAN_THREADS - 1];
  __syncthreads();
  return incl - v;
}

template <typename TI, typename T>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(const TI* in, int64_t n, T* tmp) {
  __shared__ T sh[SCAN_THREADS];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  T s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k)
    if (base + k < n) s += (T)in[base + k];
  T tot;
  block_exclusive<T>(s, sh, &tot);
  if (threadIdx.x == 0) tmp[blockIdx.x] = tot;
}

template <typename TI, typename T>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_down(const TI* in, T* out, int64_t n,
                                                            const T* tmp, T* total) {
  __shared__ T sh[SCAN_THREADS];
  // the totals of the tiles before this one, in a fixed order
  T pre = 0;
  for (int64_t i = threadIdx.x; i < (int64_t)blockIdx.x; i += SCAN_THREADS) pre += tmp[i];
  T prefix;
  block_exclusive<T>(pre, sh, &prefix);
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  T v[SCAN_ITEMS];
  T s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = base + k < n ? (T)in[base + k] : T(0);
    s += v[k];
  }
  T tot;
  T run = block_exclusive<T>(s, sh, &tot) + prefix;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = prefix + tot;
}

template <typename T>
__global__ void k_zero_total(T* total) {
  *total = 0;
}

template <typename TI, typename T>
void scan_impl(const TI* in, T* out, int64_t n, T* total, T* tmp, hipStream_t s) {
  if (n <= 0) {
    k_zero_total<T><<<1, 1, 0, s>>>(total);
    return;
  }
  int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  k_scan_reduce<TI, T><<<(unsigned)nb, SCAN_THREADS, 0, s>>>(in, n, tmp);
  k_scan_down<TI, T><<<(unsigned)nb, SCAN_THREADS, 0, s>>>(in, out, n, tmp, total);
}

}  // namespace

size_t scan_tmp_elems(int64_t n) { return (size_t)((n + SCAN_TILE - 1) / SCAN_TILE) + 1; }

void scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, uint32_t* tmp,
              hipStream_t s) {
  scan_impl<uint32_t, uint32_t>(in, out, n, total, tmp, s);
}

void scan_u64(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* total, uint64_t* tmp,
              hipStream_t s) {
  scan_impl<uint64_t, uint64_t>(in, out, n, total, tmp, s);
}

void scan_u32_u64(const uint32_t* in, uint64_t* out, int64_t n, uint64_t* total, uint64_t* tmp,
                  hipStream_t s) {
  scan_impl<uint32_t, uint64_t>(in, out, n, total, tmp, s);
}

}  // namespace sfmm
