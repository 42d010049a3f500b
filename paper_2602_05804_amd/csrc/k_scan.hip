// k_scan.hip -- exclusive prefix sums (u32, u64) used to size and place the
// tree's nodes, the radix-sort digits and the per-leaf interaction lists.
// One block for short inputs; otherwise tile totals, then tile scans that
// add the totals of the tiles before them (a scan of the totals by one block
// in between for very long inputs).  Deterministic (integer arithmetic,
// fixed order).
#include "sfmm_internal.h"

namespace sfmm {
namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;
// one block of SMALL_THREADS threads scans up to SMALL_THREADS * SMALL_ITEMS
// values; up to TWO_PASS_TILES tiles take two passes (tile totals, then tile
// scans that add the totals before them); beyond that three passes
constexpr int SMALL_THREADS = 1024;
constexpr int SMALL_ITEMS = 16;
constexpr int64_t TWO_PASS_TILES = 4096;

template <typename T>
__device__ __forceinline__ T wave_incl(T x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

// exclusive scan over a block of NT threads (wave scans, then the wave
// totals); returns this thread's exclusive prefix and the block total
template <typename T, int NT>
__device__ __forceinline__ T block_exclusive(T v, T* total) {
  constexpr int W = NT / 64;
  __shared__ T wt[W];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const T inc = wave_incl<T>(v);
  if (lane == 63) wt[w] = inc;
  __syncthreads();
  T pre = inc - v, tot = 0;
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const T t = wt[k];
    if (k < w) pre += t;
    tot += t;
  }
  *total = tot;
  __syncthreads();
  return pre;
}

template <typename T>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_reduce(const T* in, int64_t n, T* tmp) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  T s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k)
    if (base + k < n) s += in[base + k];
  T tot;
  block_exclusive<T, SCAN_THREADS>(s, &tot);
  if (threadIdx.x == 0) tmp[blockIdx.x] = tot;
}

template <typename T>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_top(T* tmp, int64_t nb, T* total) {
  T carry = 0;
  for (int64_t base = 0; base < nb; base += SCAN_THREADS) {
    int64_t i = base + threadIdx.x;
    T v = i < nb ? tmp[i] : T(0);
    T tot;
    T ex = block_exclusive<T, SCAN_THREADS>(v, &tot);
    if (i < nb) tmp[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) *total = carry;
}

// tile scan; the tile's offset is tmp[blockIdx.x] (scanned totals), or, with
// SUM_BEFORE, the sum of the raw totals of the tiles before it (and the last
// tile writes the grand total)
template <typename T, bool SUM_BEFORE>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_down(const T* in, T* out, int64_t n,
                                                            const T* tmp, T* total) {
  T before;
  if (SUM_BEFORE) {
    T c = 0;
    for (int64_t t = threadIdx.x; t < (int64_t)blockIdx.x; t += SCAN_THREADS) c += tmp[t];
    block_exclusive<T, SCAN_THREADS>(c, &before);
  } else {
    before = tmp[blockIdx.x];
  }
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  T v[SCAN_ITEMS];
  T s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = base + k < n ? in[base + k] : T(0);
    s += v[k];
  }
  T tot;
  T run = block_exclusive<T, SCAN_THREADS>(s, &tot) + before;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (SUM_BEFORE && threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) *total = before + tot;
}

// the whole scan in one block (n <= SMALL_THREADS * SMALL_ITEMS)
template <typename T>
__global__ __launch_bounds__(SMALL_THREADS) void k_scan_small(const T* in, T* out, int64_t n,
                                                              T* total) {
  const int per = (int)((n + SMALL_THREADS - 1) / SMALL_THREADS);
  const int64_t base = (int64_t)threadIdx.x * per;
  T v[SMALL_ITEMS];
  T s = 0;
#pragma unroll
  for (int k = 0; k < SMALL_ITEMS; ++k) {
    v[k] = (k < per && base + k < n) ? in[base + k] : T(0);
    s += v[k];
  }
  T tot;
  T run = block_exclusive<T, SMALL_THREADS>(s, &tot);
#pragma unroll
  for (int k = 0; k < SMALL_ITEMS; ++k) {
    if (k < per && base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) *total = tot;
}

template <typename T>
__global__ void k_zero_total(T* total) {
  *total = 0;
}

template <typename T>
void scan_impl(const T* in, T* out, int64_t n, T* total, T* tmp, hipStream_t s) {
  if (n <= 0) {
    k_zero_total<T><<<1, 1, 0, s>>>(total);
    return;
  }
  if (n <= (int64_t)SMALL_THREADS * SMALL_ITEMS) {
    k_scan_small<T><<<1, SMALL_THREADS, 0, s>>>(in, out, n, total);
    return;
  }
  int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  k_scan_reduce<T><<<(unsigned)nb, SCAN_THREADS, 0, s>>>(in, n, tmp);
  if (nb <= TWO_PASS_TILES) {
    k_scan_down<T, true><<<(unsigned)nb, SCAN_THREADS, 0, s>>>(in, out, n, tmp, total);
  } else {
    k_scan_top<T><<<1, SCAN_THREADS, 0, s>>>(tmp, nb, total);
    k_scan_down<T, false><<<(unsigned)nb, SCAN_THREADS, 0, s>>>(in, out, n, tmp, total);
  }
}

}  // namespace

size_t scan_tmp_elems(int64_t n) { return (size_t)((n + SCAN_TILE - 1) / SCAN_TILE) + 1; }

void scan_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, uint32_t* tmp,
              hipStream_t s) {
  scan_impl<uint32_t>(in, out, n, total, tmp, s);
}

void scan_u64(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* total, uint64_t* tmp,
              hipStream_t s) {
  scan_impl<uint64_t>(in, out, n, total, tmp, s);
}

}  // namespace sfmm
