// k_scan.hip -- exclusive prefix sums (u32, u64) used to size and place the
// tree's nodes, the radix-sort digits and the per-leaf interaction lists.
// Three passes: tile totals, scan of the totals by one block, tile scan with
// the tile's offset.  Deterministic (integer arithmetic, fixed order).
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

template <typename T>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_top(T* tmp, int64_t nb, T* total) {
  __shared__ T sh[SCAN_THREADS];
  T carry = 0;
  for (int64_t base = 0; base < nb; base += SCAN_THREADS) {
    int64_t i = base + threadIdx.x;
    T v = i < nb ? tmp[i] : T(0);
    T tot;
    T ex = block_exclusive<T>(v, sh, &tot);
    if (i < nb) tmp[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) *total = carry;
}

template <typename TI, typename T>
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_down(const TI* in, T* out, int64_t n,
                                                            const T* tmp) {
  __shared__ T sh[SCAN_THREADS];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  T v[SCAN_ITEMS];
  T s = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = base + k < n ? (T)in[base + k] : T(0);
    s += v[k];
  }
  T tot;
  T run = block_exclusive<T>(s, sh, &tot) + tmp[blockIdx.x];
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
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
  k_scan_top<T><<<1, SCAN_THREADS, 0, s>>>(tmp, nb, total);
  k_scan_down<TI, T><<<(unsigned)nb, SCAN_THREADS, 0, s>>>(in, out, n, tmp);
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
