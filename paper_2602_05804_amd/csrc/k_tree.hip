// k_tree.hip -- tree construction on the GPU.
//
//   bbox + Morton keys  cubic box, 21-bit cells per axis, x > y > z interleave
//   radix sort          stable LSD sort of (key, caller index), 8-bit digits
//   binary radix tree   Karras-style parallel build on the sorted keys; equal
//                       keys split on the bits of their sorted positions
//   leaf collapse       a node with <= leaf_size particles is a leaf
//   geometry + moments  leaves sum their particles; internal nodes combine
//                       their two children bottom-up (M2M, Appendix A.1)
//   node size l         largest distance from the centre of mass to a
//                       particle of the node (read of Sect. 3's l_tgt/l_src)
//
// The whole library is compiled with -ffp-contract=off: the centres of mass,
// sizes and the acceptance test below round exactly as written, so every
// node-pair decision matches a CPU evaluation of the same formulas.
#include "sfmm_internal.h"

namespace sfmm {
namespace {

constexpr int BBOX_THREADS = 256;
constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;

__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// per-block min/max of each axis; input validation on the side
__global__ __launch_bounds__(BBOX_THREADS) void k_bbox_partial(int n, const double* __restrict__ x,
                                                               const double* __restrict__ m,
                                                               const double* __restrict__ h,
                                                               double* __restrict__ part,
                                                               int* status, int check) {
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  int bad = 0;
  for (int i = blockIdx.x * BBOX_THREADS + threadIdx.x; i < n; i += gridDim.x * BBOX_THREADS) {
    for (int d = 0; d < 3; ++d) {
      double v = x[3 * (int64_t)i + d];
      mn[d] = fmin(mn[d], v);
      mx[d] = fmax(mx[d], v);
      if (check && !isfinite(v)) bad = 1;
    }
    if (check && !(m[i] > 0.0 && h[i] > 0.0 && isfinite(m[i]) && isfinite(h[i]))) bad = 1;
  }
  if (bad) atomicOr(status, ST_NONFINITE);
  __shared__ double sh[6][BBOX_THREADS / 64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int d = 0; d < 3; ++d) {
    double a = wave_min(mn[d]), b = wave_max(mx[d]);
    if (lane == 0) { sh[d][w] = a; sh[3 + d][w] = b; }
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double v = sh[threadIdx.x][0];
    for (int k = 1; k < BBOX_THREADS / 64; ++k)
      v = threadIdx.x < 3 ? fmin(v, sh[threadIdx.x][k]) : fmax(v, sh[threadIdx.x][k]);
    part[6 * blockIdx.x + threadIdx.x] = v;
  }
}

// box[0..2] = min corner, box[3] = cube extent, box[4] = 2^21 / extent (0 if flat)
__global__ __launch_bounds__(256) void k_bbox_final(int nb, const double* __restrict__ part,
                                                    double* __restrict__ box) {
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int b = threadIdx.x; b < nb; b += 256)
    for (int d = 0; d < 3; ++d) {
      mn[d] = fmin(mn[d], part[6 * b + d]);
      mx[d] = fmax(mx[d], part[6 * b + 3 + d]);
    }
  __shared__ double sh[6][4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int d = 0; d < 3; ++d) {
    const double a = wave_min(mn[d]), c = wave_max(mx[d]);
    if (lane == 0) { sh[d][w] = a; sh[3 + d][w] = c; }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int d = 0; d < 3; ++d) {
    mn[d] = fmin(fmin(sh[d][0], sh[d][1]), fmin(sh[d][2], sh[d][3]));
    mx[d] = fmax(fmax(sh[3 + d][0], sh[3 + d][1]), fmax(sh[3 + d][2], sh[3 + d][3]));
  }
  double ext = 0.0;
  for (int d = 0; d < 3; ++d) {
    double e = mx[d] - mn[d];
    if (e > ext) ext = e;
  }
  for (int d = 0; d < 3; ++d) box[d] = mn[d];
  box[3] = ext;
  box[4] = ext > 0.0 ? 2097152.0 / ext : 0.0;
}

// ---- several systems (forest) -----------------------------------------------
// box of system s: one block per system; same box[] layout as k_bbox_final
__global__ __launch_bounds__(256) void k_bbox_sys(const int64_t* __restrict__ off,
                                                  const double* __restrict__ x,
                                                  const double* __restrict__ m,
                                                  const double* __restrict__ h,
                                                  double* __restrict__ boxes, int* status,
                                                  int check) {
  const int sidx = blockIdx.x;
  const int64_t b = off[sidx], e = off[sidx + 1];
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  int bad = 0;
  for (int64_t i = b + threadIdx.x; i < e; i += 256) {
    for (int d = 0; d < 3; ++d) {
      const double v = x[3 * i + d];
      mn[d] = fmin(mn[d], v);
      mx[d] = fmax(mx[d], v);
      if (check && !isfinite(v)) bad = 1;
    }
    if (check && !(m[i] > 0.0 && h[i] > 0.0 && isfinite(m[i]) && isfinite(h[i]))) bad = 1;
  }
  if (bad) atomicOr(status, ST_NONFINITE);
  __shared__ double sh[6][4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int d = 0; d < 3; ++d) {
    const double a = wave_min(mn[d]), c = wave_max(mx[d]);
    if (lane == 0) { sh[d][w] = a; sh[3 + d][w] = c; }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double ext = 0.0;
  double* box = boxes + 8 * sidx;
  for (int d = 0; d < 3; ++d) {
    const double lo = fmin(fmin(sh[d][0], sh[d][1]), fmin(sh[d][2], sh[d][3]));
    const double hi = fmax(fmax(sh[3 + d][0], sh[3 + d][1]), fmax(sh[3 + d][2], sh[3 + d][3]));
    box[d] = lo;
    if (hi - lo > ext) ext = hi - lo;
  }
  box[3] = ext;
  box[4] = ext > 0.0 ? 2097152.0 / ext : 0.0;
}

__device__ __forceinline__ uint64_t spread3(uint64_t v);

// Morton key of each particle in its own system's box; sys[i] = its system
__global__ void k_keys_sys(int n, int nsys, const int64_t* __restrict__ off,
                           const double* __restrict__ x, const double* __restrict__ boxes,
                           uint64_t* __restrict__ key, uint32_t* __restrict__ idx,
                           uint32_t* __restrict__ sys) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int lo = 0, hi = nsys - 1;  // last s with off[s] <= i
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  const double* box = boxes + 8 * lo;
  uint64_t c[3] = {0, 0, 0};
  if (box[3] > 0.0) {
    for (int d = 0; d < 3; ++d) {
      const double f = floor((x[3 * (int64_t)i + d] - box[d]) * box[4]);
      c[d] = f > 2097151.0 ? 2097151ull : (uint64_t)f;
    }
  }
  key[i] = (spread3(c[0]) << 2) | (spread3(c[1]) << 1) | spread3(c[2]);
  idx[i] = (uint32_t)i;
  sys[i] = (uint32_t)lo;
}

// after the key sort: the system of each key-sorted position, as a sort key
__global__ void k_sys_sortkey(int n, const uint32_t* __restrict__ perm1,
                              const uint32_t* __restrict__ sys, uint64_t* __restrict__ skey,
                              uint32_t* __restrict__ pos) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  skey[i] = sys[perm1[i]];
  pos[i] = (uint32_t)i;
}

// final order = (system, key, caller index): gather permutation, keys, systems
__global__ void k_sys_final(int n, const uint32_t* __restrict__ q, const uint32_t* __restrict__ perm1,
                            const uint64_t* __restrict__ key1, const uint32_t* __restrict__ sys,
                            uint32_t* __restrict__ perm, uint64_t* __restrict__ key,
                            uint32_t* __restrict__ sys_sorted) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t p = q[i];
  const uint32_t o = perm1[p];
  perm[i] = o;
  key[i] = key1[p];
  sys_sorted[i] = sys[o];
}

__global__ void k_sys_start(int nsys, const int64_t* __restrict__ off, int32_t* __restrict__ start) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nsys) start[s] = (int32_t)off[s];
}

// 0: the node spans two systems (never walked); 1: the root of a system; 2: other
__global__ void k_node_flags(int nn, const NodeInfo* __restrict__ info,
                             const uint32_t* __restrict__ sys, uint8_t* __restrict__ flag) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nn) return;
  const NodeInfo ni = info[v];
  const bool within = !sys || sys[ni.lo] == sys[ni.lo + ni.cnt - 1];
  bool root = ni.parent < 0;
  if (!root && sys) {
    const NodeInfo pi = info[ni.parent];
    root = sys[pi.lo] != sys[pi.lo + pi.cnt - 1];
  }
  flag[v] = !within ? 0 : (root ? 1 : 2);
}

__device__ __forceinline__ uint64_t spread3(uint64_t v) {
  v &= 0x1fffffull;
  v = (v | (v << 32)) & 0x1f00000000ffffull;
  v = (v | (v << 16)) & 0x1f0000ff0000ffull;
  v = (v | (v << 8)) & 0x100f00f00f00f00full;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

__global__ void k_keys(int n, const double* __restrict__ x, const double* __restrict__ box,
                       uint64_t* __restrict__ key, uint32_t* __restrict__ idx) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double scale = box[4];
  uint64_t c[3] = {0, 0, 0};
  if (box[3] > 0.0) {
    for (int d = 0; d < 3; ++d) {
      double f = floor((x[3 * (int64_t)i + d] - box[d]) * scale);
      c[d] = f > 2097151.0 ? 2097151ull : (uint64_t)f;
    }
  }
  key[i] = (spread3(c[0]) << 2) | (spread3(c[1]) << 1) | spread3(c[2]);
  idx[i] = (uint32_t)i;
}

// ---- radix sort -----------------------------------------------------------
__global__ __launch_bounds__(RS_THREADS) void k_radix_hist(int n, const uint64_t* __restrict__ key,
                                                           int shift, uint32_t* __restrict__ hist,
                                                           int nb) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ITEMS; ++r) {
    int64_t i = base + r * RS_THREADS + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(key[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter: elements of the tile are ranked in their original order;
// equal digits inside a wave are found with eight ballots.
__global__ __launch_bounds__(RS_THREADS) void k_radix_scatter(
    int n, const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint64_t* __restrict__ kout, uint32_t* __restrict__ vout, int shift,
    const uint32_t* __restrict__ offs, int nb) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t base[256];
  __shared__ uint32_t wc[RS_THREADS / 64][256];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  run[t] = 0;
  base[t] = offs[(int64_t)t * nb + blockIdx.x];
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < RS_ITEMS; ++r) {
    for (int q = 0; q < RS_THREADS / 64; ++q) wc[q][t] = 0;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * RS_TILE + r * RS_THREADS + t;
    const bool valid = i < n;
    uint64_t k = valid ? kin[i] : 0ull;
    uint32_t v = valid ? vin[i] : 0u;
    uint32_t d = (uint32_t)((k >> shift) & 255u);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && rank == 0) wc[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = base[d] + run[d] + rank;
      for (int q = 0; q < w; ++q) pos += wc[q][d];
      kout[pos] = k;
      vout[pos] = v;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int q = 0; q < RS_THREADS / 64; ++q) add += wc[q][t];
    run[t] += add;
    __syncthreads();
  }
}

__global__ void k_gather(int n, const uint32_t* __restrict__ perm, const double* __restrict__ x,
                         const double* __restrict__ m, const double* __restrict__ h,
                         double* __restrict__ xs, double* __restrict__ ys,
                         double* __restrict__ zs, double* __restrict__ ms,
                         double* __restrict__ hs, double* __restrict__ his,
                         double* __restrict__ p4) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t j = perm[i];
  const double px = x[3 * j], py = x[3 * j + 1], pz = x[3 * j + 2], pm = m[j], ph = h[j];
  const double phi = 1.0 / ph;
  xs[i] = px;
  ys[i] = py;
  zs[i] = pz;
  ms[i] = pm;
  hs[i] = ph;
  his[i] = phi;
  double2* r = reinterpret_cast<double2*>(p4 + 4 * (int64_t)i);
  r[0] = make_double2(px, py);
  r[1] = make_double2(pz, pm);
}

// ---- binary radix tree (Karras 2012) ----------------------------------------
// delta = length of the common prefix of the augmented keys
// (system, key, position within the system); sys == nullptr: one system
__device__ __forceinline__ int delta(const uint64_t* __restrict__ k, const uint32_t* __restrict__ sys,
                                     const int32_t* __restrict__ sys_start, int n, int i, int j) {
  if (j < 0 || j >= n) return -1;
  uint32_t si = 0, sj = 0;
  if (sys) {
    si = sys[i];
    sj = sys[j];
    if (si != sj) return __clz((int)(si ^ sj));
  }
  const uint64_t a = k[i], b = k[j];
  if (a != b) return 32 + __clzll((long long)(a ^ b));
  const int s0 = sys ? sys_start[si] : 0;
  return 96 + __clz((int)((uint32_t)(i - s0) ^ (uint32_t)(j - s0)));
}

// internal node i (0..n-2); child codes: >= 0 internal node, < 0 leaf -(pos+1)
__global__ void k_karras(int n, const uint64_t* __restrict__ key, const uint32_t* __restrict__ sys,
                         const int32_t* __restrict__ sys_start, int leaf_size,
                         int32_t* __restrict__ kfirst, int32_t* __restrict__ klast,
                         int32_t* __restrict__ kleft, int32_t* __restrict__ kright,
                         int32_t* __restrict__ kpar, int32_t* __restrict__ kside,
                         uint32_t* __restrict__ kept) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n - 1) return;
  const int d = (delta(key, sys, sys_start, n, i, i + 1) - delta(key, sys, sys_start, n, i, i - 1)) >= 0 ? 1 : -1;
  const int dmin = delta(key, sys, sys_start, n, i, i - d);
  int lmax = 2;
  while (delta(key, sys, sys_start, n, i, i + lmax * d) > dmin) lmax *= 2;
  int l = 0;
  for (int t = lmax / 2; t >= 1; t /= 2)
    if (delta(key, sys, sys_start, n, i, i + (l + t) * d) > dmin) l += t;
  const int j = i + l * d;
  const int dnode = delta(key, sys, sys_start, n, i, j);
  int s = 0;
  for (int div = 2;; div *= 2) {
    int t = (l + div - 1) / div;
    if (delta(key, sys, sys_start, n, i, i + (s + t) * d) > dnode) s += t;
    if (t <= 1) break;
  }
  const int gamma = i + s * d + (d < 0 ? -1 : 0);
  const int first = min(i, j), last = max(i, j);
  const int left = (first == gamma) ? -(gamma + 1) : gamma;
  const int right = (last == gamma + 1) ? -(gamma + 2) : gamma + 1;
  kfirst[i] = first;
  klast[i] = last;
  kleft[i] = left;
  kright[i] = right;
  if (left >= 0) { kpar[left] = i; kside[left] = 0; }
  if (right >= 0) { kpar[right] = i; kside[right] = 1; }
  // a node over particles of two systems never becomes a leaf
  const bool spans = sys && sys[first] != sys[last];
  kept[i] = ((last - first + 1) > leaf_size || spans) ? 1u : 0u;
  if (i == 0) kpar[0] = -1;
}

// final node ids: root 0; the children of the kept internal node with
// compact index c sit at 1 + 2c (left) and 2 + 2c (right)
__device__ __forceinline__ int final_id(int i, const int32_t* kpar, const int32_t* kside,
                                        const uint32_t* cidx) {
  return i == 0 ? 0 : 1 + 2 * (int)cidx[kpar[i]] + kside[i];
}

__global__ void k_assign(int n, int leaf_size, const uint32_t* __restrict__ sys,
                         const int32_t* __restrict__ kfirst,
                         const int32_t* __restrict__ klast, const int32_t* __restrict__ kleft,
                         const int32_t* __restrict__ kright, const int32_t* __restrict__ kpar,
                         const int32_t* __restrict__ kside, const uint32_t* __restrict__ cidx,
                         NodeInfo* __restrict__ info, uint32_t* __restrict__ leaf_flag,
                         int32_t* __restrict__ leaf_at) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n - 1) return;
  const int first = kfirst[i], last = klast[i];
  const bool spans = sys && sys[first] != sys[last];
  if (last - first + 1 <= leaf_size && !spans) return;  // not a kept internal node
  const int me = final_id(i, kpar, kside, cidx);
  const int par = i == 0 ? -1 : final_id(kpar[i], kpar, kside, cidx);
  const int base = 1 + 2 * (int)cidx[i];
  NodeInfo ni;
  ni.lo = first; ni.cnt = last - first + 1; ni.child = base; ni.parent = par;
  info[me] = ni;
  const int ch[2] = {kleft[i], kright[i]};
  for (int side = 0; side < 2; ++side) {
    int c = ch[side], lo, cnt;
    if (c < 0) { lo = -c - 1; cnt = 1; }
    else { lo = kfirst[c]; cnt = klast[c] - kfirst[c] + 1; }
    const bool child_spans = sys && sys[lo] != sys[lo + cnt - 1];
    if (cnt <= leaf_size && !child_spans) {
      NodeInfo li;
      li.lo = lo; li.cnt = cnt; li.child = -1; li.parent = me;
      info[base + side] = li;
      leaf_flag[lo] = 1u;
      leaf_at[lo] = base + side;
    }
  }
}

__global__ void k_leaf_fill(int n, const uint32_t* __restrict__ leaf_flag,
                            const uint32_t* __restrict__ leaf_scan,
                            const int32_t* __restrict__ leaf_at, int32_t* __restrict__ leaf_node) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  if (leaf_flag[p]) leaf_node[leaf_scan[p]] = leaf_at[p];
}

__global__ void k_single_leaf(int n, NodeInfo* info, int32_t* leaf_node) {
  NodeInfo ni;
  ni.lo = 0; ni.cnt = n; ni.child = -1; ni.parent = -1;
  info[0] = ni;
  leaf_node[0] = 0;
}

// (node_depth: every node's depth, from the level grouping)
__global__ void k_leaf_depth(int nleaves, const int32_t* __restrict__ leaf_node,
                             const NodeInfo* __restrict__ info,
                             const int32_t* __restrict__ node_depth, int32_t* __restrict__ leaf_depth,
                             int32_t* __restrict__ p_leaf, int* maxdepth) {
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nleaves) return;
  const int node = leaf_node[l];
  const int d = node_depth[node];
  leaf_depth[l] = d;
  atomicMax(maxdepth, d);
  const NodeInfo ni = info[node];
  for (int p = ni.lo; p < ni.lo + ni.cnt; ++p) p_leaf[p] = l;
}

// ---- geometry, moments (bottom-up, one level after the other) --------------
// A leaf sums its particles in sorted order; an internal node combines its
// two children (children first: the deepest level comes first).
template <int P>
__device__ __forceinline__ void geom_node(int v, const NodeInfo* __restrict__ info,
                                          const double* __restrict__ xs,
                                          const double* __restrict__ ys,
                                          const double* __restrict__ zs,
                                          const double* __restrict__ ms,
                                          const double* __restrict__ hs, double* rec) {
  using E = Exp<P>;
  constexpr int NQ = E::NQ;
  constexpr int RS = rec_stride(P);
  const NodeInfo ni = info[v];
  double* r = rec + (int64_t)v * RS;
  double Q[NQ];
#pragma unroll
  for (int k = 0; k < NQ; ++k) Q[k] = 0.0;
  if (ni.child < 0) {
    double M = 0.0, S0 = 0.0, S1 = 0.0, S2 = 0.0, hm = 0.0;
    for (int j = ni.lo; j < ni.lo + ni.cnt; ++j) {
      const double mj = ms[j];
      M += mj;
      S0 += mj * xs[j];
      S1 += mj * ys[j];
      S2 += mj * zs[j];
      hm = fmax(hm, hs[j]);
    }
    const double s0 = S0 / M, s1 = S1 / M, s2 = S2 / M;
    double d2max = 0.0;
    for (int j = ni.lo; j < ni.lo + ni.cnt; ++j) {
      const double b[3] = {xs[j] - s0, ys[j] - s1, zs[j] - s2};
      const double d2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
      d2max = fmax(d2max, d2);
      E::p2m_add(b, ms[j], Q);
    }
    r[0] = s0; r[1] = s1; r[2] = s2; r[3] = sqrt(d2max); r[4] = hm; r[5] = M;
  } else {
    const double* rl = rec + (int64_t)ni.child * RS;
    const double* rr = rl + RS;
    const double ML = rl[5], MR = rr[5];
    const double M = ML + MR;
    double s[3];
    for (int d = 0; d < 3; ++d) s[d] = (ML * rl[d] + MR * rr[d]) / M;
    const double hm = fmax(rl[4], rr[4]);
    double Qc[NQ];
    {
      const double g[3] = {rl[0] - s[0], rl[1] - s[1], rl[2] - s[2]};
#pragma unroll
      for (int k = 0; k < NQ; ++k) Qc[k] = rl[8 + k];
      E::m2m_add(g, Qc, Q);
    }
    {
      const double g[3] = {rr[0] - s[0], rr[1] - s[1], rr[2] - s[2]};
#pragma unroll
      for (int k = 0; k < NQ; ++k) Qc[k] = rr[8 + k];
      E::m2m_add(g, Qc, Q);
    }
    r[0] = s[0]; r[1] = s[1]; r[2] = s[2]; r[4] = hm; r[5] = M;
  }
#pragma unroll
  for (int k = 0; k < NQ; ++k) r[8 + k] = Q[k];
}

// one level, a thread per node
template <int P>
__global__ void k_geom_level(const int32_t* __restrict__ level_nodes, uint32_t beg, uint32_t end,
                             const NodeInfo* __restrict__ info, const double* __restrict__ xs,
                             const double* __restrict__ ys, const double* __restrict__ zs,
                             const double* __restrict__ ms, const double* __restrict__ hs,
                             double* __restrict__ rec) {
  const uint32_t idx = beg + blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= end) return;
  geom_node<P>(level_nodes[idx], info, xs, ys, zs, ms, hs, rec);
}

// a run of small levels, deepest first, in one block: a barrier between
// levels makes the children's records (written by this block) visible
constexpr int GEOM_RUN_THREADS = 512;
constexpr uint32_t GEOM_RUN_MAX = 1024;  // nodes of a level that a run takes
template <int P>
__global__ __launch_bounds__(GEOM_RUN_THREADS) void k_geom_run(
    const int32_t* __restrict__ level_nodes, const uint32_t* __restrict__ level_off, int kdeep,
    int ktop, const NodeInfo* __restrict__ info, const double* __restrict__ xs,
    const double* __restrict__ ys, const double* __restrict__ zs, const double* __restrict__ ms,
    const double* __restrict__ hs, double* rec) {
  for (int k = kdeep; k >= ktop; --k) {
    const uint32_t beg = level_off[k], end = level_off[k + 1];
    for (uint32_t idx = beg + threadIdx.x; idx < end; idx += GEOM_RUN_THREADS)
      geom_node<P>(level_nodes[idx], info, xs, ys, zs, ms, hs, rec);
    __syncthreads();
  }
}

__global__ void k_extent_count(int nn, const NodeInfo* __restrict__ info,
                               uint32_t* __restrict__ chunks) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nn) return;
  const NodeInfo ni = info[v];
  chunks[v] = ni.child >= 0 ? (uint32_t)((ni.cnt + kExtentChunk - 1) / kExtentChunk) : 0u;
}

// one wave per chunk of an internal node: largest squared distance to the
// node's centre of mass, folded in with an integer max on the FP64 bits
// (non-negative doubles order like their bit patterns)
// the node of each chunk (thread per node)
__global__ void k_extent_map(int nn, int nitems, const uint32_t* __restrict__ chunk_off,
                             uint32_t* __restrict__ item_node) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nn) return;
  const uint32_t b = chunk_off[v], e = v + 1 < nn ? chunk_off[v + 1] : (uint32_t)nitems;
  for (uint32_t t = b; t < e; ++t) item_node[t] = (uint32_t)v;
}

template <int RS>
__global__ __launch_bounds__(256) void k_extent(int nn, int nitems, const NodeInfo* __restrict__ info,
                                                const uint32_t* __restrict__ chunk_off,
                                                const uint32_t* __restrict__ item_node,
                                                const double* __restrict__ xs,
                                                const double* __restrict__ ys,
                                                const double* __restrict__ zs,
                                                const double* __restrict__ rec,
                                                unsigned long long* l2bits) {
  const int item = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (item >= nitems) return;
  const int v = (int)item_node[item];
  const NodeInfo ni = info[v];
  const int c = item - (int)chunk_off[v];
  const int beg = ni.lo + c * kExtentChunk;
  const int end = min(ni.lo + ni.cnt, beg + kExtentChunk);
  const double s0 = rec[(int64_t)v * RS], s1 = rec[(int64_t)v * RS + 1], s2 = rec[(int64_t)v * RS + 2];
  double d2max = 0.0;
  for (int j = beg + lane; j < end; j += 64) {
    const double dx = xs[j] - s0, dy = ys[j] - s1, dz = zs[j] - s2;
    d2max = fmax(d2max, dx * dx + dy * dy + dz * dz);
  }
  d2max = wave_max(d2max);
  if (lane == 0) atomicMax(&l2bits[v], (unsigned long long)__double_as_longlong(d2max));
}

template <int RS>
__global__ void k_extent_final(int nn, const NodeInfo* __restrict__ info,
                               const unsigned long long* __restrict__ l2bits, double* rec) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nn) return;
  if (info[v].child < 0) return;
  rec[(int64_t)v * RS + 3] = sqrt(__longlong_as_double((long long)l2bits[v]));
}


}  // namespace

int bbox_blocks(int64_t n) {
  int64_t b = (n + BBOX_THREADS * 8 - 1) / (BBOX_THREADS * 8);
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return (int)b;
}

void launch_bbox(int n, const double* x, const double* m, const double* h, double* part,
                 double* box, int* status, int check, hipStream_t s) {
  int nb = bbox_blocks(n);
  k_bbox_partial<<<nb, BBOX_THREADS, 0, s>>>(n, x, m, h, part, status, check);
  k_bbox_final<<<1, 256, 0, s>>>(nb, part, box);
}

void launch_keys(int n, const double* x, const double* box, uint64_t* key, uint32_t* idx,
                 hipStream_t s) {
  k_keys<<<blocks_for(n, 256), 256, 0, s>>>(n, x, box, key, idx);
}

int radix_blocks(int64_t n) { return (int)((n + RS_TILE - 1) / RS_TILE); }

void radix_pass(int n, const uint64_t* kin, const uint32_t* vin, uint64_t* kout, uint32_t* vout,
                int shift, uint32_t* hist, uint32_t* hist_tmp, uint32_t* scratch_total,
                hipStream_t s) {
  const int nb = radix_blocks(n);
  k_radix_hist<<<nb, RS_THREADS, 0, s>>>(n, kin, shift, hist, nb);
  scan_u32(hist, hist, (int64_t)256 * nb, scratch_total, hist_tmp, s);
  k_radix_scatter<<<nb, RS_THREADS, 0, s>>>(n, kin, vin, kout, vout, shift, hist, nb);
}

void radix_sort(int n, uint64_t* key0, uint32_t* val0, uint64_t* key1, uint32_t* val1,
                uint32_t* hist, uint32_t* hist_tmp, uint32_t* scratch_total, hipStream_t s) {
  const int nb = radix_blocks(n);
  uint64_t *kin = key0, *kout = key1;
  uint32_t *vin = val0, *vout = val1;
  for (int shift = 0; shift < 64; shift += 8) {  // 8 passes: result lands in key0/val0
    k_radix_hist<<<nb, RS_THREADS, 0, s>>>(n, kin, shift, hist, nb);
    scan_u32(hist, hist, (int64_t)256 * nb, scratch_total, hist_tmp, s);
    k_radix_scatter<<<nb, RS_THREADS, 0, s>>>(n, kin, vin, kout, vout, shift, hist, nb);
    std::swap(kin, kout);
    std::swap(vin, vout);
  }
}

void launch_sys_keys(int n, int nsys, const int64_t* off, const double* x, const double* m,
                     const double* h, double* boxes, int* status, int check, uint64_t* key,
                     uint32_t* idx, uint32_t* sys, int32_t* sys_start, hipStream_t s) {
  k_bbox_sys<<<nsys, 256, 0, s>>>(off, x, m, h, boxes, status, check);
  k_keys_sys<<<blocks_for(n, 256), 256, 0, s>>>(n, nsys, off, x, boxes, key, idx, sys);
  k_sys_start<<<blocks_for(nsys, 256), 256, 0, s>>>(nsys, off, sys_start);
}

void launch_sys_sortkey(int n, const uint32_t* perm1, const uint32_t* sys, uint64_t* skey,
                        uint32_t* pos, hipStream_t s) {
  k_sys_sortkey<<<blocks_for(n, 256), 256, 0, s>>>(n, perm1, sys, skey, pos);
}

void launch_sys_final(int n, const uint32_t* q, const uint32_t* perm1, const uint64_t* key1,
                      const uint32_t* sys, uint32_t* perm, uint64_t* key, uint32_t* sys_sorted,
                      hipStream_t s) {
  k_sys_final<<<blocks_for(n, 256), 256, 0, s>>>(n, q, perm1, key1, sys, perm, key, sys_sorted);
}

void launch_node_flags(int nn, const NodeInfo* info, const uint32_t* sys, uint8_t* flag,
                       hipStream_t s) {
  k_node_flags<<<blocks_for(nn, 256), 256, 0, s>>>(nn, info, sys, flag);
}

void launch_gather(int n, const uint32_t* perm, const double* x, const double* m,
                   const double* h, double* xs, double* ys, double* zs, double* ms,
                   double* hs, double* his, double* p4, hipStream_t s) {
  k_gather<<<blocks_for(n, 256), 256, 0, s>>>(n, perm, x, m, h, xs, ys, zs, ms, hs, his, p4);
}

void launch_karras(int n, const uint64_t* key, const uint32_t* sys, const int32_t* sys_start,
                   int leaf_size, int32_t* kfirst, int32_t* klast, int32_t* kleft,
                   int32_t* kright, int32_t* kpar, int32_t* kside, uint32_t* kept, hipStream_t s) {
  k_karras<<<blocks_for(n - 1, 256), 256, 0, s>>>(n, key, sys, sys_start, leaf_size, kfirst, klast,
                                                  kleft, kright, kpar, kside, kept);
}

void launch_assign(int n, int leaf_size, const uint32_t* sys, const int32_t* kfirst,
                   const int32_t* klast, const int32_t* kleft, const int32_t* kright,
                   const int32_t* kpar, const int32_t* kside, const uint32_t* cidx, NodeInfo* info,
                   uint32_t* leaf_flag, int32_t* leaf_at, hipStream_t s) {
  k_assign<<<blocks_for(n - 1, 256), 256, 0, s>>>(n, leaf_size, sys, kfirst, klast, kleft, kright,
                                                  kpar, kside, cidx, info, leaf_flag, leaf_at);
}

void launch_leaf_fill(int n, const uint32_t* leaf_flag, const uint32_t* leaf_scan,
                      const int32_t* leaf_at, int32_t* leaf_node, hipStream_t s) {
  k_leaf_fill<<<blocks_for(n, 256), 256, 0, s>>>(n, leaf_flag, leaf_scan, leaf_at, leaf_node);
}

void launch_single_leaf(int n, NodeInfo* info, int32_t* leaf_node, hipStream_t s) {
  k_single_leaf<<<1, 1, 0, s>>>(n, info, leaf_node);
}

void launch_leaf_depth(int nleaves, const int32_t* leaf_node, const NodeInfo* info,
                       const int32_t* node_depth, int32_t* leaf_depth, int32_t* p_leaf,
                       int* maxdepth, hipStream_t s) {
  k_leaf_depth<<<blocks_for(nleaves, 256), 256, 0, s>>>(nleaves, leaf_node, info, node_depth,
                                                        leaf_depth, p_leaf, maxdepth);
}

template <int P>
void geometry_order(int maxdepth, const uint32_t* off_h, const uint32_t* off_d,
                    const int32_t* level_nodes, const NodeInfo* info, const double* xs,
                    const double* ys, const double* zs, const double* ms, const double* hs,
                    double* rec, hipStream_t s) {
  // runs of four or more consecutive levels of at most GEOM_RUN_MAX nodes
  // (the top of the tree) go to one block, the others one launch each
  int k = maxdepth;
  while (k >= 0) {
    const uint32_t size = off_h[k + 1] - off_h[k];
    if (size <= GEOM_RUN_MAX) {
      int top = k;
      while (top - 1 >= 0 && off_h[top] - off_h[top - 1] <= GEOM_RUN_MAX) --top;
      // (a run pays off from four levels on: one level in the block takes
      // about two thirds of a launch of its own)
      if (k - top >= 3) {
        k_geom_run<P><<<1, GEOM_RUN_THREADS, 0, s>>>(level_nodes, off_d, k, top, info, xs, ys,
                                                     zs, ms, hs, rec);
        k = top - 1;
        continue;
      }
    }
    if (size > 0)
      k_geom_level<P><<<blocks_for(size, 128), 128, 0, s>>>(level_nodes, off_h[k], off_h[k + 1],
                                                             info, xs, ys, zs, ms, hs, rec);
    --k;
  }
}

void launch_geometry(int order, int maxdepth, const uint32_t* level_off_host,
                     const uint32_t* level_off_dev, const int32_t* level_nodes,
                     const NodeInfo* info, const double* xs, const double* ys, const double* zs,
                     const double* ms, const double* hs, double* rec, hipStream_t s) {
  switch (order) {
#define GEOM_CASE(P)                                                                         \
  case P:                                                                                    \
    geometry_order<P>(maxdepth, level_off_host, level_off_dev, level_nodes, info, xs, ys, zs, \
                      ms, hs, rec, s);                                                       \
    break;
    GEOM_CASE(0) GEOM_CASE(1) GEOM_CASE(2) GEOM_CASE(3) GEOM_CASE(4)
#undef GEOM_CASE
  }
}

void launch_extent_count(int nn, const NodeInfo* info, uint32_t* chunks, hipStream_t s) {
  k_extent_count<<<blocks_for(nn, 256), 256, 0, s>>>(nn, info, chunks);
}

void launch_extent(int order, int nn, int nitems, const NodeInfo* info,
                   const uint32_t* chunk_off, uint32_t* item_node, const double* xs,
                   const double* ys, const double* zs, double* rec, unsigned long long* l2bits,
                   hipStream_t s) {
  if (nitems <= 0) return;
  k_extent_map<<<blocks_for(nn, 256), 256, 0, s>>>(nn, nitems, chunk_off, item_node);
  const unsigned nb = blocks_for(nitems, 4);
#define SFMM_EXTENT(RS) \
  k_extent<RS><<<nb, 256, 0, s>>>(nn, nitems, info, chunk_off, item_node, xs, ys, zs, rec, l2bits)
  switch (rec_stride(order)) {
    case 16: SFMM_EXTENT(16); break;
    case 24: SFMM_EXTENT(24); break;
    case 32: SFMM_EXTENT(32); break;
    case 48: SFMM_EXTENT(48); break;
  }
#undef SFMM_EXTENT
}

void launch_extent_final(int order, int nn, const NodeInfo* info,
                         const unsigned long long* l2bits, double* rec, hipStream_t s) {
  const unsigned nb = blocks_for(nn, 256);
  switch (rec_stride(order)) {
    case 16: k_extent_final<16><<<nb, 256, 0, s>>>(nn, info, l2bits, rec); break;
    case 24: k_extent_final<24><<<nb, 256, 0, s>>>(nn, info, l2bits, rec); break;
    case 32: k_extent_final<32><<<nb, 256, 0, s>>>(nn, info, l2bits, rec); break;
    case 48: k_extent_final<48><<<nb, 256, 0, s>>>(nn, info, l2bits, rec); break;
  }
}

}  // namespace sfmm
