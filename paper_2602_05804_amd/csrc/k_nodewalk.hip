// k_nodewalk.hip -- level-synchronous form of the dual tree walk.
//
// In Algorithm 1 (Sect. 3) every leaf walks from (root, root) down its own
// branch; the pairs a leaf tests against its ancestor p_k, and their outcome,
// depend only on p_k, so all leaves below p_k repeat them.  Here each node
// is visited once, level by level from the root:
//   tested(v) = expand(opened(parent(v)))   (a leaf source stays, an
//               internal source is replaced by its two children; for the
//               root, tested = {root})
// and each tested source is, as in Algorithm 2,
//   the node itself            -> opened
//   accepted (MAC + softening) -> M2L entry of v
//   otherwise                  -> opened
// An internal v hands its opened list to its children.  A leaf v lowers
// its opened sources in place: a leaf source becomes a P2P entry, an
// internal one is replaced by its children and tested against v again.
// The list of leaf L in Algorithm 1 is exactly the concatenation of the
// M2L lists of p_0 .. p_d plus L's P2P list (same pairs; the order inside a
// depth differs).
//
// One wave (a 64-thread block) per node; lanes take 64 sources at a time,
// and entries are written in lane order.  An internal node's M2L and opened
// lists together are its tested list, whose size its parent records while
// walking (opened leaves once, opened internal nodes twice).  So one region
// of the M2L pool holds both lists, M2L entries from the front and opened
// entries from the back, and its size is known before the node is walked:
// the region is the node's fixed slot, or a piece of an arena when larger.
// Each level is then one launch.  The leaves come after all levels, in one
// pass that writes each leaf's lists into fixed per-leaf slots (or a few
// large slots).  A second pass, at exact offsets, takes only the leaves that
// fit neither.
#include "sfmm_internal.h"

namespace sfmm {
namespace {

__device__ __forceinline__ bool accept(const double* __restrict__ rt, const double* __restrict__ rs,
                                       double theta2, double r_kern) {
  const double dx = rs[0] - rt[0];
  const double dy = rs[1] - rt[1];
  const double dz = rs[2] - rt[2];
  const double d2 = dx * dx + dy * dy + dz * dz;
  const double lsum = rt[3] + rs[3];
  const double hm = fmax(rt[4], rs[4]);
  const double rsum = lsum + r_kern * hm;
  return (lsum * lsum < theta2 * d2) && (d2 >= rsum * rsum);
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// exclusive prefix over the wave of a small non-negative count (< 8) and the
// wave total
__device__ __forceinline__ uint32_t wave_prefix(uint32_t c, uint32_t& total) {
  uint32_t pre = 0;
  total = 0;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const uint64_t m = __ballot((c >> b) & 1u);
    // set bits of m below this lane
    pre += __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u))
           << b;
    total += (uint32_t)__popcll(m) << b;
  }
  return pre;
}

__global__ void k_node_depth(int nn, const NodeInfo* __restrict__ info, int32_t* __restrict__ depth,
                             uint64_t* __restrict__ key, uint32_t* __restrict__ ids) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nn) return;
  int d = 0;
  for (int u = info[v].parent; u >= 0; u = info[u].parent) ++d;
  depth[v] = d;
  // grouped by depth, and within a depth the internal nodes first
  key[v] = (uint64_t)min(2 * d + (info[v].child < 0 ? 1 : 0), 255);
  ids[v] = (uint32_t)v;
}

// level k spans [level_off[k], level_off[k + 1]), its internal nodes
// [level_off[k], level_int[k]) (the scanned histogram of the sort keys)
__global__ void k_level_offsets(int nlev, int nb, int nn, const uint32_t* __restrict__ hist,
                                uint32_t* __restrict__ level_off, uint32_t* __restrict__ level_int) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > nlev) return;
  level_off[k] = k < nlev ? hist[(int64_t)(2 * k) * nb] : (uint32_t)nn;
  level_int[k] = k < nlev ? hist[(int64_t)(2 * k + 1) * nb] : (uint32_t)nn;
}

// ---- one level -----------------------------------------------------------------
struct Emit {
  // reserved bases (uniform, 64-bit) and running offsets
  uint64_t m2l_base, open_base, p2p_base;
  uint32_t m2l_run, open_run, p2p_run;
  // leaf P2P lists: pairs that may fall inside a kernel from the front,
  // pairs beyond both kernels (plain_run of them so far) from the back of
  // the leaf's p2p_total entries
  uint32_t plain_run, p2p_total;
  // internal node: opened entries go backwards from open_base - 1 (the end
  // of its region); exp_lane sums this lane's opened entries, an internal
  // one counted twice
  uint32_t exp_lane;
  // leaf: this lane's share of the particles of the P2P entries
  uint32_t src_lane;
  // leaf, slot mode: the sizes of the slots written, and the entries beyond
  // both kernels staged in LDS (in rank order) until the leaf's P2P count is
  // known, or in global memory (plain_g) once the leaf has a large slot
  uint32_t slot_m, slot_p;
  uint32_t* plain;
  uint32_t* plain_g;
  bool big_m, big_p;  // a large slot was asked for (M2L, P2P)
};

template <bool WRITE>
__device__ __forceinline__ void emit_lists(const NodeWalkArgs& a, Emit& e, uint32_t s0, uint32_t s1,
                                           uint32_t nm, uint32_t sel_m, uint32_t no,
                                           uint32_t sel_o, bool to_p2p) {
  // nm entries (first from s0 if sel_m & 1, then s1 if sel_m & 2) go to M2L;
  // no entries to the opened (or P2P) list likewise
  uint32_t tm, to;
  const uint32_t pm = wave_prefix(nm, tm);
  const uint32_t po = wave_prefix(no, to);
  if (WRITE) {
    uint64_t k = e.m2l_base + e.m2l_run + pm;
    if (sel_m & 1u) { if (k < a.m2l_cap) a.m2l_pool[k] = s0; ++k; }
    if (sel_m & 2u) { if (k < a.m2l_cap) a.m2l_pool[k] = s1; }
    if (to_p2p) {
      uint64_t q = e.p2p_base + e.p2p_run + po;
      if (sel_o & 1u) { if (q < a.p2p_cap) a.p2p_pool[q] = s0; ++q; }
      if (sel_o & 2u) { if (q < a.p2p_cap) a.p2p_pool[q] = s1; }
    } else {
      // rank from the end of the node's region (r < region <= open_base)
      uint32_t r = e.open_run + po;
      if (sel_o & 1u) {
        const uint64_t q = e.open_base - 1u - r;
        if (q < a.open_cap) a.open_pool[q] = s0;
        ++r;
      }
      if (sel_o & 2u) {
        const uint64_t q = e.open_base - 1u - r;
        if (q < a.open_cap) a.open_pool[q] = s1;
      }
    }
  }
  e.m2l_run += tm;
  if (to_p2p) e.p2p_run += to; else e.open_run += to;
}

// a leaf's lists: nm M2L entries (sel_m), np P2P entries that may need
// softening (sel_p) and nq P2P entries beyond both kernels (sel_q); the
// latter are written from the end of the leaf's range, so the P2P kernel
// meets the softened pairs first and the rest in whole chunks without them.
// W = kLeafExact writes at the leaf's exact offsets (its P2P count known);
// W = kLeafSlot writes the M2L and softening entries into the leaf's fixed
// slots as far as they fit and stages the others in LDS
constexpr int kLeafExact = 1;
constexpr int kLeafSlot = 2;

// slot mode: a leaf whose M2L list outgrows its slot moves it to one of the
// large slots (a.nbig of a.big_m entries after all slots), in one piece; with
// none left it keeps its slot (and is walked again afterwards)
__device__ __forceinline__ void promote_m2l(const NodeWalkArgs& a, Emit& e) {
  const uint32_t lane = threadIdx.x & 63;
  uint32_t b = 0;
  if (lane == 0) b = (uint32_t)atomicAdd(reinterpret_cast<unsigned long long*>(a.run + 8), 1ull);
  b = __builtin_amdgcn_readfirstlane(b);
  e.big_m = true;
  if (b >= a.nbig) return;
  const uint64_t nb = a.leaf_base + (uint64_t)a.nleaves * a.slot_m + (uint64_t)b * a.big_m;
  __threadfence();  // the wave's own slot entries, read back below
  for (uint32_t i = lane; i < e.m2l_run; i += 64)
    if (nb + i < a.m2l_cap && e.m2l_base + i < a.m2l_cap) a.m2l_pool[nb + i] = a.m2l_pool[e.m2l_base + i];
  e.m2l_base = nb;
  e.slot_m = a.big_m;
}

// the same for the P2P list: its entries that may need softening move to a
// large P2P slot, the staged ones to that slot's global staging area
__device__ __forceinline__ void promote_p2p(const NodeWalkArgs& a, Emit& e) {
  const uint32_t lane = threadIdx.x & 63;
  uint32_t b = 0;
  if (lane == 0) b = (uint32_t)atomicAdd(reinterpret_cast<unsigned long long*>(a.run + 9), 1ull);
  b = __builtin_amdgcn_readfirstlane(b);
  e.big_p = true;
  if (b >= a.nbig) return;
  const uint64_t nb = (uint64_t)a.nleaves * a.slot_p + (uint64_t)b * a.big_p;
  uint32_t* g = a.big_plain + (uint64_t)b * a.big_p;
  __syncthreads();  // the staged entries (LDS)
  __threadfence();  // the wave's own slot entries
  for (uint32_t i = lane; i < e.p2p_run; i += 64)
    if (nb + i < a.p2p_cap && e.p2p_base + i < a.p2p_cap) a.p2p_pool[nb + i] = a.p2p_pool[e.p2p_base + i];
  for (uint32_t i = lane; i < e.plain_run; i += 64) g[i] = e.plain[i];
  e.p2p_base = nb;
  e.slot_p = a.big_p;
  e.plain_g = g;
}

template <int W>
__device__ __forceinline__ void emit_leaf_lists(const NodeWalkArgs& a, Emit& e, uint32_t s0,
                                                uint32_t s1, uint32_t nm, uint32_t sel_m,
                                                uint32_t np, uint32_t sel_p, uint32_t nq,
                                                uint32_t sel_q) {
  uint32_t tm, tp, tq;
  const uint32_t pm = wave_prefix(nm, tm);
  const uint32_t pp = wave_prefix(np, tp);
  const uint32_t pq = wave_prefix(nq, tq);
  if (W == kLeafSlot) {
    // (uniform tests: the wave's totals)
    if (!e.big_m && e.m2l_run + tm > e.slot_m) promote_m2l(a, e);
    if (!e.big_p && e.p2p_run + tp + e.plain_run + tq > e.slot_p) promote_p2p(a, e);
    uint32_t k = e.m2l_run + pm;
    if (sel_m & 1u) { if (k < e.slot_m && e.m2l_base + k < a.m2l_cap) a.m2l_pool[e.m2l_base + k] = s0; ++k; }
    if (sel_m & 2u) { if (k < e.slot_m && e.m2l_base + k < a.m2l_cap) a.m2l_pool[e.m2l_base + k] = s1; }
    uint32_t q = e.p2p_run + pp;
    if (sel_p & 1u) { if (q < e.slot_p && e.p2p_base + q < a.p2p_cap) a.p2p_pool[e.p2p_base + q] = s0; ++q; }
    if (sel_p & 2u) { if (q < e.slot_p && e.p2p_base + q < a.p2p_cap) a.p2p_pool[e.p2p_base + q] = s1; }
    uint32_t r = e.plain_run + pq;
    uint32_t* pl = e.plain_g ? e.plain_g : e.plain;
    if (sel_q & 1u) { if (r < e.slot_p) pl[r] = s0; ++r; }
    if (sel_q & 2u) { if (r < e.slot_p) pl[r] = s1; }
  }
  if (W == kLeafExact) {
    uint64_t k = e.m2l_base + e.m2l_run + pm;
    if (sel_m & 1u) { if (k < a.m2l_cap) a.m2l_pool[k] = s0; ++k; }
    if (sel_m & 2u) { if (k < a.m2l_cap) a.m2l_pool[k] = s1; }
    uint64_t q = e.p2p_base + e.p2p_run + pp;
    if (sel_p & 1u) { if (q < a.p2p_cap) a.p2p_pool[q] = s0; ++q; }
    if (sel_p & 2u) { if (q < a.p2p_cap) a.p2p_pool[q] = s1; }
    uint32_t r = e.plain_run + pq;  // rank from the back
    for (int b = 0; b < 2; ++b) {
      if (!(sel_q & (1u << b))) continue;
      if (r < e.p2p_total) {
        const uint64_t t = e.p2p_base + (e.p2p_total - 1u - r);
        if (t < a.p2p_cap) a.p2p_pool[t] = b ? s1 : s0;
      }
      ++r;
    }
  }
  e.m2l_run += tm;
  e.p2p_run += tp;
  e.plain_run += tq;
}

// classification of one tested source against target v
// returns 0 = M2L, 1 = opened (no branches: the self pair is selected out)
__device__ __forceinline__ int classify(const NodeWalkArgs& a, int v, const double* rv, uint32_t s) {
  const bool acc = accept(rv, a.rec + (int64_t)s * a.stride, a.theta2, a.r_kern);
  return ((int)s != v && acc) ? 0 : 1;
}

// the same test for a leaf target, from one evaluation of d^2: 0 = M2L,
// 1 = opened (or P2P that may need softening), 2 = opened although beyond
// both kernels (only the opening angle failed; a P2P pair of leaves then
// needs no softening), 3 = opened, and every node below s would fail the
// softening test against v too: s lies inside v's own kernel reach,
// d + l_s < l_v + R_kern h_max(v) (any node below s has its centre within
// l_s of s's and h_max >= 0), so the lowering would end with all of s's
// leaves as P2P sources; the margin keeps rounding in the tests the
// lowering would make from deciding otherwise
__device__ __forceinline__ int classify3(const NodeWalkArgs& a, int v, const double* rv,
                                         uint32_t s) {
  const double* rs = a.rec + (int64_t)s * a.stride;
  const double dx = rs[0] - rv[0];
  const double dy = rs[1] - rv[1];
  const double dz = rs[2] - rv[2];
  const double d2 = dx * dx + dy * dy + dz * dz;
  const double lsum = rv[3] + rs[3];
  const double rsum = lsum + a.r_kern * fmax(rv[4], rs[4]);
  const double reach = rv[3] + a.r_kern * rv[4] - rs[3];
  const bool beyond = d2 >= rsum * rsum;
  const bool whole = reach > 0.0 && d2 < reach * reach * (1.0 - 1e-9);
  const bool mac = lsum * lsum < a.theta2 * d2;
  const int k = beyond ? (mac ? 0 : 2) : (whole ? 3 : 1);
  return (int)s == v ? 1 : k;  // selects, no branches
}

// internal target: the tested sources, 64 * kWalkBatch at a time; every
// load of a batch (list entries, then children, then records) is issued
// before the classification, so a node waits for one chain of dependent
// loads per batch instead of one per 64 sources; entries are emitted in
// the order of the tested list
constexpr int kWalkBatch = 4;

template <bool WRITE>
__device__ void walk_internal(const NodeWalkArgs& a, int v, const double* rv, const uint32_t* src,
                              uint32_t nsrc, Emit& e) {
  const uint32_t lane = threadIdx.x & 63;
  for (uint32_t base = 0; base < nsrc; base += 64 * kWalkBatch) {
    uint32_t sb[kWalkBatch];
#pragma unroll
    for (int u = 0; u < kWalkBatch; ++u) {
      const uint32_t i = base + 64u * u + lane;
      sb[u] = i < nsrc ? src[i] : 0xffffffffu;
    }
    // invalid slots read node v (a valid index) and are masked afterwards,
    // so the loads and tests need no branches
    int cb[kWalkBatch];
#pragma unroll
    for (int u = 0; u < kWalkBatch; ++u) {
      const bool ok = sb[u] != 0xffffffffu;
      cb[u] = a.info[ok ? sb[u] : (uint32_t)v].child;
      if (!ok) cb[u] = -2;
    }
    uint32_t selm[kWalkBatch], selo[kWalkBatch], nm[kWalkBatch], no[kWalkBatch];
    uint32_t t0[kWalkBatch], t1[kWalkBatch];
#pragma unroll
    for (int u = 0; u < kWalkBatch; ++u) {
      const bool ok = cb[u] != -2;
      const bool two = cb[u] >= 0;
      t0[u] = two ? (uint32_t)cb[u] : (ok ? sb[u] : (uint32_t)v);
      t1[u] = two ? (uint32_t)cb[u] + 1u : (uint32_t)v;
      const bool m0 = classify(a, v, rv, t0[u]) == 0;
      const bool m1 = classify(a, v, rv, t1[u]) == 0;
      const uint32_t v0 = ok ? 1u : 0u, v1 = two ? 1u : 0u;
      selm[u] = (m0 ? v0 : 0u) | ((m1 ? v1 : 0u) << 1);
      selo[u] = (m0 ? 0u : v0) | ((m1 ? 0u : v1) << 1);
      nm[u] = (m0 ? v0 : 0u) + (m1 ? v1 : 0u);
      no[u] = (m0 ? 0u : v0) + (m1 ? 0u : v1);
      // the children's tested list: an opened leaf once, an internal node twice
      const uint32_t x0 = a.info[t0[u]].child >= 0 ? 2u : 1u;
      const uint32_t x1 = a.info[t1[u]].child >= 0 ? 2u : 1u;
      e.exp_lane += ((selo[u] & 1u) ? x0 : 0u) + ((selo[u] & 2u) ? x1 : 0u);
    }
#pragma unroll
    for (int u = 0; u < kWalkBatch; ++u) {
      if (base + 64u * u >= nsrc) break;  // uniform
      emit_lists<WRITE>(a, e, t0[u], t1[u], nm[u], selm[u], no[u], selo[u], false);
    }
  }
}

// leaf target: U groups of 64 tested sources per step (all their loads
// issued before the classification); opened internal sources are pushed on
// the lowering stack (in LDS), which is drained 64 entries per step after
// each batch of the tested list, so the stack stays within a few chunks per
// tree level.  Returns false when the stack would overflow (the walk is then
// rerun with a larger stack).
template <int W, int U>
__device__ __forceinline__ bool leaf_step(const NodeWalkArgs& a, int v, const double* rv,
                                          const uint32_t (&t0)[U], const uint32_t (&t1)[U],
                                          const int (&nt)[U], Emit& e, uint32_t* stk,
                                          uint32_t& sp) {
  int kk[U][2], cc[U][2], pc[U][2];
#pragma unroll
  for (int u = 0; u < U; ++u) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const bool valid = q < nt[u];
      const uint32_t t = valid ? (q ? t1[u] : t0[u]) : (uint32_t)v;  // a valid index
      const int k = classify3(a, v, rv, t);
      const NodeInfo ti = a.info[t];
      kk[u][q] = valid ? k : -1;
      cc[u][q] = valid ? ti.child : 0;
      pc[u][q] = ti.cnt;
    }
  }
  bool ok = true;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    uint32_t selm = 0, selp = 0, selq = 0, nm = 0, np = 0, nq = 0;
    bool open0 = false, open1 = false;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int k = kk[u][q];
      if (k < 0) continue;
      if (k == 0) { selm |= 1u << q; ++nm; continue; }
      if (cc[u][q] < 0 || k == 3) {
        // a leaf, or a whole subtree of P2P sources kept as one entry
        if (k == 2) { selq |= 1u << q; ++nq; }
        else { selp |= 1u << q; ++np; }
        e.src_lane += (uint32_t)pc[u][q];
      } else {
        if (q) open1 = true; else open0 = true;
      }
    }
    emit_leaf_lists<W>(a, e, t0[u], t1[u], nm, selm, np, selp, nq, selq);
    const uint32_t npush = (open0 ? 2u : 0u) + (open1 ? 2u : 0u);
    uint32_t tpush;
    const uint32_t pp = wave_prefix(npush, tpush);
    if (!ok || sp + tpush > a.stack_cap) { ok = false; continue; }  // uniform
    uint32_t w = sp + pp;
    if (open0) { stk[w] = (uint32_t)cc[u][0]; stk[w + 1] = (uint32_t)cc[u][0] + 1u; w += 2; }
    if (open1) { stk[w] = (uint32_t)cc[u][1]; stk[w + 1] = (uint32_t)cc[u][1] + 1u; }
    sp += tpush;
  }
  __syncthreads();
  return ok;
}

template <int W>
__device__ void walk_leaf(const NodeWalkArgs& a, int v, const double* rv, const uint32_t* src,
                          uint32_t nsrc, bool root, Emit& e, uint32_t* stk, int* status) {
  // three groups of 64 tested sources per step: the leaf kernels then fit
  // 128 registers (four waves per SIMD for this latency-bound walk; four
  // groups took 137 and left three)
  constexpr int U = 3;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t n0 = root ? 1u : nsrc;
  uint32_t sp = 0;
  bool ok = true;
  for (uint32_t base = 0; base < n0 && ok; base += 64 * U) {
    uint32_t sb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t i = base + 64u * u + lane;
      sb[u] = i < n0 ? (root ? (uint32_t)v : src[i]) : 0xffffffffu;
    }
    int cb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) cb[u] = (sb[u] != 0xffffffffu && !root) ? a.info[sb[u]].child : -1;
    uint32_t t0[U], t1[U];
    int nt[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      t0[u] = t1[u] = 0;
      nt[u] = 0;
      if (sb[u] == 0xffffffffu) continue;
      if (cb[u] < 0) { t0[u] = sb[u]; nt[u] = 1; }
      else { t0[u] = (uint32_t)cb[u]; t1[u] = (uint32_t)cb[u] + 1u; nt[u] = 2; }
    }
    ok = leaf_step<W, U>(a, v, rv, t0, t1, nt, e, stk, sp);
    // the stack is drained U groups of 64 at a time while it holds more than
    // one group and has room for what they may push (2 per entry), else one
    // group at a time (the leaves with the longest lists lower deep stacks,
    // and their walks set the pass's time)
    while (ok && sp > 0) {
      const uint32_t kw = sp < 64u * U ? sp : 64u * U;
      if (sp > 64u && sp + kw <= a.stack_cap) {  // (uniform)
        uint32_t d0[U], d1[U];
        int dn[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          d1[u] = 0;
          dn[u] = 64u * u + lane < kw ? 1 : 0;
          d0[u] = dn[u] ? stk[sp - kw + 64u * u + lane] : 0u;
        }
        __syncthreads();
        sp -= kw;
        ok = leaf_step<W, U>(a, v, rv, d0, d1, dn, e, stk, sp);
      } else {
        const uint32_t k = sp < 64u ? sp : 64u;
        uint32_t d0[1] = {0}, d1[1] = {0};
        int dn[1] = {lane < k ? 1 : 0};
        if (dn[0]) d0[0] = stk[sp - k + lane];
        __syncthreads();
        sp -= k;
        ok = leaf_step<W, 1>(a, v, rv, d0, d1, dn, e, stk, sp);
      }
    }
  }
  if (!ok && lane == 0) atomicOr(status, ST_OVERFLOW);
}

// ---- internal nodes, level by level ---------------------------------------
// The M2L pool region of an internal node is its tested list (1 for a root,
// else exp[parent]), known before the node is walked: the node's fixed slot
// of int_slot entries (by its rank among the internal nodes), or for a
// larger region a piece of the arena of int_big entries after all slots
// (run[0] entries of it taken, by run[10] nodes).  Leaves take no room at
// their level (they are walked after all levels); a node over two systems
// gets empty lists.
__global__ __launch_bounds__(64) void k_nodewalk_internal(NodeWalkArgs a, int level, uint32_t rank0) {
  const uint32_t beg = a.level_off[level], end = a.level_int[level];
  const uint32_t b = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t idx = beg + b;
  if (idx >= end) return;
  const int v = a.level_nodes[idx];
  const NodeInfo vi = a.info[v];
  // a node over two systems (several systems solved together) is never
  // walked; the walk of each system starts at its own root
  const int flag = a.node_flag ? (int)a.node_flag[v] : (vi.parent < 0 ? 1 : 2);
  const uint32_t lane = threadIdx.x & 63;
  if (flag == 0) {
    if (lane == 0) {
      a.m2l_cnt[v] = 0; a.open_cnt[v] = 0; a.p2p_cnt[v] = 0;
      a.m2l_off[v] = 0; a.open_off[v] = 0; a.p2p_off[v] = 0;
    }
    return;
  }
  if (vi.child < 0) return;  // (the level's internal nodes come first)
  if (lane == 0) { a.p2p_cnt[v] = 0; a.p2p_off[v] = 0; }
  const bool root = flag == 1;
  const double* rv = a.rec + (int64_t)v * a.stride;
  const uint32_t region = root ? 1u : a.exp[vi.parent];
  Emit e{};
  bool fits = true;
  if (region <= a.int_slot) {
    e.m2l_base = (uint64_t)(rank0 + b) * a.int_slot;
  } else {
    uint64_t t = 0;
    if (lane == 0) {
      t = atomicAdd(reinterpret_cast<unsigned long long*>(a.run), (unsigned long long)region);
      atomicAdd(reinterpret_cast<unsigned long long*>(a.run + 10), 1ull);
    }
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)t);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(t >> 32));
    t = ((uint64_t)hi << 32) | lo;
    e.m2l_base = (uint64_t)a.int_nodes * a.int_slot + t;
    fits = t + region <= a.int_big;
  }
  e.open_base = e.m2l_base + region;
  // a region that does not fit gets no offset (the walk goes on counting,
  // the host grows the pool and walks again)
  fits = fits && e.open_base <= a.m2l_cap;
  if (lane == 0) a.m2l_off[v] = fits ? (uint32_t)e.m2l_base : kNoList;
  if (root) {
    // (root, root) is opened: both root children meet both root children
    if (lane == 0) {
      if (fits) a.open_pool[e.m2l_base] = (uint32_t)v;
      a.m2l_cnt[v] = 0;
      a.open_cnt[v] = 1;
      a.open_off[v] = fits ? (uint32_t)e.m2l_base : kNoList;
      a.exp[v] = 2;
    }
    return;
  }
  const uint32_t po = a.open_off[vi.parent];
  uint32_t nsrc = a.open_cnt[vi.parent];
  if ((uint64_t)po + nsrc > a.open_cap) nsrc = 0;  // pool too small: the walk is rerun
  walk_internal<true>(a, v, rv, a.open_pool + po, nsrc, e);
  uint32_t ex = e.exp_lane;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) ex += (uint32_t)__shfl_xor((int)ex, o, 64);
  if (lane == 0) {
    a.m2l_cnt[v] = e.m2l_run;
    a.open_cnt[v] = e.open_run;
    a.open_off[v] = fits ? (uint32_t)(e.open_base - e.open_run) : kNoList;
    a.exp[v] = ex;
  }
}

// ---- leaves, all levels at once ---------------------------------------------
// A leaf's lists depend only on its parent's opened list, so the leaves are
// walked after every level's internal nodes, in leaf order (one wave per
// leaf).  One pass writes each leaf's lists into fixed slots (slot_m M2L
// entries per leaf after the internal nodes' regions in the M2L pool, slot_p
// P2P entries per leaf at the front of the P2P pool).  A leaf whose lists do
// not fit its slots is listed (in one of kXcds lists by its leaf range,
// run[11 + range] of them) and walked again by a second
// pass, which writes its lists after all slots, at offsets from scans of
// such leaves' counts.
template <bool OVF>
__device__ void leaf_lists(const NodeWalkArgs& a, int l, uint32_t* stk) {
  const int v = a.leaf_node[l];
  const NodeInfo vi = a.info[v];
  const int flag = a.node_flag ? (int)a.node_flag[v] : (vi.parent < 0 ? 1 : 2);
  const uint32_t lane = threadIdx.x & 63;
  if (flag == 0) {  // (a leaf never spans two systems; kept for safety)
    if (lane == 0) {
      a.m2l_cnt[v] = 0; a.open_cnt[v] = 0; a.p2p_cnt[v] = 0;
      a.m2l_off[v] = 0; a.open_off[v] = 0; a.p2p_off[v] = 0;
      a.leaf_m2l_cnt[l] = 0; a.leaf_p2p_cnt[l] = 0;
      a.src_total[l] = 0; a.item_cnt[l] = 1;
    }
    return;
  }
  const bool root = flag == 1;
  const double* rv = a.rec + (int64_t)v * a.stride;
  const uint32_t* src = nullptr;
  uint32_t nsrc = 0;
  if (!root) {
    const uint32_t po = a.open_off[vi.parent];
    nsrc = a.open_cnt[vi.parent];
    src = a.open_pool + po;
    if ((uint64_t)po + nsrc > a.open_cap) nsrc = 0;  // pool too small: the walk is rerun
  }
  const uint64_t nl = (uint64_t)a.nleaves;
  Emit e{};
  if (OVF) {
    e.m2l_base = a.leaf_base + nl * a.slot_m + (uint64_t)a.nbig * a.big_m + a.leaf_m2l_off[l];
    e.p2p_base = nl * a.slot_p + (uint64_t)a.nbig * a.big_p + a.leaf_p2p_off[l];
    e.p2p_total = a.p2p_cnt[v];  // from the first pass
    if (lane == 0) {
      const bool fm = e.m2l_base + a.m2l_cnt[v] <= a.m2l_cap;
      const bool fp = e.p2p_base + e.p2p_total <= a.p2p_cap;
      a.m2l_off[v] = fm ? (uint32_t)e.m2l_base : kNoList;
      a.p2p_off[v] = fp ? (uint32_t)e.p2p_base : kNoList;
    }
    walk_leaf<kLeafExact>(a, v, rv, src, nsrc, root, e, stk, a.status);
    __syncthreads();  // (the stack is reused by the wave's next leaf)
    return;
  }
  e.m2l_base = a.leaf_base + (uint64_t)l * a.slot_m;
  e.p2p_base = (uint64_t)l * a.slot_p;
  e.slot_m = a.slot_m;
  e.slot_p = a.slot_p;
  e.plain = stk + a.stack_cap;
  walk_leaf<kLeafSlot>(a, v, rv, src, nsrc, root, e, stk, a.status);
  uint32_t ns = e.src_lane;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) ns += (uint32_t)__shfl_xor((int)ns, o, 64);
  const uint32_t nm = e.m2l_run, np = e.p2p_run, nq = e.plain_run;
  const bool fits = nm <= e.slot_m && np + nq <= e.slot_p;  // uniform
  __syncthreads();  // the staged entries are complete
  if (e.plain_g) __threadfence();  // (staged in global memory by this wave)
  if (fits) {
    // the entries beyond both kernels after the others, in reverse rank
    // order (as the exact pass writes them)
    const uint32_t* pl = e.plain_g ? e.plain_g : e.plain;
    for (uint32_t i = lane; i < nq; i += 64) {
      const uint64_t t = e.p2p_base + np + i;
      if (t < a.p2p_cap) a.p2p_pool[t] = pl[nq - 1u - i];
    }
  }
  if (lane == 0) {
    a.m2l_cnt[v] = nm;
    a.p2p_cnt[v] = np + nq;
    a.open_cnt[v] = 0;
    a.open_off[v] = 0;
    if (fits) {
      a.m2l_off[v] = e.m2l_base + nm <= a.m2l_cap ? (uint32_t)e.m2l_base : kNoList;
      a.p2p_off[v] = e.p2p_base + np + nq <= a.p2p_cap ? (uint32_t)e.p2p_base : kNoList;
    } else {
      // (the list of its range of leaves, the range this XCD walks here and
      // walks again in the second pass: its lists' sources stay in its L2)
      const uint32_t seg = ((uint32_t)a.nleaves + kXcds - 1) / kXcds;
      const uint32_t part = (uint32_t)l / seg;
      const unsigned long long k =
          atomicAdd(reinterpret_cast<unsigned long long*>(a.run + 11 + part), 1ull);
      a.ovf_leaf[(uint64_t)part * seg + k] = (uint32_t)l;
    }
    // lists left for the second pass (none when they fit)
    a.leaf_m2l_cnt[l] = fits ? 0u : nm;
    a.leaf_p2p_cnt[l] = fits ? 0u : np + nq;
    // P2P work items of the leaf: runs of at most kP2PItem source particles
    a.src_total[l] = ns;
    const uint32_t k = (ns + kP2PItem - 1) / kP2PItem;
    a.item_cnt[l] = k > 0 ? k : 1u;
  }
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_nodewalk_leaves(NodeWalkArgs a) {
  extern __shared__ uint32_t stk[];
  const int l = (int)xcd_block(blockIdx.x, gridDim.x);
  if (l < a.nleaves) leaf_lists<false>(a, l, stk);
}

// the second pass: a fixed grid of waves takes the listed leaves in turn
constexpr unsigned kOvfWaves = 4096;

__global__ __launch_bounds__(64) void k_nodewalk_leaves_ovf(NodeWalkArgs a) {
  extern __shared__ uint32_t stk[];
  // block b runs on XCD b % kXcds (the hardware's round-robin) and takes
  // that range's list
  const uint32_t part = blockIdx.x % kXcds, stride = gridDim.x / kXcds;
  const uint32_t seg = ((uint32_t)a.nleaves + kXcds - 1) / kXcds;
  const uint64_t nov = a.run[11 + part];
  for (uint64_t i = blockIdx.x / kXcds; i < nov; i += stride)
    leaf_lists<true>(a, (int)a.ovf_leaf[(uint64_t)part * seg + i], stk);
}

__global__ void k_leaf_stats(LeafStatArgs a) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= a.nleaves) return;
  const int leaf = a.leaf_node[l];
  const int d = a.leaf_depth[l];
  const NodeInfo li = a.info[leaf];
  int v = 0;
  uint64_t m2l = a.m2l_cnt[0];
  int kfirst = m2l > 0 ? 0 : -1;
  for (int k = 1; k <= d; ++k) {
    const int c = a.info[v].child;
    v = (li.lo < a.info[c + 1].lo) ? c : c + 1;
    const uint32_t mc = a.m2l_cnt[v];
    if (mc > 0 && kfirst < 0) kfirst = k;
    m2l += mc;
  }
  uint64_t src = 0;
  const uint32_t off = a.p2p_off[leaf], cnt = a.p2p_cnt[leaf];
  for (uint32_t q = 0; q < cnt; ++q) src += (uint64_t)a.info[a.p2p_pool[off + q]].cnt;
  a.m2l[l] = m2l;
  a.l2l[l] = kfirst < 0 ? 0u : (uint64_t)(d - kfirst);
  a.pairs[l] = src * (uint64_t)li.cnt - (uint64_t)li.cnt;
}

// one thread per node: the lists a consumer reads (M2L of every node, P2P
// of every leaf) must lie inside the part of the pools this walk wrote, and
// (check_entries) hold only node ids below nn.  Also the walk's totals:
// run[1] += M2L entries, run[4] += P2P entries, run[6] / run[7] = max with
// the longest M2L / P2P list of a leaf.
template <bool ENTRIES>
__global__ __launch_bounds__(256) void k_check_lists(NodeWalkArgs a, int nn) {
  __shared__ uint64_t red[4][4];
  const uint64_t nl = (uint64_t)a.nleaves;
  const uint64_t used_m = a.leaf_base + nl * a.slot_m + (uint64_t)a.nbig * a.big_m + a.run[3];
  const uint64_t used_p = nl * a.slot_p + (uint64_t)a.nbig * a.big_p + a.run[2];
  const uint64_t lim_m = used_m < a.m2l_cap ? used_m : a.m2l_cap;
  const uint64_t lim_p = used_p < a.p2p_cap ? used_p : a.p2p_cap;
  bool bad = false;
  uint64_t sm = 0, sp = 0, xm = 0, xp = 0;
  // (a grid of a few blocks, so that few atomics meet at the totals)
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < nn; v += gridDim.x * blockDim.x) {
    const uint32_t mc = a.m2l_cnt[v];
    sm += mc;
    if (mc > 0) {
      const uint64_t off = a.m2l_off[v];
      if (off + mc > lim_m) bad = true;
      else if (ENTRIES)
        for (uint32_t k = 0; k < mc; ++k) bad |= (a.m2l_pool[off + k] & kSrcMask) >= (uint32_t)nn;
    }
    if (a.info[v].child < 0) {
      const uint32_t pc = a.p2p_cnt[v];
      sp += pc;
      xm = max(xm, (uint64_t)mc);
      xp = max(xp, (uint64_t)pc);
      if (pc > 0) {
        const uint64_t off = a.p2p_off[v];
        if (off + pc > lim_p) bad = true;
        else if (ENTRIES)
          for (uint32_t k = 0; k < pc; ++k) bad |= a.p2p_pool[off + k] >= (uint32_t)nn;
      }
    }
  }
  if (bad) atomicOr(a.status, ST_BADLIST);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    sm += __shfl_xor(sm, o, 64);
    sp += __shfl_xor(sp, o, 64);
    xm = max(xm, (uint64_t)__shfl_xor(xm, o, 64));
    xp = max(xp, (uint64_t)__shfl_xor(xp, o, 64));
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { red[0][w] = sm; red[1][w] = sp; red[2][w] = xm; red[3][w] = xp; }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t[4] = {red[0][0], red[1][0], red[2][0], red[3][0]};
    for (int k = 1; k < 4; ++k) {
      t[0] += red[0][k]; t[1] += red[1][k];
      t[2] = max(t[2], red[2][k]); t[3] = max(t[3], red[3][k]);
    }
    auto* run = reinterpret_cast<unsigned long long*>(a.run);
    if (t[0]) atomicAdd(run + 1, (unsigned long long)t[0]);
    if (t[1]) atomicAdd(run + 4, (unsigned long long)t[1]);
    if (t[2]) atomicMax(run + 6, (unsigned long long)t[2]);
    if (t[3]) atomicMax(run + 7, (unsigned long long)t[3]);
  }
}

}  // namespace

void launch_check_lists(const NodeWalkArgs& a, int nn, bool check_entries, hipStream_t s) {
  if (nn <= 0) return;
  const unsigned nb = std::min<unsigned>(128, blocks_for(nn, 256));
  if (check_entries) k_check_lists<true><<<nb, 256, 0, s>>>(a, nn);
  else k_check_lists<false><<<nb, 256, 0, s>>>(a, nn);
}

void launch_leaf_stats(const LeafStatArgs& a, hipStream_t s) {
  if (a.nleaves <= 0) return;
  k_leaf_stats<<<(a.nleaves + 127) / 128, 128, 0, s>>>(a);
}

void launch_node_depth(int nn, const NodeInfo* info, int32_t* depth, uint64_t* key,
                       uint32_t* ids, hipStream_t s) {
  k_node_depth<<<(nn + 255) / 256, 256, 0, s>>>(nn, info, depth, key, ids);
}

void launch_level_offsets(int nlev, int nb, int nn, const uint32_t* hist_scanned,
                          uint32_t* level_off, uint32_t* level_int, hipStream_t s) {
  k_level_offsets<<<(nlev + 1 + 255) / 256, 256, 0, s>>>(nlev, nb, nn, hist_scanned, level_off,
                                                          level_int);
}

void launch_nodewalk_level(const NodeWalkArgs& a, int level, int nodes_in_level, uint32_t rank0,
                           hipStream_t s) {
  // (nodes_in_level: the level's internal nodes, rank0 those of the levels above)
  if (nodes_in_level <= 0) return;
  k_nodewalk_internal<<<nodes_in_level, 64, 0, s>>>(a, level, rank0);
}

void launch_nodewalk_leaves(const NodeWalkArgs& a, uint32_t* scan_tmp, hipStream_t s) {
  if (a.nleaves <= 0) return;
  const size_t lds = a.stack_cap * sizeof(uint32_t);
  k_nodewalk_leaves<<<a.nleaves, 64, lds + a.slot_p * sizeof(uint32_t), s>>>(a);
  scan_u32_u64(a.leaf_m2l_cnt, a.leaf_m2l_off, a.nleaves, a.run + 3,
               reinterpret_cast<uint64_t*>(scan_tmp), s);
  scan_u32_u64(a.leaf_p2p_cnt, a.leaf_p2p_off, a.nleaves, a.run + 2,
               reinterpret_cast<uint64_t*>(scan_tmp), s);
  // P2P work items: item_off[nleaves] = their total (read back with the walk's)
  scan_u32(a.item_cnt, a.item_off, a.nleaves, a.item_off + a.nleaves, scan_tmp, s);
  const unsigned ng = std::min<unsigned>(kOvfWaves, ((unsigned)a.nleaves + kXcds - 1) / kXcds * kXcds);
  k_nodewalk_leaves_ovf<<<ng, 64, lds, s>>>(a);
}

}  // namespace sfmm
