// k_far.hip -- far field of each leaf: M2L on every ancestor, the L2L chain
// down the branch and L2P at the leaf's particles (Sect. 2.2, Algorithm 1,
// Appendix A.2).
//
// A group of SPLIT lanes per leaf.  The leaf's M2L list is grouped by the
// depth of the target ancestor; the lanes of the group take every SPLIT-th
// entry of each depth and keep a partial local expansion in registers: at
// depth k it is re-centred from p_{k-1} to p_k (exact for the polynomial)
// and the lane's M2L terms for p_k are added.  Re-centring is linear, so the
// group's partial expansions are summed at the leaf and evaluated at its
// particles.  Every leaf still evaluates all M2L interactions of all of its
// ancestors.  Neighbouring leaves (Morton order) share their upper
// ancestors, so lanes mostly read the same source records.
#include <algorithm>

#include "sfmm_internal.h"

namespace sfmm {
namespace {

template <int P, bool NODE, int SPLIT, int WAVES>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WAVES))) void k_far(FarArgs a) {
  using E = Exp<P>;
  constexpr int NQ = E::NQ;
  constexpr int NL = E::NL;
  constexpr int RS = rec_stride(P);
  const int lane = threadIdx.x;
  const int sub = lane % SPLIT;
  const int l = blockIdx.x * (64 / SPLIT) + lane / SPLIT;
  const bool active = l < a.nleaves;
  const NodeInfo* __restrict__ info = a.info;
  const double* __restrict__ rec = a.rec;
  const int leaf = active ? a.leaf_node[l] : 0;
  const int d = active ? a.leaf_depth[l] : -1;
  const int lo = info[leaf].lo;
  const int cnt = active ? info[leaf].cnt : 0;

  double L[NL];
#pragma unroll
  for (int q = 0; q < NL; ++q) L[q] = 0.0;
  bool have = false;
  // list range of depth k for this lane: entries base + sub, base + sub + SPLIT, ...
  const uint32_t* list = NODE ? a.node_m2l_pool : a.m2l_list;
  const uint32_t* dc = NODE ? nullptr : a.depth_cnt + (active ? a.leaf_doff[l] : 0);
  uint64_t seg = NODE ? 0 : (active ? a.m2l_off[l] : 0);  // per-leaf lists: start of depth k
  uint64_t e = 0, ne = 0;
  int v = 0, k = 0;
  double sv[3] = {rec[0], rec[1], rec[2]};
  if (d >= 0) {
    if (NODE) { e = a.node_m2l_off[0]; ne = e + a.node_m2l_cnt[0]; }
    else { e = seg; ne = seg + dc[0]; }
    e += sub;
  }
  // one loop per lane: an M2L while the current depth has entries left,
  // else a step down the branch (L2L), until the leaf's list is done.  The
  // source record of the next entry and the list index of the one after it
  // are loaded while the current M2L is computed.
  double cs[3], cq[NQ];
  uint32_t idx_next = 0;
  auto load_rec = [&](uint32_t ent, double* sd, double* qd) {
    const double* rs = rec + (int64_t)(ent & kSrcMask) * RS;
    sd[0] = rs[0]; sd[1] = rs[1]; sd[2] = rs[2];
#pragma unroll
    for (int q = 0; q < NQ; ++q) qd[q] = rs[8 + q];
  };
  // at the top of the loop, when e < ne: (cs, cq) hold entry e's source and
  // idx_next the list index of the following entry (the last one repeated
  // when there is none)
  auto start_depth = [&]() {
    if (e < ne) {
      load_rec(list[e], cs, cq);
      idx_next = list[e + SPLIT < ne ? e + SPLIT : ne - 1];
    }
  };
  start_depth();
  for (;;) {
    if (e < ne) {
      const uint64_t en = e + SPLIT;
      double ns[3], nq[NQ];
      load_rec(idx_next, ns, nq);
      idx_next = list[en + SPLIT < ne ? en + SPLIT : ne - 1];
      const double r[3] = {cs[0] - sv[0], cs[1] - sv[1], cs[2] - sv[2]};
      E::m2l_add(r, cq, L);
      have = true;
      e = en;
      cs[0] = ns[0]; cs[1] = ns[1]; cs[2] = ns[2];
#pragma unroll
      for (int q = 0; q < NQ; ++q) cq[q] = nq[q];
    } else if (k < d) {
      const int c = info[v].child;
      const int nv = (lo < info[c + 1].lo) ? c : c + 1;
      const double* rn = rec + (int64_t)nv * RS;
      const double sn[3] = {rn[0], rn[1], rn[2]};
      if (have) {
        const double hv[3] = {sn[0] - sv[0], sn[1] - sv[1], sn[2] - sv[2]};
        E::l2l(hv, L);
      }
      v = nv;
      sv[0] = sn[0]; sv[1] = sn[1]; sv[2] = sn[2];
      ++k;
      if (NODE) {
        e = a.node_m2l_off[v];
        ne = e + a.node_m2l_cnt[v];
      } else {
        seg += dc[k - 1];
        e = seg;
        ne = seg + dc[k];
      }
      e += sub;
      start_depth();
    } else {
      break;
    }
  }
  // the SPLIT lanes of a leaf hold partial expansions about the same centre
#pragma unroll
  for (int o = SPLIT / 2; o > 0; o >>= 1) {
#pragma unroll
    for (int q = 0; q < NL; ++q) L[q] += __shfl_xor(L[q], o, 64);
    // every lane must take part in the shuffle (no short-circuit around it)
    const int other = __shfl_xor((int)have, o, 64);
    have = have || other != 0;
  }
  for (int j = lo + sub; j < lo + cnt; j += SPLIT) {
    const double off[3] = {a.xs[j] - sv[0], a.ys[j] - sv[1], a.zs[j] - sv[2]};
    double f[3] = {0.0, 0.0, 0.0}, phi = 0.0;
    if (have) E::l2p(off, L, f, phi);
    double* o = a.far + 4 * (int64_t)j;
    o[0] = f[0]; o[1] = f[1]; o[2] = f[2]; o[3] = phi;
  }
}

// ---- shared far field -------------------------------------------------------
// The caching of shared interactions of Sect. 5: the M2L list of node v (the
// pairs the level walk accepted with v as target) is evaluated once into
// LN[v]; a leaf's far field is then the root-to-leaf chain
//   L <- L2L(L, s_v - s_parent) (when L is non-zero), L <- L + LN[v],
// and L2P at its particles -- the same terms as the per-leaf form, whose
// replicated evaluation of every ancestor's list is what this removes.
//
// k_m2l_nodes: SPLIT lanes per node, nodes taken in level order (neighbours
// in a wave have similar list lengths); each lane sums every SPLIT-th entry,
// the group's partial sums are added with shuffles, and lane q of the group
// stores the coefficients q, q + SPLIT, ...  With F32 the contraction of a
// target at depth >= top runs on FP32 terms (FP64 sums), as in the per-leaf
// FP32C kernel.
constexpr int kSharedSplit = 8;  // lanes per node in k_m2l_nodes

template <int P, int SPLIT, bool F32, int WAVES>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WAVES))) void k_m2l_nodes(
    SharedFarArgs a) {
  using E = Exp<P>;
  constexpr int NQ = E::NQ;
  constexpr int NL = E::NL;
  constexpr int RS = rec_stride(P), RS32 = rec32_stride(P);
  const int lane = threadIdx.x;
  const int sub = lane % SPLIT;
  // (no XCD-contiguous mapping here: the cost per node varies with the
  // level, and the hardware's round-robin keeps the XCDs balanced)
  const int g = blockIdx.x * (64 / SPLIT) + lane / SPLIT;
  const bool active = g < a.nn;
  const int v = active ? a.level_nodes[g] : 0;
  const uint32_t cnt = active ? a.m2l_cnt[v] : 0u;
  const uint32_t off = active ? a.m2l_off[v] : 0u;
  const double* __restrict__ rec = a.rec;
  const double sv[3] = {rec[(int64_t)v * RS], rec[(int64_t)v * RS + 1], rec[(int64_t)v * RS + 2]};
  const bool f32 = F32 && active && a.depth[v] >= a.top;
  double L[NL];
#pragma unroll
  for (int q = 0; q < NL; ++q) L[q] = 0.0;
  for (uint32_t e = off + sub; e < off + cnt; e += SPLIT) {
    const uint32_t src = a.pool[e] & kSrcMask;
    const double* rs = rec + (int64_t)src * RS;
    if (F32 && f32) {
      const float r[3] = {(float)(rs[0] - sv[0]), (float)(rs[1] - sv[1]), (float)(rs[2] - sv[2])};
      const float* r32 = a.rec32 + (int64_t)src * RS32;
      float Q[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) Q[q] = r32[q];
      E::m2l_add_f32(r, Q, L);
    } else {
      const double r[3] = {rs[0] - sv[0], rs[1] - sv[1], rs[2] - sv[2]};
      double Q[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) Q[q] = rs[8 + q];
      E::m2l_add(r, Q, L);
    }
  }
#pragma unroll
  for (int o = SPLIT / 2; o > 0; o >>= 1) {
#pragma unroll
    for (int q = 0; q < NL; ++q) L[q] += __shfl_xor(L[q], o, 64);
  }
  if (active && cnt > 0) {
    double* out = a.ln + (int64_t)v * NL;
#pragma unroll
    for (int q = 0; q < NL; ++q)
      if (q % SPLIT == sub) out[q] = L[q];
  }
}

// The one-sided symmetric M2L (Sect. 5 notes that an interaction can be
// applied to both nodes of a pair): every unordered pair of the interaction
// set -- node v's M2L list holds s exactly when s's holds v -- is evaluated
// once, by the node with the smaller id, with one derivative tensor D(r) for
// both directions (Exp<P>::m2l_pair): the owner's side is summed in
// registers as in k_m2l_nodes, the partner's side is added to the partner's
// local coefficients with FP64 atomic adds, and the owner adds its own sum
// last, also atomically.  ln must hold zeros before.  The order of the
// atomic additions is not fixed, so results agree with the directed form to
// rounding, not bit for bit.
template <int P, int SPLIT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1))) void k_m2l_mutual(
    SharedFarArgs a) {
  using E = Exp<P>;
  constexpr int NQ = E::NQ;
  constexpr int NL = E::NL;
  constexpr int RS = rec_stride(P);
  const int lane = threadIdx.x;
  const int sub = lane % SPLIT;
  const int g = blockIdx.x * (64 / SPLIT) + lane / SPLIT;
  const bool active = g < a.nn;
  const int v = active ? a.level_nodes[g] : 0;
  const uint32_t cnt = active ? a.m2l_cnt[v] : 0u;
  const uint32_t off = active ? a.m2l_off[v] : 0u;
  const double* __restrict__ rec = a.rec;
  const double* rv = rec + (int64_t)v * RS;
  const double sv[3] = {rv[0], rv[1], rv[2]};
  // the owner's moments with odd degrees negated (its side of D(-r))
  double QTs[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) QTs[q] = rv[8 + q];
  {
    int k = 0;
#pragma unroll
    for (int n = 0; n <= P; ++n)
#pragma unroll
      for (int c = 0; c < (n + 1) * (n + 2) / 2; ++c, ++k)
        if (n & 1) QTs[k] = -QTs[k];
  }
  double L[NL];
#pragma unroll
  for (int q = 0; q < NL; ++q) L[q] = 0.0;
  for (uint32_t e = off + sub; e < off + cnt; e += SPLIT) {
    const uint32_t src = a.pool[e] & kSrcMask;
    if ((int)src <= v) continue;  // the partner owns this pair
    const double* rs = rec + (int64_t)src * RS;
    const double r[3] = {rs[0] - sv[0], rs[1] - sv[1], rs[2] - sv[2]};
    double QS[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) QS[q] = rs[8 + q];
    E::m2l_pair(r, QS, QTs, L, a.ln + (int64_t)src * NL);
  }
#pragma unroll
  for (int o = SPLIT / 2; o > 0; o >>= 1) {
#pragma unroll
    for (int q = 0; q < NL; ++q) L[q] += __shfl_xor(L[q], o, 64);
  }
  if (active && cnt > 0) {
    double* out = a.ln + (int64_t)v * NL;
#pragma unroll
    for (int q = 0; q < NL; ++q)
      if (q % SPLIT == sub) unsafeAtomicAdd(&out[q], L[q]);
  }
}

// Sort key of the node at level position g for the shared M2L: the number
// of SPLIT-entry steps its list takes, longest first (clamped at 127 steps),
// after a group bit that puts FP32 targets (FP32C, depth >= top) behind the
// FP64 ones.  A stable pass on this key gives every wave nodes that take the
// same number of steps, where level order leaves lanes idle until the
// longest list of the wave ends; each node's own sum is unchanged.
__global__ void k_m2l_order_keys(int nn, int split, const int32_t* __restrict__ level_nodes,
                                 const uint32_t* __restrict__ cnt,
                                 const int32_t* __restrict__ depth, int top, int f32,
                                 uint64_t* __restrict__ key, uint32_t* __restrict__ ids) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nn) return;
  const int v = level_nodes[g];
  const uint32_t steps = (cnt[v] + (uint32_t)split - 1) / (uint32_t)split;
  const uint32_t c = steps < 127u ? steps : 127u;
  const uint32_t grp = (f32 && depth[v] >= top) ? 1u : 0u;
  key[g] = (uint64_t)((grp << 7) | (127u - c));
  ids[g] = (uint32_t)v;
}

__global__ void k_zero_f64(int64_t n, double* __restrict__ p) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// k_far_shared: one lane per leaf walks its branch from the root
template <int P>
__global__ __launch_bounds__(64) void k_far_shared(FarArgs a, const double* __restrict__ ln) {
  using E = Exp<P>;
  constexpr int NL = E::NL;
  constexpr int RS = rec_stride(P);
  const int l = xcd_block(blockIdx.x, gridDim.x) * 64 + threadIdx.x;
  if (l >= a.nleaves) return;
  const NodeInfo* __restrict__ info = a.info;
  const double* __restrict__ rec = a.rec;
  const int leaf = a.leaf_node[l];
  const int d = a.leaf_depth[l];
  const int lo = info[leaf].lo;
  const int cnt = info[leaf].cnt;
  double L[NL];
#pragma unroll
  for (int q = 0; q < NL; ++q) L[q] = 0.0;
  bool have = false;
  int v = 0;
  double sv[3] = {rec[0], rec[1], rec[2]};
  auto add_node = [&](int u) {
    if (a.node_m2l_cnt[u] == 0) return;
    const double* lu = ln + (int64_t)u * NL;
#pragma unroll
    for (int q = 0; q < NL; ++q) L[q] += lu[q];
    have = true;
  };
  add_node(0);
  for (int k = 0; k < d; ++k) {
    const int c = info[v].child;
    const int nv = (lo < info[c + 1].lo) ? c : c + 1;
    const double* rn = rec + (int64_t)nv * RS;
    const double sn[3] = {rn[0], rn[1], rn[2]};
    if (have) {
      const double hv[3] = {sn[0] - sv[0], sn[1] - sv[1], sn[2] - sv[2]};
      E::l2l(hv, L);
    }
    v = nv;
    sv[0] = sn[0]; sv[1] = sn[1]; sv[2] = sn[2];
    add_node(v);
  }
  for (int j = lo; j < lo + cnt; ++j) {
    const double off[3] = {a.xs[j] - sv[0], a.ys[j] - sv[1], a.zs[j] - sv[2]};
    double f[3] = {0.0, 0.0, 0.0}, phi = 0.0;
    if (have) E::l2p(off, L, f, phi);
    double* o = a.far + 4 * (int64_t)j;
    o[0] = f[0]; o[1] = f[1]; o[2] = f[2]; o[3] = phi;
  }
}

template <int P, int SPLIT, int WAVES>
void shared_order(const FarArgs& f, const SharedFarArgs& a, bool f32, hipStream_t s) {
  if (a.nn > 0) {
    const unsigned nb = (unsigned)((a.nn + 64 / SPLIT - 1) / (64 / SPLIT));
    if (f32) k_m2l_nodes<P, SPLIT, true, WAVES><<<nb, 64, 0, s>>>(a);
    else k_m2l_nodes<P, SPLIT, false, WAVES><<<nb, 64, 0, s>>>(a);
  }
  if (f.nleaves > 0) k_far_shared<P><<<(unsigned)((f.nleaves + 63) / 64), 64, 0, s>>>(f, a.ln);
}

template <int P>
void mutual_order(const FarArgs& f, const SharedFarArgs& a, hipStream_t s) {
  if (a.nn > 0) {
    const int64_t nz = (int64_t)a.nn * Exp<P>::NL;
    k_zero_f64<<<(unsigned)std::min<int64_t>((nz + 255) / 256, 4096), 256, 0, s>>>(nz, a.ln);
    constexpr int SPLIT = 8;
    k_m2l_mutual<P, SPLIT><<<(unsigned)((a.nn + 64 / SPLIT - 1) / (64 / SPLIT)), 64, 0, s>>>(a);
  }
  if (f.nleaves > 0) k_far_shared<P><<<(unsigned)((f.nleaves + 63) / 64), 64, 0, s>>>(f, a.ln);
}

template <int SPLIT, int WAVES>
void shared_split(int order, const FarArgs& f, const SharedFarArgs& a, bool f32, hipStream_t s) {
  switch (order) {
    case 0: shared_order<0, SPLIT, WAVES>(f, a, f32, s); break;
    case 1: shared_order<1, SPLIT, WAVES>(f, a, f32, s); break;
    case 2: shared_order<2, SPLIT, WAVES>(f, a, f32, s); break;
    case 3: shared_order<3, SPLIT, WAVES>(f, a, f32, s); break;
    case 4: shared_order<4, SPLIT, WAVES>(f, a, f32, s); break;
  }
}

}  // namespace

void launch_far_shared(int order, const FarArgs& f, const SharedFarArgs& a, bool f32,
                       hipStream_t s) {
  // 8 lanes per node; the FP64 contraction fits a two-wave register budget
  // without spilling, the FP32 one does not
  if (f32) shared_split<kSharedSplit, 1>(order, f, a, f32, s);
  else shared_split<kSharedSplit, 2>(order, f, a, f32, s);
}

void launch_m2l_order(const SharedFarArgs& a, bool f32, const M2LOrderBufs& b, hipStream_t s) {
  if (a.nn <= 0) return;
  k_m2l_order_keys<<<(unsigned)((a.nn + 255) / 256), 256, 0, s>>>(
      a.nn, kSharedSplit, a.level_nodes, a.m2l_cnt, a.depth, a.top, f32 ? 1 : 0, b.key0, b.ids0);
  radix_pass(a.nn, b.key0, b.ids0, b.key1, b.ids1, 0, b.hist, b.hist_tmp, b.total, s);
}

void launch_far_mutual(int order, const FarArgs& f, const SharedFarArgs& a, hipStream_t s) {
  switch (order) {
    case 0: mutual_order<0>(f, a, s); break;
    case 1: mutual_order<1>(f, a, s); break;
    case 2: mutual_order<2>(f, a, s); break;
    case 3: mutual_order<3>(f, a, s); break;
    case 4: mutual_order<4>(f, a, s); break;
  }
}

template <bool NODE, int SPLIT, int WAVES>
void far_dispatch(int order, const FarArgs& a, hipStream_t s) {
  const unsigned nb = (unsigned)((a.nleaves + 64 / SPLIT - 1) / (64 / SPLIT));
  switch (order) {
    case 0: k_far<0, NODE, SPLIT, WAVES><<<nb, 64, 0, s>>>(a); break;
    case 1: k_far<1, NODE, SPLIT, WAVES><<<nb, 64, 0, s>>>(a); break;
    case 2: k_far<2, NODE, SPLIT, WAVES><<<nb, 64, 0, s>>>(a); break;
    case 3: k_far<3, NODE, SPLIT, WAVES><<<nb, 64, 0, s>>>(a); break;
    case 4: k_far<4, NODE, SPLIT, WAVES><<<nb, 64, 0, s>>>(a); break;
  }
}

void launch_far(int order, bool node_lists, const FarArgs& a, hipStream_t s) {
  if (a.nleaves <= 0) return;
  // 4 lanes per leaf, one wave per SIMD
  if (node_lists) far_dispatch<true, 4, 1>(order, a, s);
  else far_dispatch<false, 4, 1>(order, a, s);
}

}  // namespace sfmm
