// k_far.hip -- far field of each leaf: M2L on every ancestor, the L2L chain
// down the branch and L2P at the leaf's particles (Sect. 2.2, Algorithm 1's
// propagate_to_next_parent, Appendix A.2).
//
// One thread per leaf.  The leaf's M2L list is grouped by the depth of the
// target ancestor, so the thread keeps one local expansion in registers:
// at depth k it re-centres the expansion from p_{k-1} to p_k (exact for the
// polynomial) and adds the M2L of every source listed for p_k.  Leaves of a
// wave share their upper ancestors, so the upper part of the lists is the
// same for all lanes and the source records are read once per wave.
#include "sfmm_internal.h"

namespace sfmm {
namespace {

template <int P, bool NODE>
__global__ __launch_bounds__(128) void k_far(FarArgs a) {
  using E = Exp<P>;
  constexpr int NQ = E::NQ;
  constexpr int NL = E::NL;
  constexpr int RS = rec_stride(P);
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
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
  uint64_t e = NODE ? 0 : a.m2l_off[l];
  const uint64_t end = NODE ? 0 : a.m2l_off[l + 1];
  int v = 0;
  double sv[3] = {rec[0], rec[1], rec[2]};
  for (int k = 0; k <= d; ++k) {
    if (k > 0) {
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
    }
    uint64_t ne = end;
    const uint32_t* list = a.m2l_list;
    if (NODE) {
      e = a.node_m2l_off[v];
      ne = e + a.node_m2l_cnt[v];
      list = a.node_m2l_pool;
    }
    while (e < ne) {
      const uint32_t ent = list[e];
      if (!NODE && (int)(ent >> kSrcBits) != k) break;
      const double* rs = rec + (int64_t)(ent & kSrcMask) * RS;
      const double r[3] = {rs[0] - sv[0], rs[1] - sv[1], rs[2] - sv[2]};
      double Q[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) Q[q] = rs[8 + q];
      E::m2l_add(r, Q, L);
      have = true;
      ++e;
    }
  }
  for (int j = lo; j < lo + cnt; ++j) {
    const double off[3] = {a.xs[j] - sv[0], a.ys[j] - sv[1], a.zs[j] - sv[2]};
    double f[3] = {0.0, 0.0, 0.0}, phi = 0.0;
    if (have) E::l2p(off, L, f, phi);
    double* o = a.far + 4 * (int64_t)j;
    o[0] = f[0]; o[1] = f[1]; o[2] = f[2]; o[3] = phi;
  }
}

}  // namespace

template <bool NODE>
void far_dispatch(int order, const FarArgs& a, hipStream_t s) {
  const unsigned nb = (unsigned)((a.nleaves + 127) / 128);
  switch (order) {
    case 0: k_far<0, NODE><<<nb, 128, 0, s>>>(a); break;
    case 1: k_far<1, NODE><<<nb, 128, 0, s>>>(a); break;
    case 2: k_far<2, NODE><<<nb, 128, 0, s>>>(a); break;
    case 3: k_far<3, NODE><<<nb, 128, 0, s>>>(a); break;
    case 4: k_far<4, NODE><<<nb, 128, 0, s>>>(a); break;
  }
}

void launch_far(int order, bool node_lists, const FarArgs& a, hipStream_t s) {
  if (a.nleaves <= 0) return;
  if (node_lists) far_dispatch<true>(order, a, s);
  else far_dispatch<false>(order, a, s);
}

}  // namespace sfmm
