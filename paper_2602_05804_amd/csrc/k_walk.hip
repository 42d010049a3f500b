// k_walk.hip -- the per-leaf dual tree walk (Sect. 3, Algorithms 1 and 2).
//
// One thread per leaf (leaves in Morton order, so a wave walks 64
// neighbouring leaves whose branches share their upper part).  Each thread
//   1. descends from the root to its leaf to get the branch p_0 .. p_d,
//   2. runs the stack walk from (root, root): a node met with itself is
//      opened; an accepted pair is an M2L of the source on the ancestor p_k;
//      a rejected pair is opened -- two leaves become a P2P entry, a leaf
//      source meets the next ancestor, an internal source splits and its
//      children meet the next ancestor (or the leaf itself once the target
//      is the leaf: the lowering of shallow leaves).
// Acceptance: (l_t + l_s)^2 < theta^2 d^2 (opening angle) and
// d^2 >= (l_t + l_s + R_kern max(h_max))^2 (softening: every pair inside a
// kernel stays a particle pair), d the distance between centres of mass.
//
// The walk runs twice: a count pass (per-depth M2L counts, P2P count) and,
// after the host has sized the lists, a fill pass that writes the entries
// grouped by depth.  Both passes visit the same pairs in the same order.
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

template <int MAXD, bool FILL>
__global__ __launch_bounds__(128) void k_walk(WalkArgs a) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= a.nleaves) return;
  const int leaf = a.leaf_node[l];
  const int d = a.leaf_depth[l];
  if (d > MAXD) {
    atomicOr(a.status, ST_DEPTH);
    return;
  }
  const NodeInfo* __restrict__ info = a.info;
  const double* __restrict__ rec = a.rec;
  const int RS = a.stride;
  const int lo = info[leaf].lo;
  const int my_cnt = info[leaf].cnt;

  int branch[MAXD + 1];
  branch[0] = 0;
  {
    int v = 0;
    for (int k = 1; k <= d; ++k) {
      const int c = info[v].child;
      v = (lo < info[c + 1].lo) ? c : c + 1;
      branch[k] = v;
    }
  }
  uint32_t cur[MAXD + 1];
  uint64_t base = 0;
  if (FILL) {
    uint32_t run = 0;
    const uint32_t* dc = a.depth_cnt + a.leaf_doff[l];
    for (int k = 0; k <= d; ++k) {
      cur[k] = run;
      run += dc[k];
    }
    base = a.m2l_cnt[l];  // offsets after the scan
  } else {
    for (int k = 0; k <= d; ++k) cur[k] = 0;
  }
  uint64_t np2p = 0, npairs = 0;
  const uint64_t p2p_base = FILL ? a.p2p_cnt[l] : 0;

  constexpr int CAP = MAXD + 2;
  uint32_t stack[CAP];
  int sp = 0;
  stack[sp++] = 0u;  // (depth 0, root)
  while (sp > 0) {
    const uint32_t e = stack[--sp];
    const int k = (int)(e >> kSrcBits);
    const int src = (int)(e & kSrcMask);
    const int tgt = branch[k];
    bool open;
    if (tgt == src) {
      open = true;
    } else if (accept(rec + (int64_t)tgt * RS, rec + (int64_t)src * RS, a.theta2, a.r_kern)) {
      if (FILL) a.m2l_list[base + cur[k]] = ((uint32_t)k << kSrcBits) | (uint32_t)src;
      cur[k]++;
      open = false;
    } else {
      open = true;
    }
    if (!open) continue;
    const NodeInfo si = info[src];
    if (si.child < 0) {
      if (k == d) {
        if (FILL) a.p2p_list[p2p_base + np2p] = src;
        np2p++;
        npairs += (uint64_t)si.cnt * (uint64_t)my_cnt;
      } else {
        if (sp >= CAP) { atomicOr(a.status, ST_OVERFLOW); break; }
        stack[sp++] = ((uint32_t)(k + 1) << kSrcBits) | (uint32_t)src;
      }
    } else {
      const uint32_t kk = (uint32_t)(k == d ? k : k + 1);
      if (sp + 2 > CAP) { atomicOr(a.status, ST_OVERFLOW); break; }
      stack[sp++] = (kk << kSrcBits) | (uint32_t)si.child;
      stack[sp++] = (kk << kSrcBits) | (uint32_t)(si.child + 1);
    }
  }
  if (!FILL) {
    uint32_t* dc = a.depth_cnt + a.leaf_doff[l];
    uint64_t tot = 0;
    int kfirst = -1;
    for (int k = 0; k <= d; ++k) {
      dc[k] = cur[k];
      tot += cur[k];
      if (kfirst < 0 && cur[k] > 0) kfirst = k;
    }
    a.l2l_cnt[l] = kfirst < 0 ? 0u : (uint64_t)(d - kfirst);
    a.m2l_cnt[l] = tot;
    a.p2p_cnt[l] = np2p;
    a.pair_cnt[l] = npairs - (uint64_t)my_cnt;  // the self pairs j == i are skipped
  }
}

__global__ void k_leaf_doff(int nleaves, const int32_t* __restrict__ leaf_depth,
                            uint64_t* __restrict__ out) {
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < nleaves) out[l] = (uint64_t)leaf_depth[l] + 1u;
}

template <int MAXD>
void walk_dispatch(const WalkArgs& a, bool fill, hipStream_t s) {
  const unsigned nb = (unsigned)((a.nleaves + 127) / 128);
  if (fill) k_walk<MAXD, true><<<nb, 128, 0, s>>>(a);
  else k_walk<MAXD, false><<<nb, 128, 0, s>>>(a);
}

}  // namespace

void launch_walk(const WalkArgs& a, int maxdepth, bool fill, hipStream_t s) {
  if (a.nleaves <= 0) return;
  if (maxdepth <= 24) walk_dispatch<24>(a, fill, s);
  else if (maxdepth <= 40) walk_dispatch<40>(a, fill, s);
  else if (maxdepth <= 64) walk_dispatch<64>(a, fill, s);
  else walk_dispatch<kMaxDepthCap>(a, fill, s);
}

void launch_leaf_doff(int nleaves, const int32_t* leaf_depth, uint64_t* out, hipStream_t s) {
  k_leaf_doff<<<(nleaves + 255) / 256, 256, 0, s>>>(nleaves, leaf_depth, out);
}

}  // namespace sfmm
