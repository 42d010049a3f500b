// k_p2p_tile.hip -- P2P, the softened direct sum of Sect. 2 (Eq.
// softdirectsum) over the source leaves the walk cached for a leaf, with the
// leaf's targets held in lanes and the sources streamed through LDS.
//
// One wave per work item (a leaf and a run of at most kP2PItem of its
// flattened sources, as for the other P2P kernels).  With nt targets, the
// wave's lanes form NS = min(64 / nt, 32) stripes of nt lanes: lane
// (s, t) = s * nt + t holds target t in registers and, at every step, meets
// source s of the step, so a step evaluates NS sources against all targets
// and nearly every lane does useful work for any leaf size.
//
// Sources are staged 64 at a time: their particle indices are flattened into
// LDS, then each lane loads one source record (x, y, z, m, h) (the next
// batch's records load while the current batch's steps run) and tests it
// against the target leaf's sphere (centre of mass c, size l, largest
// softening length h_max):
//   |x_j - c| >= l + 2 max(h_max, h_j)  ->  r_ij >= 2 max(h_i, h_j) for every
//   target i of the leaf: no pair with j lies inside a kernel ("far");
// otherwise the source is "near".  The batch is stored near sources first.
// A far step is the plain pair m/r^3 (dx, dy, dz), m/r.  A near step tests
// each pair against both kernels, r^2 < 4 max(h_i, h_j)^2: a pair beyond
// them is plain, a pair inside gets 1/r = 0 and its source goes to a ring
// queue of its target in LDS (the self pair j = i is skipped).  Queued pairs
// are evaluated in soft passes, lane (s, t) taking entry s of target t's
// queue, so each lane adds to its own target and the spline kernels run on
// mostly busy lanes; a pass runs when a queue could overflow, and at the end
// of the item until every queue is empty.  The pair kernels are the formulas
// of softening.h: the mean of the two particles' kernels, so each pair force
// stays antisymmetric.
//
// Per-lane sums are reduced over the stripes in stripe order at the end of
// the item (a fixed order: the results do not depend on timing), and the
// item's partial sums are added per target by k_p2p_reduce in item order.
#include <type_traits>

#include "sfmm_internal.h"
#include "softening.h"

namespace sfmm {
namespace {

constexpr int kWin = 256;        // flattened source indices staged per window
constexpr int kMaxStripes = 32;  // NS <= 32
constexpr int kQueue = 64;       // ring queue slots per target (a power of two)

__device__ __forceinline__ int wave_incl_scan_i(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// a wave-uniform int kept in a scalar register
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint32_t popc64(uint64_t m) { return (uint32_t)__popcll(m); }

// a batch source's softening length squared and particle index (16 bytes,
// like the other batch arrays, so that one address serves all three)
struct SrcHJ {
  double h2;
  int j;
  int pad;
};

template <int LS>
struct TileLds {
  uint32_t sidx[kWin];           // flattened source particle indices of the window
  double2 b_xy[64], b_zm[64];    // the batch: x, y | z, m
  SrcHJ b_hj[64];                //            h^2, particle index
  int queue[LS][kQueue];         // per target: ring of sources whose pair lies inside a kernel
};

template <int LS, bool NODE>
__global__ __launch_bounds__(64) void k_p2p_tile(NearArgs a) {
  __shared__ TileLds<LS> sh;
  const int lane = threadIdx.x;
  const uint32_t item = xcd_block(blockIdx.x, gridDim.x);
  if (item >= a.item_off[a.nleaves]) return;  // the grid is an upper bound
  const int l = a.item_leaf[item];
  const uint32_t kitem = a.item_k[item];
  const int node = a.leaf_node[l];
  const NodeInfo ti = a.info[node];
  const int nt = uni(ti.cnt);  // 1 .. LS
  const int ns = uni(min(64 / nt, kMaxStripes));
  const int s = lane / nt, t = lane - s * nt;
  const bool lane_ok = s < ns;
  // this lane's target (lanes past the stripes repeat target 0 and add nothing)
  const int tq = lane_ok ? t : 0;
  // the stripe this lane reads a batch source for (lanes past the stripes
  // read stripe 0's and keep sums nobody reads: full steps need no masks)
  const int sq = lane_ok ? s : 0;
  const int it = ti.lo + tq;
  const double xi = a.xs[it], yi = a.ys[it], zi = a.zs[it];
  const double hi = a.hs[it], hiinv = a.his[it];
  const double h4i = 4.0 * hi * hi;
  // the lanes of this lane's target, and those below this lane
  uint64_t tmask = 0;
  for (int q = 0; q < ns; ++q) tmask |= 1ull << (q * nt + tq);
  if (!lane_ok) tmask = 0;
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  // this lane's target queue: first slot and length (the same on its stripes)
  int qhead = 0, qlen = 0;
  const int qcap = uni(kQueue - ns);  // a near step adds at most ns to a queue
  // the target leaf's sphere: centre of mass, size, largest softening length
  const double* rl = a.rec + (int64_t)node * a.rec_stride;
  const double cx = rl[0], cy = rl[1], cz = rl[2], ll = rl[3], lh = rl[4];
  double fx = 0.0, fy = 0.0, fz = 0.0, ph = 0.0;
  uint32_t nsoft = 0;

  // up to ns queued sources of every target, each against its own target
  auto soft_pass = [&]() {
    const bool v = lane_ok && s < qlen;
    const int j = v ? sh.queue[tq][(qhead + s) & (kQueue - 1)] : it;
    const double2* rj = reinterpret_cast<const double2*>(a.p4 + 4 * (int64_t)j);
    const double2 xy = rj[0], zm = rj[1];
    const double hj = a.hs[j], hjinv = a.his[j];
    const double dx = xi - xy.x, dy = yi - xy.y, dz = zi - zm.x;
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const double rinv = rsqrt_pair(r2);  // 0 for coincident particles
    const double rinv3 = rinv * rinv * rinv;
    const double r = r2 * rinv;
    double g1, p1, g2, p2;
    soft_sel(r * hiinv, hiinv, hi * rinv, rinv, rinv3, g1, p1);
    soft_sel(r * hjinv, hjinv, hj * rinv, rinv, rinv3, g2, p2);
    const double w = v ? zm.y : 0.0;
    const double mg = w * (0.5 * (g1 + g2));
    fx = fma(mg, dx, fx);
    fy = fma(mg, dy, fy);
    fz = fma(mg, dz, fz);
    ph = fma(w, 0.5 * (p1 + p2), ph);
    const int take = min(qlen, ns);
    qhead = (qhead + take) & (kQueue - 1);
    qlen -= take;
  };

  // one far step over batch sources b0 .. b0 + navail - 1 (navail <= ns):
  // every pair beyond both kernels; a full step (navail == ns) needs no mask
  auto far_step = [&](int b0, int navail, auto fullc) {
    constexpr bool FULL = decltype(fullc)::value;
    const bool v = FULL || (lane_ok && s < navail);
    const int q = b0 + (FULL ? sq : (v ? s : 0));
    const double2 xy = sh.b_xy[q], zm = sh.b_zm[q];
    const double w = FULL ? zm.y : (v ? zm.y : 0.0);
    const double dx = xi - xy.x, dy = yi - xy.y, dz = zi - zm.x;
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const double rinv = rsqrt_refined(r2);  // r2 >= 4 h^2 > 0 for a far source
    const double mr = w * rinv;
    const double mg = mr * (rinv * rinv);
    fx = fma(mg, dx, fx);
    fy = fma(mg, dy, fy);
    fz = fma(mg, dz, fz);
    ph += mr;
  };

  // one near step: pairs inside a kernel go to their target's queue; in a
  // full step the self pair needs no mask either (r^2 = 0 is inside a
  // kernel, so its 1/r is 0)
  auto near_step = [&](int b0, int navail, auto fullc) {
    constexpr bool FULL = decltype(fullc)::value;
    const bool v = FULL ? lane_ok : (lane_ok && s < navail);
    const int q = b0 + (FULL ? sq : (v ? s : 0));
    const double2 xy = sh.b_xy[q], zm = sh.b_zm[q];
    const SrcHJ hj = sh.b_hj[q];
    const int j = hj.j;
    const double dx = xi - xy.x, dy = yi - xy.y, dz = zi - zm.x;
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    // r^2 < 4 h_i^2 or r^2 < 4 h_j^2, the second as r^2 / 4 < h_j^2 (scaling
    // by 4 is exact, so the decision is the same; with two different left
    // sides the compiler keeps two compares instead of a max that would
    // canonicalise its operands)
    const bool inside = r2 < h4i || r2 * 0.25 < hj.h2;
    const bool use = v && j != it;
    const double rinv = inside ? 0.0 : rsqrt_refined(r2);
    const double w = FULL ? zm.y : (use ? zm.y : 0.0);
    const double mr = w * rinv;
    const double mg = mr * (rinv * rinv);
    fx = fma(mg, dx, fx);
    fy = fma(mg, dy, fy);
    fz = fma(mg, dz, fz);
    ph += mr;
    const bool push = use && inside;
    const uint64_t bal = __ballot(push);
    if (bal) {
      const uint64_t mine = bal & tmask;
      if (push) sh.queue[tq][(qhead + qlen + (int)popc64(mine & below)) & (kQueue - 1)] = j;
      qlen += (int)popc64(mine);
      nsoft += popc64(bal);
    }
  };

  uint64_t e0, e1;
  const int32_t* list;
  if (NODE) {
    e0 = a.node_p2p_off[node];
    e1 = e0 + a.node_p2p_cnt[node];
    list = reinterpret_cast<const int32_t*>(a.node_p2p_pool);
  } else {
    e0 = a.p2p_off[l];
    e1 = a.p2p_off[l + 1];
    list = a.p2p_list;
  }
  // this item's run [f_lo, f_hi) of the leaf's flattened sources, from the
  // list entry that holds its first source
  const uint32_t f_lo = kitem * kP2PItem;
  const uint32_t ftot = a.src_total[l];
  const uint32_t f_hi = f_lo + kP2PItem < ftot ? f_lo + kP2PItem : ftot;
  uint32_t carry = 0;
  if (kitem > 0) { e0 = a.item_e0[item]; carry = a.item_c0[item]; }
  for (uint64_t c0 = e0; c0 < e1; c0 += 64) {
    // 64 list entries: their particle ranges in the flattened order, clipped
    // to the run: [pre, pre + cnt) of this group's sources start at particle lo
    int cnt = 0, lo = 0;
    uint32_t fb = 0xffffffffu;
    const bool in = c0 + lane < e1;
    NodeInfo si{};
    if (in) si = a.info[list[c0 + lane]];
    const int sincl = wave_incl_scan_i(in ? si.cnt : 0);
    if (in) {
      const uint32_t fe = carry + (uint32_t)sincl;
      fb = fe - (uint32_t)si.cnt;
      const uint32_t b = fb > f_lo ? fb : f_lo;
      const uint32_t en = fe < f_hi ? fe : f_hi;
      if (en > b) { cnt = (int)(en - b); lo = si.lo + (int)(b - fb); }
    }
    carry += (uint32_t)__builtin_amdgcn_readlane(sincl, 63);
    // lane 0 always holds an entry (c0 < e1)
    if ((uint32_t)__builtin_amdgcn_readfirstlane(fb) >= f_hi) break;  // the run is done
    const int incl = wave_incl_scan_i(cnt);
    const int pre = incl - cnt;
    const int total = __builtin_amdgcn_readlane(incl, 63);
    for (int w0 = 0; w0 < total; w0 += kWin) {
      const int wn = uni(min(kWin, total - w0));
      // flatten: each entry writes its part of the window; entries of at most
      // 16 sources in the window one index per iteration, larger ones by the
      // whole wave
      const int ab = max(pre, w0), ae = min(pre + cnt, w0 + kWin);
      const int nw = ae > ab ? ae - ab : 0;
      const bool big = nw > 16;
      for (int k = 0; k < 16; ++k) {
        if (!__any(k < nw && !big)) break;
        if (k < nw && !big) sh.sidx[ab - w0 + k] = (uint32_t)(lo + (ab - pre) + k);
      }
      uint64_t bigm = __ballot(big);
      while (bigm) {
        const int k = __builtin_ctzll(bigm);
        bigm &= bigm - 1;
        const int kb = __builtin_amdgcn_readlane(ab, k), kn = __builtin_amdgcn_readlane(nw, k);
        const int klo = __builtin_amdgcn_readlane(lo, k) + (kb - __builtin_amdgcn_readlane(pre, k));
        for (int q = lane; q < kn; q += 64) sh.sidx[kb - w0 + q] = (uint32_t)(klo + q);
      }
      __syncthreads();
      // batches of 64 sources; the next batch's records load during the steps
      auto load_src = [&](int u0, int& j, double2& xy, double2& zm, double& hj) {
        j = u0 + lane < wn ? (int)sh.sidx[u0 + lane] : ti.lo;
        const double2* rj = reinterpret_cast<const double2*>(a.p4 + 4 * (int64_t)j);
        xy = rj[0];
        zm = rj[1];
        hj = a.hs[j];
      };
      int j;
      double2 xy, zm;
      double hj;
      load_src(0, j, xy, zm, hj);
      for (int u0 = 0; u0 < wn; u0 += 64) {
        const int nb = uni(min(64, wn - u0));
        const bool sv = lane < nb;
        const double ex = xy.x - cx, ey = xy.y - cy, ez = zm.x - cz;
        const double d2 = fma(ex, ex, fma(ey, ey, ez * ez));
        const double reach = ll + 2.0 * fmax(lh, hj);
        // (a relative margin keeps rounding from making a near source far)
        const bool near = d2 < reach * reach * (1.0 + 1e-9);
        const uint64_t bn = __ballot(sv && near), bf = __ballot(sv && !near);
        const int nn = uni((int)popc64(bn));
        if (sv) {
          const int q = near ? (int)popc64(bn & below) : nn + (int)popc64(bf & below);
          sh.b_xy[q] = xy;
          sh.b_zm[q] = zm;
          sh.b_hj[q] = SrcHJ{hj * hj, j, 0};
        }
        if (u0 + 64 < wn) load_src(u0 + 64, j, xy, zm, hj);
        __syncthreads();
        // (before a near step every queue holds at most qcap = kQueue - ns,
        // the step adds at most ns to each, and a soft pass takes ns from
        // every queue above qcap (qcap >= 32 >= ns): one pass restores it)
        int b0 = 0;
        for (; b0 + ns <= nn; b0 += ns) {
          near_step(b0, ns, std::true_type{});
          if (__any(qlen > qcap)) soft_pass();
        }
        if (b0 < nn) {
          near_step(b0, nn - b0, std::false_type{});
          if (__any(qlen > qcap)) soft_pass();
        }
        for (b0 = nn; b0 + ns <= nb; b0 += ns) far_step(b0, ns, std::true_type{});
        if (b0 < nb) far_step(b0, nb - b0, std::false_type{});
        __syncthreads();  // the batch may be written next
      }
    }
  }
  // the queued pairs left
  while (__any(qlen > 0)) soft_pass();
  // sums over the stripes, in stripe order, per target
  __syncthreads();
  double2* red = sh.b_xy;  // 64 x (fx, fy), then 64 x (fz, ph) in b_zm
  double2* red2 = sh.b_zm;
  red[lane] = make_double2(fx, fy);
  red2[lane] = make_double2(fz, ph);
  __syncthreads();
  if (lane < nt) {
    double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0;
    for (int q = 0; q < ns; ++q) {
      const double2 u = red[q * nt + lane], v = red2[q * nt + lane];
      sx += u.x; sy += u.y; sz += v.x; sp += v.y;
    }
    double* o = a.part + (item * (int64_t)LS + lane) * 4;
    o[0] = sx; o[1] = sy; o[2] = sz; o[3] = sp;
  }
  if (lane == 0 && nsoft) atomicAdd(a.soft_pairs, (unsigned long long)nsoft);
}

}  // namespace

void launch_p2p_tile(bool node_lists, int ls, const NearArgs& a, int64_t items, hipStream_t s) {
  if (a.n <= 0 || items <= 0) return;
  const unsigned nbl = (unsigned)items;
  if (ls == 10) {
    if (node_lists) k_p2p_tile<10, true><<<nbl, 64, 0, s>>>(a);
    else k_p2p_tile<10, false><<<nbl, 64, 0, s>>>(a);
  } else if (ls == 16) {
    if (node_lists) k_p2p_tile<16, true><<<nbl, 64, 0, s>>>(a);
    else k_p2p_tile<16, false><<<nbl, 64, 0, s>>>(a);
  } else {
    if (node_lists) k_p2p_tile<32, true><<<nbl, 64, 0, s>>>(a);
    else k_p2p_tile<32, false><<<nbl, 64, 0, s>>>(a);
  }
}

}  // namespace sfmm
