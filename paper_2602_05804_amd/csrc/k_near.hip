// k_near.hip -- near field (P2P) and the output in the caller's order, plus
// the FP64 momentum diagnostics.
//
// P2P is the softened direct sum of Sect. 2, Eq. (softdirectsum), over the
// source leaves the walk cached for the particle's leaf (the self leaf
// included, j != i).  Softening: cubic spline with support 2h; for a pair
// with unequal h the two kernels are averaged, which keeps the pair force
// antisymmetric (Newton's third law).  Kernel shapes, with q = r/h:
//   force  f(q)/q:  4/3 - 6/5 q^2 + 1/2 q^3                       (q < 1)
//                   8/3 - 3 q + 6/5 q^2 - 1/6 q^3 - 1/(15 q^3)     (1 <= q < 2)
//                   1/q^3                                          (q >= 2)
//   potential:      7/5 - 2/3 q^2 + 3/10 q^4 - 1/10 q^5            (q < 1)
//                   8/5 - 4/3 q^2 + q^3 - 3/10 q^4 + 1/30 q^5 - 1/(15 q)
//                   1/q                                            (q >= 2)
// (force per unit separation = shape / h^3, potential = shape / h).
#include "sfmm_internal.h"
#include "softening.h"

namespace sfmm {
namespace {

template <bool NODE>
__global__ __launch_bounds__(256) void k_near(NearArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const double xi = a.xs[i], yi = a.ys[i], zi = a.zs[i], hi = a.hs[i];
  const double hinv_i = 1.0 / hi;
  const int leaf = a.p_leaf[i];
  uint64_t e0, e1;
  const int32_t* list;
  if (NODE) {
    const int node = a.leaf_node[leaf];
    e0 = a.node_p2p_off[node];
    e1 = e0 + a.node_p2p_cnt[node];
    list = reinterpret_cast<const int32_t*>(a.node_p2p_pool);
  } else {
    e0 = a.p2p_off[leaf];
    e1 = a.p2p_off[leaf + 1];
    list = a.p2p_list;
  }
  double fx = 0.0, fy = 0.0, fz = 0.0, ph = 0.0;
  for (uint64_t e = e0; e < e1; ++e) {
    const NodeInfo si = a.info[list[e]];
    for (int j = si.lo; j < si.lo + si.cnt; ++j) {
      if (j == i) continue;
      const double dx = xi - a.xs[j], dy = yi - a.ys[j], dz = zi - a.zs[j];
      const double r2 = dx * dx + dy * dy + dz * dz;
      const double hj = a.hs[j], mj = a.ms[j];
      const double hm = fmax(hi, hj);
      double gs, ps;
      if (r2 >= 4.0 * hm * hm) {
        const double rinv = rsqrt(r2);
        gs = rinv * rinv * rinv;
        ps = rinv;
      } else {
        const double r = sqrt(r2);
        double g1, p1, g2, p2;
        if (r >= 2.0 * hi) {
          const double rinv = 1.0 / r;
          g1 = rinv * rinv * rinv; p1 = rinv;
        } else {
          soft(r, hinv_i, g1, p1);
        }
        if (r >= 2.0 * hj) {
          const double rinv = 1.0 / r;
          g2 = rinv * rinv * rinv; p2 = rinv;
        } else {
          soft(r, 1.0 / hj, g2, p2);
        }
        gs = 0.5 * (g1 + g2);
        ps = 0.5 * (p1 + p2);
      }
      const double mg = mj * gs;
      fx = fma(mg, dx, fx);
      fy = fma(mg, dy, fy);
      fz = fma(mg, dz, fz);
      ph = fma(mj, ps, ph);
    }
  }
  if (a.include_self) ph = fma(a.ms[i], 1.4 * hinv_i, ph);
  // far[] holds the L2P field F and potential polynomial (acc = -G F); the
  // near sums above use the same convention: acc = -G (F + f), pot = -G (P + ph).
  const double* fr = a.far + 4 * (int64_t)i;
  const double G = a.G;
  const int64_t o = a.perm[i];
  a.acc[3 * o] = -G * (fr[0] + fx);
  a.acc[3 * o + 1] = -G * (fr[1] + fy);
  a.acc[3 * o + 2] = -G * (fr[2] + fz);
  a.pot[o] = -G * (fr[3] + ph);
}

// ---- wave per target leaf ----------------------------------------------------
// The leaf's particles (at most LS) are wave-uniform and held in registers;
// the lanes walk the flattened list of source particles of the leaf's P2P
// sources, 64 at a time, and each lane accumulates the field of its source on
// every target.  A butterfly reduction then gives each target its total.
__device__ __forceinline__ int wave_incl_scan(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Targets in LDS, in passes of TG targets each, fully unrolled (static
// accumulator indices; nt is the same on every lane, so the guard is a scalar
// branch); the sources are read once per pass.  Pairs inside a kernel are not
// evaluated in the wave's pass over the sources (where most lanes would idle
// through the softening branch) but queued in LDS as (target, source); every
// 64 queued pairs are evaluated together, one per lane, and added to the same
// per-target accumulators.
template <int LS, bool NODE, int TG>
__global__ __launch_bounds__(64) void k_p2p_leaf(NearArgs a) {
  constexpr int NA = TG;  // accumulators per pass
  const int lane = threadIdx.x;
  const uint32_t item = blockIdx.x;
  if (item >= a.item_off[a.nleaves]) return;  // the grid is an upper bound
  const int l = a.item_leaf[item];
  const uint32_t kitem = a.item_k[item];
  const int node = a.leaf_node[l];
  const NodeInfo ti = a.info[node];
  const int nt = ti.cnt;
  // targets in LDS (read back as broadcasts): x, y, z, 1/h, h
  __shared__ double tg[LS][5];
  if (lane < nt) {
    const int j = ti.lo + lane;
    tg[lane][0] = a.xs[j]; tg[lane][1] = a.ys[j]; tg[lane][2] = a.zs[j];
    tg[lane][3] = a.his[j]; tg[lane][4] = a.hs[j];
  }
  __syncthreads();
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
  uint32_t carry0 = 0;
  if (kitem > 0) { e0 = a.item_e0[item]; carry0 = a.item_c0[item]; }
  __shared__ int qj[128];
  __shared__ int qi[128];
  uint32_t qn = 0;     // queued softened pairs (the same on every lane)
  uint32_t nsoft = 0;  // softened pairs of this item
  for (int t0 = 0; t0 < nt; t0 += NA) {
    double fx[NA], fy[NA], fz[NA], ph[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) { fx[i] = 0.0; fy[i] = 0.0; fz[i] = 0.0; ph[i] = 0.0; }
    // the softened pairs of queue slots [0, count), one per lane, into the
    // accumulators of their targets; the rest of the queue moves to the front
    auto flush = [&](uint32_t count) {
      __syncthreads();
      const bool act = (uint32_t)lane < count;
      const int j2 = act ? qj[lane] : ti.lo;
      const int i2 = act ? qi[lane] : 0;
      const double thi = tg[i2][3];
      const double dx = tg[i2][0] - a.xs[j2], dy = tg[i2][1] - a.ys[j2], dz = tg[i2][2] - a.zs[j2];
      const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
      const double rinv = rsqrt_pair(r2);
      const double rinv3 = rinv * rinv * rinv;
      const double r = r2 * rinv;
      const double hj = a.hs[j2], hjinv = a.his[j2];
      double g1, p1, g2, p2;
      soft_sel(r * thi, thi, tg[i2][4] * rinv, rinv, rinv3, g1, p1);
      soft_sel(r * hjinv, hjinv, hj * rinv, rinv, rinv3, g2, p2);
      const double w = act ? a.ms[j2] : 0.0;
      const double mg = w * (0.5 * (g1 + g2));
      const double cx = mg * dx, cy = mg * dy, cz = mg * dz, cp = w * (0.5 * (p1 + p2));
#pragma unroll
      for (int ii = 0; ii < NA; ++ii) {
        if (act && i2 == t0 + ii) {
          fx[ii] += cx; fy[ii] += cy; fz[ii] += cz; ph[ii] += cp;
        }
      }
      const uint32_t rem = qn - count;
      int tj = 0, tq = 0;
      if ((uint32_t)lane < rem) { tj = qj[count + lane]; tq = qi[count + lane]; }
      __syncthreads();
      if ((uint32_t)lane < rem) { qj[lane] = tj; qi[lane] = tq; }
      qn = rem;
      __syncthreads();
    };
    uint32_t carry = carry0;  // sources of the list entries before c0
    for (uint64_t c0 = e0; c0 < e1; c0 += 64) {
      // 64 list entries: their particle ranges [fb, fe) in the flattened
      // order, then clipped to the run
      int cnt = 0, lo = 0;
      uint32_t fb = 0xffffffffu;
      NodeInfo si{};
      if (c0 + lane < e1) si = a.info[list[c0 + lane]];
      const int sincl = wave_incl_scan(c0 + lane < e1 ? si.cnt : 0);
      if (c0 + lane < e1) {
        const uint32_t fe = carry + (uint32_t)sincl;
        fb = fe - (uint32_t)si.cnt;
        const uint32_t b = fb > f_lo ? fb : f_lo;
        const uint32_t en = fe < f_hi ? fe : f_hi;
        if (en > b) { cnt = (int)(en - b); lo = si.lo + (int)(b - fb); }
      }
      carry += (uint32_t)__shfl(sincl, 63, 64);
      if (__shfl((int)fb, 0, 64) >= (int)f_hi) break;  // the run is done (uniform)
      const int incl = wave_incl_scan(cnt);
      const int pre = incl - cnt;
      const int total = __shfl(incl, 63, 64);
      for (int f0 = 0; f0 < total; f0 += 64) {
        const int f = f0 + lane;
        // owner lane k: the last lane with pre <= f (binary search over lanes)
        int k = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1) {
          const int pk = __shfl(pre, k + step, 64);
          if (pk <= f) k += step;
        }
        const int jj = __shfl(lo, k, 64) + (f - __shfl(pre, k, 64));
        // lanes past the window's end stay in step with the others (the queue
        // count and its barriers are per wave) and contribute nothing
        const bool fv = f < total;
        const int j = fv ? jj : ti.lo;
        const double xj = a.xs[j], yj = a.ys[j], zj = a.zs[j], mj = a.ms[j];
        const double hjinv = a.his[j];
        const double hj2inv = hjinv * hjinv;
#pragma unroll
        for (int ii = 0; ii < NA; ++ii) {
          const int i = t0 + ii;
          if (i >= nt) continue;
          const double w = (!fv || j == ti.lo + i) ? 0.0 : mj;  // the pair (i, i) is skipped
          const double thi = tg[i][3];
          const double dx = tg[i][0] - xj, dy = tg[i][1] - yj, dz = tg[i][2] - zj;
          const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
          const double rinv = rsqrt_pair(r2);
          const double rinv3 = rinv * rinv * rinv;
          const bool inside = fv && ((r2 * (thi * thi) < 4.0) || (r2 * hj2inv < 4.0));
          const bool push = inside && w != 0.0;
          const uint64_t bal = __ballot(push);
          if (bal) {
            const uint32_t below =
                __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
            if (push) { qj[qn + below] = j; qi[qn + below] = i; }
            qn += (uint32_t)__popcll(bal);
            nsoft += (uint32_t)__popcll(bal);
          }
          // both kernels at q >= 2 outside; a pair inside went to the queue
          const double wq = inside ? 0.0 : w;
          const double mg = wq * rinv3;
          fx[ii] = fma(mg, dx, fx[ii]);
          fy[ii] = fma(mg, dy, fy[ii]);
          fz[ii] = fma(mg, dz, fz[ii]);
          ph[ii] = fma(wq, rinv, ph[ii]);
          if (qn >= 64) flush(64);
        }
      }
    }
    if (qn > 0) flush(qn);
#pragma unroll
    for (int ii = 0; ii < NA; ++ii) {
      const int i = t0 + ii;
      if (i >= nt) break;
      const double sx = wave_sum(fx[ii]), sy = wave_sum(fy[ii]), sz = wave_sum(fz[ii]);
      const double sp = wave_sum(ph[ii]);
      if (lane == i) {
        double* o = a.part + ((int64_t)item * LS + i) * 4;
        o[0] = sx; o[1] = sy; o[2] = sz; o[3] = sp;
      }
    }
  }
  if (lane == 0 && nsoft) atomicAdd(a.soft_pairs, (unsigned long long)nsoft);
}

// Wave per item, targets held in scalar registers.  The same sums as
// k_p2p_leaf with less work per pair: the loop control is wave-uniform
// (scalar), the targets of a pass are wave-uniform values, a pair is inside
// a kernel when r^2 < max(4 h_i^2, 4 h_j^2), and the field of a pair beyond
// both kernels is m/r^3 (dx, dy, dz) and m/r, with the refined 1/r replaced
// by 0 for pairs inside a kernel (the self pair and coincident particles
// included: r^2 = 0 is always inside).  Pairs inside a kernel, other than
// the self pair, go to a queue per target in LDS and are evaluated 64 at a
// time, each batch for one target (so its data stay wave-uniform), after
// each group of 64 sources has met the pass's targets.  A leaf's targets
// are taken in passes of TG and one pass of the remainder, each with a fixed
// target count (no per-target exits inside the unrolled loop).
struct WaveItem {
  int tlo, nt;
  uint64_t e0, e1;
  const int32_t* list;
  uint32_t f_lo, f_hi;
  uint32_t carry0;  // the flattened start of entry e0
  int64_t item;
};

constexpr uint32_t kTQ = 192;  // queue slots per target (63 + 64 U, U <= 2)

// U groups of 64 sources per step: their index searches and loads are
// independent, so a wave keeps U chains of latency in flight
template <int K, int LS, int U>
__device__ __forceinline__ void p2p_wave_pass(const NearArgs& a, const WaveItem& w, int t0,
                                              int* q, uint32_t& nsoft) {
  const int lane = threadIdx.x;
  const int tlo = w.tlo;
  double tx[K], ty[K], tz[K], t4[K];
  double fx[K], fy[K], fz[K], ph[K];
  uint32_t qh[K], qn[K];  // per-target ring queue head and length (wave-uniform)
#pragma unroll
  for (int ii = 0; ii < K; ++ii) {
    const int it = tlo + t0 + ii;
    tx[ii] = wave_uniform(a.xs[it]);
    ty[ii] = wave_uniform(a.ys[it]);
    tz[ii] = wave_uniform(a.zs[it]);
    const double hu = wave_uniform(a.hs[it]);
    t4[ii] = 4.0 * hu * hu;
    fx[ii] = 0.0; fy[ii] = 0.0; fz[ii] = 0.0; ph[ii] = 0.0;
    qh[ii] = 0; qn[ii] = 0;
  }
  // the first `count` queued sources of target ii, one per lane
  auto flush = [&](auto iic, uint32_t count) {
    constexpr int ii = decltype(iic)::value;
    __syncthreads();
    const bool act = (uint32_t)lane < count;
    uint32_t slot = qh[ii] + (uint32_t)lane;
    if (slot >= kTQ) slot -= kTQ;
    const int j2 = act ? q[ii * kTQ + slot] : tlo;
    const int it = tlo + t0 + ii;  // wave-uniform
    const double hi = wave_uniform(a.hs[it]), hiinv = wave_uniform(a.his[it]);
    const double2* rj = reinterpret_cast<const double2*>(a.p4 + 4 * (int64_t)j2);
    const double2 sxy = rj[0], szm = rj[1];
    const double dx = tx[ii] - sxy.x, dy = ty[ii] - sxy.y, dz = tz[ii] - szm.x;
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const double rinv = rsqrt_pair(r2);
    const double rinv3 = rinv * rinv * rinv;
    const double r = r2 * rinv;
    const double hj = a.hs[j2], hjinv = a.his[j2];
    double g1, p1, g2, p2;
    soft_sel(r * hiinv, hiinv, hi * rinv, rinv, rinv3, g1, p1);
    soft_sel(r * hjinv, hjinv, hj * rinv, rinv, rinv3, g2, p2);
    const double wm = act ? szm.y : 0.0;
    const double mg = wm * (0.5 * (g1 + g2));
    fx[ii] = fma(mg, dx, fx[ii]);
    fy[ii] = fma(mg, dy, fy[ii]);
    fz[ii] = fma(mg, dz, fz[ii]);
    ph[ii] = fma(wm, 0.5 * (p1 + p2), ph[ii]);
    qh[ii] += count;
    if (qh[ii] >= kTQ) qh[ii] -= kTQ;
    qn[ii] -= count;
  };
  uint32_t carry = w.carry0;  // sources of the list entries before c0 (wave-uniform)
  for (uint64_t c0 = w.e0; c0 < w.e1; c0 += 64) {
    // 64 list entries: their particle ranges [fb, fe) in the flattened
    // order, then clipped to the run
    int cnt = 0, lo = 0;
    uint32_t fb = 0xffffffffu;
    NodeInfo si{};
    const bool in = c0 + lane < w.e1;
    if (in) si = a.info[w.list[c0 + lane]];
    const int sincl = wave_incl_scan(in ? si.cnt : 0);
    if (in) {
      const uint32_t fe = carry + (uint32_t)sincl;
      fb = fe - (uint32_t)si.cnt;
      const uint32_t b = fb > w.f_lo ? fb : w.f_lo;
      const uint32_t en = fe < w.f_hi ? fe : w.f_hi;
      if (en > b) { cnt = (int)(en - b); lo = si.lo + (int)(b - fb); }
    }
    carry += (uint32_t)__builtin_amdgcn_readlane(sincl, 63);
    // lane 0 always holds an entry (c0 < e1)
    if ((uint32_t)__builtin_amdgcn_readfirstlane(fb) >= w.f_hi) break;  // the run is done
    const int incl = wave_incl_scan(cnt);
    const int pre = incl - cnt;
    const int total = __builtin_amdgcn_readlane(incl, 63);
    for (int f0 = 0; f0 < total; f0 += 64 * U) {
      int j[U];
      bool fv[U];
      double xj[U], yj[U], zj[U], mj[U], h4j[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int f = f0 + 64 * u + lane;
        // owner lane k: the last lane with pre <= f (binary search over lanes)
        int k = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1) {
          const int pk = __shfl(pre, k + step, 64);
          if (pk <= f) k += step;
        }
        const int jj = __shfl(lo, k, 64) + (f - __shfl(pre, k, 64));
        fv[u] = f < total;
        j[u] = fv[u] ? jj : tlo;  // a valid index; contributes nothing
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double2* rj = reinterpret_cast<const double2*>(a.p4 + 4 * (int64_t)j[u]);
        const double2 sxy = rj[0], szm = rj[1];
        const double hj = a.hs[j[u]];
        xj[u] = sxy.x;
        yj[u] = sxy.y;
        zj[u] = szm.x;
        mj[u] = fv[u] ? szm.y : 0.0;
        h4j[u] = 4.0 * hj * hj;
      }
#pragma unroll
      for (int ii = 0; ii < K; ++ii) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const double dx = tx[ii] - xj[u], dy = ty[ii] - yj[u], dz = tz[ii] - zj[u];
          const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
          const bool inside = r2 < fmax(t4[ii], h4j[u]);
          const double rinv = inside ? 0.0 : rsqrt_refined(r2);
          const double mr = mj[u] * rinv;
          const double mg = mr * (rinv * rinv);
          fx[ii] = fma(mg, dx, fx[ii]);
          fy[ii] = fma(mg, dy, fy[ii]);
          fz[ii] = fma(mg, dz, fz[ii]);
          ph[ii] += mr;
          // (an empty statement that reads the sums: keeps this target's
          // arithmetic ahead of the queue branch below, so that the compiler
          // does not move it past the branches of the later targets and hold
          // every target's separation vector at once)
          asm volatile("" ::"v"(fx[ii]), "v"(fy[ii]), "v"(fz[ii]), "v"(ph[ii]));
          const bool push = inside && fv[u] && j[u] != tlo + t0 + ii;
          const uint64_t bal = __builtin_amdgcn_ballot_w64(push);
          if (bal) {
            if (push) {
              const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                  (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
              uint32_t sl = qh[ii] + qn[ii] + below;
              if (sl >= kTQ) sl -= kTQ;
              q[ii * kTQ + sl] = j[u];
            }
            const uint32_t c = (uint32_t)__popcll(bal);
            qn[ii] += c;
            nsoft += c;
          }
        }
      }
      // a queue holds at most 63 + 64 U entries here
      static_for<K>([&](auto iic) {
        constexpr int ii = decltype(iic)::value;
        while (qn[ii] >= 64) flush(iic, 64);
      });
    }
  }
  static_for<K>([&](auto iic) {
    constexpr int ii = decltype(iic)::value;
    if (qn[ii] > 0) flush(iic, qn[ii]);
  });
#pragma unroll
  for (int ii = 0; ii < K; ++ii) {
    const double sx = wave_sum(fx[ii]), sy = wave_sum(fy[ii]), sz = wave_sum(fz[ii]);
    const double sp = wave_sum(ph[ii]);
    if (lane == t0 + ii) {
      double* o = a.part + (w.item * LS + t0 + ii) * 4;
      o[0] = sx; o[1] = sy; o[2] = sz; o[3] = sp;
    }
  }
}

template <int LS, bool NODE, int TG, int WPE, int U>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE))) void k_p2p_wave(
    NearArgs a) {
  const int lane = threadIdx.x;
  const uint32_t item = xcd_block(blockIdx.x, gridDim.x);
  if (item >= a.item_off[a.nleaves]) return;  // the grid is an upper bound
  const int l = a.item_leaf[item];
  const uint32_t kitem = a.item_k[item];
  const int node = a.leaf_node[l];
  const NodeInfo ti = a.info[node];
  WaveItem w;
  w.tlo = ti.lo;
  w.nt = ti.cnt;
  w.item = item;
  if (NODE) {
    w.e0 = a.node_p2p_off[node];
    w.e1 = w.e0 + a.node_p2p_cnt[node];
    w.list = reinterpret_cast<const int32_t*>(a.node_p2p_pool);
  } else {
    w.e0 = a.p2p_off[l];
    w.e1 = a.p2p_off[l + 1];
    w.list = a.p2p_list;
  }
  // this item's run [f_lo, f_hi) of the leaf's flattened sources, from the
  // list entry that holds its first source
  w.f_lo = kitem * kP2PItem;
  const uint32_t ftot = a.src_total[l];
  w.f_hi = w.f_lo + kP2PItem < ftot ? w.f_lo + kP2PItem : ftot;
  w.carry0 = 0;
  if (kitem > 0) { w.e0 = a.item_e0[item]; w.carry0 = a.item_c0[item]; }
  __shared__ int q[TG * kTQ];
  uint32_t nsoft = 0;
  int t0 = 0;
  for (; t0 + TG <= w.nt; t0 += TG) p2p_wave_pass<TG, LS, U>(a, w, t0, q, nsoft);
  // the remainder, a pass with a fixed target count (uniform branches)
  static_for<TG>([&](auto rc) {
    constexpr int r = decltype(rc)::value;
    if (r > 0 && w.nt - t0 == r) p2p_wave_pass<(r > 0 ? r : 1), LS, U>(a, w, t0, q, nsoft);
  });
  if (lane == 0 && nsoft) atomicAdd(a.soft_pairs, (unsigned long long)nsoft);
}

// per leaf, the particles over its P2P list entries and its work items:
// max(1, ceil(sources / kP2PItem)).  One wave per leaf.  (The level walk
// computes both in its leaf pass.)
template <bool NODE>
__global__ __launch_bounds__(64) void k_p2p_items_count(NearArgs a, uint32_t* __restrict__ src_total,
                                                        uint32_t* __restrict__ cnt) {
  const int l = blockIdx.x;
  const int lane = threadIdx.x;
  uint64_t e0, e1;
  const int32_t* list;
  if (NODE) {
    const int node = a.leaf_node[l];
    e0 = a.node_p2p_off[node];
    e1 = e0 + a.node_p2p_cnt[node];
    list = reinterpret_cast<const int32_t*>(a.node_p2p_pool);
  } else {
    e0 = a.p2p_off[l];
    e1 = a.p2p_off[l + 1];
    list = a.p2p_list;
  }
  uint32_t carry = 0;
  for (uint64_t c0 = e0; c0 < e1; c0 += 64) {
    const bool in = c0 + lane < e1;
    const int c = in ? a.info[list[c0 + lane]].cnt : 0;
    const int incl = wave_incl_scan(c);
    carry += (uint32_t)__shfl(incl, 63, 64);
  }
  if (lane == 0) {
    src_total[l] = carry;
    const uint32_t k = (carry + kP2PItem - 1) / kP2PItem;
    cnt[l] = k > 0 ? k : 1u;
  }
}

// item_leaf / item_k of every item, and for each item after a leaf's first
// the list entry holding its first source and that entry's start in the
// flattened order (item k starts at source k * kP2PItem).  One wave per
// kFillLeaves leaves: a lane per leaf for the first two, then the whole wave
// scans the list of each of its leaves with more than one item (a few in a
// hundred, so a wave meets about one).
constexpr int kFillLeaves = 16;
constexpr int kFillGroups = 8;
template <bool NODE>
__global__ __launch_bounds__(64) void k_p2p_items_fill(NearArgs a, int32_t* __restrict__ item_leaf,
                                                       uint32_t* __restrict__ item_k,
                                                       uint32_t* __restrict__ item_e0,
                                                       uint32_t* __restrict__ item_c0) {
  const int lane = threadIdx.x;
  const int lme = blockIdx.x * kFillLeaves + lane;
  uint32_t nb = 0, ne = 0;
  if (lane < kFillLeaves && lme < a.nleaves) {
    nb = a.item_off[lme];
    ne = a.item_off[lme + 1];
    for (uint32_t t = nb; t < ne; ++t) {
      item_leaf[t] = lme;
      item_k[t] = t - nb;
    }
  }
  uint64_t multi = __ballot(ne - nb > 1);
  while (multi) {
    const int q = __builtin_ctzll(multi);
    multi &= multi - 1;
    const int l = blockIdx.x * kFillLeaves + q;
    const uint32_t b = (uint32_t)__shfl((int)nb, q, 64), e = (uint32_t)__shfl((int)ne, q, 64);
    uint64_t e0, e1;
    const int32_t* list;
    if (NODE) {
      const int node = a.leaf_node[l];
      e0 = a.node_p2p_off[node];
      e1 = e0 + a.node_p2p_cnt[node];
      list = reinterpret_cast<const int32_t*>(a.node_p2p_pool);
    } else {
      e0 = a.p2p_off[l];
      e1 = a.p2p_off[l + 1];
      list = a.p2p_list;
    }
    // kFillGroups groups of 64 entries per step, their loads issued together
    // (the longest lists, a few thousand entries, set this kernel's time)
    uint32_t carry = 0;
    for (uint64_t c0 = e0; c0 < e1; c0 += 64 * kFillGroups) {
      int src[kFillGroups];
#pragma unroll
      for (int u = 0; u < kFillGroups; ++u) src[u] = c0 + 64 * u + lane < e1 ? list[c0 + 64 * u + lane] : -1;
      uint32_t cu[kFillGroups];
#pragma unroll
      for (int u = 0; u < kFillGroups; ++u) cu[u] = src[u] >= 0 ? (uint32_t)a.info[src[u]].cnt : 0u;
#pragma unroll
      for (int u = 0; u < kFillGroups; ++u) {
        const uint64_t g0 = c0 + 64 * u;
        if (g0 >= e1) break;  // (uniform)
        const bool in = g0 + lane < e1;
        const uint32_t c = cu[u];
        const int incl = wave_incl_scan((int)c);
        const uint32_t fe = carry + (uint32_t)incl, fb = fe - c;
        if (in && c > 0) {
          uint32_t k = (fb + kP2PItem - 1) / kP2PItem;
          if (k == 0) k = 1;
          for (; k * kP2PItem < fe && b + k < e; ++k) {
            item_e0[b + k] = (uint32_t)(g0 + lane);
            item_c0[b + k] = fb;
          }
        }
        carry += (uint32_t)__shfl(incl, 63, 64);
      }
    }
  }
}

// one thread per sorted particle: its items' partial sums in item order,
// the far field and the self term, in the caller's order
__global__ void k_p2p_reduce(NearArgs a, int ls) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n) return;
  const int l = a.p_leaf[j];
  const uint32_t t0 = a.item_off[l], t1 = a.item_off[l + 1];
  const int i = j - a.info[a.leaf_node[l]].lo;
  double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0;
  for (uint32_t t = t0; t < t1; ++t) {
    const double* q = a.part + ((int64_t)t * ls + i) * 4;
    sx += q[0]; sy += q[1]; sz += q[2]; sp += q[3];
  }
  if (a.include_self) sp = fma(a.ms[j], 1.4 * a.his[j], sp);
  const double* fr = a.far + 4 * (int64_t)j;
  const int64_t o = a.perm[j];
  const double G = a.G;
  a.acc[3 * o] = -G * (fr[0] + sx);
  a.acc[3 * o + 1] = -G * (fr[1] + sy);
  a.acc[3 * o + 2] = -G * (fr[2] + sz);
  a.pot[o] = -G * (fr[3] + sp);
}

constexpr int MOM_THREADS = 256;

__global__ __launch_bounds__(MOM_THREADS) void k_momentum_partial(int n, const double* __restrict__ m,
                                                                  const double* __restrict__ acc,
                                                                  double* __restrict__ part) {
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = blockIdx.x * MOM_THREADS + threadIdx.x; i < n; i += gridDim.x * MOM_THREADS) {
    const double F0 = m[i] * acc[3 * (int64_t)i], F1 = m[i] * acc[3 * (int64_t)i + 1],
                 F2 = m[i] * acc[3 * (int64_t)i + 2];
    s[0] += F0; s[1] += F1; s[2] += F2;
    s[3] += sqrt(F0 * F0 + F1 * F1 + F2 * F2);
  }
  __shared__ double sh[4][MOM_THREADS];
  for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] = s[c];
  __syncthreads();
  for (int w = MOM_THREADS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < 4; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) part[4 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_momentum_final(int nb, const double* __restrict__ part,
                                                        double* __restrict__ out) {
  // fixed summation tree: thread t sums partials t, t+64, ... of component
  // t / 64, then a fixed pairwise reduction
  __shared__ double sh[256];
  const int c = threadIdx.x >> 6, t = threadIdx.x & 63;
  double s = 0.0;
  for (int b = t; b < nb; b += 64) s += part[4 * b + c];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 32; w > 0; w >>= 1) {
    if (t < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (t == 0) out[c] = sh[threadIdx.x];
}

}  // namespace

#define WAVE_LAUNCH(LS, TG, WPE)                                           \
  do {                                                                     \
    if (node_lists) k_p2p_wave<LS, true, TG, WPE, 1><<<nbl, 64, 0, s>>>(a); \
    else k_p2p_wave<LS, false, TG, WPE, 1><<<nbl, 64, 0, s>>>(a);          \
    record_mark(km.end, s);                                                \
    if (!km.skip_reduce) launch_p2p_reduce(a, LS, s);                      \
  } while (0)

#define NEAR_LAUNCH(LS, TG)                                                \
  do {                                                                     \
    if (node_lists) k_p2p_leaf<LS, true, TG><<<nbl, 64, 0, s>>>(a);        \
    else k_p2p_leaf<LS, false, TG><<<nbl, 64, 0, s>>>(a);                  \
    record_mark(km.end, s);                                                \
    if (!km.skip_reduce) launch_p2p_reduce(a, LS, s);                      \
  } while (0)

void launch_p2p_items_count(bool node_lists, const NearArgs& a, uint32_t* src_total,
                            uint32_t* item_cnt, hipStream_t s) {
  if (a.nleaves <= 0) return;
  if (node_lists) k_p2p_items_count<true><<<a.nleaves, 64, 0, s>>>(a, src_total, item_cnt);
  else k_p2p_items_count<false><<<a.nleaves, 64, 0, s>>>(a, src_total, item_cnt);
}

void launch_p2p_items_fill(bool node_lists, const NearArgs& a, int32_t* item_leaf,
                           uint32_t* item_k, uint32_t* item_e0, uint32_t* item_c0, hipStream_t s) {
  if (a.nleaves <= 0) return;
  const unsigned nb = (unsigned)((a.nleaves + kFillLeaves - 1) / kFillLeaves);
  if (node_lists)
    k_p2p_items_fill<true><<<nb, 64, 0, s>>>(a, item_leaf, item_k, item_e0, item_c0);
  else
    k_p2p_items_fill<false><<<nb, 64, 0, s>>>(a, item_leaf, item_k, item_e0, item_c0);
}

void launch_p2p_reduce(const NearArgs& a, int ls, hipStream_t s) {
  if (a.n <= 0) return;
  k_p2p_reduce<<<blocks_for(a.n, 256), 256, 0, s>>>(a, ls);
}

void launch_near(bool node_lists, int leaf_size, int variant, const NearArgs& a, int64_t items,
                 hipStream_t s, KernelMarks km) {
  if (a.n <= 0) return;
  const unsigned nbl = (unsigned)items;
  record_mark(km.begin, s);
  if (variant == 1) leaf_size = 1 << 20;  // particle per thread
  // variant (the shapes are listed with sfmm_config.near_kernel)
  if (leaf_size <= 32 && variant == 13) {
    launch_p2p_tile(node_lists, p2p_leaf_slots(leaf_size), a, items, s);
    record_mark(km.end, s);
    if (!km.skip_reduce) launch_p2p_reduce(a, p2p_leaf_slots(leaf_size), s);
    return;
  }
  // leaf_size <= 10: five targets per pass at four waves per SIMD; <= 16:
  // six at four (the shapes that won on the polytrope and Plummer workloads);
  // <= 32: eight at three
  if (leaf_size <= 10) {
    if (variant == 6) NEAR_LAUNCH(10, 5);
    else WAVE_LAUNCH(10, 5, 4);
  } else if (leaf_size <= 16) {
    if (variant == 6) NEAR_LAUNCH(16, 8);
    else WAVE_LAUNCH(16, 6, 4);
  } else if (leaf_size <= 32) {
    if (variant == 6) NEAR_LAUNCH(32, 8);
    else WAVE_LAUNCH(32, 8, 3);
  } else {
    if (node_lists) k_near<true><<<(a.n + 255) / 256, 256, 0, s>>>(a);
    else k_near<false><<<(a.n + 255) / 256, 256, 0, s>>>(a);
    record_mark(km.end, s);
  }
}

// leapfrog update of one system: v += kick * acc; x += drift * v
__global__ void k_leapfrog(int64_t n3, double* __restrict__ x, double* __restrict__ v,
                           const double* __restrict__ acc, double kick, double drift) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n3) return;
  // separate multiply and add (no contraction), as the update is written
  const double vi = v[i] + kick * acc[i];
  v[i] = vi;
  x[i] = x[i] + drift * vi;
}

void launch_leapfrog(int64_t n, double* x, double* v, const double* acc, double kick, double drift,
                     hipStream_t s) {
  if (n <= 0) return;
  const int64_t n3 = 3 * n;
  k_leapfrog<<<(unsigned)((n3 + 255) / 256), 256, 0, s>>>(n3, x, v, acc, kick, drift);
}

int momentum_blocks(int64_t n) {
  int64_t b = (n + MOM_THREADS * 8 - 1) / (MOM_THREADS * 8);
  if (b < 1) b = 1;
  if (b > 512) b = 512;
  return (int)b;
}

void launch_momentum(int n, const double* m, const double* acc, double* part, double* out,
                     hipStream_t s) {
  const int nb = momentum_blocks(n);
  k_momentum_partial<<<nb, MOM_THREADS, 0, s>>>(n, m, acc, part);
  k_momentum_final<<<1, 256, 0, s>>>(nb, part, out);
}

}  // namespace sfmm
