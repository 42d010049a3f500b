// k_f32c.hip -- the FP32-compensated form (SFMM_FP32C) of the far field and
// of P2P.
//
// Geometry, moments, the L2L chain and L2P stay in FP64.  The bulk terms run
// in FP32 and every term is added into an FP64 accumulator, which bounds the
// summation error below that of an FP32 hi/lo (TwoSum) pair at a lower cost
// here (an FP64 add issues at the FP32 rate).
//   M2L  targets at depth < top: FP64 as in k_far; deeper targets: the
//        separation of the two centres is formed in FP64 and rounded, the
//        moments are an FP32 copy, the derivatives and the contraction are
//        FP32 (Exp<P>::m2l_add_f32).
//   P2P  each particle carries its FP32 offset from its leaf's centre; a pair
//        (i in A, j in B) uses d = fl32(c_A - c_B) + (o_i - o_j), which is
//        exactly minus the separation seen from j, so each pair force is
//        antisymmetric.
#include "sfmm_internal.h"

namespace sfmm {
namespace {

template <int P>
__global__ void k_prep_nodes32(int nn, const double* __restrict__ rec,
                               const int32_t* __restrict__ node_depth, float* __restrict__ rec32) {
  constexpr int NQ = Exp<P>::NQ;
  constexpr int RS = rec_stride(P), RS32 = rec32_stride(P);
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nn) return;
  const double* r = rec + (int64_t)v * RS;
  float* o = rec32 + (int64_t)v * RS32;
#pragma unroll
  for (int k = 0; k < NQ; ++k) o[k] = (float)r[8 + k];
  o[NQ] = __int_as_float(node_depth[v]);
}

template <int RS>
__global__ void k_prep_particles32(int nleaves, const int32_t* __restrict__ leaf_node,
                                   const NodeInfo* __restrict__ info, const double* __restrict__ rec,
                                   const double* __restrict__ xs, const double* __restrict__ ys,
                                   const double* __restrict__ zs, const double* __restrict__ ms,
                                   const double* __restrict__ hs, float4* __restrict__ pf,
                                   float2* __restrict__ ph) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nleaves) return;
  const int v = leaf_node[l];
  const NodeInfo ni = info[v];
  const double* r = rec + (int64_t)v * RS;
  for (int j = ni.lo; j < ni.lo + ni.cnt; ++j) {
    pf[j] = make_float4((float)(xs[j] - r[0]), (float)(ys[j] - r[1]), (float)(zs[j] - r[2]),
                        (float)ms[j]);
    ph[j] = make_float2((float)hs[j], (float)(1.0 / hs[j]));
  }
}

// ---- far field -----------------------------------------------------------------
template <int P, bool NODE, int SPLIT>
__global__ __launch_bounds__(64) void k_far32(FarArgs a, const float* __restrict__ rec32, int top) {
  using E = Exp<P>;
  constexpr int NQ = E::NQ;
  constexpr int NL = E::NL;
  constexpr int RS = rec_stride(P), RS32 = rec32_stride(P);
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
  const uint32_t* list = NODE ? a.node_m2l_pool : a.m2l_list;
  const uint32_t* dc = NODE ? nullptr : a.depth_cnt + (active ? a.leaf_doff[l] : 0);
  uint64_t seg = NODE ? 0 : (active ? a.m2l_off[l] : 0);
  uint64_t e = 0, ne = 0;
  int v = 0, k = 0;
  double sv[3] = {rec[0], rec[1], rec[2]};
  if (d >= 0) {
    if (NODE) { e = a.node_m2l_off[0]; ne = e + a.node_m2l_cnt[0]; }
    else { e = seg; ne = seg + dc[0]; }
    e += sub;
  }
  // FP32 entries: source centre (FP64) and FP32 moments of the current entry,
  // with the next entry prefetched
  double cs[3] = {0.0, 0.0, 0.0};
  float cq[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) cq[q] = 0.f;
  uint32_t idx_next = 0;
  auto load32 = [&](uint32_t ent, double* sd, float* qd) {
    const uint32_t s = ent & kSrcMask;
    const double* rs = rec + (int64_t)s * RS;
    sd[0] = rs[0]; sd[1] = rs[1]; sd[2] = rs[2];
    const float* r32 = rec32 + (int64_t)s * RS32;
#pragma unroll
    for (int q = 0; q < NQ; ++q) qd[q] = r32[q];
  };
  auto start_depth = [&]() {
    if (k >= top && e < ne) {
      load32(list[e], cs, cq);
      idx_next = list[e + SPLIT < ne ? e + SPLIT : ne - 1];
    }
  };
  start_depth();
  for (;;) {
    if (e < ne) {
      if (k < top) {
        const double* rs = rec + (int64_t)(list[e] & kSrcMask) * RS;
        const double r[3] = {rs[0] - sv[0], rs[1] - sv[1], rs[2] - sv[2]};
        double Q[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) Q[q] = rs[8 + q];
        E::m2l_add(r, Q, L);
        e += SPLIT;
      } else {
        const uint64_t en = e + SPLIT;
        double ns[3];
        float nq[NQ];
        load32(idx_next, ns, nq);
        idx_next = list[en + SPLIT < ne ? en + SPLIT : ne - 1];
        const float r[3] = {(float)(cs[0] - sv[0]), (float)(cs[1] - sv[1]), (float)(cs[2] - sv[2])};
        E::m2l_add_f32(r, cq, L);
        e = en;
        cs[0] = ns[0]; cs[1] = ns[1]; cs[2] = ns[2];
#pragma unroll
        for (int q = 0; q < NQ; ++q) cq[q] = nq[q];
      }
      have = true;
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
#pragma unroll
  for (int o = SPLIT / 2; o > 0; o >>= 1) {
#pragma unroll
    for (int q = 0; q < NL; ++q) L[q] += __shfl_xor(L[q], o, 64);
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

// ---- P2P ------------------------------------------------------------------------
__device__ __forceinline__ void soft32(float q, float hinv, float qi, float rinv, float rinv3,
                                       float& g, float& psi) {
  const float q2 = q * q;
  const float h3 = hinv * hinv * hinv;
  const float gA = h3 * fmaf(q2, fmaf(0.5f, q, -1.2f), 4.0f / 3.0f);
  const float pA = hinv * fmaf(q2, fmaf(q2, fmaf(-0.1f, q, 0.3f), -2.0f / 3.0f), 1.4f);
  const float qi3 = qi * qi * qi;
  const float gB = h3 * (fmaf(q, fmaf(q, fmaf(q, -1.0f / 6.0f, 1.2f), -3.0f), 8.0f / 3.0f) -
                         qi3 * (1.0f / 15.0f));
  const float pB = hinv * (fmaf(q2, fmaf(q, fmaf(q, fmaf(q, 1.0f / 30.0f, -0.3f), 1.0f), -4.0f / 3.0f), 1.6f) -
                           qi * (1.0f / 15.0f));
  g = q >= 2.0f ? rinv3 : (q < 1.0f ? gA : gB);
  psi = q >= 2.0f ? rinv : (q < 1.0f ? pA : pB);
}

__device__ __forceinline__ int wave_incl_scan32(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// targets in passes of TG, each pass unrolled (static accumulator indices);
// the sources are read once per pass
template <int LS, bool NODE, int RS, int TG>
__global__ __launch_bounds__(64) void k_p2p_leaf32(NearArgs a, const float4* __restrict__ pf,
                                                   const float2* __restrict__ phh) {
  const int lane = threadIdx.x;
  const uint32_t item = blockIdx.x;
  if (item >= a.item_off[a.nleaves]) return;  // the grid is an upper bound
  const int l = a.item_leaf[item];
  const uint32_t kitem = a.item_k[item];
  const int node = a.leaf_node[l];
  const NodeInfo ti = a.info[node];
  const int nt = ti.cnt;
  const double* rt = a.rec + (int64_t)node * RS;
  const double ct0 = rt[0], ct1 = rt[1], ct2 = rt[2];
  __shared__ float tg[LS][5];  // offset x, y, z, 1/h, h
  if (lane < nt) {
    const float4 o = pf[ti.lo + lane];
    const float2 hh = phh[ti.lo + lane];
    tg[lane][0] = o.x; tg[lane][1] = o.y; tg[lane][2] = o.z;
    tg[lane][3] = hh.y; tg[lane][4] = hh.x;
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
  // this item's run [f_lo, f_hi) of the leaf's flattened sources
  const uint32_t f_lo = kitem * kP2PItem;
  const uint32_t ftot = a.src_total[l];
  const uint32_t f_hi = f_lo + kP2PItem < ftot ? f_lo + kP2PItem : ftot;
  uint32_t carry0 = 0;  // from the list entry that holds the run's first source
  if (kitem > 0) { e0 = a.item_e0[item]; carry0 = a.item_c0[item]; }
  uint32_t nsoft = 0;  // pairs inside a kernel (complete on lane 0)
  for (int t0 = 0; t0 < nt; t0 += TG) {
    double fx[TG], fy[TG], fz[TG], ph[TG];
#pragma unroll
    for (int i = 0; i < TG; ++i) { fx[i] = 0.0; fy[i] = 0.0; fz[i] = 0.0; ph[i] = 0.0; }
    uint32_t carry = carry0;  // sources of the list entries before c0
    for (uint64_t c0 = e0; c0 < e1; c0 += 64) {
      int cnt = 0, lo = 0, sub = 0;
      uint32_t fb = 0xffffffffu;
      float dcx = 0.f, dcy = 0.f, dcz = 0.f;
      const bool in = c0 + lane < e1;
      const int src = in ? list[c0 + lane] : 0;
      NodeInfo si{};
      if (in) si = a.info[src];
      const int sincl = wave_incl_scan32(in ? si.cnt : 0);
      if (in) {
        const uint32_t fe = carry + (uint32_t)sincl;
        fb = fe - (uint32_t)si.cnt;
        const uint32_t b = fb > f_lo ? fb : f_lo;
        const uint32_t en = fe < f_hi ? fe : f_hi;
        if (en > b) { cnt = (int)(en - b); lo = si.lo + (int)(b - fb); }
        // a whole subtree: its particles' offsets are relative to their own
        // leaves, whose centres are looked up per particle
        sub = si.child >= 0 ? 1 : 0;
        const double* rs = a.rec + (int64_t)src * RS;
        dcx = (float)(ct0 - rs[0]);
        dcy = (float)(ct1 - rs[1]);
        dcz = (float)(ct2 - rs[2]);
      }
      carry += (uint32_t)__shfl(sincl, 63, 64);
      if (__shfl((int)fb, 0, 64) >= (int)f_hi) break;  // the run is done (uniform)
      const int incl = wave_incl_scan32(cnt);
      const int pre = incl - cnt;
      const int total = __shfl(incl, 63, 64);
      for (int f0 = 0; f0 < total; f0 += 64) {
        const int f = f0 + lane;
        int k = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1) {
          const int pk = __shfl(pre, k + step, 64);
          if (pk <= f) k += step;
        }
        const int j = __shfl(lo, k, 64) + (f - __shfl(pre, k, 64));
        float cx = __shfl(dcx, k, 64), cy = __shfl(dcy, k, 64), cz = __shfl(dcz, k, 64);
        const int jsub = __shfl(sub, k, 64);
        if (f >= total) continue;
        if (jsub) {
          const double* rl = a.rec + (int64_t)a.leaf_node[a.p_leaf[j]] * RS;
          cx = (float)(ct0 - rl[0]);
          cy = (float)(ct1 - rl[1]);
          cz = (float)(ct2 - rl[2]);
        }
        const float4 oj = pf[j];
        const float2 hj = phh[j];
        const float hj2inv = hj.y * hj.y;
#pragma unroll
        for (int ii = 0; ii < TG; ++ii) {
          const int i = t0 + ii;
          if (i >= nt) continue;
          const float w = (j == ti.lo + i) ? 0.f : oj.w;
          const float thi = tg[i][3];
          const float dx = cx + (tg[i][0] - oj.x);
          const float dy = cy + (tg[i][1] - oj.y);
          const float dz = cz + (tg[i][2] - oj.z);
          const float r2 = dx * dx + dy * dy + dz * dz;
          const float rinv = r2 > 0.f ? __frsqrt_rn(r2) : 0.f;
          const float rinv3 = rinv * rinv * rinv;
          float gs = rinv3, ps = rinv;
          const bool inside = (r2 * (thi * thi) < 4.0f) || (r2 * hj2inv < 4.0f);
          nsoft += (uint32_t)__popcll(__ballot(inside && w != 0.f));  // lane 0 is always active
          if (__ballot(inside)) {
            const float r = r2 * rinv;
            float g1, p1, g2, p2;
            soft32(r * thi, thi, tg[i][4] * rinv, rinv, rinv3, g1, p1);
            soft32(r * hj.y, hj.y, hj.x * rinv, rinv, rinv3, g2, p2);
            if (inside) {
              gs = 0.5f * (g1 + g2);
              ps = 0.5f * (p1 + p2);
            }
          }
          const float mg = w * gs;
          fx[ii] += (double)(mg * dx);
          fy[ii] += (double)(mg * dy);
          fz[ii] += (double)(mg * dz);
          ph[ii] += (double)(w * ps);
        }
      }
    }
#pragma unroll
    for (int ii = 0; ii < TG; ++ii) {
      const int i = t0 + ii;
      if (i >= nt) break;
      const double sx = wave_sum64(fx[ii]), sy = wave_sum64(fy[ii]), sz = wave_sum64(fz[ii]);
      const double sp = wave_sum64(ph[ii]);
      if (lane == i) {
        double* o = a.part + ((int64_t)item * LS + i) * 4;
        o[0] = sx; o[1] = sy; o[2] = sz; o[3] = sp;
      }
    }
  }
  if (lane == 0 && nsoft) atomicAdd(a.soft_pairs, (unsigned long long)nsoft);
}

// ---- P2P, wave per item with the targets in scalar registers -------------------
// The FP32 form of k_p2p_wave (k_near.hip): wave-uniform loop control, the
// targets of a pass (FP32 offsets and 4 h^2) as wave-uniform values, the
// field of a pair beyond both kernels as m/r^3 (dx, dy, dz) and m/r with 1/r
// replaced by 0 inside a kernel, and the pairs inside a kernel queued per
// target (with the pair's FP32 centre difference) and evaluated 64 at a
// time.  Every term is added into FP64 sums.
__device__ __forceinline__ float wave_uniform_f(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

struct Wave32Item {
  int tlo, nt;
  uint64_t e0, e1;
  const int32_t* list;
  uint32_t f_lo, f_hi, carry0;
  int64_t item;
  double ct0, ct1, ct2;  // the target leaf's centre
};

constexpr uint32_t kTQ32 = 128;  // queue slots per target (63 + 64)

// Sums of FP32 pair terms: each term added to an FP64 accumulator (AccD, the
// default), or compensated in FP32 (AccT: Knuth's TwoSum keeps the rounding
// error of every addition, hi + lo is rounded to FP64 once at the end).
struct AccD {
  double v = 0.0;
  __device__ __forceinline__ void add(float x) { v += (double)x; }
  __device__ __forceinline__ double get() const { return v; }
  __device__ __forceinline__ void keep() { asm volatile("" ::"v"(v)); }
};
struct AccT {
  float hi = 0.f, lo = 0.f;
  __device__ __forceinline__ void add(float x) {
    const float s = hi + x;
    const float bb = s - hi;
    const float e = (hi - (s - bb)) + (x - bb);
    hi = s;
    lo += e;
  }
  __device__ __forceinline__ double get() const { return (double)hi + (double)lo; }
  __device__ __forceinline__ void keep() { asm volatile("" ::"v"(hi), "v"(lo)); }
};

template <int K, int LS, int RS, typename Acc>
__device__ __forceinline__ void p2p_wave32_pass(const NearArgs& a, const float4* __restrict__ pf,
                                                const float2* __restrict__ phh, const Wave32Item& w,
                                                int t0, int* qj, float* qc, uint32_t& nsoft) {
  const int lane = threadIdx.x;
  const int tlo = w.tlo;
  float tx[K], ty[K], tz[K], t4[K];
  Acc fx[K], fy[K], fz[K], ph[K];
  uint32_t qn[K];
#pragma unroll
  for (int ii = 0; ii < K; ++ii) {
    const float4 o = pf[tlo + t0 + ii];
    tx[ii] = wave_uniform_f(o.x);
    ty[ii] = wave_uniform_f(o.y);
    tz[ii] = wave_uniform_f(o.z);
    const float hu = wave_uniform_f(phh[tlo + t0 + ii].x);
    t4[ii] = 4.0f * hu * hu;
    fx[ii] = Acc(); fy[ii] = Acc(); fz[ii] = Acc(); ph[ii] = Acc();
    qn[ii] = 0;
  }
  // the first `count` queued pairs of target ii (the rest moves down)
  auto flush = [&](auto iic, uint32_t count) {
    constexpr int ii = decltype(iic)::value;
    __syncthreads();
    const bool act = (uint32_t)lane < count;
    int* qjt = qj + ii * kTQ32;
    float* qct = qc + ii * kTQ32 * 3;
    const int j2 = act ? qjt[lane] : tlo;
    const float cx = act ? qct[3 * lane] : 0.f, cy = act ? qct[3 * lane + 1] : 0.f,
                cz = act ? qct[3 * lane + 2] : 0.f;
    const float2 th = phh[tlo + t0 + ii];
    const float hi = wave_uniform_f(th.x), hiinv = wave_uniform_f(th.y);
    const float4 oj = pf[j2];
    const float2 hj = phh[j2];
    const float dx = cx + (tx[ii] - oj.x), dy = cy + (ty[ii] - oj.y), dz = cz + (tz[ii] - oj.z);
    const float r2 = dx * dx + dy * dy + dz * dz;
    const float rinv = r2 > 0.f ? __frsqrt_rn(r2) : 0.f;
    const float rinv3 = rinv * rinv * rinv;
    const float r = r2 * rinv;
    float g1, p1, g2, p2;
    soft32(r * hiinv, hiinv, hi * rinv, rinv, rinv3, g1, p1);
    soft32(r * hj.y, hj.y, hj.x * rinv, rinv, rinv3, g2, p2);
    const float wm = act ? oj.w : 0.f;
    const float mg = wm * (0.5f * (g1 + g2));
    fx[ii].add(mg * dx);
    fy[ii].add(mg * dy);
    fz[ii].add(mg * dz);
    ph[ii].add(wm * (0.5f * (p1 + p2)));
    // the remainder moves to the front of the queue
    const uint32_t rem = qn[ii] - count;
    int tj = 0;
    float ta = 0.f, tb = 0.f, tc = 0.f;
    if ((uint32_t)lane < rem) {
      tj = qjt[count + lane];
      ta = qct[3 * (count + lane)]; tb = qct[3 * (count + lane) + 1]; tc = qct[3 * (count + lane) + 2];
    }
    __syncthreads();
    if ((uint32_t)lane < rem) {
      qjt[lane] = tj;
      qct[3 * lane] = ta; qct[3 * lane + 1] = tb; qct[3 * lane + 2] = tc;
    }
    qn[ii] = rem;
  };
  uint32_t carry = w.carry0;  // sources of the list entries before c0 (wave-uniform)
  for (uint64_t c0 = w.e0; c0 < w.e1; c0 += 64) {
    // 64 list entries: their particle ranges [fb, fe) in the flattened
    // order, clipped to the run; a leaf entry's FP32 centre difference
    int cnt = 0, lo = 0, sub = 0;
    uint32_t fb = 0xffffffffu;
    float dcx = 0.f, dcy = 0.f, dcz = 0.f;
    const bool in = c0 + lane < w.e1;
    const int src = in ? w.list[c0 + lane] : 0;
    NodeInfo si{};
    if (in) si = a.info[src];
    const int sincl = wave_incl_scan32(in ? si.cnt : 0);
    if (in) {
      const uint32_t fe = carry + (uint32_t)sincl;
      fb = fe - (uint32_t)si.cnt;
      const uint32_t b = fb > w.f_lo ? fb : w.f_lo;
      const uint32_t en = fe < w.f_hi ? fe : w.f_hi;
      if (en > b) { cnt = (int)(en - b); lo = si.lo + (int)(b - fb); }
      // a whole subtree: its particles' offsets are relative to their own
      // leaves, whose centres are looked up per particle
      sub = si.child >= 0 ? 1 : 0;
      const double* rs = a.rec + (int64_t)src * RS;
      dcx = (float)(w.ct0 - rs[0]);
      dcy = (float)(w.ct1 - rs[1]);
      dcz = (float)(w.ct2 - rs[2]);
    }
    carry += (uint32_t)__builtin_amdgcn_readlane(sincl, 63);
    // lane 0 always holds an entry (c0 < e1)
    if ((uint32_t)__builtin_amdgcn_readfirstlane(fb) >= w.f_hi) break;  // the run is done
    const int incl = wave_incl_scan32(cnt);
    const int pre = incl - cnt;
    const int total = __builtin_amdgcn_readlane(incl, 63);
    for (int f0 = 0; f0 < total; f0 += 64) {
      const int f = f0 + lane;
      int k = 0;
#pragma unroll
      for (int step = 32; step > 0; step >>= 1) {
        const int pk = __shfl(pre, k + step, 64);
        if (pk <= f) k += step;
      }
      const int jj = __shfl(lo, k, 64) + (f - __shfl(pre, k, 64));
      float cx = __shfl(dcx, k, 64), cy = __shfl(dcy, k, 64), cz = __shfl(dcz, k, 64);
      const int jsub = __shfl(sub, k, 64);
      const bool fv = f < total;
      const int j = fv ? jj : tlo;  // a valid index; contributes nothing
      if (fv && jsub) {
        const double* rl = a.rec + (int64_t)a.leaf_node[a.p_leaf[j]] * RS;
        cx = (float)(w.ct0 - rl[0]);
        cy = (float)(w.ct1 - rl[1]);
        cz = (float)(w.ct2 - rl[2]);
      }
      const float4 oj = pf[j];
      const float hj = phh[j].x;
      const float mj = fv ? oj.w : 0.f;
      const float h4j = 4.0f * hj * hj;
#pragma unroll
      for (int ii = 0; ii < K; ++ii) {
        const float dx = cx + (tx[ii] - oj.x), dy = cy + (ty[ii] - oj.y), dz = cz + (tz[ii] - oj.z);
        const float r2 = dx * dx + dy * dy + dz * dz;
        const bool inside = r2 < fmaxf(t4[ii], h4j);
        const float rinv = inside ? 0.f : __builtin_amdgcn_rsqf(r2);
        const float mr = mj * rinv;
        const float mg = mr * (rinv * rinv);
        fx[ii].add(mg * dx);
        fy[ii].add(mg * dy);
        fz[ii].add(mg * dz);
        ph[ii].add(mr);
        // (keeps this target's arithmetic ahead of the queue branch)
        fx[ii].keep(); fy[ii].keep(); fz[ii].keep(); ph[ii].keep();
        const bool push = inside && fv && j != tlo + t0 + ii;
        const uint64_t bal = __builtin_amdgcn_ballot_w64(push);
        if (bal) {
          if (push) {
            const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
            const uint32_t sl = qn[ii] + below;
            qj[ii * kTQ32 + sl] = j;
            float* qq = qc + (ii * kTQ32 + sl) * 3;
            qq[0] = cx; qq[1] = cy; qq[2] = cz;
          }
          const uint32_t c = (uint32_t)__popcll(bal);
          qn[ii] += c;
          nsoft += c;
        }
      }
      // a queue holds at most 63 + 64 entries here
      static_for<K>([&](auto iic) {
        constexpr int ii = decltype(iic)::value;
        if (qn[ii] >= 64) flush(iic, 64);
      });
    }
  }
  static_for<K>([&](auto iic) {
    constexpr int ii = decltype(iic)::value;
    if (qn[ii] > 0) flush(iic, qn[ii]);
  });
#pragma unroll
  for (int ii = 0; ii < K; ++ii) {
    const double sx = wave_sum64(fx[ii].get()), sy = wave_sum64(fy[ii].get());
    const double sz = wave_sum64(fz[ii].get()), sp = wave_sum64(ph[ii].get());
    if (lane == t0 + ii) {
      double* o = a.part + (w.item * LS + t0 + ii) * 4;
      o[0] = sx; o[1] = sy; o[2] = sz; o[3] = sp;
    }
  }
}

template <int LS, bool NODE, int RS, int TG, int WPE, typename Acc>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE))) void k_p2p_wave32(
    NearArgs a, const float4* __restrict__ pf, const float2* __restrict__ phh) {
  const int lane = threadIdx.x;
  const uint32_t item = xcd_block(blockIdx.x, gridDim.x);
  if (item >= a.item_off[a.nleaves]) return;  // the grid is an upper bound
  const int l = a.item_leaf[item];
  const uint32_t kitem = a.item_k[item];
  const int node = a.leaf_node[l];
  const NodeInfo ti = a.info[node];
  Wave32Item w;
  w.tlo = ti.lo;
  w.nt = ti.cnt;
  w.item = item;
  const double* rt = a.rec + (int64_t)node * RS;
  w.ct0 = rt[0]; w.ct1 = rt[1]; w.ct2 = rt[2];
  if (NODE) {
    w.e0 = a.node_p2p_off[node];
    w.e1 = w.e0 + a.node_p2p_cnt[node];
    w.list = reinterpret_cast<const int32_t*>(a.node_p2p_pool);
  } else {
    w.e0 = a.p2p_off[l];
    w.e1 = a.p2p_off[l + 1];
    w.list = a.p2p_list;
  }
  w.f_lo = kitem * kP2PItem;
  const uint32_t ftot = a.src_total[l];
  w.f_hi = w.f_lo + kP2PItem < ftot ? w.f_lo + kP2PItem : ftot;
  w.carry0 = 0;
  if (kitem > 0) { w.e0 = a.item_e0[item]; w.carry0 = a.item_c0[item]; }
  __shared__ int qj[TG * kTQ32];
  __shared__ float qc[TG * kTQ32 * 3];
  uint32_t nsoft = 0;
  int t0 = 0;
  for (; t0 + TG <= w.nt; t0 += TG)
    p2p_wave32_pass<TG, LS, RS, Acc>(a, pf, phh, w, t0, qj, qc, nsoft);
  // the remainder, a pass with a fixed target count (uniform branches)
  static_for<TG>([&](auto rc) {
    constexpr int r = decltype(rc)::value;
    if (r > 0 && w.nt - t0 == r)
      p2p_wave32_pass<(r > 0 ? r : 1), LS, RS, Acc>(a, pf, phh, w, t0, qj, qc, nsoft);
  });
  if (lane == 0 && nsoft) atomicAdd(a.soft_pairs, (unsigned long long)nsoft);
}

constexpr int kFarSplit32 = 2;

template <int P>
void far32_order(bool node_lists, const FarArgs& a, const float* rec32, int top, hipStream_t s) {
  const unsigned nb = (unsigned)((a.nleaves + 64 / kFarSplit32 - 1) / (64 / kFarSplit32));
  if (node_lists) k_far32<P, true, kFarSplit32><<<nb, 64, 0, s>>>(a, rec32, top);
  else k_far32<P, false, kFarSplit32><<<nb, 64, 0, s>>>(a, rec32, top);
}

template <int RS>
void prep_particles(int nleaves, const int32_t* leaf_node, const NodeInfo* info, const double* rec,
                    const double* xs, const double* ys, const double* zs, const double* ms,
                    const double* hs, float4* pf, float2* ph, hipStream_t s) {
  k_prep_particles32<RS><<<(nleaves + 127) / 128, 128, 0, s>>>(nleaves, leaf_node, info, rec, xs, ys,
                                                               zs, ms, hs, pf, ph);
}

// variant 0: the wave kernel with scalar-register targets; 7: the same with
// TwoSum-compensated FP32 sums instead of FP64 ones; 6: the earlier shape
// (targets in LDS, the softened branch taken in the pass)
template <int LS, int RS>
void p2p32(bool node_lists, int variant, const NearArgs& a, const float4* pf, const float2* ph,
           int64_t items, hipStream_t s, KernelMarks km) {
  constexpr int TG = LS <= 10 ? 5 : 8;
  const unsigned nb = (unsigned)items;
  record_mark(km.begin, s);
  if (variant == 6) {
    if (node_lists) k_p2p_leaf32<LS, true, RS, TG><<<nb, 64, 0, s>>>(a, pf, ph);
    else k_p2p_leaf32<LS, false, RS, TG><<<nb, 64, 0, s>>>(a, pf, ph);
  } else if (variant == 7) {
    if (node_lists) k_p2p_wave32<LS, true, RS, TG, 4, AccT><<<nb, 64, 0, s>>>(a, pf, ph);
    else k_p2p_wave32<LS, false, RS, TG, 4, AccT><<<nb, 64, 0, s>>>(a, pf, ph);
  } else {
    if (node_lists) k_p2p_wave32<LS, true, RS, TG, 4, AccD><<<nb, 64, 0, s>>>(a, pf, ph);
    else k_p2p_wave32<LS, false, RS, TG, 4, AccD><<<nb, 64, 0, s>>>(a, pf, ph);
  }
  record_mark(km.end, s);
  if (!km.skip_reduce) launch_p2p_reduce(a, LS, s);
}

}  // namespace

void launch_prep32(int order, int nn, int nleaves, const int32_t* leaf_node, const NodeInfo* info,
                   const double* rec, const int32_t* node_depth, const double* xs, const double* ys,
                   const double* zs, const double* ms, const double* hs, float* rec32, float4* pf,
                   float2* ph, hipStream_t s) {
  const unsigned nb = (unsigned)((nn + 255) / 256);
  switch (order) {
    case 0: k_prep_nodes32<0><<<nb, 256, 0, s>>>(nn, rec, node_depth, rec32); break;
    case 1: k_prep_nodes32<1><<<nb, 256, 0, s>>>(nn, rec, node_depth, rec32); break;
    case 2: k_prep_nodes32<2><<<nb, 256, 0, s>>>(nn, rec, node_depth, rec32); break;
    case 3: k_prep_nodes32<3><<<nb, 256, 0, s>>>(nn, rec, node_depth, rec32); break;
    case 4: k_prep_nodes32<4><<<nb, 256, 0, s>>>(nn, rec, node_depth, rec32); break;
  }
  switch (rec_stride(order)) {
    case 16: prep_particles<16>(nleaves, leaf_node, info, rec, xs, ys, zs, ms, hs, pf, ph, s); break;
    case 24: prep_particles<24>(nleaves, leaf_node, info, rec, xs, ys, zs, ms, hs, pf, ph, s); break;
    case 32: prep_particles<32>(nleaves, leaf_node, info, rec, xs, ys, zs, ms, hs, pf, ph, s); break;
    case 48: prep_particles<48>(nleaves, leaf_node, info, rec, xs, ys, zs, ms, hs, pf, ph, s); break;
  }
}

void launch_far32(int order, bool node_lists, const FarArgs& a, const float* rec32, int top,
                  hipStream_t s) {
  if (a.nleaves <= 0) return;
  switch (order) {
    case 0: far32_order<0>(node_lists, a, rec32, top, s); break;
    case 1: far32_order<1>(node_lists, a, rec32, top, s); break;
    case 2: far32_order<2>(node_lists, a, rec32, top, s); break;
    case 3: far32_order<3>(node_lists, a, rec32, top, s); break;
    case 4: far32_order<4>(node_lists, a, rec32, top, s); break;
  }
}

bool launch_near32(int order, bool node_lists, int leaf_size, int variant, const NearArgs& a,
                   const float4* pf, const float2* ph, int64_t items, hipStream_t s,
                   KernelMarks km) {
  if (a.n <= 0) return true;
  const int RS = rec_stride(order);
  if (leaf_size > 16) return false;
#define SFMM_P2P32(LS)                                                   \
  switch (RS) {                                                          \
    case 16: p2p32<LS, 16>(node_lists, variant, a, pf, ph, items, s, km); break;      \
    case 24: p2p32<LS, 24>(node_lists, variant, a, pf, ph, items, s, km); break;      \
    case 32: p2p32<LS, 32>(node_lists, variant, a, pf, ph, items, s, km); break;      \
    case 48: p2p32<LS, 48>(node_lists, variant, a, pf, ph, items, s, km); break;      \
  }
  if (leaf_size <= 10) { SFMM_P2P32(10) } else { SFMM_P2P32(16) }
#undef SFMM_P2P32
  return true;
}

}  // namespace sfmm
