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

namespace sfmm {
namespace {

__device__ __forceinline__ void soft(double r, double hinv, double& g, double& psi) {
  const double q = r * hinv;
  const double h3 = hinv * hinv * hinv;
  if (q < 1.0) {
    const double q2 = q * q;
    g = h3 * fma(q2, fma(0.5, q, -1.2), 4.0 / 3.0);
    psi = hinv * fma(q2, fma(q2, fma(-0.1, q, 0.3), -2.0 / 3.0), 1.4);
  } else {
    const double q2 = q * q;
    const double qi = 1.0 / q;
    const double qi3 = qi * qi * qi;
    // 8/3 - 3q + 6/5 q^2 - 1/6 q^3 - 1/(15 q^3)
    g = h3 * (fma(q, fma(q, fma(q, -1.0 / 6.0, 1.2), -3.0), 8.0 / 3.0) - qi3 * (1.0 / 15.0));
    // 8/5 - 4/3 q^2 + q^3 - 3/10 q^4 + 1/30 q^5 - 1/(15 q)
    psi = hinv * (fma(q2, fma(q, fma(q, fma(q, 1.0 / 30.0, -0.3), 1.0), -4.0 / 3.0), 1.6) -
                  qi * (1.0 / 15.0));
  }
}

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

void launch_near(bool node_lists, const NearArgs& a, hipStream_t s) {
  if (a.n <= 0) return;
  if (node_lists) k_near<true><<<(a.n + 255) / 256, 256, 0, s>>>(a);
  else k_near<false><<<(a.n + 255) / 256, 256, 0, s>>>(a);
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
