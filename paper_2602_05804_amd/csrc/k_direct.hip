// k_direct.hip -- the softened direct sum of Sect. 2, Eq. (softdirectsum),
// over all N sources for a set of targets: the O(N^2) reference the SFMM
// approximates (accuracy sweeps against the opening angle, the paper's
// Plummer and homogeneous-sphere tests).
//
// One thread per target; the sources stream through LDS in tiles of 256
// (x, y, z, m, h, 1/h), read back as broadcasts.  Pairs with j == i are
// skipped; unequal h are averaged as in P2P.  Sources are summed in index
// order, so the result is reproducible.
#include "sfmm_internal.h"
#include "softening.h"

namespace sfmm {
namespace {

constexpr int kDirTile = 256;

__global__ __launch_bounds__(kDirTile) void k_direct(int64_t n, const double* __restrict__ x,
                                                     const double* __restrict__ m,
                                                     const double* __restrict__ h, int64_t nt,
                                                     const int64_t* __restrict__ targets,
                                                     double G, int include_self,
                                                     double* __restrict__ acc,
                                                     double* __restrict__ pot, int* status) {
  __shared__ double sx[kDirTile], sy[kDirTile], sz[kDirTile], sm[kDirTile], sh[kDirTile],
      shi[kDirTile];
  const int64_t t = (int64_t)blockIdx.x * kDirTile + threadIdx.x;
  const int64_t it = t < nt ? (targets ? targets[t] : t) : 0;
  const bool valid = it >= 0 && it < n;  // a bad index is reported, never read
  if (t < nt && !valid) atomicOr(status, ST_OVERFLOW);
  const bool active = t < nt && valid;
  const int64_t i = valid ? it : 0;
  const double xi = x[3 * i], yi = x[3 * i + 1], zi = x[3 * i + 2];
  const double hinv_i = 1.0 / h[i];
  const double h_i = h[i];
  double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
  for (int64_t base = 0; base < n; base += kDirTile) {
    const int64_t j = base + threadIdx.x;
    if (j < n) {
      sx[threadIdx.x] = x[3 * j];
      sy[threadIdx.x] = x[3 * j + 1];
      sz[threadIdx.x] = x[3 * j + 2];
      sm[threadIdx.x] = m[j];
      sh[threadIdx.x] = h[j];
      shi[threadIdx.x] = 1.0 / h[j];
    }
    __syncthreads();
    const int cnt = (int)((n - base) < kDirTile ? (n - base) : kDirTile);
    for (int k = 0; k < cnt; ++k) {
      const double w = (base + k == i) ? 0.0 : sm[k];
      const double dx = xi - sx[k], dy = yi - sy[k], dz = zi - sz[k];
      const double r2 = dx * dx + dy * dy + dz * dz;
      const double rinv = r2 > 0.0 ? rsqrt(r2) : 0.0;
      const double rinv3 = rinv * rinv * rinv;
      double gs = rinv3, ps = rinv;
      const double hj = sh[k], hjinv = shi[k];
      const bool inside = (r2 * (hinv_i * hinv_i) < 4.0) || (r2 * (hjinv * hjinv) < 4.0);
      if (__ballot(inside)) {
        const double r = r2 * rinv;
        double g1, p1, g2, p2;
        soft_sel(r * hinv_i, hinv_i, h_i * rinv, rinv, rinv3, g1, p1);
        soft_sel(r * hjinv, hjinv, hj * rinv, rinv, rinv3, g2, p2);
        if (inside) {
          gs = 0.5 * (g1 + g2);
          ps = 0.5 * (p1 + p2);
        }
      }
      const double mg = w * gs;
      ax = fma(mg, dx, ax);
      ay = fma(mg, dy, ay);
      az = fma(mg, dz, az);
      ph = fma(w, ps, ph);
    }
    __syncthreads();
  }
  if (!active) return;
  if (include_self) ph = fma(m[i], 1.4 * hinv_i, ph);
  acc[3 * t] = -G * ax;
  acc[3 * t + 1] = -G * ay;
  acc[3 * t + 2] = -G * az;
  pot[t] = -G * ph;
}

}  // namespace

void launch_direct(int64_t n, const double* x, const double* m, const double* h, int64_t nt,
                   const int64_t* targets, double G, int include_self, double* acc, double* pot,
                   int* status, hipStream_t s) {
  if (nt <= 0 || n <= 0) return;
  const unsigned nb = (unsigned)((nt + kDirTile - 1) / kDirTile);
  k_direct<<<nb, kDirTile, 0, s>>>(n, x, m, h, nt, targets, G, include_self, acc, pot, status);
}

}  // namespace sfmm
