// k_direct.hip -- the softened direct sum of Sect. 2, Eq. (softdirectsum),
// over all N sources for a set of targets: the O(N^2) reference the SFMM
// approximates (accuracy sweeps against the opening angle, the paper's
// Plummer and homogeneous-sphere tests).
//
// One thread per target, the sources split into chunks: block (b, c) sums
// chunk c of the sources for targets b * 256 .. b * 256 + 255, streaming them
// through LDS in tiles of 256 (x, y, z, m, h, 1/h) read back as broadcasts,
// and writes its partial sums to a buffer [chunk][target][4]; a second kernel
// adds each target's partials in chunk order.  Pairs with j == i are skipped;
// unequal h are averaged as in P2P.  The summation order is fixed, so the
// result is reproducible.  With few targets the chunks keep the chip busy.
#include "sfmm_internal.h"
#include "softening.h"

namespace sfmm {
namespace {

constexpr int kDirTile = 256;

__global__ __launch_bounds__(kDirTile) void k_direct_part(int64_t n, const double* __restrict__ x,
                                                          const double* __restrict__ m,
                                                          const double* __restrict__ h,
                                                          int64_t nt,
                                                          const int64_t* __restrict__ targets,
                                                          int64_t chunk, double* __restrict__ part,
                                                          int* status) {
  __shared__ double sx[kDirTile], sy[kDirTile], sz[kDirTile], sm[kDirTile], sh[kDirTile],
      shi[kDirTile];
  const int64_t t = (int64_t)blockIdx.x * kDirTile + threadIdx.x;
  const int64_t it = t < nt ? (targets ? targets[t] : t) : 0;
  const bool valid = it >= 0 && it < n;  // a bad index is reported, never read
  if (t < nt && !valid && blockIdx.y == 0) atomicOr(status, ST_OVERFLOW);
  const int64_t i = valid ? it : 0;
  const double xi = x[3 * i], yi = x[3 * i + 1], zi = x[3 * i + 2];
  const double hinv_i = 1.0 / h[i];
  const double h_i = h[i];
  double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
  const int64_t j0 = (int64_t)blockIdx.y * chunk;
  const int64_t j1 = j0 + chunk < n ? j0 + chunk : n;
  for (int64_t base = j0; base < j1; base += kDirTile) {
    const int64_t j = base + threadIdx.x;
    if (j < j1) {
      sx[threadIdx.x] = x[3 * j];
      sy[threadIdx.x] = x[3 * j + 1];
      sz[threadIdx.x] = x[3 * j + 2];
      sm[threadIdx.x] = m[j];
      sh[threadIdx.x] = h[j];
      shi[threadIdx.x] = 1.0 / h[j];
    }
    __syncthreads();
    const int cnt = (int)((j1 - base) < kDirTile ? (j1 - base) : kDirTile);
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
  if (t >= nt) return;
  double* o = part + ((int64_t)blockIdx.y * nt + t) * 4;
  o[0] = ax; o[1] = ay; o[2] = az; o[3] = ph;
}

// per target: the chunks' partial sums in chunk order, the self term, -G
__global__ void k_direct_final(int64_t n, const double* __restrict__ m,
                               const double* __restrict__ h, int64_t nt,
                               const int64_t* __restrict__ targets, int nchunk,
                               const double* __restrict__ part, double G, int include_self,
                               double* __restrict__ acc, double* __restrict__ pot) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const int64_t it = targets ? targets[t] : t;
  if (it < 0 || it >= n) return;  // reported by the first kernel
  double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
  for (int c = 0; c < nchunk; ++c) {
    const double* q = part + ((int64_t)c * nt + t) * 4;
    ax += q[0]; ay += q[1]; az += q[2]; ph += q[3];
  }
  if (include_self) ph = fma(m[it], 1.4 * (1.0 / h[it]), ph);
  acc[3 * t] = -G * ax;
  acc[3 * t + 1] = -G * ay;
  acc[3 * t + 2] = -G * az;
  pot[t] = -G * ph;
}

__global__ void k_clear_int(int* p) { *p = 0; }

}  // namespace

int direct_chunks(int64_t n, int64_t nt, uint64_t max_part_bytes) {
  if (n <= 0 || nt <= 0) return 1;
  const int64_t nb = (nt + kDirTile - 1) / kDirTile;
  int64_t c = (4096 + nb - 1) / nb;                      // about 4096 blocks in all
  const int64_t tiles = (n + kDirTile - 1) / kDirTile;   // at least one tile per chunk
  if (c > tiles) c = tiles;
  const int64_t fit = (int64_t)(max_part_bytes / ((uint64_t)nt * 4 * sizeof(double)));
  if (c > fit) c = fit;
  if (c > 65535) c = 65535;  // (grid y)
  return (int)c;             // 0: not even one chunk fits
}

void launch_direct(int64_t n, const double* x, const double* m, const double* h, int64_t nt,
                   const int64_t* targets, double G, int include_self, double* acc, double* pot,
                   int* status, double* part, int nchunk, hipStream_t s) {
  k_clear_int<<<1, 1, 0, s>>>(status);
  if (nt <= 0 || n <= 0 || nchunk < 1) return;
  // chunks of whole tiles
  const int64_t tiles = (n + kDirTile - 1) / kDirTile;
  const int64_t chunk = ((tiles + nchunk - 1) / nchunk) * kDirTile;
  const int nc = (int)((n + chunk - 1) / chunk);
  const dim3 grid((unsigned)((nt + kDirTile - 1) / kDirTile), (unsigned)nc);
  k_direct_part<<<grid, kDirTile, 0, s>>>(n, x, m, h, nt, targets, chunk, part, status);
  k_direct_final<<<(unsigned)((nt + 255) / 256), 256, 0, s>>>(n, m, h, nt, targets, nc, part, G,
                                                               include_self, acc, pot);
}

}  // namespace sfmm
