// softening.h -- cubic-spline (M4) softened pair kernels, FP64, shared by
// the P2P kernels and the direct sum.  With q = r/h (support 2h):
//   g   = f(q)/(q h^3):  4/3 - 6/5 q^2 + 1/2 q^3                     (q < 1)
//                        8/3 - 3 q + 6/5 q^2 - 1/6 q^3 - 1/(15 q^3)   (1 <= q < 2)
//                        1/q^3                                        (q >= 2)   (times 1/h^3)
//   psi = psi(q)/h:      7/5 - 2/3 q^2 + 3/10 q^4 - 1/10 q^5          (q < 1)
//                        8/5 - 4/3 q^2 + q^3 - 3/10 q^4 + 1/30 q^5 - 1/(15 q)
//                        1/q                                          (q >= 2)   (times 1/h)
// (Sect. 2, the softened direct sum; the kernel shapes follow from the M4
// spline's enclosed mass and potential.)
#pragma once
#include <hip/hip_runtime.h>

namespace sfmm {

// 1/sqrt(r2) for r2 > 0, 0 for r2 == 0: the hardware estimate refined once
// with the third-order step y' = y (1 + e/2 + 3e^2/8), e = 1 - r2 y^2 (the
// series of (1 - e)^(-1/2)); no branch
__device__ __forceinline__ double rsqrt_pair(double r2) {
  const double y = __builtin_amdgcn_rsq(r2);
  const double e = fma(-r2 * y, y, 1.0);
  const double r = fma(y * e, fma(e, 0.375, 0.5), y);
  return r2 > 0.0 ? r : 0.0;
}

// the same refined 1/sqrt(r2) for r2 > 0 only (r2 == 0 gives NaN): for a
// caller that replaces the value of every pair inside a kernel anyway
__device__ __forceinline__ double rsqrt_refined(double r2) {
  const double y = __builtin_amdgcn_rsq(r2);
  const double e = fma(-r2 * y, y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
}

// a wave-uniform double read from the first active lane (kept in scalar
// registers by the compiler)
__device__ __forceinline__ double wave_uniform(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

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

// g = f(q)/(q h^3) and psi = psi(q)/h for one particle's kernel at q = r/h,
// without branches; qi = 1/q (= h/r), rinv = 1/r, rinv3 = 1/r^3
__device__ __forceinline__ void soft_sel(double q, double hinv, double qi, double rinv,
                                         double rinv3, double& g, double& psi) {
  const double q2 = q * q;
  const double h3 = hinv * hinv * hinv;
  const double gA = h3 * fma(q2, fma(0.5, q, -1.2), 4.0 / 3.0);
  const double pA = hinv * fma(q2, fma(q2, fma(-0.1, q, 0.3), -2.0 / 3.0), 1.4);
  const double qi3 = qi * qi * qi;
  const double gB = h3 * (fma(q, fma(q, fma(q, -1.0 / 6.0, 1.2), -3.0), 8.0 / 3.0) -
                          qi3 * (1.0 / 15.0));
  const double pB = hinv * (fma(q2, fma(q, fma(q, fma(q, 1.0 / 30.0, -0.3), 1.0), -4.0 / 3.0), 1.6) -
                            qi * (1.0 / 15.0));
  g = q >= 2.0 ? rinv3 : (q < 1.0 ? gA : gB);
  psi = q >= 2.0 ? rinv : (q < 1.0 ? pA : pB);
}

}  // namespace sfmm
