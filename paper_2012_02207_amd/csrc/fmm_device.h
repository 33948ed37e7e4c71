// Device helpers shared by the gfx950 kernels of this library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fmm_internal.h"

namespace fmm {

constexpr int WAVE = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// wave-wide broadcast of a double from lane `src`
__device__ __forceinline__ double shfl_d(double v, int src) { return __shfl(v, src, WAVE); }

// full-wave sum (every lane receives the total); butterfly over xor partners
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
  return v;
}

// Regular solid harmonics Y_n^m(x), m >= 0, in exactly the rounding sequence
// of their defining two-term recurrences (no contraction; used where results
// feed the acceptance test):
//   Y_0^0 = 1, Y_n^n = -(x + i y) Y_{n-1}^{n-1} / (2n),
//   Y_n^m = ((2n-1) z Y_{n-1}^m - r^2 Y_{n-2}^m) / ((n+m)(n-m)).
// Values are written to re[cidx(n,m)*stride], im[cidx(n,m)*stride].
__device__ inline void regular_exact(int p, double x, double y, double z, double* re, double* im,
                                     int stride) {
  double r2 = (x * x + y * y) + z * z;
  re[0] = 1.0;
  im[0] = 0.0;
  double pr = 1.0, pi = 0.0;
  for (int n = 1; n <= p; n++) {
    double tr = x * pr - y * pi;
    double ti = x * pi + y * pr;
    double den = (double)(2 * n);
    pr = (-tr) / den;
    pi = (-ti) / den;
    re[cidx(n, n) * stride] = pr;
    im[cidx(n, n) * stride] = pi;
  }
  for (int m = 0; m < p; m++) {
    double ar2 = 0.0, ai2 = 0.0;  // Y_{n-2}^m
    double ar1 = re[cidx(m, m) * stride], ai1 = im[cidx(m, m) * stride];
    for (int n = m + 1; n <= p; n++) {
      double k = (double)(2 * n - 1) * z;
      double ar = k * ar1;
      double ai = k * ai1;
      double nr = ar, ni = ai;
      if (n - 2 >= m) {
        double br = r2 * ar2;
        double bi = r2 * ai2;
        nr = ar - br;
        ni = ai - bi;
      }
      double den = (double)((n + m) * (n - m));
      double vr = nr / den, vi = ni / den;
      re[cidx(n, m) * stride] = vr;
      im[cidx(n, m) * stride] = vi;
      ar2 = ar1;
      ai2 = ai1;
      ar1 = vr;
      ai1 = vi;
    }
  }
}

// coefficient (n, m) for either sign of m from m >= 0 storage (exact)
__device__ __forceinline__ void cget(const double* re, const double* im, int stride, int n, int m,
                                     double& a, double& b) {
  if (m >= 0) {
    a = re[cidx(n, m) * stride];
    b = im[cidx(n, m) * stride];
  } else {
    double s = (m & 1) ? -1.0 : 1.0;
    a = s * re[cidx(n, -m) * stride];
    b = -s * im[cidx(n, -m) * stride];
  }
}

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// n! in FP64 by repeated multiplication (evaluation-side normalisations only)
__device__ __forceinline__ double fmm_fact_dev(int n) {
  double r = 1.0;
  for (int i = 2; i <= n; i++) r *= (double)i;
  return r;
}

}  // namespace fmm
