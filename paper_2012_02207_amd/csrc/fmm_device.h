// Device helpers shared by the gfx950 kernels of this library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "fmm_internal.h"

namespace fmm {

constexpr int WAVE = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Workgroup i runs on XCD i mod 8.  Per-sink kernels take their sinks in
// chunks of XCD_CHUNK consecutive workgroups, the chunks dealt to the XCDs in
// turn: each XCD gets an even share of the work (sinks in one range of the
// list differ in cost) while neighbouring sinks, which share sources, still
// run on the same XCD.  The grid is a whole number of rounds (xcd_grid).
constexpr int XCD_CHUNK = 8;  // measured: 1, 4 and 8 within 0.7%; 32 and 128 slower (2.9%, 1.4%)
__device__ __forceinline__ int xcd_block() {
  int j = blockIdx.x >> 3, x = blockIdx.x & 7;
  return ((j / XCD_CHUNK) * 8 + x) * XCD_CHUNK + j % XCD_CHUNK;
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

// grid for xcd_block(): nblk blocks rounded up to whole rounds of 8 chunks
inline unsigned xcd_grid(int64_t nblk) {
  int64_t r = 8 * (int64_t)XCD_CHUNK;
  return (unsigned)(r * ceil_div(nblk, r));
}

// n! in FP64 by repeated multiplication (evaluation-side normalisations only)
__device__ __forceinline__ double fmm_fact_dev(int n) {
  double r = 1.0;
  for (int i = 2; i <= n; i++) r *= (double)i;
  return r;
}


// ---- cross-lane transpose-reduce (the M2L kernels) ------------------------
// D values per lane summed over the 64 lanes in six halving steps with
// partner distances 32, 16, 8, 4, 2, 1.  With L values left, a lane keeps the
// first ceil(L/2) of them or the rest, by that bit of its lane id, and adds its
// partner's copy of the kept part; once a single value is left the steps are
// plain butterflies.  A lane on the upper side of an odd L keeps one slot more
// than there are values: that pad slot holds an unused sum, and pads only ever
// meet pads (partners share every earlier bit), so they need no clearing.
// The total of value j ends in lane reduce_owner(D, j).
constexpr int reduce_len(int D, int t) {
  int L = D;
  for (int k = 0; k < t; k++) L = (L + 1) / 2;
  return L;
}
constexpr int reduce_owner(int D, int j) {
  int lane = 0, L = D;
  for (int t = 0; t < 6; t++) {
    if (L >= 2) {
      int h = (L + 1) / 2;
      if (j >= h) {
        lane |= 32 >> t;
        j -= h;
      }
      L = h;
    }
  }
  return lane;
}

// reduce_owner inverted: the value j whose total this lane ends with, and
// whether that is a real value (not a pad)
template <int D>
__device__ __forceinline__ void reduce_slot(int lane, int& j, int& real) {
  j = 0;
  int left = D;  // real values in this lane's part
  bool ok = true;
#pragma unroll
  for (int t = 0; t < 6; t++) {
    int L = reduce_len(D, t);
    bool bit = (lane & (32 >> t)) != 0;
    if (L >= 2) {
      int H = (L + 1) / 2;
      j += bit ? H : 0;
      left = bit ? left - H : (left < H ? left : H);
    } else {
      ok = ok && !bit;
    }
  }
  real = ok && left >= 1;
}

// DPP control of the steps at distances 8, 4, 2, 1 (t = 2..5): row mirror,
// half-row mirror, quad_perm [2,3,0,1], quad_perm [1,0,3,2]; each pairs lanes
// that differ in that bit
constexpr int reduce_dpp_ctrl(int t) { return t == 2 ? 0x140 : t == 3 ? 0x141 : t == 4 ? 0x4E : 0xB1; }

// lanes 32..63 of a <-> lanes 0..31 of b (T = 0), or the odd 16-lane rows of a
// <-> the even rows of b (T = 1)
template <int T>
__device__ __forceinline__ void lane_swap(uint32_t& a, uint32_t& b) {
  if constexpr (T == 0) {
    auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    a = (uint32_t)r[0];
    b = (uint32_t)r[1];
  } else {
    auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    a = (uint32_t)r[0];
    b = (uint32_t)r[1];
  }
}
template <int T>
__device__ __forceinline__ void lane_swap(float& a, float& b) {
  uint32_t ua = __builtin_bit_cast(uint32_t, a), ub = __builtin_bit_cast(uint32_t, b);
  lane_swap<T>(ua, ub);
  a = __builtin_bit_cast(float, ua);
  b = __builtin_bit_cast(float, ub);
}
template <int T>
__device__ __forceinline__ void lane_swap(double& a, double& b) {
  uint64_t ua = __builtin_bit_cast(uint64_t, a), ub = __builtin_bit_cast(uint64_t, b);
  uint32_t alo = (uint32_t)ua, ahi = (uint32_t)(ua >> 32), blo = (uint32_t)ub, bhi = (uint32_t)(ub >> 32);
  lane_swap<T>(alo, blo);
  lane_swap<T>(ahi, bhi);
  a = __builtin_bit_cast(double, ((uint64_t)ahi << 32) | alo);
  b = __builtin_bit_cast(double, ((uint64_t)bhi << 32) | blo);
}

// the value of v in the lane that DPP control CTRL selects
template <int CTRL>
__device__ __forceinline__ float dpp_read(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_read(double v) {
  uint64_t u = __builtin_bit_cast(uint64_t, v);
  int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, false);
  int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// compile-time loop: f(std::integral_constant<int, i>) for i in [I, E)
template <int I, int E, class F>
__device__ __forceinline__ void unroll_for(F&& f) {
  if constexpr (I < E) {
    f(std::integral_constant<int, I>{});
    unroll_for<I + 1, E>(f);
  }
}

// x[0..D) of every lane -> the cross-lane totals (in place, see above); each
// lane adds its last value to *acc_slot, meaningful in the owner lanes only
template <int D, class T>
__device__ __forceinline__ void reduce_lanes(T* x, double* acc_slot, int lane) {
  unroll_for<0, 6>([&](auto tc) {
    constexpr int t = tc;
    constexpr int L = reduce_len(D, t);
    constexpr int H = (L + 1) / 2;
    if constexpr (t < 2) {
      unroll_for<0, H>([&](auto ic) {
        constexpr int i = ic;
        T a = x[i], b = x[i];  // L == 1 (or the pad of an odd L): a butterfly
        if constexpr (i + H < L) b = x[i + H];
        lane_swap<t>(a, b);
        x[i] = a + b;
      });
    } else {
      constexpr int CTRL = reduce_dpp_ctrl(t);
      bool hi = (lane & (32 >> t)) != 0;
      unroll_for<0, H>([&](auto ic) {
        constexpr int i = ic;
        T r = x[i] + dpp_read<CTRL>(x[i]);
        if constexpr (i + H < L) {
          T q = x[i + H] + dpp_read<CTRL>(x[i + H]);
          r = hi ? q : r;
        }
        x[i] = r;
      });
    }
  });
  *acc_slot += (double)x[0];
}

}  // namespace fmm
