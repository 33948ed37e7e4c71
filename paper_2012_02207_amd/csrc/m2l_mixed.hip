// Mixed-precision M2L on gfx950: the rotation-accelerated operator of section
// 2.4 in FP32 for cell pairs below the root levels (the FP64 kernel handles
// pairs that touch a cell above level root_levels).
//
// Range and conditioning: the FP32 operands are the moments in the
// rotation-invariant normalised real basis, scaled by the source size,
//   N_n^m = G_n^m M_n^m / rho_A^n,  G_n^0 = n!,  G_n^m = sqrt(2 (n-m)!(n+m)!),
// for which ||N_n|| = P_n / rho_A^n <= M_A (the P_n of section 2.3), and in
// which the swap matrices G W_n G^-1 are orthogonal (entries in [-1, 1]).  The
// translation along z becomes
//   Lt_n^m = sum_k N'_k^m T(n,k,m) (rho_B/r)^n (rho_A/r)^k / r,
//   T(n,k,m) = (-1)^(n+m) (n+k)! G_n^m / ((n-m)!(n+m)! G_k^m),
// with (rho_A + rho_B) < r, so every factor is O(1).  The result
// Lt = rho_B^n G L / ((n-m)!(n+m)!) is summed per sink in FP64 and converted
// back to the standard local coefficients in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "fmm_device.h"
#include "fmm_tables.h"

namespace fmm {

namespace mx {

template <int I, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < E) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, E>(f);
  }
}

constexpr double cfact(int n) {
  double r = 1.0;
  for (int i = 2; i <= n; i++) r *= (double)i;
  return r;
}
constexpr int rb_m(int j) { return (j + 1) >> 1; }
constexpr bool rb_re(int j) { return j == 0 || (j & 1); }
constexpr bool swap_nz(int n, int i, int j) {
  return rb_re(i) == rb_re(j) && (((rb_m(i) + rb_m(j) + n) & 1) == (rb_re(i) ? 0 : 1));
}
constexpr int crank(int n, int i, int j) {
  int c = 0;
  for (int t = 0; t < j; t++) c += swap_nz(n, i, t) ? 1 : 0;
  return c;
}
constexpr int swoff(int n) { return n * (4 * n * n - 1) / 3; }

// normalisation G_n^m of real-basis entry j of order n (m = rb_m(j))
constexpr double csqrt_newton(double x) {
  if (x <= 0) return 0;
  double r = x > 1 ? x : 1;
  for (int i = 0; i < 200; i++) r = 0.5 * (r + x / r);
  return r;
}
constexpr double gnorm_eval(int n, int m) {
  return m == 0 ? cfact(n) : csqrt_newton(2.0 * cfact(n - m) * cfact(n + m));
}
// evaluated once per translation unit (the swap and translation constants of
// every kernel read it at compile time)
struct GnormTable {
  double v[FMM_GPU_PMAX + 1][FMM_GPU_PMAX + 1];
};
constexpr GnormTable make_gnorm_table() {
  GnormTable t{};
  for (int n = 0; n <= FMM_GPU_PMAX; n++)
    for (int m = 0; m <= n; m++) t.v[n][m] = gnorm_eval(n, m);
  return t;
}
inline constexpr GnormTable kGnorm = make_gnorm_table();
constexpr double gnorm(int n, int m) { return kGnorm.v[n][m]; }
// translation constant T(n, k, m)
constexpr double tconst(int n, int k, int m) {
  double s = ((n + m) & 1) ? -1.0 : 1.0;
  return s * cfact(n + k) * gnorm(n, m) / (cfact(n - m) * cfact(n + m) * gnorm(k, m));
}

// entry (i, j) of the orthogonal swap matrix G W_n G^-1 in FP32 (structural
// non-zeros only are used): a compile-time constant, so every product takes
// its matrix entry as an instruction operand instead of a load
constexpr float swap_w32(int n, int i, int j) {
  return (float)(fmm_swap_table[swoff(n) + i * (2 * n + 1) + j] * gnorm(n, rb_m(i)) / gnorm(n, rb_m(j)));
}

template <int N>
__device__ __forceinline__ void swap_apply(float* v) {
  constexpr int D = 2 * N + 1;
  float out[D];
  static_for<0, D>([&](auto ic) {
    constexpr int i = ic;
    float s = 0.f;
    static_for<0, D>([&](auto jc) {
      constexpr int j = jc;
      if constexpr (swap_nz(N, i, j)) {
        constexpr float w = swap_w32(N, i, j);
        if constexpr (crank(N, i, j) == 0)
          s = w * v[j];
        else
          s = fmaf(w, v[j], s);
      }
    });
    out[i] = s;
  });
  static_for<0, D>([&](auto ic) { v[ic] = out[ic]; });
}

// rotation about z: (C, S)_m <- (C cos ma - S sin ma, C sin ma + S cos ma),
// with (cos ma, sin ma), m = 1..N, from tables built once per pair by the
// angle-addition recurrence; sgn = -1 rotates by -a
template <int N>
__device__ __forceinline__ void zrot_tab(float* v, const float* cm, const float* sm, float sgn) {
  static_for<1, N + 1>([&](auto mc) {
    constexpr int m = mc;
    float c = cm[m], sn = sgn * sm[m];
    float C = v[2 * m - 1], S = v[2 * m];
    v[2 * m - 1] = fmaf(C, c, -S * sn);
    v[2 * m] = fmaf(C, sn, S * c);
  });
}

template <int P>
__device__ __forceinline__ void angle_table(float c1, float s1, float* cm, float* sm) {
  cm[0] = 1.f;
  sm[0] = 0.f;
  if constexpr (P >= 1) {
    cm[1] = c1;
    sm[1] = s1;
  }
  static_for<2, P + 1>([&](auto mc) {
    constexpr int m = mc;
    cm[m] = fmaf(cm[m - 1], c1, -sm[m - 1] * s1);
    sm[m] = fmaf(sm[m - 1], c1, cm[m - 1] * s1);
  });
}

}  // namespace mx

constexpr int MX_WAVES = 4;

// first source of [b, e) whose id is >= first_lo (ids are breadth first, so the
// sources above the root levels form a prefix of the ascending list)
__device__ __forceinline__ int split_point(const int* src, int b, int e, int first_lo) {
  int lo = b, hi = e;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (src[mid] < first_lo)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// One wavefront per sink (or wps of them, each with a contiguous part of the
// list), a source per lane.  Up to p = 10, four waves per
// SIMD (at most 128 VGPRs: a few bytes spill at p = 10, measured faster than
// three waves without); p = 11, 12 take three (p = 12 in 168 VGPRs, 6% faster
// than two waves on the 2^22-body workload) and higher orders two.
// The FP64 per-order sums live in LDS (a slot per lane), not in registers,
// which would spill at that budget.
// The angle multiples cos ma, sin ma of the two z-rotations come from tables
// built once per pair (rebuilding them in every order's rotation cost ~13% of
// the kernel's instructions at p = 10).
template <int P>
__global__ void __launch_bounds__(64 * MX_WAVES) __attribute__((amdgpu_waves_per_eu(P <= 10 ? 4 : P <= 12 ? 3 : 2))) k_m2l_fp32(int ncell, int first_lo,
                                                            const int* __restrict__ off,
                                                            const int* __restrict__ src,
                                                            const double* __restrict__ cx,
                                                            const double* __restrict__ cy,
                                                            const double* __restrict__ cz,
                                                            const double* __restrict__ scale,
                                                            const float* __restrict__ nmult,
                                                            double* __restrict__ loc, int wps, M2lSeg sg) {
  using namespace mx;
  constexpr int NC = ncoef(P);
  constexpr int NR = (P + 1) * (P + 1);
  // wps wavefronts per sink: the sink's list, in batches of 64 sources, is
  // split into wps contiguous parts; each wave sums its part, and the parts
  // are added in order at the end (through LDS, one barrier)
  // With one wave per sink and a plan (sg.nseg), the items are the sinks and
  // the later segments of long lists (see M2lSeg): a segment writes a partial
  // expansion, added to the sink's in segment order afterwards.
  int spb = MX_WAVES / wps;    // sinks per workgroup
  int nlo = ncell - first_lo;  // sinks below the root levels
  int nitems = sg.nseg ? sg.max_items : nlo;
  int nblk = (nitems + spb - 1) / spb;
  int blk = xcd_block();
  int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: B and its data in SGPRs
  int slot = wv / wps, part = wv - slot * wps;
  int it = blk * spb + slot, seg = 0;
  if (wps == 1 && (blk >= nblk || it >= nitems)) return;  // (no barrier below for one wave per sink)
  int B = first_lo + it;
  if (sg.nseg && it >= nlo) {  // a later segment of a long list (one wave per sink)
    int x = it - nlo;
    if (x >= *sg.nextra) return;
    int2 v = sg.extra[x];
    B = v.x;
    seg = v.y;
  }
  bool live = blk < nblk && B < ncell;
  int b = 0, e = 0;
  double* out = loc + (size_t)B * NC * 2;
  if (live) {
    e = off[B + 1];
    b = split_point(src, off[B], e, first_lo);
    if (sg.nseg && sg.nseg[B] > 1) {
      b += seg * sg.K;
      e = min(e, b + sg.K);
      if (seg > 0) out = sg.part + (size_t)(sg.pbase[B] + seg - 1) * NC * 2;
    }
  }
  int lane = threadIdx.x & 63;
  if (wps == 1 && b == e) {  // no FP32 pair: the sink's expansion starts at zero
    for (int k = lane; k < NC * 2; k += 64) out[k] = 0.0;
    return;
  }
  int nbat = (e - b + 63) >> 6;
  int pb = b + 64 * (nbat * part / wps), pe = min(e, b + 64 * (nbat * (part + 1) / wps));
  __shared__ double accs[MX_WAVES][P + 1][64];
  double* acc = &accs[wv][0][0] + lane;
#pragma unroll
  for (int t = 0; t <= P; t++) acc[64 * t] = 0.0;
  double bx = 0.0, by = 0.0, bz = 0.0, sB = 1.0;
  if (live) {
    bx = cx[B];
    by = cy[B];
    bz = cz[B];
    sB = scale[B];
  }

  for (int base = pb; base < pe; base += 64) {
    int k = base + lane;
    bool act = k < pe;
    int A = act ? src[k] : src[pb];
    // geometry in FP64, rounded once
    double Rx = bx - cx[A], Ry = by - cy[A], Rz = bz - cz[A];
    double rho2 = Rx * Rx + Ry * Ry;
    double r = sqrt(rho2 + Rz * Rz);
    double rho = sqrt(rho2);
    double rinv = 1.0 / r;
    float ca, sa;
    if (rho > 0.0) {
      double ri = 1.0 / rho;
      ca = (float)(Ry * ri);
      sa = (float)(Rx * ri);
    } else {
      ca = 0.f;
      sa = 1.f;
    }
    float cb = (float)(Rz * rinv), sb = (float)(-rho * rinv);
    float tca[P + 1], tsa[P + 1], tcb[P + 1], tsb[P + 1];
    angle_table<P>(ca, sa, tca, tsa);
    angle_table<P>(cb, sb, tcb, tsb);
    auto rotA = [&](auto nc, float* v, float sgn) { zrot_tab<decltype(nc)::value>(v, tca, tsa, sgn); };
    auto rotB = [&](auto nc, float* v, float sgn) { zrot_tab<decltype(nc)::value>(v, tcb, tsb, sgn); };
    // an inactive lane (past the end of the list) gets zero factors, so all its
    // outputs are zero
    float tA = (float)(scale[A] * rinv), tB = (float)(sB * rinv), fr = act ? (float)rinv : 0.f;
    float pA[P + 1], pB[P + 1];
    pA[0] = 1.f;
    pB[0] = fr;
#pragma unroll
    for (int j = 1; j <= P; j++) {
      pA[j] = pA[j - 1] * tA;
      pB[j] = pB[j - 1] * tB;
    }
    const float* Mv = nmult + (size_t)A * NR;
    constexpr int K0 = (P + 2) / 2;
    constexpr int NLP = (P - K0 + 1) * (P - K0 + 1);
    float Lp[NLP];
#pragma unroll
    for (int t = 0; t < NLP; t++) Lp[t] = 0.f;
    static_for<K0, P + 1>([&](auto kc) {
      constexpr int kk = kc;
      __builtin_amdgcn_sched_barrier(0);
      const float* Mo = Mv + kk * kk;
      asm volatile("" : "+v"(Mo));
      float v[2 * kk + 1];
      static_for<0, 2 * kk + 1>([&](auto jc) { v[jc] = Mo[jc]; });
      rotA(kc, v, 1.f);
      swap_apply<kk>(v);
      rotB(kc, v, 1.f);
      swap_apply<kk>(v);
      // fold into the partial local expansion: orders n <= P - kk
      static_for<0, 2 * kk + 1>([&](auto jc) { v[jc] *= pA[kk]; });
      static_for<0, P - kk + 1>([&](auto nc) {
        constexpr int n = nc;
        static_for<0, (n < kk ? n : kk) + 1>([&](auto mc) {
          constexpr int m = mc;
          constexpr float T = (float)tconst(n, kk, m);
          if constexpr (m == 0) {
            Lp[n * n] = fmaf(v[0], T, Lp[n * n]);
          } else {
            Lp[n * n + 2 * m - 1] = fmaf(v[2 * m - 1], T, Lp[n * n + 2 * m - 1]);
            Lp[n * n + 2 * m] = fmaf(v[2 * m], T, Lp[n * n + 2 * m]);
          }
        });
      });
    });
    float Mp[K0 * K0];
    static_for<0, K0>([&](auto nc) {
      constexpr int n = nc;
      __builtin_amdgcn_sched_barrier(0);
      const float* Mo = Mv + n * n;
      asm volatile("" : "+v"(Mo));
      float* v = Mp + n * n;
      static_for<0, 2 * n + 1>([&](auto jc) { v[jc] = Mo[jc]; });
      rotA(nc, v, 1.f);
      swap_apply<n>(v);
      rotB(nc, v, 1.f);
      swap_apply<n>(v);
      static_for<0, 2 * n + 1>([&](auto jc) { v[jc] *= pA[n]; });
    });
    static_for<0, P + 1>([&](auto nc) {
      constexpr int n = nc;
      __builtin_amdgcn_sched_barrier(0);
      float w[2 * n + 1];
      static_for<0, n + 1>([&](auto mc) {
        constexpr int m = mc;
        if constexpr (m <= P - n) {
          float sC = 0.f, sS = 0.f;
          if constexpr (n <= P - K0) {
            sC = Lp[n * n + (m == 0 ? 0 : 2 * m - 1)];
            if constexpr (m > 0) sS = Lp[n * n + 2 * m];
          }
          constexpr int KMAX = (P - n) < (K0 - 1) ? (P - n) : (K0 - 1);
          static_for<m, KMAX + 1>([&](auto kc) {
            constexpr int kk = kc;
            constexpr float T = (float)tconst(n, kk, m);
            sC = fmaf(Mp[kk * kk + (m == 0 ? 0 : 2 * m - 1)], T, sC);
            if constexpr (m > 0) sS = fmaf(Mp[kk * kk + 2 * m], T, sS);
          });
          if constexpr (m == 0) {
            w[0] = sC * pB[n];
          } else {
            w[2 * m - 1] = sC * pB[n];
            w[2 * m] = sS * pB[n];
          }
        } else {
          w[2 * m - 1] = 0.f;
          w[2 * m] = 0.f;
        }
      });
      swap_apply<n>(w);
      rotB(nc, w, -1.f);
      swap_apply<n>(w);
      rotA(nc, w, -1.f);
      reduce_lanes<2 * n + 1>(w, &acc[64 * n], lane);
    });
  }
  if (wps > 1) {
    __syncthreads();  // every part's sums are in LDS
    if (!live || part != 0) return;
    if (b == e) {
      for (int k = lane; k < NC * 2; k += 64) out[k] = 0.0;
      return;
    }
  }
  // back to standard coefficients: L_n^0 = Lt n! / rho_B^n,
  // L_n^m = Lt sqrt((n-m)!(n+m)!/2) / rho_B^n; real-basis entry j of order n
  // is held by lane reduce_owner(2n+1, j) (the cross-lane sum in fmm_device.h)
  double isB = 1.0 / sB, pw = 1.0;
  static_for<0, P + 1>([&](auto nc) {
    constexpr int n = nc;
    int j, real;
    reduce_slot<2 * n + 1>(lane, j, real);
    if (real) {
      int m = (j + 1) >> 1;
      bool im = j > 0 && !(j & 1);
      double f = (m == 0 ? 1.0 : sqrt(0.5)) * sqrt(fmm_fact_dev(n - m) * fmm_fact_dev(n + m)) * pw;
      double t = acc[64 * n];
      for (int k = 1; k < wps; k++) t += accs[wv + k][n][lane];  // the other parts, in order
      out[2 * cidx(n, m) + (im ? 1 : 0)] = t * f;
      if (j == 0) out[2 * cidx(n, 0) + 1] = 0.0;
    }
    pw *= isB;
  });
}

// normalised, size-scaled FP32 moments of every cell (real basis, (P+1)^2 per cell)
__global__ void k_normalize32(int p, int ncell, const double* mult, const double* scale, float* nmult) {
  int nr = (p + 1) * (p + 1);
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)ncell * nr) return;
  int c = (int)(t / nr), j = (int)(t % nr);
  int n = 0;
  while ((n + 1) * (n + 1) <= j) n++;
  int jj = j - n * n, m = (jj + 1) >> 1;
  bool im = jj > 0 && !(jj & 1);
  double g = m == 0 ? fmm_fact_dev(n) : sqrt(2.0 * fmm_fact_dev(n - m) * fmm_fact_dev(n + m));
  double v = mult[(size_t)c * ncoef(p) * 2 + 2 * cidx(n, m) + (im ? 1 : 0)];
  double is = 1.0 / scale[c], pw = 1.0;  // scale^-n by repeated products (as on the local side)
  for (int k = 0; k < n; k++) pw *= is;
  nmult[t] = (float)(v * g * pw);
}

// expansion scale per cell: its radius, or 1 for a point-like cell
__global__ void k_scale(int ncell, const double* rad, double* scale) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncell) scale[c] = rad[c] > 0.0 ? rad[c] : 1.0;
}

// The segment plan of the FP32 M2L (one thread per sink below the root
// levels; its FP32 pairs are the list's suffix from split_point); ctr[0]
// counts the extra items (zero on entry).
__global__ void k_m2l32_plan(int ncell, int first_lo, const int* __restrict__ off, const int* __restrict__ src,
                             int K, int* nseg, int* pbase, int2* extra, int* ctr) {
  int B = first_lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (B >= ncell) return;
  int e = off[B + 1];
  int len = e - split_point(src, off[B], e, first_lo);
  int ns = len > K ? (len + K - 1) / K : 1;
  nseg[B] = ns;
  if (ns > 1) {
    int x = atomicAdd(ctr, ns - 1);
    for (int k = 1; k < ns; k++) extra[x + k - 1] = make_int2(B, k);
    pbase[B] = x;
  }
}

// partial expansions of split sinks added in segment order (threads of each
// sink's first extra item, one per coefficient)
__global__ void k_m2l32_combine(int ncd, int max_extra, const int* __restrict__ nseg, const int* __restrict__ pbase,
                                const int2* __restrict__ extra, const int* __restrict__ nextra,
                                const double* __restrict__ part, double* loc) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int x = (int)(t / ncd), k = (int)(t % ncd);
  if (x >= max_extra || x >= *nextra) return;
  int2 v = extra[x];
  if (v.y != 1) return;
  int B = v.x, ns = nseg[B];
  double s = loc[(size_t)B * ncd + k];
  for (int g = 1; g < ns; g++) s += part[(size_t)(pbase[B] + g - 1) * ncd + k];
  loc[(size_t)B * ncd + k] = s;
}

constexpr int M2L32_SEG_MIN = 512;   // FP32 pairs per segment, at least
constexpr int M2L32_SEG_DIV = 8192;  // and at least the list total / M2L32_SEG_DIV

template <int P>
static void launch_p32(Ctx& c, int first_lo) {
  int nc = (int)c.ncell;
  int nlo = nc - first_lo;
  if (nlo <= 0) return;
  int wps = c.prm.m2l_waves;
  int spb = MX_WAVES / wps;
  M2lSeg sg{};
  int64_t extra_max = 0;
  if (wps == 1) {  // long lists in segments (see M2lSeg)
    int64_t cnt = c.m2l.count;
    int K = (int)std::max<int64_t>(M2L32_SEG_MIN, ceil_div(cnt, M2L32_SEG_DIV));
    // split sinks hold len > K pairs in ceil(len / K) < 2 len / K segments:
    // fewer than cnt / K <= M2L32_SEG_DIV extra items
    extra_max = std::min<int64_t>(M2L32_SEG_DIV, ceil_div(cnt, K));
    size_t ncd = (size_t)ncoef(P) * 2;
    ensure(c.ws, c.m2l_nseg, (size_t)nc + 1);
    ensure(c.ws, c.m2l_pbase, (size_t)nc + 1);
    ensure(c.ws, c.m2l_extra, (size_t)extra_max + 1);
    ensure(c.ws, c.m2l_part, (size_t)(extra_max + 1) * ncd);
    ensure(c.ws, c.counters, 512);
    int* ctr = c.counters.p + 46;
    zero_fill(c, ctr, sizeof(int));
    hipLaunchKernelGGL(k_m2l32_plan, dim3((unsigned)ceil_div(nlo, 256)), dim3(256), 0, c.stream, nc, first_lo,
                       c.m2l.off.p, c.m2l.src.p, K, c.m2l_nseg.p, c.m2l_pbase.p, c.m2l_extra.p, ctr);
    HIPCHK(hipGetLastError());
    sg = M2lSeg{c.m2l_nseg.p, c.m2l_pbase.p, c.m2l_extra.p, ctr, c.m2l_part.p, K, (int)(nlo + extra_max)};
  }
  int nitems = sg.nseg ? sg.max_items : nlo;
  int nblk = (nitems + spb - 1) / spb;
  unsigned grid = xcd_grid(nblk);
  hipLaunchKernelGGL(k_m2l_fp32<P>, dim3(grid), dim3(64 * MX_WAVES), 0, c.stream, nc, first_lo,
                     c.m2l.off.p, c.m2l.src.p, c.c_cx.p, c.c_cy.p, c.c_cz.p, c.scale.p, c.nmult.p, c.loc.p,
                     wps, sg);
  if (sg.nseg && extra_max > 0) {
    int ncd = ncoef(P) * 2;
    hipLaunchKernelGGL(k_m2l32_combine, dim3((unsigned)ceil_div(extra_max * ncd, 256)), dim3(256), 0, c.stream,
                       ncd, (int)extra_max, sg.nseg, sg.pbase, sg.extra, sg.nextra, sg.part, c.loc.p);
  }
}

template <int P>
static bool dispatch32(Ctx& c, int first_lo) {
  if constexpr (P > FMM_GPU_PMAX) {
    return false;
  } else {
    if (c.p == P) {
      launch_p32<P>(c, first_lo);
      return true;
    }
    return dispatch32<P + 1>(c, first_lo);
  }
}

bool mixed_supported(int p) { return p >= 1 && p <= FMM_GPU_PMAX; }

void launch_m2l_fp64_range(Ctx& c, int first_lo);

void launch_m2l_mixed_lo(Ctx& c) {
  int nc = (int)c.ncell;
  int first_lo = mixed_first_lo(c);
  if (first_lo >= nc) {
    if (c.have_events) {  // no FP32 pairs: the main M2L kernel time is zero
      HIPCHK(hipEventRecord(c.ev[9], c.stream));
      HIPCHK(hipEventRecord(c.ev[10], c.stream));
    }
    return;
  }
  if (c.have_events) HIPCHK(hipEventRecord(c.ev[9], c.stream));
  if (!dispatch32<1>(c, first_lo)) throw hip_error{hipErrorInvalidValue, "M2L order not compiled"};
  HIPCHK(hipGetLastError());
  if (c.have_events) HIPCHK(hipEventRecord(c.ev[10], c.stream));
}

// expansion scales and normalised FP32 moments of every cell (mixed
// precision); run with the upward pass, as soon as the multipoles exist
void launch_normalize32(Ctx& c) {
  int nc = (int)c.ncell;
  ensure(c.ws, c.scale, (size_t)nc);
  ensure(c.ws, c.nmult, (size_t)nc * (c.p + 1) * (c.p + 1));
  hipLaunchKernelGGL(k_scale, dim3((nc + 255) / 256), dim3(256), 0, c.stream, nc, c.c_rad.p, c.scale.p);
  int64_t tot = (int64_t)nc * (c.p + 1) * (c.p + 1);
  hipLaunchKernelGGL(k_normalize32, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, c.stream, c.p, nc,
                     c.mult.p, c.scale.p, c.nmult.p);
  HIPCHK(hipGetLastError());
}

// first cell below the root levels (ids are breadth first)
int mixed_first_lo(Ctx& c) {
  // orders without an FP32 kernel: every M2L pair in FP64 (the near field
  // stays FP32)
  if (!mixed_supported(c.p)) return (int)c.ncell;
  int K = c.prm.root_levels;
  return K <= c.depth ? c.lvl_first[K] : (int)c.ncell;
}

// sinks with at least one FP64 pair: every sink above first_lo with a
// non-empty list, and those below whose (ascending) list starts above it.
// The list order depends on the atomics; each sink's result does not.
__global__ void k_root_sinks(int ncell, int first_lo, const int* __restrict__ off, const int* __restrict__ src,
                             int* __restrict__ sinks, int* __restrict__ count) {
  int B = blockIdx.x * blockDim.x + threadIdx.x;
  if (B >= ncell) return;
  int b = off[B], e = off[B + 1];
  bool has = b < e && (B < first_lo || src[b] < first_lo);
  if (has) sinks[atomicAdd(count, 1)] = B;
}

// loc[B] += loc64[B] for the listed sinks (grid-stride over coefficients)
__global__ void k_add_sinks(const int* __restrict__ sinks, const int* __restrict__ count, int ncd,
                            double* __restrict__ loc, const double* __restrict__ loc64) {
  int64_t tot = (int64_t)(*count) * ncd;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
    size_t k = (size_t)sinks[t / ncd] * ncd + (size_t)(t % ncd);
    loc[k] += loc64[k];
  }
}

// FP64 M2L of every pair touching a root-level cell into loc64, for the sinks
// that have such pairs (listed in c.root_sinks, count at counters[64]); the
// other sinks' entries of loc64 are not written
void launch_m2l_mixed_root(Ctx& c, double* loc64) {
  int nc = (int)c.ncell;
  ensure(c.ws, c.root_sinks, (size_t)nc);
  ensure(c.ws, c.counters, 512);
  int* count = c.counters.p + 64;
  zero_fill(c, count, sizeof(int));
  int first_lo = mixed_first_lo(c);
  hipLaunchKernelGGL(k_root_sinks, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, c.stream, nc, first_lo,
                     c.m2l.off.p, c.m2l.src.p, c.root_sinks.p, count);
  HIPCHK(hipGetLastError());
  launch_m2l_fp64_sinks(c, first_lo, c.mult.p, loc64, c.root_sinks.p, count);
}

// loc += loc64 over the sinks launch_m2l_mixed_root listed
void add_root_locals(Ctx& c, double* loc, const double* loc64) {
  hipLaunchKernelGGL(k_add_sinks, dim3(1024), dim3(256), 0, c.stream, c.root_sinks.p, c.counters.p + 64,
                     ncoef(c.p) * 2, loc, loc64);
  HIPCHK(hipGetLastError());
}

}  // namespace fmm
