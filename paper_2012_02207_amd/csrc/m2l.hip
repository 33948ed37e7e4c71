// Rotation-accelerated M2L on gfx950 (section 2.4), FP64.
//
// For a directed pair A -> B with R = z_B - z_A, the source moments are
// rotated so that R lies along +z (rotate about z by alpha = pi/2 - phi, swap
// x <-> z, rotate about z by beta = -theta, swap x <-> z), translated along z,
// where only T_j^0(r z) = j!/r^{j+1} is non-zero (O(p^3) instead of O(p^4)),
// and rotated back.  Locals transform with the transposed map; in the scaled
// basis Lhat_n^m = L_n^m / ((n-m)!(n+m)!) that transpose is again
// "swap, rotate, swap, rotate" with negated angles in reverse order, so one
// table of swap matrices W_n (exact dyadic rationals, u(z,y,x) = W_n u(x,y,z))
// serves both directions.  Real basis per order n: index 0 = Re c^0,
// 2m-1 = Re c^m, 2m = Im c^m.  W_n never mixes Re with Im parts and couples
// Re^m with Re^m' only when m + m' + n is even (Im parts: odd); those zeros are
// skipped at compile time.
//
// Work mapping: one wavefront owns one sink cell B and keeps its local
// expansion (scaled basis) distributed over the lanes; each lane evaluates the
// whole rotated M2L of one source of B's list, and every output order is
// summed across the wavefront before it is added.  The order p is a template
// parameter so that all coefficient arrays live in registers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "fmm_device.h"
#include "fmm_tables.h"

namespace fmm {

constexpr int swoff(int n) { return n * (4 * n * n - 1) / 3; }

static __constant__ double c_fact_m2l[2 * FMM_GPU_PMAX + 2];
static bool g_m2l_tables[64] = {};  // per device

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

// real-basis index helpers
constexpr int rb_m(int j) { return (j + 1) >> 1; }
constexpr bool rb_re(int j) { return j == 0 || (j & 1); }
constexpr bool swap_nz(int n, int i, int j) {
  return rb_re(i) == rb_re(j) && (((rb_m(i) + rb_m(j) + n) & 1) == (rb_re(i) ? 0 : 1));
}

// position of entry j among the structural non-zeros of row i of W_n (the
// first one starts each row's sum)
constexpr int crank(int n, int i, int j) {
  int c = 0;
  for (int t = 0; t < j; t++) c += swap_nz(n, i, t) ? 1 : 0;
  return c;
}

// v (order-n slice, 2n+1 values) <- W_n v.  The structural non-zeros are
// compile-time constants (dyadic rationals, most of them exact as the 32-bit
// literal operand of v_fmac_f64), so no product loads its matrix entry.
template <int N, class T>
__device__ __forceinline__ void swap_apply(T* v) {
  constexpr int D = 2 * N + 1;
  T out[D];
  static_for<0, D>([&](auto ic) {
    constexpr int i = ic;
    T s = 0;
    static_for<0, D>([&](auto jc) {
      constexpr int j = jc;
      if constexpr (swap_nz(N, i, j)) {
        constexpr double wc = fmm_swap_table[swoff(N) + i * (2 * N + 1) + j];
        T w = (T)wc;
        if constexpr (crank(N, i, j) == 0)
          s = w * v[j];
        else
          s = fma(w, v[j], s);
      }
    });
    out[i] = s;
  });
  static_for<0, D>([&](auto ic) { v[ic] = out[ic]; });
}

// rotation about z: (C, S)_m <- (C cos m a - S sin m a, C sin m a + S cos m a);
// cos m a, sin m a by the angle-addition recurrence from (c1, s1)
template <int N, class T>
__device__ __forceinline__ void zrot(T* v, T c1, T s1) {
  T cm = c1, sm = s1;
  static_for<1, N + 1>([&](auto mc) {
    constexpr int m = mc;
    if constexpr (m > 1) {
      T c2 = fma(cm, c1, -sm * s1);
      sm = fma(sm, c1, cm * s1);
      cm = c2;
    }
    T C = v[2 * m - 1], S = v[2 * m];
    v[2 * m - 1] = fma(C, cm, -S * sm);
    v[2 * m] = fma(C, sm, S * cm);
  });
}

// Transpose-reduce of D values per lane over the 64 lanes: at each butterfly
// step a lane keeps half of its remaining values and adds the partner's copy
// of that half (about D + 6 shuffles instead of 6 D).  Afterwards the total of
// value j sits in lane j * (64 / Dp) (Dp = D rounded up to a power of two),
// which adds it to its accumulator acc_slot.
constexpr int M2L_WAVES = 4;  // sinks per workgroup (one per wavefront)

// M2L of the pairs src[b .. e) of one sink cell B (one wavefront; lane =
// lane id) into the expansion out (NC complex coefficients; zeros when b == e)
template <int P>
__device__ __forceinline__ void m2l_range_fp64(int B, int b, int e, int lane, const int* __restrict__ src,
                                               const double* __restrict__ cx, const double* __restrict__ cy,
                                               const double* __restrict__ cz, const double* __restrict__ mult,
                                               double* __restrict__ out, double* acc) {
  constexpr int NC = ncoef(P);
  if (b == e) {  // no pair: the sink's expansion starts at zero (never a listed sink)
    for (int k = lane; k < NC * 2; k += 64) out[k] = 0.0;
    return;
  }
  // per-order sums, one LDS slot per lane: acc[64 n]
#pragma unroll
  for (int t = 0; t <= P; t++) acc[64 * t] = 0.0;
  double bx = cx[B], by = cy[B], bz = cz[B];

  for (int base = b; base < e; base += 64) {
    int k = base + lane;
    bool act = k < e;
    int A = act ? src[k] : src[b];
    double Rx = bx - cx[A], Ry = by - cy[A], Rz = bz - cz[A];
    double rho2 = fma(Rx, Rx, Ry * Ry);
    double r2 = fma(Rz, Rz, rho2);
    double rinv = 1.0 / sqrt(r2);
    double rho = sqrt(rho2);
    double ca, sa;
    if (rho > 0.0) {
      double ri = 1.0 / rho;
      ca = Ry * ri;
      sa = Rx * ri;
    } else {
      ca = 0.0;
      sa = 1.0;
    }
    double cb = Rz * rinv, sb = -rho * rinv;
    // translation factors g_j = j! / r^{j+1}
    // (an inactive lane, past the end of the list, gets zero factors, so all
    // its outputs are zero)
    double g[P + 1];
    {
      double rp = act ? rinv : 0.0;
#pragma unroll
      for (int j = 0; j <= P; j++) {
        g[j] = cfact(j) * rp;
        rp *= rinv;
      }
    }
    const double* M = mult + (size_t)A * NC * 2;
    // Source orders k >= K0 reach only output orders n <= P - k < K0: rotate
    // them first and fold them at once into a partial local expansion Lp
    // (orders 0..P-K0), so that only the low orders of the rotated multipole
    // stay live.  Same terms, summed in a different order.
    constexpr int K0 = (P + 2) / 2;
    constexpr int NLP = (P - K0 + 1) * (P - K0 + 1);
    double Lp[NLP];
#pragma unroll
    for (int t = 0; t < NLP; t++) Lp[t] = 0.0;
    static_for<K0, P + 1>([&](auto kc) {
      constexpr int kk = kc;
      __builtin_amdgcn_sched_barrier(0);
      double v[2 * kk + 1];
      // an opaque per-order pointer keeps the loads of this order from being
      // merged with (and hoisted along with) those of other orders
      const double* Mo = M + 2 * cidx(kk, 0);
      asm volatile("" : "+v"(Mo));
      v[0] = Mo[0];
      static_for<1, kk + 1>([&](auto mc) {
        constexpr int m = mc;
        v[2 * m - 1] = Mo[2 * m];
        v[2 * m] = Mo[2 * m + 1];
      });
      zrot<kk>(v, ca, sa);
      swap_apply<kk>(v);
      zrot<kk>(v, cb, sb);
      swap_apply<kk>(v);
      static_for<0, P - kk + 1>([&](auto nc) {
        constexpr int n = nc;
        static_for<0, (n < kk ? n : kk) + 1>([&](auto mc) {
          constexpr int m = mc;
          if constexpr (m == 0) {
            Lp[n * n] = fma(v[0], g[n + kk], Lp[n * n]);
          } else {
            Lp[n * n + 2 * m - 1] = fma(v[2 * m - 1], g[n + kk], Lp[n * n + 2 * m - 1]);
            Lp[n * n + 2 * m] = fma(v[2 * m], g[n + kk], Lp[n * n + 2 * m]);
          }
        });
      });
    });
    // low source orders: rotate and keep
    double Mp[K0 * K0];
    static_for<0, K0>([&](auto nc) {
      constexpr int n = nc;
      __builtin_amdgcn_sched_barrier(0);
      double* v = Mp + n * n;
      const double* Mo = M + 2 * cidx(n, 0);
      asm volatile("" : "+v"(Mo));
      v[0] = Mo[0];
      static_for<1, n + 1>([&](auto mc) {
        constexpr int m = mc;
        v[2 * m - 1] = Mo[2 * m];
        v[2 * m] = Mo[2 * m + 1];
      });
      zrot<n>(v, ca, sa);
      swap_apply<n>(v);
      zrot<n>(v, cb, sb);
      swap_apply<n>(v);
    });
    // complete the translation, rotate back and reduce, one output order at a time
    static_for<0, P + 1>([&](auto nc) {
      constexpr int n = nc;
      __builtin_amdgcn_sched_barrier(0);
      double w[2 * n + 1];
      static_for<0, n + 1>([&](auto mc) {
        constexpr int m = mc;
        if constexpr (m <= P - n) {
          double sC = 0.0, sS = 0.0;
          if constexpr (n <= P - K0) {
            sC = Lp[n * n + (m == 0 ? 0 : 2 * m - 1)];
            if constexpr (m > 0) sS = Lp[n * n + 2 * m];
          }
          constexpr int KMAX = (P - n) < (K0 - 1) ? (P - n) : (K0 - 1);
          static_for<m, KMAX + 1>([&](auto kc) {
            constexpr int kk = kc;
            sC = fma(Mp[kk * kk + (m == 0 ? 0 : 2 * m - 1)], g[n + kk], sC);
            if constexpr (m > 0) sS = fma(Mp[kk * kk + 2 * m], g[n + kk], sS);
          });
          constexpr double f = (((n + m) & 1) ? -1.0 : 1.0) / (cfact(n - m) * cfact(n + m));
          if constexpr (m == 0) {
            w[0] = sC * f;
          } else {
            w[2 * m - 1] = sC * f;
            w[2 * m] = sS * f;
          }
        } else {
          w[2 * m - 1] = 0.0;
          w[2 * m] = 0.0;
        }
      });
      swap_apply<n>(w);
      zrot<n>(w, cb, -sb);
      swap_apply<n>(w);
      zrot<n>(w, ca, -sa);
      reduce_lanes<2 * n + 1>(w, &acc[64 * n], lane);
    });
  }
  // back to the unscaled basis: L_n^m = (n-m)!(n+m)! Lhat_n^m; real-basis
  // entry j of order n is held by lane reduce_owner(2n+1, j) (the cross-lane
  // sum in fmm_device.h)
  static_for<0, P + 1>([&](auto nc) {
    constexpr int n = nc;
    int j, real;
    reduce_slot<2 * n + 1>(lane, j, real);
    if (real) {
      int m = (j + 1) >> 1;
      bool im = j > 0 && !(j & 1);
      double f = c_fact_m2l[n - m] * c_fact_m2l[n + m];
      out[2 * cidx(n, m) + (im ? 1 : 0)] = acc[64 * n] * f;
      if (j == 0) out[2 * cidx(n, 0) + 1] = 0.0;
    }
  });
}

// M2L of the list of one sink cell B; with B >= first_lo only the sources
// below first_lo are taken
template <int P>
__device__ __forceinline__ void m2l_sink_fp64(int B, int first_lo, int lane, const int* __restrict__ off,
                                              const int* __restrict__ src, const double* __restrict__ cx,
                                              const double* __restrict__ cy, const double* __restrict__ cz,
                                              const double* __restrict__ mult, double* __restrict__ loc,
                                              double* acc) {
  constexpr int NC = ncoef(P);
  int b = off[B], e = off[B + 1];
  if (B >= first_lo) {
    // mixed precision: only the sources above the root levels (a prefix of
    // the ascending, breadth-first list) are handled in FP64
    int lo = b, hi = e;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (src[mid] < first_lo)
        lo = mid + 1;
      else
        hi = mid;
    }
    e = lo;
  }
  m2l_range_fp64<P>(B, b, e, lane, src, cx, cy, cz, mult, loc + (size_t)B * NC * 2, acc);
}

// All sinks (one wavefront each; consecutive workgroups, which the hardware
// hands to the eight XCDs in turn, take consecutive sinks, so that every XCD
// gets an even share of the work), or, with LIST, the sinks[0 .. *nsinks) in
// a grid-stride loop.  Up to p = 12, two waves per SIMD (256 registers each;
// at p = 12 84 B spill, and the 2^22-body FP64 evaluation still takes 49.2 ms
// instead of 55.0 with one wave).  Higher orders take one wave.  The per-order
// sums live in LDS and the sink index is wave-uniform (its data in SGPRs).
template <int P, bool LIST>
__global__ void __launch_bounds__(64 * M2L_WAVES) __attribute__((amdgpu_waves_per_eu(P <= 12 ? 2 : 1))) k_m2l_fp64(int ncell, int first_lo, const int* __restrict__ sinks,
                                                             const int* __restrict__ nsinks,
                                                             const int* __restrict__ off,
                                                             const int* __restrict__ src,
                                                             const double* __restrict__ cx,
                                                             const double* __restrict__ cy,
                                                             const double* __restrict__ cz,
                                                             const double* __restrict__ mult,
                                                             double* __restrict__ loc, M2lSeg sg) {
  constexpr int NC = ncoef(P);
  int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  __shared__ double accs[M2L_WAVES][P + 1][64];
  double* acc = &accs[wv][0][0] + lane;
  if constexpr (LIST) {
    int cnt = *nsinks;
    for (int it = blockIdx.x * M2L_WAVES + wv; it < cnt; it += gridDim.x * M2L_WAVES)
      m2l_sink_fp64<P>(sinks[it], first_lo, lane, off, src, cx, cy, cz, mult, loc, acc);
  } else {
    int nitems = sg.nseg ? sg.max_items : ncell;
    int nblk = (nitems + M2L_WAVES - 1) / M2L_WAVES;
    int blk = xcd_block();
    int it = blk * M2L_WAVES + wv;
    if (blk >= nblk || it >= nitems) return;
    if (!sg.nseg) {
      m2l_sink_fp64<P>(it, first_lo, lane, off, src, cx, cy, cz, mult, loc, acc);
      return;
    }
    // whole lists, long ones in segments of K pairs
    int B = it, seg = 0;
    if (it >= ncell) {
      int x = it - ncell;
      if (x >= *sg.nextra) return;
      int2 v = sg.extra[x];
      B = v.x;
      seg = v.y;
    }
    int b = off[B], e = off[B + 1];
    double* out = loc + (size_t)B * NC * 2;
    if (sg.nseg[B] > 1) {
      b += seg * sg.K;
      e = min(e, b + sg.K);
      if (seg > 0) out = sg.part + (size_t)(sg.pbase[B] + seg - 1) * NC * 2;
    }
    m2l_range_fp64<P>(B, b, e, lane, src, cx, cy, cz, mult, out, acc);
  }
}

// The segment plan of the M2L over whole lists (one thread per sink); ctr[0]
// counts the extra items (zero on entry), and a split sink's partial slots
// follow its extra items.
__global__ void k_m2l_plan(int ncell, const int* __restrict__ off, int K, int* nseg, int* pbase, int2* extra,
                           int* ctr) {
  int B = blockIdx.x * blockDim.x + threadIdx.x;
  if (B >= ncell) return;
  int len = off[B + 1] - off[B];
  int ns = len > K ? (len + K - 1) / K : 1;
  nseg[B] = ns;
  if (ns > 1) {
    int x = atomicAdd(ctr, ns - 1);
    for (int k = 1; k < ns; k++) extra[x + k - 1] = make_int2(B, k);
    pbase[B] = x;
  }
}

// the partial expansions of split sinks added in segment order (threads of
// each sink's first extra item, one per coefficient)
__global__ void k_m2l_combine(int ncd, int max_extra, const int* __restrict__ nseg, const int* __restrict__ pbase,
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

constexpr int M2L_SEG_MIN = 512;    // pairs per segment, at least
constexpr int M2L_SEG_DIV = 8192;   // and at least the list total / M2L_SEG_DIV

// the plan for the M2L over whole lists (on c.stream)
static M2lSeg plan_m2l(Ctx& c) {
  int nc = (int)c.ncell;
  int64_t cnt = c.m2l.count;
  int K = (int)std::max<int64_t>(M2L_SEG_MIN, ceil_div(cnt, M2L_SEG_DIV));
  // a split sink holds len > K pairs in ceil(len / K) < 2 len / K segments, so
  // the extra items number fewer than cnt / K <= M2L_SEG_DIV
  int64_t extra_max = std::min<int64_t>(M2L_SEG_DIV, ceil_div(cnt, K));
  size_t ncd = (size_t)ncoef(c.p) * 2;
  ensure(c.ws, c.m2l_nseg, (size_t)nc + 1);
  ensure(c.ws, c.m2l_pbase, (size_t)nc + 1);
  ensure(c.ws, c.m2l_extra, (size_t)extra_max + 1);
  ensure(c.ws, c.m2l_part, (size_t)(extra_max + 1) * ncd);
  ensure(c.ws, c.counters, 512);
  int* ctr = c.counters.p + 46;
  zero_fill(c, ctr, sizeof(int));
  hipLaunchKernelGGL(k_m2l_plan, dim3((unsigned)ceil_div(nc, 256)), dim3(256), 0, c.stream, nc, c.m2l.off.p, K,
                     c.m2l_nseg.p, c.m2l_pbase.p, c.m2l_extra.p, ctr);
  HIPCHK(hipGetLastError());
  return M2lSeg{c.m2l_nseg.p, c.m2l_pbase.p, c.m2l_extra.p, ctr, c.m2l_part.p, K, (int)(nc + extra_max)};
}

// sinks == nullptr: every sink cell; otherwise the listed sinks (count on the
// device, so the launch needs no host synchronisation)
template <int P>
static void launch_p(Ctx& c, int first_lo, const double* mult, double* loc, const int* sinks, const int* nsinks) {
  int nc = (int)c.ncell;
  if (sinks) {
    constexpr unsigned LIST_BLOCKS = 512;
    hipLaunchKernelGGL((k_m2l_fp64<P, true>), dim3(LIST_BLOCKS), dim3(64 * M2L_WAVES), 0, c.stream, nc, first_lo,
                       sinks, nsinks, c.m2l.off.p, c.m2l.src.p, c.c_cx.p, c.c_cy.p, c.c_cz.p, mult, loc, M2lSeg{});
    return;
  }
  M2lSeg sg{};
  if (first_lo >= nc) sg = plan_m2l(c);  // whole lists: long ones in segments
  int nitems = sg.nseg ? sg.max_items : nc;
  int nblk = (nitems + M2L_WAVES - 1) / M2L_WAVES;
  unsigned grid = xcd_grid(nblk);
  hipLaunchKernelGGL((k_m2l_fp64<P, false>), dim3(grid), dim3(64 * M2L_WAVES), 0, c.stream, nc, first_lo,
                     (const int*)nullptr, (const int*)nullptr, c.m2l.off.p, c.m2l.src.p, c.c_cx.p, c.c_cy.p,
                     c.c_cz.p, mult, loc, sg);
  if (sg.nseg) {
    int ncd = ncoef(P) * 2, max_extra = sg.max_items - nc;
    if (max_extra > 0)
      hipLaunchKernelGGL(k_m2l_combine, dim3((unsigned)ceil_div((int64_t)max_extra * ncd, 256)), dim3(256), 0,
                         c.stream, ncd, max_extra, sg.nseg, sg.pbase, sg.extra, sg.nextra, sg.part, loc);
  }
}

template <int P>
static bool dispatch(Ctx& c, int first_lo, const double* mult, double* loc, const int* sinks, const int* nsinks) {
  if constexpr (P > FMM_GPU_PMAX) {
    return false;
  } else {
    if (c.p == P) {
      launch_p<P>(c, first_lo, mult, loc, sinks, nsinks);
      return true;
    }
    return dispatch<P + 1>(c, first_lo, mult, loc, sinks, nsinks);
  }
}

void launch_m2l_fp64(Ctx& c) {
  if (c.have_events) HIPCHK(hipEventRecord(c.ev[9], c.stream));
  launch_m2l_fp64_range(c, (int)c.ncell);
  if (c.have_events) HIPCHK(hipEventRecord(c.ev[10], c.stream));
}

// FP64 M2L for all pairs whose sink is above first_lo or whose source is
// (first_lo = ncell: every pair); writes loc, which must be zeroed before
void launch_m2l_fp64_range(Ctx& c, int first_lo) {
  launch_m2l_fp64_buffers(c, first_lo, c.mult.p, c.loc.p);
}

static bool& m2l_tables_flag() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  return g_m2l_tables[dev & 63];
}

void upload_m2l_tables() {
  bool& done = m2l_tables_flag();
  if (done) return;
  HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_fact_m2l), fmm_fact_table, sizeof(double) * (2 * FMM_GPU_PMAX + 2)));
  done = true;
}

// the same over other expansion buffers (same tree and list)
void launch_m2l_fp64_buffers(Ctx& c, int first_lo, const double* mult, double* loc) {
  if (c.p > FMM_GPU_PMAX) return launch_m2l_hi(c, first_lo, mult, loc, nullptr, nullptr);
  upload_m2l_tables();
  if (!dispatch<1>(c, first_lo, mult, loc, nullptr, nullptr))
    throw hip_error{hipErrorInvalidValue, "M2L order not compiled"};
  HIPCHK(hipGetLastError());
}

// only the sinks sinks[0 .. *nsinks) (device memory); every coefficient of a
// listed sink is written, the others are left untouched
void launch_m2l_fp64_sinks(Ctx& c, int first_lo, const double* mult, double* loc, const int* sinks,
                           const int* nsinks) {
  if (c.p > FMM_GPU_PMAX) return launch_m2l_hi(c, first_lo, mult, loc, sinks, nsinks);
  upload_m2l_tables();
  if (!dispatch<1>(c, first_lo, mult, loc, sinks, nsinks))
    throw hip_error{hipErrorInvalidValue, "M2L order not compiled"};
  HIPCHK(hipGetLastError());
}

}  // namespace fmm
