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

#include <type_traits>

#include "fmm_device.h"
#include "fmm_tables.h"

namespace fmm {

constexpr int swoff(int n) { return n * (4 * n * n - 1) / 3; }
constexpr int SWAP_DOUBLES = swoff(FMM_GPU_PMAX + 1);

static __constant__ double c_swap[SWAP_DOUBLES];
static bool g_m2l_tables = false;

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

// v (order-n slice, 2n+1 values) <- W_n v
template <int N, class T>
__device__ __forceinline__ void swap_apply(T* v) {
  constexpr int D = 2 * N + 1;
  T out[D];
  static_for<0, D>([&](auto ic) {
    constexpr int i = ic;
    T s = 0;
    bool first = true;
    static_for<0, D>([&](auto jc) {
      constexpr int j = jc;
      if constexpr (swap_nz(N, i, j)) {
        T w = (T)c_swap[swoff(N) + i * D + j];
        if (first) {
          s = w * v[j];
          first = false;
        } else {
          s = fma(w, v[j], s);
        }
      }
    });
    out[i] = s;
  });
  static_for<0, D>([&](auto ic) { v[ic] = out[ic]; });
}

// rotation about z: (C, S)_m <- (C cos m a - S sin m a, C sin m a + S cos m a)
template <int N, class T>
__device__ __forceinline__ void zrot(T* v, const T* cm, const T* sm, T sgn) {
  static_for<1, N + 1>([&](auto mc) {
    constexpr int m = mc;
    T C = v[2 * m - 1], S = v[2 * m];
    T s = sgn * sm[m];
    v[2 * m - 1] = fma(C, cm[m], -S * s);
    v[2 * m] = fma(C, s, S * cm[m]);
  });
}

template <int P>
__global__ void __launch_bounds__(64) k_m2l_fp64(int ncell, const int* __restrict__ off,
                                                 const int* __restrict__ src,
                                                 const double* __restrict__ cx,
                                                 const double* __restrict__ cy,
                                                 const double* __restrict__ cz,
                                                 const double* __restrict__ mult,
                                                 double* __restrict__ loc) {
  constexpr int NC = ncoef(P);
  constexpr int NR = (P + 1) * (P + 1);      // real-basis length
  constexpr int NSLOT = (NR + 63) / 64;
  // XCD-aware mapping: consecutive workgroups land on different XCDs, so give
  // each XCD a contiguous range of sinks (neighbouring sinks share sources)
  int per = (ncell + 7) >> 3;
  int B = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (B >= ncell) return;
  int b = off[B], e = off[B + 1];
  if (b == e) return;
  int lane = threadIdx.x;
  double accum[NSLOT];
#pragma unroll
  for (int t = 0; t < NSLOT; t++) accum[t] = 0.0;
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
    double cam[P + 1], sam[P + 1], cbm[P + 1], sbm[P + 1];
    cam[0] = 1.0;
    sam[0] = 0.0;
    cbm[0] = 1.0;
    sbm[0] = 0.0;
#pragma unroll
    for (int m = 1; m <= P; m++) {
      cam[m] = fma(cam[m - 1], ca, -sam[m - 1] * sa);
      sam[m] = fma(sam[m - 1], ca, cam[m - 1] * sa);
      cbm[m] = fma(cbm[m - 1], cb, -sbm[m - 1] * sb);
      sbm[m] = fma(sbm[m - 1], cb, cbm[m - 1] * sb);
    }
    // translation factors g_j = j! / r^{j+1}
    double g[P + 1];
    {
      double rp = rinv;
#pragma unroll
      for (int j = 0; j <= P; j++) {
        g[j] = cfact(j) * rp;
        rp *= rinv;
      }
    }
    // forward rotation of the source moments, order by order
    double Mp[NR];
    const double* M = mult + (size_t)A * NC * 2;
    static_for<0, P + 1>([&](auto nc) {
      constexpr int n = nc;
      double* v = Mp + n * n;
      v[0] = M[2 * cidx(n, 0)];
      static_for<1, n + 1>([&](auto mc) {
        constexpr int m = mc;
        v[2 * m - 1] = M[2 * cidx(n, m)];
        v[2 * m] = M[2 * cidx(n, m) + 1];
      });
      zrot<n>(v, cam, sam, 1.0);
      swap_apply<n>(v);
      zrot<n>(v, cbm, sbm, 1.0);
      swap_apply<n>(v);
    });
    // translate along z, rotate back and reduce, one output order at a time
    static_for<0, P + 1>([&](auto nc) {
      constexpr int n = nc;
      double w[2 * n + 1];
      static_for<0, n + 1>([&](auto mc) {
        constexpr int m = mc;
        if constexpr (m <= P - n) {
          double sC = 0.0, sS = 0.0;
          static_for<m, P - n + 1>([&](auto kc) {
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
      zrot<n>(w, cbm, sbm, -1.0);
      swap_apply<n>(w);
      zrot<n>(w, cam, sam, -1.0);
      static_for<0, 2 * n + 1>([&](auto jc) {
        constexpr int j = jc;
        constexpr int idx = n * n + j;
        double tot = wave_sum(act ? w[j] : 0.0);
        if (lane == (idx & 63)) accum[idx >> 6] += tot;
      });
    });
  }
  // back to the unscaled basis: L_n^m = (n-m)!(n+m)! Lhat_n^m
  double* out = loc + (size_t)B * NC * 2;
  static_for<0, P + 1>([&](auto nc) {
    constexpr int n = nc;
    static_for<0, 2 * n + 1>([&](auto jc) {
      constexpr int j = jc;
      constexpr int idx = n * n + j;
      constexpr int m = rb_m(j);
      constexpr double f = cfact(n - m) * cfact(n + m);
      if (lane == (idx & 63)) {
        double v = accum[idx >> 6] * f;
        if constexpr (j == 0) {
          out[2 * cidx(n, 0)] = v;
          out[2 * cidx(n, 0) + 1] = 0.0;
        } else if constexpr (rb_re(j)) {
          out[2 * cidx(n, m)] = v;
        } else {
          out[2 * cidx(n, m) + 1] = v;
        }
      }
    });
  });
}

template <int P>
static void launch_p(Ctx& c) {
  int nc = (int)c.ncell;
  unsigned grid = 8u * (unsigned)((nc + 7) / 8);
  hipLaunchKernelGGL(k_m2l_fp64<P>, dim3(grid), dim3(64), 0, c.stream, nc, c.m2l.off.p, c.m2l.src.p,
                     c.c_cx.p, c.c_cy.p, c.c_cz.p, c.mult.p, c.loc.p);
}

template <int P>
static bool dispatch(Ctx& c) {
  if constexpr (P > FMM_GPU_PMAX) {
    return false;
  } else {
    if (c.p == P) {
      launch_p<P>(c);
      return true;
    }
    return dispatch<P + 1>(c);
  }
}

void launch_m2l_fp64(Ctx& c) {
  if (!g_m2l_tables) {
    HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_swap), fmm_swap_table, sizeof(double) * SWAP_DOUBLES));
    g_m2l_tables = true;
  }
  if (!dispatch<1>(c)) throw hip_error{hipErrorInvalidValue, "M2L order not compiled"};
  HIPCHK(hipGetLastError());
}

}  // namespace fmm
