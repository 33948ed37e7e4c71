// Rotation-accelerated M2L for any order up to 30 (section 2.4), FP64.
//
// The same operator as k_m2l_fp64 (m2l.hip): for a directed pair A -> B the
// source moments are rotated about z by alpha = pi/2 - phi, their x and z
// swapped, rotated about z by -theta and swapped again, so that R = z_B - z_A
// lies along +z; translated along z, where only T_j^0(r z) = j!/r^{j+1} is
// non-zero; then rotated back with the transposed sequence in the scaled basis
// Lhat_n^m = L_n^m / ((n-m)!(n+m)!).  Real basis per order n: index 0 = Re c^0,
// 2m-1 = Re c^m, 2m = Im c^m; W_n couples Re^m with Re^m' only when
// m + m' + n is even (Im parts: odd), and those zeros are never stored.
//
// The register-resident kernel holds a whole expansion per lane, which stops
// fitting beyond p = 16 (441 values at p = 20, 961 at p = 30).  Here the
// order is a run-time value and the wavefront works on one pair at a time:
// the 64 lanes share the (p+1)^2 real coefficients of the rotated moments,
// which live in LDS between the steps (every swap mixes the coefficients of
// one order), and each lane keeps a fixed slice of the sink's local
// expansion in registers.  One wavefront per workgroup and per sink, so the
// steps are separated by workgroup barriers of a single wave.
#include <hip/hip_runtime.h>

#include <vector>

#include "fmm_device.h"
#include "fmm_tables.h"

namespace fmm {

namespace hi {

constexpr int PMAX = FMM_TABLE_PMAX;  // orders with swap tables (section 2.4: p <= 30)
constexpr int SMAX = (PMAX + 1) * (PMAX + 1);
constexpr int TMAX = (SMAX + 63) / 64;  // local-expansion entries per lane

constexpr int rb_m(int j) { return (j + 1) >> 1; }
constexpr bool rb_re(int j) { return j == 0 || (j & 1); }
constexpr bool swap_nz(int n, int i, int j) {
  return rb_re(i) == rb_re(j) && (((rb_m(i) + rb_m(j) + n) & 1) == (rb_re(i) ? 0 : 1));
}
constexpr int nnz_upto(int p) {  // structural non-zeros of W_0 .. W_p
  int c = 0;
  for (int n = 0; n <= p; n++)
    for (int i = 0; i < 2 * n + 1; i++)
      for (int j = 0; j < 2 * n + 1; j++) c += swap_nz(n, i, j) ? 1 : 0;
  return c;
}
constexpr int CSW = nnz_upto(PMAX);

}  // namespace hi

// compacted W_n (n <= 30), row by row, columns ascending; offset of row i of
// order n at [n^2 + i]
static __device__ double g_cswap_hi[hi::CSW];
static __device__ int g_rowoff_hi[hi::SMAX];
static __constant__ double c_fact_hi[2 * hi::PMAX + 2];
static bool g_hi_tables[64] = {};  // per device

// Row i of order n: the first structurally non-zero column's order m0 and the
// number of non-zeros; the columns are orders m0, m0 + 2, ... of the same part
// (Re: column index 0 for m = 0, 2m - 1 otherwise; Im: 2m).
__device__ __forceinline__ void hi_row(int n, int i, int& m0, int& cnt, bool& re) {
  re = i == 0 || (i & 1);
  int mi = (i + 1) >> 1;
  if (re) {
    m0 = (n + mi) & 1;
  } else {
    m0 = ((n + mi + 1) & 1) ? 1 : 2;
  }
  cnt = m0 <= n ? (n - m0) / 2 + 1 : 0;
}

// out[n^2 + i] = sum_j W_n[i][j] v[n^2 + j] for every row of orders 0..p
__device__ __forceinline__ void hi_swap(int S, const double* __restrict__ v, double* __restrict__ out, int lane) {
  for (int u = lane; u < S; u += 64) {
    int n = (int)sqrtf((float)u);
    while (n * n > u) n--;
    while ((n + 1) * (n + 1) <= u) n++;
    int i = u - n * n;
    int m0, cnt;
    bool re;
    hi_row(n, i, m0, cnt, re);
    const double* w = g_cswap_hi + g_rowoff_hi[u];
    const double* vn = v + n * n;
    double s = 0.0;
    for (int t = 0; t < cnt; t++) {
      int m = m0 + 2 * t;
      int j = re ? (m == 0 ? 0 : 2 * m - 1) : 2 * m;
      s = fma(w[t], vn[j], s);
    }
    out[u] = s;
  }
}

// rotation about z of every order: (C, S)_m <- (C cos ma - S sin ma, C sin ma + S cos ma)
// with (cos ma, sin ma) from the table cs[m]; sgn = -1 rotates by -a
__device__ __forceinline__ void hi_zrot(int S, double* v, const double2* cs, double sgn, int lane) {
  for (int u = lane; u < S; u += 64) {
    int n = (int)sqrtf((float)u);
    while (n * n > u) n--;
    while ((n + 1) * (n + 1) <= u) n++;
    int j = u - n * n;
    if (j & 1) {  // Re c^m at j = 2m - 1, Im c^m next to it
      int m = (j + 1) >> 1;
      double cm = cs[m].x, sm = sgn * cs[m].y;
      double C = v[u], Sv = v[u + 1];
      v[u] = fma(C, cm, -Sv * sm);
      v[u + 1] = fma(C, sm, Sv * cm);
    }
  }
}

// M2L of the list of sink B; with B >= first_lo only the sources below
// first_lo are taken (the FP64 part of mixed precision)
template <bool LIST>
__global__ void __launch_bounds__(64) k_m2l_hi(int p, int ncell, int first_lo, const int* __restrict__ sinks,
                                               const int* __restrict__ nsinks, const int* __restrict__ off,
                                               const int* __restrict__ src, const double* __restrict__ cx,
                                               const double* __restrict__ cy, const double* __restrict__ cz,
                                               const double* __restrict__ mult, double* __restrict__ loc) {
  extern __shared__ double lds[];
  const int S = (p + 1) * (p + 1), NC = ncoef(p);
  double* V = lds;
  double* U = lds + S;
  double2* ca_t = (double2*)(lds + 2 * S);  // (cos m alpha, sin m alpha), m = 0..p
  double2* cb_t = ca_t + (p + 1);           // (cos m theta', sin m theta') of -theta
  double* g = (double*)(cb_t + (p + 1));    // g_j = j! / r^{j+1}, j = 0..p
  const int lane = threadIdx.x;
  int count = LIST ? *nsinks : ncell;
  for (int it = blockIdx.x; it < count; it += gridDim.x) {
    int B = LIST ? sinks[it] : it;
    int b = off[B], e = off[B + 1];
    if (B >= first_lo) {
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
    double* out = loc + (size_t)B * NC * 2;
    if (b == e) {
      for (int k = lane; k < NC * 2; k += 64) out[k] = 0.0;
      continue;
    }
    double acc[hi::TMAX];
#pragma unroll
    for (int t = 0; t < hi::TMAX; t++) acc[t] = 0.0;
    double bx = cx[B], by = cy[B], bz = cz[B];
    for (int k = b; k < e; k++) {
      int A = src[k];
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
      // angle tables by the angle-addition recurrence, one lane per order m
      // (lanes 0..p for alpha, 32..32+p for -theta), and the translation
      // factors (lanes 0..p)
      {
        int m = lane & 31;
        if (m <= p) {
          double c1 = lane < 32 ? ca : cb, s1 = lane < 32 ? sa : sb;
          double cm = 1.0, sm = 0.0;
          for (int q = 1; q <= m; q++) {
            double c2 = fma(cm, c1, -sm * s1);
            sm = fma(sm, c1, cm * s1);
            cm = c2;
          }
          (lane < 32 ? ca_t : cb_t)[m] = make_double2(cm, sm);
          if (lane < 32) {
            double rp = rinv;
            for (int q = 0; q < m; q++) rp *= rinv;
            g[m] = c_fact_hi[m] * rp;
          }
        }
      }
      // source moments in the real basis
      const double* M = mult + (size_t)A * NC * 2;
      for (int u = lane; u < S; u += 64) {
        int n = (int)sqrtf((float)u);
        while (n * n > u) n--;
        while ((n + 1) * (n + 1) <= u) n++;
        int j = u - n * n, m = (j + 1) >> 1;
        bool im = j > 0 && !(j & 1);
        V[u] = M[2 * cidx(n, m) + (im ? 1 : 0)];
      }
      __syncthreads();
      hi_zrot(S, V, ca_t, 1.0, lane);
      __syncthreads();
      hi_swap(S, V, U, lane);
      __syncthreads();
      hi_zrot(S, U, cb_t, 1.0, lane);
      __syncthreads();
      hi_swap(S, U, V, lane);
      __syncthreads();
      // translation along z in the scaled basis:
      // Lhat_n^m = (-1)^{n+m} / ((n-m)!(n+m)!) sum_{k=m}^{p-n} M'_k^m g_{n+k}
      for (int u = lane; u < S; u += 64) {
        int n = (int)sqrtf((float)u);
        while (n * n > u) n--;
        while ((n + 1) * (n + 1) <= u) n++;
        int j = u - n * n, m = (j + 1) >> 1;
        double s = 0.0;
        if (m <= p - n) {
          for (int kk = m; kk <= p - n; kk++) s = fma(V[kk * kk + j], g[n + kk], s);
          double f = (((n + m) & 1) ? -1.0 : 1.0) / (c_fact_hi[n - m] * c_fact_hi[n + m]);
          s = s * f;
        }
        U[u] = s;
      }
      __syncthreads();
      hi_swap(S, U, V, lane);
      __syncthreads();
      hi_zrot(S, V, cb_t, -1.0, lane);
      __syncthreads();
      hi_swap(S, V, U, lane);
      __syncthreads();
      hi_zrot(S, U, ca_t, -1.0, lane);
      __syncthreads();
#pragma unroll
      for (int t = 0; t < hi::TMAX; t++) {
        int u = lane + 64 * t;
        if (u < S) acc[t] += U[u];
      }
      __syncthreads();  // U and the tables are rewritten by the next pair
    }
    // back to the unscaled basis: L_n^m = (n-m)!(n+m)! Lhat_n^m
#pragma unroll
    for (int t = 0; t < hi::TMAX; t++) {
      int u = lane + 64 * t;
      if (u < S) {
        int n = (int)sqrtf((float)u);
        while (n * n > u) n--;
        while ((n + 1) * (n + 1) <= u) n++;
        int j = u - n * n, m = (j + 1) >> 1;
        bool im = j > 0 && !(j & 1);
        out[2 * cidx(n, m) + (im ? 1 : 0)] = acc[t] * (c_fact_hi[n - m] * c_fact_hi[n + m]);
        if (j == 0) out[2 * cidx(n, 0) + 1] = 0.0;
      }
    }
  }
}

void upload_hi_tables() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (g_hi_tables[dev & 63]) return;
  std::vector<double> cs;
  std::vector<int> ro(hi::SMAX, 0);
  cs.reserve(hi::CSW);
  for (int n = 0; n <= hi::PMAX; n++) {
    int D = 2 * n + 1, sw = n * (4 * n * n - 1) / 3;  // dense table offset of order n
    for (int i = 0; i < D; i++) {
      ro[n * n + i] = (int)cs.size();
      for (int j = 0; j < D; j++)
        if (hi::swap_nz(n, i, j)) cs.push_back(fmm_swap_table[sw + i * D + j]);
    }
  }
  if ((int)cs.size() != hi::CSW) throw hip_error{hipErrorInvalidValue, "compacted swap table size"};
  HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(g_cswap_hi), cs.data(), sizeof(double) * cs.size()));
  HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(g_rowoff_hi), ro.data(), sizeof(int) * ro.size()));
  HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_fact_hi), fmm_fact_table, sizeof(double) * (2 * hi::PMAX + 2)));
  g_hi_tables[dev & 63] = true;
}

size_t m2l_hi_lds_bytes(int p) {
  size_t S = (size_t)(p + 1) * (p + 1);
  return sizeof(double) * (2 * S + 5 * (size_t)(p + 1));
}

// any order up to 30; sinks == nullptr: every sink cell, else the listed ones
void launch_m2l_hi(Ctx& c, int first_lo, const double* mult, double* loc, const int* sinks,
                   const int* nsinks) {
  if (c.p > hi::PMAX) throw unsupported_error{"expansion order above 30"};
  upload_hi_tables();
  int nc = (int)c.ncell;
  size_t lds = m2l_hi_lds_bytes(c.p);
  if (sinks) {
    hipLaunchKernelGGL((k_m2l_hi<true>), dim3(2048), dim3(64), lds, c.stream, c.p, nc, first_lo, sinks, nsinks,
                       c.m2l.off.p, c.m2l.src.p, c.c_cx.p, c.c_cy.p, c.c_cz.p, mult, loc);
  } else {
    hipLaunchKernelGGL((k_m2l_hi<false>), dim3((unsigned)std::max(nc, 1)), dim3(64), lds, c.stream, c.p, nc,
                       first_lo, (const int*)nullptr, (const int*)nullptr, c.m2l.off.p, c.m2l.src.p, c.c_cx.p,
                       c.c_cy.p, c.c_cz.p, mult, loc);
  }
  HIPCHK(hipGetLastError());
}

}  // namespace fmm
