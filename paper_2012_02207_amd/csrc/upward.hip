// Upward pass on gfx950: P2M at the leaves, M2M towards the root and the
// per-order norms P_k of every cell's multipole.
//
// P2M: M_n^m = sum_i m_i Y_n^m(x_i - z) over the cell's bodies (section 2.2,
// multipole-moment equation).  M2M shifts each child's moments to the parent
// centre with the regular addition theorem (section 2.1).  P_k^2 =
// sum_{m=-k..k} (k-m)!(k+m)! |M_k^m|^2 (section 2.3).  These values enter the
// acceptance test, so every sum runs sequentially in a fixed order with
// separately rounded products: bodies in sorted order, children in octant
// order, terms in (k, l) order.  A wavefront owns one cell: lanes evaluate the
// harmonics of different bodies (or children) into LDS, then lanes owning
// different coefficients accumulate over the bodies in order.
#include <hip/hip_runtime.h>

#include "fmm_device.h"
#include "fmm_tables.h"

namespace fmm {

static __constant__ double c_fact[2 * FMM_TABLE_PMAX + 2];
static __constant__ double c_binom[FMM_TABLE_PMAX + 1][FMM_TABLE_PMAX + 1];
static bool g_up_tables = false;

// LDS budget per P2M workgroup (dynamic, sized from p so that several
// workgroups share a CU)
constexpr int P2M_LDS_DOUBLES = 2560;  // 20 KB

// bodies handled per LDS batch so that 2 * ncoef * batch doubles fit
__host__ __device__ inline int p2m_batch(int p) {
  int nc = ncoef(p), b = 64;
  while (b > 1 && 2 * nc * b > P2M_LDS_DOUBLES) b >>= 1;
  return b;
}

constexpr int M2M_T = 128;  // threads per M2M workgroup: one per coefficient (p <= 14)

__global__ void __launch_bounds__(64) k_p2m(int p, const int* leaves, int nleaves, const int* cb,
                                            const int* ce, const double* sx, const double* sy,
                                            const double* sz, const double* sm, const double* cx,
                                            const double* cy, const double* cz, double* mult) {
  extern __shared__ double lds[];
  int li = blockIdx.x;
  if (li >= nleaves) return;
  int c = leaves[li];
  int nc = ncoef(p);
  int batch = p2m_batch(p);
  double* yre = lds;
  double* yim = lds + nc * batch;
  int lane = threadIdx.x;
  double x0 = cx[c], y0 = cy[c], z0 = cz[c];
  int b = cb[c], e = ce[c];
  // each lane keeps the running sums of coefficients lane, lane+64, ...
  constexpr int MAXK = (ncoef(FMM_TABLE_PMAX) + 63) / 64;
  double acr[MAXK], aci[MAXK];
  for (int t = 0; t < MAXK; t++) acr[t] = aci[t] = 0.0;
  for (int i0 = b; i0 < e; i0 += batch) {
    int cnt = min(batch, e - i0);
    if (lane < cnt) {
      int i = i0 + lane;
      regular_exact(p, sx[i] - x0, sy[i] - y0, sz[i] - z0, yre + lane, yim + lane, batch);
    }
    __syncthreads();
    for (int t = 0; t < MAXK; t++) {
      int k = lane + 64 * t;
      if (k < nc) {
        double sr = acr[t], si = aci[t];
        for (int j = 0; j < cnt; j++) {
          double m = sm[i0 + j];
          double tr = m * yre[k * batch + j];
          double ti = m * yim[k * batch + j];
          sr = sr + tr;
          si = si + ti;
        }
        acr[t] = sr;
        aci[t] = si;
      }
    }
    __syncthreads();
  }
  double* out = mult + (size_t)c * nc * 2;
  for (int t = 0; t < MAXK; t++) {
    int k = lane + 64 * t;
    if (k < nc) {
      out[2 * k] = acr[t];
      out[2 * k + 1] = aci[t];
    }
  }
}

__global__ void __launch_bounds__(M2M_T) k_m2m(int p, int first, int count, const int* c0,
                                                const int* nch, const double* cx, const double* cy,
                                                const double* cz, double* mult) {
  extern __shared__ double lds[];
  int c = first + blockIdx.x;
  if (blockIdx.x >= count || nch[c] == 0) return;
  int nc = ncoef(p);
  int k0 = c0[c], kn = nch[c];
  double* yre = lds;             // child j at stride 8
  double* yim = lds + nc * 8;
  double* mch = lds + 2 * nc * 8;  // children's moments, contiguous ids -> contiguous rows
  int lane = threadIdx.x;
  if (lane < kn) {
    int ch = k0 + lane;
    regular_exact(p, cx[ch] - cx[c], cy[ch] - cy[c], cz[ch] - cz[c], yre + lane, yim + lane, 8);
  }
  const double* src = mult + (size_t)k0 * nc * 2;
  for (int t = lane; t < kn * nc * 2; t += M2M_T) mch[t] = src[t];
  __syncthreads();
  double* out = mult + (size_t)c * nc * 2;
  for (int t = lane; t < nc; t += M2M_T) {
    // coefficient index t -> (n, m)
    int n = 0;
    while (cidx(n + 1, 0) <= t) n++;
    int m = t - cidx(n, 0);
    double sr = 0.0, si = 0.0;
    for (int j = 0; j < kn; j++) {
      const double* cm = mch + j * nc * 2;
      for (int k = 0; k <= n; k++) {
        int jj = n - k;
        // l ranges over |l| <= k with |m - l| <= jj
        int lo = max(-k, m - jj), hi = min(k, m + jj);
        for (int l = lo; l <= hi; l++) {
          int q = m - l;
          double ar, ai;
          cget(yre + j, yim + j, 8, k, l, ar, ai);
          double br, bi;
          if (q >= 0) {
            br = cm[2 * cidx(jj, q)];
            bi = cm[2 * cidx(jj, q) + 1];
          } else {
            double s = (q & 1) ? -1.0 : 1.0;
            br = s * cm[2 * cidx(jj, -q)];
            bi = -s * cm[2 * cidx(jj, -q) + 1];
          }
          double tr = ar * br - ai * bi;
          double ti = ar * bi + ai * br;
          sr = sr + tr;
          si = si + ti;
        }
      }
    }
    out[2 * t] = sr;
    out[2 * t + 1] = si;
  }
}

// P_k = sqrt( (k!)^2 |M_k^0|^2 + sum_{m=1..k} 2 (k-m)!(k+m)! |M_k^m|^2 ), and the
// product C(p, k) P_k used by the acceptance test
__global__ void k_pk(int p, int ncell, const double* mult, double* pk, double* pkb) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)ncell * (p + 1)) return;
  int c = (int)(t / (p + 1)), k = (int)(t % (p + 1));
  const double* M = mult + (size_t)c * ncoef(p) * 2;
  double acc = 0.0;
  for (int m = 0; m <= k; m++) {
    double re = M[2 * cidx(k, m)], im = M[2 * cidx(k, m) + 1];
    double w = (m == 0) ? (c_fact[k] * c_fact[k]) : (2.0 * (c_fact[k - m] * c_fact[k + m]));
    acc = acc + w * (re * re + im * im);
  }
  double P = sqrt(acc);
  pk[t] = P;
  pkb[t] = c_binom[p][k] * P;
}

__global__ void k_list_leaves(const int* nch, int ncell, int* flag) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncell) flag[c] = nch[c] == 0 ? 1 : 0;
}

__global__ void k_compact_leaves(const int* flag, const int* off, int ncell, int* leaves) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncell && flag[c]) leaves[off[c]] = c;
}

void upward_pass(Ctx& c) {
  if (!g_up_tables) {
    HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_fact), fmm_fact_table, sizeof(fmm_fact_table)));
    HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_binom), fmm_binom_table, sizeof(fmm_binom_table)));
    g_up_tables = true;
  }
  hipStream_t s = c.stream;
  int p = c.p, nc = (int)c.ncell;
  ensure(c.ws, c.mult, (size_t)nc * ncoef(p) * 2);
  ensure(c.ws, c.pk, (size_t)nc * (p + 1));
  // leaf list
  ensure(c.ws, c.c_split, (size_t)2 * nc + 64);
  ensure(c.ws, c.leaves, (size_t)nc);
  int* flag = c.c_split.p;
  int* off = flag + nc + 32;
  int* leaves = c.leaves.p;
  long long* tot = (long long*)c.counters.p;
  hipLaunchKernelGGL(k_list_leaves, dim3((nc + 255) / 256), dim3(256), 0, s, c.c_nchild.p, nc, flag);
  exclusive_scan(c, flag, off, nc, tot);
  hipLaunchKernelGGL(k_compact_leaves, dim3((nc + 255) / 256), dim3(256), 0, s, flag, off, nc, leaves);
  c.nleaf = read_total(c, tot);
  size_t p2m_lds = sizeof(double) * 2 * ncoef(p) * p2m_batch(p);
  hipLaunchKernelGGL(k_p2m, dim3((unsigned)c.nleaf), dim3(64), p2m_lds, s, p, leaves, (int)c.nleaf,
                     c.c_begin.p, c.c_end.p, c.sx.p, c.sy.p, c.sz.p, c.sm.p, c.c_cx.p, c.c_cy.p,
                     c.c_cz.p, c.mult.p);
  HIPCHK(hipGetLastError());
  for (int level = c.depth - 1; level >= 0; level--) {
    int first = c.lvl_first[level], count = c.lvl_count[level];
    size_t m2m_lds = sizeof(double) * 32 * ncoef(p);  // harmonics of 8 children + their moments
    hipLaunchKernelGGL(k_m2m, dim3(count), dim3(M2M_T), m2m_lds, s, p, first, count, c.c_child0.p,
                       c.c_nchild.p, c.c_cx.p, c.c_cy.p, c.c_cz.p, c.mult.p);
    HIPCHK(hipGetLastError());
  }
  int64_t npk = (int64_t)nc * (p + 1);
  ensure(c.ws, c.pkb, (size_t)npk);
  hipLaunchKernelGGL(k_pk, dim3((unsigned)ceil_div(npk, 256)), dim3(256), 0, s, p, nc, c.mult.p, c.pk.p,
                     c.pkb.p);
  HIPCHK(hipGetLastError());
}

}  // namespace fmm
