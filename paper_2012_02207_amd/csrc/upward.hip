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
static bool g_up_tables[64] = {};  // per device

// Column m of the regular harmonics of (x, y, z) in the exact rounding
// sequence of the full recurrence (the same arithmetic as regular_exact): the
// diagonal Y_1^1 .. Y_m^m, then Y_n^m for n = m+1..p.  Lanes evaluate
// different columns (and bodies) in parallel.
template <class Store>
__device__ inline void regular_column_exact(int p, int m, double x, double y, double z, Store store) {
  double r2 = (x * x + y * y) + z * z;
  double pr = 1.0, pi = 0.0;
  for (int n = 1; n <= m; n++) {
    double tr = x * pr - y * pi;
    double ti = x * pi + y * pr;
    double den = (double)(2 * n);
    pr = (-tr) / den;
    pi = (-ti) / den;
  }
  store(m, pr, pi);
  double ar2 = 0.0, ai2 = 0.0, ar1 = pr, ai1 = pi;
  for (int n = m + 1; n <= p; n++) {
    double k = (double)(2 * n - 1) * z;
    double nr = k * ar1, ni = k * ai1;
    if (n - 2 >= m) {
      double br = r2 * ar2, bi = r2 * ai2;
      nr = nr - br;
      ni = ni - bi;
    }
    double den = (double)((n + m) * (n - m));
    double vr = nr / den, vi = ni / den;
    store(n, vr, vi);
    ar2 = ar1;
    ai2 = ai1;
    ar1 = vr;
    ai1 = vi;
  }
}

// (n, m) of coefficient index t
__device__ __forceinline__ void coef_nm(int t, int& n, int& m) {
  n = 0;
  while (cidx(n + 1, 0) <= t) n++;
  m = t - cidx(n, 0);
}

// P2M: one workgroup per leaf; bodies in batches of P2M_T / (p+1), lane
// (body, column) evaluates one harmonic column into LDS, then lanes owning
// coefficients accumulate over the batch in sorted body order.
constexpr int P2M_T = 256;

__host__ __device__ inline int p2m_batch(int p) { return P2M_T / (p + 1); }

__global__ void __launch_bounds__(P2M_T) k_p2m(int p, const int* leaves, int nleaves, const int* cb,
                                               const int* ce, const double* sx, const double* sy,
                                               const double* sz, const double* sm, const double* cx,
                                               const double* cy, const double* cz, double* mult) {
  extern __shared__ double lds[];
  int li = blockIdx.x;
  if (li >= nleaves) return;
  int c = leaves[li];
  int nc = ncoef(p);
  int batch = p2m_batch(p);
  double* yre = lds;  // [coef][body], stride batch
  double* yim = lds + nc * batch;
  double* msh = lds + 2 * nc * batch;  // masses of the batch
  int t = threadIdx.x;
  double x0 = cx[c], y0 = cy[c], z0 = cz[c];
  int b = cb[c], e = ce[c];
  constexpr int MAXK = (ncoef(FMM_TABLE_PMAX) + P2M_T - 1) / P2M_T;
  double acr[MAXK], aci[MAXK];
  for (int u = 0; u < MAXK; u++) acr[u] = aci[u] = 0.0;
  int hb = t / (p + 1), hm = t - hb * (p + 1);  // harmonic lane: body hb, column hm
  for (int i0 = b; i0 < e; i0 += batch) {
    int cnt = min(batch, e - i0);
    if (hb < cnt) {
      int i = i0 + hb;
      if (hm == 0) msh[hb] = sm[i];
      regular_column_exact(p, hm, sx[i] - x0, sy[i] - y0, sz[i] - z0, [&](int n, double vr, double vi) {
        yre[cidx(n, hm) * batch + hb] = vr;
        yim[cidx(n, hm) * batch + hb] = vi;
      });
    }
    __syncthreads();
    for (int u = 0; u < MAXK; u++) {
      int k = t + P2M_T * u;
      if (k < nc) {
        double sr = acr[u], si = aci[u];
#pragma unroll 4
        for (int j = 0; j < cnt; j++) {
          double m = msh[j];
          double tr = m * yre[k * batch + j];
          double ti = m * yim[k * batch + j];
          sr = sr + tr;
          si = si + ti;
        }
        acr[u] = sr;
        aci[u] = si;
      }
    }
    __syncthreads();
  }
  double* out = mult + (size_t)c * nc * 2;
  for (int u = 0; u < MAXK; u++) {
    int k = t + P2M_T * u;
    if (k < nc) {
      out[2 * k] = acr[u];
      out[2 * k + 1] = aci[u];
    }
  }
}

// M2M, one workgroup per parent.  The children's harmonics Y_k^l(z_c - z_P)
// and moments M_j^q are laid out in LDS for both signs of their order
// (entry n(n+1) + m, m = -n..n, the negative orders from the stored ones by
// the conjugate symmetry, exact), so that every sum is a branch-free loop in
// the defining order.  Each (child, coefficient) pair is a task: the child's
// shifted moment summed over k, then l ascending, products rounded
// separately; the parent's coefficient then adds its children's sums in
// octant order.  A sum is at most p + 1 terms of one child long, not eight
// children long, so the few parents of the top levels finish quickly.
constexpr int M2M_T = 128;
constexpr int M2M_ALL_CHILDREN_PMAX = 16;  // the eight-children layout up to this order
constexpr int M2M_TASKS = (8 * ncoef(M2M_ALL_CHILDREN_PMAX) + M2M_T - 1) / M2M_T;

__global__ void __launch_bounds__(M2M_T) k_m2m(int p, int first, int count, const int* c0,
                                                const int* nch, const double* cx, const double* cy,
                                                const double* cz, double* mult) {
  extern __shared__ double lds[];
  int c = first + blockIdx.x;
  if (blockIdx.x >= count || nch[c] == 0) return;
  int nc = ncoef(p);
  int S = (p + 1) * (p + 1);
  int k0 = c0[c], kn = nch[c];
  double2* Yx = (double2*)lds;  // [child][S]
  double2* Mx = Yx + 8 * S;     // [child][S]
  int t = threadIdx.x;
  for (int u = t; u < kn * (p + 1); u += M2M_T) {  // harmonics, both signs of l
    int j = u / (p + 1), m = u - j * (p + 1);
    int ch = k0 + j;
    double2* Y = Yx + j * S;
    double sg = (m & 1) ? -1.0 : 1.0;
    regular_column_exact(p, m, cx[ch] - cx[c], cy[ch] - cy[c], cz[ch] - cz[c],
                         [&](int n, double vr, double vi) {
                           Y[n * n + n + m] = make_double2(vr, vi);
                           if (m > 0) Y[n * n + n - m] = make_double2(sg * vr, -sg * vi);
                         });
  }
  const double* src = mult + (size_t)k0 * nc * 2;
  for (int u = t; u < kn * S; u += M2M_T) {  // moments, both signs of q
    int j = u / S, r = u - j * S;
    int n = 0;
    while ((n + 1) * (n + 1) <= r) n++;
    int q = r - n * n - n;
    const double* cm = src + (size_t)j * nc * 2;
    int aq = q < 0 ? -q : q;
    double a = cm[2 * cidx(n, aq)], bb = cm[2 * cidx(n, aq) + 1];
    if (q < 0) {
      double sg = (aq & 1) ? -1.0 : 1.0;
      a = sg * a;
      bb = -sg * bb;
    }
    Mx[u] = make_double2(a, bb);
  }
  __syncthreads();
  // per-child sums, held in registers until every task has read the tables
  double pr[M2M_TASKS], pi[M2M_TASKS];
#pragma unroll
  for (int w = 0; w < M2M_TASKS; w++) {
    pr[w] = pi[w] = 0.0;
    int u = t + M2M_T * w;
    if (u < kn * nc) {
      int j = u / nc, q = u - j * nc;
      int n, m;
      coef_nm(q, n, m);
      const double2* Y = Yx + j * S;
      const double2* M = Mx + j * S;
      double sr = 0.0, si = 0.0;
      for (int k = 0; k <= n; k++) {
        int jj = n - k;
        int lo = max(-k, m - jj), hi = min(k, m + jj);
        const double2* Yk = Y + k * k + k + lo;
        const double2* Mj = M + jj * jj + jj + m - lo;
        int cnt = hi - lo + 1;
#pragma unroll 4
        for (int r = 0; r < cnt; r++) {  // l = lo + r
          double2 a = Yk[r], bq = Mj[-r];
          double tr = a.x * bq.x - a.y * bq.y;
          double ti = a.x * bq.y + a.y * bq.x;
          sr = sr + tr;
          si = si + ti;
        }
      }
      pr[w] = sr;
      pi[w] = si;
    }
  }
  __syncthreads();
  double2* part = Yx;  // [child][coefficient], over the harmonics
#pragma unroll
  for (int w = 0; w < M2M_TASKS; w++) {
    int u = t + M2M_T * w;
    if (u < kn * nc) part[u] = make_double2(pr[w], pi[w]);
  }
  __syncthreads();
  double* out = mult + (size_t)c * nc * 2;
  for (int q = t; q < nc; q += M2M_T) {
    double sr = 0.0, si = 0.0;
    for (int j = 0; j < kn; j++) {
      double2 v = part[j * nc + q];
      sr = sr + v.x;
      si = si + v.y;
    }
    out[2 * q] = sr;
    out[2 * q + 1] = si;
  }
}

size_t m2m_lds_bytes(int p) { return sizeof(double2) * 2 * 8 * (size_t)(p + 1) * (p + 1); }

// The same M2M with one child at a time in LDS (harmonics and moments of that
// child only), for the orders whose eight children do not fit: each lane sums
// a child's shifted moment (k, then l) and adds it to its running coefficient
// child by child in octant order, so it rounds exactly as k_m2m.
constexpr int M2M_SMAXK = (ncoef(FMM_TABLE_PMAX) + M2M_T - 1) / M2M_T;

__global__ void __launch_bounds__(M2M_T) k_m2m_stream(int p, int first, int count, const int* c0,
                                                       const int* nch, const double* cx, const double* cy,
                                                       const double* cz, double* mult) {
  extern __shared__ double lds[];
  int c = first + blockIdx.x;
  if (blockIdx.x >= count || nch[c] == 0) return;
  int nc = ncoef(p);
  int S = (p + 1) * (p + 1);
  int k0 = c0[c], kn = nch[c];
  double2* Y = (double2*)lds;  // [S] harmonics of the current child
  double2* Mx = Y + S;         // [S] its moments, both signs of q
  int t = threadIdx.x;
  double sr[M2M_SMAXK], si[M2M_SMAXK];
  for (int q = 0; q < M2M_SMAXK; q++) sr[q] = si[q] = 0.0;
  for (int j = 0; j < kn; j++) {
    int ch = k0 + j;
    for (int m = t; m <= p; m += M2M_T) {
      double sg = (m & 1) ? -1.0 : 1.0;
      regular_column_exact(p, m, cx[ch] - cx[c], cy[ch] - cy[c], cz[ch] - cz[c],
                           [&](int n, double vr, double vi) {
                             Y[n * n + n + m] = make_double2(vr, vi);
                             if (m > 0) Y[n * n + n - m] = make_double2(sg * vr, -sg * vi);
                           });
    }
    const double* cm = mult + (size_t)ch * nc * 2;
    for (int r = t; r < S; r += M2M_T) {
      int n = 0;
      while ((n + 1) * (n + 1) <= r) n++;
      int q = r - n * n - n;
      int aq = q < 0 ? -q : q;
      double a = cm[2 * cidx(n, aq)], bb = cm[2 * cidx(n, aq) + 1];
      if (q < 0) {
        double sg = (aq & 1) ? -1.0 : 1.0;
        a = sg * a;
        bb = -sg * bb;
      }
      Mx[r] = make_double2(a, bb);
    }
    __syncthreads();
    for (int q = 0; q < M2M_SMAXK; q++) {
      int u = t + M2M_T * q;
      if (u >= nc) break;
      int n, m;
      coef_nm(u, n, m);
      double ar = 0.0, ai = 0.0;  // this child's sum, added to the parent's below
      for (int k = 0; k <= n; k++) {
        int jj = n - k;
        int lo = max(-k, m - jj), hi = min(k, m + jj);
        const double2* Yk = Y + k * k + k + lo;
        const double2* Mj = Mx + jj * jj + jj + m - lo;
        int cnt = hi - lo + 1;
        for (int r = 0; r < cnt; r++) {  // l = lo + r
          double2 a = Yk[r], bq = Mj[-r];
          double tr = a.x * bq.x - a.y * bq.y;
          double ti = a.x * bq.y + a.y * bq.x;
          ar = ar + tr;
          ai = ai + ti;
        }
      }
      sr[q] = sr[q] + ar;
      si[q] = si[q] + ai;
    }
    __syncthreads();
  }
  double* out = mult + (size_t)c * nc * 2;
  for (int q = 0; q < M2M_SMAXK; q++) {
    int u = t + M2M_T * q;
    if (u < nc) {
      out[2 * u] = sr[q];
      out[2 * u + 1] = si[q];
    }
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

// M2M from the deepest parents to the roots over the multipole buffer `mult`
void m2m_levels(Ctx& c, double* mult) {
  for (int level = c.depth - 1; level >= 0; level--) {
    int first = c.lvl_first[level], count = c.lvl_count[level];
    if (c.p <= M2M_ALL_CHILDREN_PMAX)
      hipLaunchKernelGGL(k_m2m, dim3(count), dim3(M2M_T), m2m_lds_bytes(c.p), c.stream, c.p, first, count,
                         c.c_child0.p, c.c_nchild.p, c.c_cx.p, c.c_cy.p, c.c_cz.p, mult);
    else
      hipLaunchKernelGGL(k_m2m_stream, dim3(count), dim3(M2M_T), m2m_lds_bytes(c.p) / 8, c.stream, c.p, first,
                         count, c.c_child0.p, c.c_nchild.p, c.c_cx.p, c.c_cy.p, c.c_cz.p, mult);
    HIPCHK(hipGetLastError());
  }
}

void upload_up_tables() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (g_up_tables[dev & 63]) return;
  HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_fact), fmm_fact_table, sizeof(fmm_fact_table)));
  HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_binom), fmm_binom_table, sizeof(fmm_binom_table)));
  g_up_tables[dev & 63] = true;
}

void upward_pass(Ctx& c) {
  upload_up_tables();
  int p = c.p, nc = (int)c.ncell;
  ensure(c.ws, c.mult, (size_t)nc * ncoef(p) * 2);
  ensure(c.ws, c.pk, (size_t)nc * (p + 1));
  // the leaf list and count come from the tree build, so nothing here waits
  // for the device
  expansions_up(c);
}

// P2M at the leaves (the list from the tree build), M2M to the roots, P_k
void expansions_up(Ctx& c) {
  hipStream_t s = c.stream;
  int p = c.p, nc = (int)c.ncell;
  const int* leaves = c.leaves.p;
  size_t p2m_lds = sizeof(double) * (2 * ncoef(p) + 1) * p2m_batch(p);
  hipLaunchKernelGGL(k_p2m, dim3((unsigned)c.nleaf), dim3(P2M_T), p2m_lds, s, p, leaves, (int)c.nleaf,
                     c.c_begin.p, c.c_end.p, c.sx.p, c.sy.p, c.sz.p, c.sm.p, c.c_cx.p, c.c_cy.p,
                     c.c_cz.p, c.mult.p);
  HIPCHK(hipGetLastError());
  m2m_levels(c, c.mult.p);
  int64_t npk = (int64_t)nc * (p + 1);
  ensure(c.ws, c.pkb, (size_t)npk);
  hipLaunchKernelGGL(k_pk, dim3((unsigned)ceil_div(npk, 256)), dim3(256), 0, s, p, nc, c.mult.p, c.pk.p,
                     c.pkb.p);
  HIPCHK(hipGetLastError());
  if (c.prm.precision == FMM_MIXED && mixed_supported(p)) launch_normalize32(c);
}

}  // namespace fmm
