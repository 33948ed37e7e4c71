// Dual-tree walks on gfx950 (section 2.1 "Dual-tree Walk", section 2.3).
//
// Both walks expand a frontier of cell pairs level-synchronously from
// (root, root).  A pair (A, A) with A a leaf is a near-field self pair; an
// internal A yields its child pairs (c_i, c_j), i <= j.  A pair A != B is
// accepted (both directed pairs recorded), or, if both are leaves, recorded as
// a near-field leaf pair in both directions, or split: B when A is a leaf or
// when B is larger and not a leaf, A otherwise (ties split A).
//   * estimate walk: accept iff (r_A + r_B) < theta_est r (the "theta < 1"
//     estimate of the scalar force, section 2.3);
//   * main walk: the error-controlled mutual criterion
//     theta < 1 and E_{A->B} M_A / r^2 < eps f_B and E_{B->A} M_B / r^2 < eps f_A
//     (section 2.3), with E from the per-order norms P_k.
// Emission order inside a step is not fixed (wave-aggregated atomics); the
// recorded pair SETS are, and every list is afterwards grouped by sink and
// sorted by source, so all consumers see a deterministic order.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fmm_device.h"
#include "fmm_tables.h"

namespace fmm {

static __constant__ double c_binom[FMM_TABLE_PMAX + 1][FMM_TABLE_PMAX + 1];
static bool g_walk_tables = false;

struct CellView {
  const int *nch, *c0;
  const double *rad, *cx, *cy, *cz, *mass, *pk, *fmin;
  int p;
  double theta, err_tol;
  int geometric;
};

__device__ __forceinline__ double com_r2(const CellView& v, int a, int b) {
  double dx = v.cx[b] - v.cx[a];
  double dy = v.cy[b] - v.cy[a];
  double dz = v.cz[b] - v.cz[a];
  return (dx * dx + dy * dy) + dz * dz;
}

// E_{A->B} M_A / r^2 with M_A cancelled; sums in the order the definition lists
__device__ double mac_lhs(const CellView& v, int A, int B, double r, double r2) {
  int p = v.p;
  double rA = v.rad[A], rB = v.rad[B];
  double rp = r;
  for (int i = 2; i <= p; i++) rp = rp * r;
  double mx = rA > rB ? rA : rB;
  double pref = (8.0 * mx) / (rA + rB);
  double pw[FMM_TABLE_PMAX + 1];
  pw[0] = 1.0;
  double powB = 1.0;
  for (int j = 1; j <= p; j++) {
    powB = powB * rB;
    pw[j] = powB;
  }
  const double* PA = v.pk + (size_t)A * (p + 1);
  double SA = 0.0;
  for (int k = 0; k <= p; k++) SA = SA + (c_binom[p][k] * PA[k]) * pw[p - k];
  return (pref * (SA / rp)) / r2;
}

template <int KIND>
__device__ bool accept(const CellView& v, int A, int B) {
  double r2 = com_r2(v, A, B);
  double r = sqrt(r2);
  double rA = v.rad[A], rB = v.rad[B];
  if (KIND == 0) return (rA + rB) < v.theta * r;
  if (!((rA + rB) < v.theta * r)) return false;
  if (v.geometric) return true;
  if (rA + rB == 0.0) return true;
  double lab = mac_lhs(v, A, B, r, r2);
  double lba = mac_lhs(v, B, A, r, r2);
  return (lab < v.err_tol * v.fmin[B]) && (lba < v.err_tol * v.fmin[A]);
}

__device__ __forceinline__ int wave_incl_scan(int x) {
  int lane = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

// one wave-aggregated allocation of `cnt` slots from counter *ctr
__device__ __forceinline__ long long wave_alloc(int cnt, int* ctr, int& excl) {
  int incl = wave_incl_scan(cnt);
  excl = incl - cnt;
  int total = __shfl(incl, 63, 64);
  int base = 0;
  if (lane_id() == 63 && total > 0) base = atomicAdd(ctr, total);
  base = __shfl(base, 63, 64);
  return base;
}

// ctr[0]: next frontier, ctr[1]: accepted pairs, ctr[2]: near-field leaf pairs
template <int KIND>
__global__ void __launch_bounds__(256) k_walk(CellView v, const int2* fin, int nin, int2* fout,
                                              int fcap, int* ctr, int2* acc_list, int acap,
                                              int2* near_list, int ncap) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  bool live = t < nin;
  int A = 0, B = 0, nkids = 0, nacc = 0, nnear = 0, mode = 0;
  // mode: 0 none, 1 self children, 2 split A, 3 split B
  if (live) {
    int2 pr = fin[t];
    A = pr.x;
    B = pr.y;
    int kA = v.nch[A], kB = v.nch[B];
    if (A == B) {
      if (kA == 0) {
        nnear = 1;
      } else {
        mode = 1;
        nkids = kA * (kA + 1) / 2;
      }
    } else if (accept<KIND>(v, A, B)) {
      nacc = 2;
    } else if (kA == 0 && kB == 0) {
      nnear = 2;
    } else {
      bool splitB = (kA == 0) || (v.rad[B] > v.rad[A] && kB != 0);
      mode = splitB ? 3 : 2;
      nkids = splitB ? kB : kA;
    }
  }
  int ek, ea, en;
  long long bk = wave_alloc(nkids, &ctr[0], ek);
  long long ba = wave_alloc(nacc, &ctr[1], ea);
  long long bn = wave_alloc(nnear, &ctr[2], en);
  if (!live) return;
  long long o = bk + ek;
  if (mode == 1) {
    int c0 = v.c0[A], k = v.nch[A];
    for (int i = 0; i < k; i++)
      for (int j = i; j < k; j++, o++)
        if (o < fcap) fout[o] = make_int2(c0 + i, c0 + j);
  } else if (mode == 2) {
    int c0 = v.c0[A];
    for (int i = 0; i < nkids; i++, o++)
      if (o < fcap) fout[o] = make_int2(c0 + i, B);
  } else if (mode == 3) {
    int c0 = v.c0[B];
    for (int j = 0; j < nkids; j++, o++)
      if (o < fcap) fout[o] = make_int2(A, c0 + j);
  }
  if (nacc) {
    long long q = ba + ea;
    if (q + 1 < acap) {
      acc_list[q] = make_int2(B, A);  // (sink, source)
      acc_list[q + 1] = make_int2(A, B);
    }
  }
  if (nnear) {
    long long q = bn + en;
    if (nnear == 1) {
      if (q < ncap) near_list[q] = make_int2(A, A);
    } else if (q + 1 < ncap) {
      near_list[q] = make_int2(B, A);
      near_list[q + 1] = make_int2(A, B);
    }
  }
}

__global__ void k_seed(int2* f) { f[0] = make_int2(0, 0); }

// ---- grouping by sink, sorted by source ----------------------------------
__global__ void k_count_sinks(const int2* raw, int64_t cnt, int* hist) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) atomicAdd(&hist[raw[i].x], 1);
}

__global__ void k_scatter_sinks(const int2* raw, int64_t cnt, const int* off, int* cursor, int* src) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  int2 pr = raw[i];
  int slot = atomicAdd(&cursor[pr.x], 1);
  src[off[pr.x] + slot] = pr.y;
}

constexpr int SEG_T = 512, SEG_CAP = 8192;

// sorts each sink's sources ascending: bitonic sort in LDS; longer segments
// fall back to a rank sort in global memory (entries within a segment are distinct)
__global__ void __launch_bounds__(SEG_T) k_sort_segments(const int* off, int nseg, int* src,
                                                         int* tmp) {
  __shared__ int sh[SEG_CAP];
  int s = blockIdx.x;
  if (s >= nseg) return;
  int b = off[s], e = off[s + 1], len = e - b;
  if (len <= 1) return;
  if (len <= SEG_CAP) {
    int P = 1;
    while (P < len) P <<= 1;
    for (int i = threadIdx.x; i < P; i += SEG_T) sh[i] = i < len ? src[b + i] : 0x7fffffff;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1)
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = threadIdx.x; i < P; i += SEG_T) {
          int ix = i ^ j;
          if (ix > i) {
            int a = sh[i], c = sh[ix];
            bool up = (i & k) == 0;
            if ((a > c) == up) {
              sh[i] = c;
              sh[ix] = a;
            }
          }
        }
        __syncthreads();
      }
    for (int i = threadIdx.x; i < len; i += SEG_T) src[b + i] = sh[i];
  } else {
    for (int i = threadIdx.x; i < len; i += SEG_T) {
      int v = src[b + i], r = 0;
      for (int j = 0; j < len; j++) r += src[b + j] < v;
      tmp[b + r] = v;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < len; i += SEG_T) src[b + i] = tmp[b + i];
  }
}

static void group_by_sink(Ctx& c, CellList& L) {
  hipStream_t s = c.stream;
  int nc = (int)c.ncell;
  ensure(c.ws, L.off, (size_t)nc + 1);
  ensure(c.ws, L.cursor, (size_t)nc + 1);
  ensure(c.ws, L.src, (size_t)std::max<int64_t>(L.count, 1));
  int* hist = L.cursor.p;
  HIPCHK(hipMemsetAsync(hist, 0, sizeof(int) * (nc + 1), s));
  if (L.count)
    hipLaunchKernelGGL(k_count_sinks, dim3((unsigned)ceil_div(L.count, 256)), dim3(256), 0, s,
                       L.raw.p, L.count, hist);
  exclusive_scan(c, hist, L.off.p, nc + 1, nullptr);
  HIPCHK(hipMemsetAsync(hist, 0, sizeof(int) * (nc + 1), s));
  if (L.count) {
    hipLaunchKernelGGL(k_scatter_sinks, dim3((unsigned)ceil_div(L.count, 256)), dim3(256), 0, s,
                       L.raw.p, L.count, L.off.p, hist, L.src.p);
    // rank-sort scratch reuses the raw pair buffer (count ints fit in count int2)
    hipLaunchKernelGGL(k_sort_segments, dim3(nc), dim3(SEG_T), 0, s, L.off.p, nc, L.src.p,
                       (int*)L.raw.p);
  }
  HIPCHK(hipGetLastError());
}

template <int KIND>
static void run_walk(Ctx& c, CellList& acc, CellList& nearl) {
  hipStream_t s = c.stream;
  CellView v{};
  v.nch = c.c_nchild.p;
  v.c0 = c.c_child0.p;
  v.rad = c.c_rad.p;
  v.cx = c.c_cx.p;
  v.cy = c.c_cy.p;
  v.cz = c.c_cz.p;
  v.mass = c.c_mass.p;
  v.pk = c.pk.p;
  v.fmin = c.fmin.p;
  v.p = c.p;
  v.theta = KIND == 0 ? c.prm.theta_est : c.prm.theta;
  v.err_tol = c.err_tol;
  v.geometric = c.prm.mac == FMM_MAC_GEOMETRIC;
  size_t fcap0 = std::max<size_t>(4096, (size_t)c.ncell * 4);
  ensure(c.ws, c.front[0], fcap0);
  ensure(c.ws, c.front[1], fcap0);
  ensure(c.ws, acc.raw, std::max<size_t>(acc.raw.cap, (size_t)c.ncell * 8 + 64));
  ensure(c.ws, nearl.raw, std::max<size_t>(nearl.raw.cap, (size_t)c.ncell * 8 + 64));
  ensure(c.ws, c.counters, 64);
  int* ctr = c.counters.p + 16;
  int* h = (int*)c.hbuf;
  hipLaunchKernelGGL(k_seed, dim3(1), dim3(1), 0, s, c.front[0].p);
  int nin = 1, cur = 0;
  int nacc = 0, nnear = 0;
  while (nin > 0) {
    for (;;) {
      int init[4] = {0, nacc, nnear, 0};
      HIPCHK(hipMemcpyAsync(ctr, init, sizeof(init), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_walk<KIND>, dim3((unsigned)ceil_div(nin, 256)), dim3(256), 0, s, v,
                         c.front[cur].p, nin, c.front[1 - cur].p, (int)c.front[1 - cur].cap, ctr,
                         acc.raw.p, (int)acc.raw.cap, nearl.raw.p, (int)nearl.raw.cap);
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(h, ctr, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      bool again = false;
      if ((size_t)h[0] > c.front[1 - cur].cap) {
        ensure(c.ws, c.front[1 - cur], (size_t)h[0] * 2);
        again = true;
      }
      if ((size_t)h[1] + 2 > acc.raw.cap) {
        ensure(c.ws, acc.raw, (size_t)h[1] * 2 + 64, true, s);
        again = true;
      }
      if ((size_t)h[2] + 2 > nearl.raw.cap) {
        ensure(c.ws, nearl.raw, (size_t)h[2] * 2 + 64, true, s);
        again = true;
      }
      if (!again) break;
    }
    nacc = h[1];
    nnear = h[2];
    nin = h[0];
    cur = 1 - cur;
    if ((size_t)nin * 36 > c.front[1 - cur].cap) ensure(c.ws, c.front[1 - cur], (size_t)nin * 8 + 4096);
  }
  acc.count = nacc;
  nearl.count = nnear;
  group_by_sink(c, acc);
  group_by_sink(c, nearl);
}

// ---- scalar-force estimate -----------------------------------------------
// F_B = sum over accepted sources A (ascending) of M_A / r^2
__global__ void k_fcell(int ncell, const int* off, const int* src, const double* mass,
                        const double* cx, const double* cy, const double* cz, double* F) {
  int B = blockIdx.x * blockDim.x + threadIdx.x;
  if (B >= ncell) return;
  double f = 0.0;
  for (int k = off[B]; k < off[B + 1]; k++) {
    int A = src[k];
    double dx = cx[B] - cx[A], dy = cy[B] - cy[A], dz = cz[B] - cz[A];
    double r2 = (dx * dx + dy * dy) + dz * dz;
    f = f + mass[A] / r2;
  }
  F[B] = f;
}

// f_i = (F summed from the root down to the leaf) + sum_{j near, j != i} m_j / d^2,
// partners in ascending id, bodies in sorted order
__global__ void __launch_bounds__(64) k_near_f(const int* leaves, int nleaves, const int* cb,
                                               const int* ce, const int* parent, const int* off,
                                               const int* src, const double* F, const double* sx,
                                               const double* sy, const double* sz, const double* sm,
                                               double* f) {
  int li = blockIdx.x;
  if (li >= nleaves) return;
  int B = leaves[li];
  double far = 0.0;
  {
    int path[FMM_MAX_LEVEL + 2];
    int len = 0;
    for (int q = B; q >= 0; q = parent[q]) path[len++] = q;
    for (int t = len - 1; t >= 0; t--) far = far + F[path[t]];
  }
  int b = cb[B], e = ce[B];
  for (int i0 = b; i0 < e; i0 += 64) {
    int i = i0 + threadIdx.x;
    bool act = i < e;
    double xi = act ? sx[i] : 0.0, yi = act ? sy[i] : 0.0, zi = act ? sz[i] : 0.0;
    double near = 0.0;
    for (int k = off[B]; k < off[B + 1]; k++) {
      int A = src[k];
      for (int j = cb[A]; j < ce[A]; j++) {
        double dx = sx[j] - xi, dy = sy[j] - yi, dz = sz[j] - zi;
        double d2 = (dx * dx + dy * dy) + dz * dz;
        if (j != i && d2 > 0.0) near = near + sm[j] / d2;
      }
    }
    if (act) f[i] = far + near;
  }
}

__global__ void k_fmin(int first, int count, const int* cb, const int* ce, const int* c0,
                       const int* nch, const double* f, double* fmin) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  int c = first + t;
  double m;
  if (nch[c] == 0) {
    m = INFINITY;
    for (int i = cb[c]; i < ce[c]; i++)
      if (f[i] < m) m = f[i];
  } else {
    m = fmin[c0[c]];
    for (int k = 1; k < nch[c]; k++)
      if (fmin[c0[c] + k] < m) m = fmin[c0[c] + k];
  }
  fmin[c] = m;
}

void estimate_walk(Ctx& c) {
  if (!g_walk_tables) {
    HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(c_binom), fmm_binom_table, sizeof(fmm_binom_table)));
    g_walk_tables = true;
  }
  hipStream_t s = c.stream;
  int nc = (int)c.ncell;
  ensure(c.ws, c.fcell, nc);
  ensure(c.ws, c.fmin, nc);
  ensure(c.ws, c.fpart, (size_t)c.n);
  run_walk<0>(c, c.est_far, c.est_near);
  hipLaunchKernelGGL(k_fcell, dim3((nc + 255) / 256), dim3(256), 0, s, nc, c.est_far.off.p,
                     c.est_far.src.p, c.c_mass.p, c.c_cx.p, c.c_cy.p, c.c_cz.p, c.fcell.p);
  // leaves list was built by the upward pass in c_split (flag | off | leaves)
  const int* leaves = c.c_split.p + 2 * (nc + 32);
  hipLaunchKernelGGL(k_near_f, dim3((unsigned)c.nleaf), dim3(64), 0, s, leaves, (int)c.nleaf,
                     c.c_begin.p, c.c_end.p, c.c_parent.p, c.est_near.off.p, c.est_near.src.p,
                     c.fcell.p, c.sx.p, c.sy.p, c.sz.p, c.sm.p, c.fpart.p);
  for (int level = c.depth; level >= 0; level--) {
    int first = c.lvl_first[level], count = c.lvl_count[level];
    hipLaunchKernelGGL(k_fmin, dim3((count + 127) / 128), dim3(128), 0, s, first, count, c.c_begin.p,
                       c.c_end.p, c.c_child0.p, c.c_nchild.p, c.fpart.p, c.fmin.p);
  }
  HIPCHK(hipGetLastError());
}

void mac_walk(Ctx& c) { run_walk<1>(c, c.m2l, c.p2p); }

}  // namespace fmm
