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

#include <functional>

#include <algorithm>
#include <climits>

#include "fmm_device.h"
#include "fmm_tables.h"

namespace fmm {


struct CellView {
  const int *nch, *c0;
  const double4* geo;  // (centre x, y, z, radius) per cell, one 32-byte record
  const double *mass, *pkb, *fmin;
  int p;
  double theta, err_tol;
  int geometric;
};

__device__ __forceinline__ double com_r2(const double4& a, const double4& b) {
  double dx = b.x - a.x;
  double dy = b.y - a.y;
  double dz = b.z - a.z;
  return (dx * dx + dy * dy) + dz * dz;
}

// E_{A->B} M_A / r^2 with M_A cancelled; sums in the order the definition
// lists (k ascending), each term (C(p,k) P_{k,A}) r_B^{p-k}, with C(p,k) P_{k,A}
// formed once per cell by the upward pass.  P = 0: the order is the run-time
// v.p (orders without an unrolled instance), with the same operations in the
// same order.
template <int P>
__device__ double mac_lhs(const CellView& v, int A, double rA, double rB, double r, double r2) {
  constexpr int PM = P > 0 ? P : FMM_TABLE_PMAX;
  const int p = P > 0 ? P : v.p;
  double rp = r;
#pragma unroll
  for (int i = 2; i <= PM; i++)
    if (i <= p) rp = rp * r;
  double mx = rA > rB ? rA : rB;
  double pref = (8.0 * mx) / (rA + rB);
  double pw[PM + 1];
  pw[0] = 1.0;
  double powB = 1.0;
#pragma unroll
  for (int j = 1; j <= PM; j++) {
    powB = powB * rB;
    pw[j] = powB;
  }
  const double* PA = v.pkb + (size_t)A * (p + 1);
  double SA = 0.0;
#pragma unroll
  for (int k = 0; k <= PM; k++)
    if (k <= p) SA = SA + PA[k] * pw[p - k];
  return (pref * (SA / rp)) / r2;
}

template <int KIND, int P>
__device__ bool accept(const CellView& v, int A, int B, const double4& gA, const double4& gB) {
  double r2 = com_r2(gA, gB);
  double r = sqrt(r2);
  double rA = gA.w, rB = gB.w;
  if constexpr (KIND == 0) {
    return (rA + rB) < v.theta * r;
  } else {
    if (!((rA + rB) < v.theta * r)) return false;
    if (v.geometric) return true;
    if (rA + rB == 0.0) return true;
    double lab = mac_lhs<P>(v, A, rA, rB, r, r2);
    double lba = mac_lhs<P>(v, B, rB, rA, r, r2);
    return (lab < v.err_tol * v.fmin[B]) && (lba < v.err_tol * v.fmin[A]);
  }
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

constexpr int WALK_T = 512;  // threads per workgroup of the walk kernels

// One workgroup-aggregated allocation of `cnt` slots from the 64-bit counter
// *ctr: a wave scan, the wave totals combined through LDS, one atomic per
// workgroup.
__device__ __forceinline__ long long block_alloc(int cnt, unsigned long long* ctr, int& excl, int* sh,
                                                 long long* shb) {
  int incl = wave_incl_scan(cnt);
  int wv = threadIdx.x >> 6;
  if (lane_id() == 63) sh[wv] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int w = 0; w < WALK_T / 64; w++) {
      int t = sh[w];
      sh[w] = run;
      run += t;
    }
    *shb = run > 0 ? (long long)atomicAdd(ctr, (unsigned long long)run) : 0;
  }
  __syncthreads();
  excl = incl - cnt + sh[wv];
  long long base = *shb;
  __syncthreads();
  return base;
}

// Device counters of a walk (64-bit, each on its own cache line, at the int
// offsets below): three rotating frontier sizes, the totals of accepted and
// near-field entries, and the largest frontier seen.  Step k reads its
// frontier size from slot k % 3, appends to slot (k+1) % 3 and clears slot
// (k+2) % 3 for the step after, so consecutive steps need no host round trip.
// 64-bit totals cannot wrap; the host rejects lists longer than the int32
// CSR arrays can index (walk_list_fits).
constexpr int WC_FRONT = 0, WC_ACC = 96, WC_NEAR = 128, WC_MAXF = 160, WC_INTS = 192;
constexpr int WALK_BLOCKS = 1024;  // persistent grid; blocks stride over the frontier

__device__ __forceinline__ unsigned long long* wc64(int* ctr, int off) {
  return reinterpret_cast<unsigned long long*>(ctr + off);
}

template <int KIND, int P>
__global__ void __launch_bounds__(WALK_T) k_walk(CellView v, int step, const int2* fin, int fin_cap,
                                              int2* fout, long long fcap, int* ctr, uint64_t* acc_list,
                                              long long acap, uint64_t* near_list, long long ncap,
                                              int bits) {
  long long nin_all = (long long)*wc64(ctr, WC_FRONT + 32 * (step % 3));
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *wc64(ctr, WC_FRONT + 32 * ((step + 2) % 3)) = 0ull;
    atomicMax(wc64(ctr, WC_MAXF), (unsigned long long)nin_all);
  }
  int nin = (int)min(nin_all, (long long)fin_cap);  // an overflowed frontier is redone by the host
  unsigned long long* fctr = wc64(ctr, WC_FRONT + 32 * ((step + 1) % 3));
  __shared__ int sh[WALK_T / 64];
  __shared__ long long shb;
  for (int base = blockIdx.x * WALK_T; base < nin; base += gridDim.x * WALK_T) {
    int t = base + threadIdx.x;
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
      } else {
        double4 gA = v.geo[A], gB = v.geo[B];
        if (accept<KIND, P>(v, A, B, gA, gB)) {
          nacc = 2;
        } else if (kA == 0 && kB == 0) {
          nnear = 2;
        } else {
          bool splitB = (kA == 0) || (gB.w > gA.w && kB != 0);
          mode = splitB ? 3 : 2;
          nkids = splitB ? kB : kA;
        }
      }
    }
    int ek, ea, en;
    long long bk = block_alloc(nkids, fctr, ek, sh, &shb);
    long long ba = block_alloc(nacc, wc64(ctr, WC_ACC), ea, sh, &shb);
    long long bn = block_alloc(nnear, wc64(ctr, WC_NEAR), en, sh, &shb);
    if (!live) continue;
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
    // list entries: (sink << bits) | source
    uint64_t kab = ((uint64_t)B << bits) | (uint64_t)A, kba = ((uint64_t)A << bits) | (uint64_t)B;
    if (nacc) {
      long long q = ba + ea;
      if (q + 1 < acap) {
        acc_list[q] = kab;
        acc_list[q + 1] = kba;
      }
    }
    if (nnear) {
      long long q = bn + en;
      if (nnear == 1) {
        if (q < ncap) near_list[q] = kab;
      } else if (q + 1 < ncap) {
        near_list[q] = kab;
        near_list[q + 1] = kba;
      }
    }
  }
}

// the walks start from (root, root) of every system; counters cleared
__global__ void k_seed(int2* f, int nsys, int* ctr) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nsys) f[s] = make_int2(s, s);
  if (s < WC_INTS) ctr[s] = s == WC_FRONT ? nsys : 0;  // low half of the 64-bit frontier size
}

// ---- grouping by sink, sorted by source ----------------------------------
// The keys (sink << bits | source) are radix-sorted (as 32-bit keys when
// 2 bits <= 32); CSR offsets come from a lower bound per sink and the sources
// are the low bits.
template <class K>
__global__ void k_csr_off(const K* keys, int64_t cnt, int nseg, int bits, int* off) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s > nseg) return;
  uint64_t t = (uint64_t)s << bits;
  int64_t lo = 0, hi = cnt;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if ((uint64_t)keys[mid] < t)
      lo = mid + 1;
    else
      hi = mid;
  }
  off[s] = (int)lo;
}

template <class K>
__global__ void k_extract_src(const K* keys, int64_t cnt, uint64_t mask, int* src) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) src[i] = (int)((uint64_t)keys[i] & mask);
}

static int list_bits(int64_t ncell) {
  int b = 1;
  while (((int64_t)1 << b) < ncell) b++;
  return b;
}

static void group_by_sink(Ctx& c, CellList& L) {
  hipStream_t s = c.stream;
  int nc = (int)c.ncell;
  int bits = list_bits(c.ncell);
  ensure(c.ws, L.off, (size_t)nc + 1);
  ensure(c.ws, L.src, (size_t)std::max<int64_t>(L.count, 1));
  ensure(c.ws, L.tmp, (size_t)std::max<int64_t>(L.count, 1));
  uint64_t mask = ((uint64_t)1 << bits) - 1;
  unsigned g = (unsigned)std::max<int64_t>(1, ceil_div(L.count, 256));
  unsigned go = (unsigned)ceil_div(nc + 1, 256);
  if (2 * bits <= 32) {
    uint32_t* b0 = (uint32_t*)L.tmp.p;  // two 32-bit buffers in the 64-bit scratch
    uint32_t* b1 = b0 + std::max<int64_t>(L.count, 1);
    const uint32_t* sorted = b0;
    if (L.count) {
      sorted = radix_sort_narrow(c, L.raw.p, b0, b1, L.count, 2 * bits);
      hipLaunchKernelGGL(k_extract_src<uint32_t>, dim3(g), dim3(256), 0, s, sorted, L.count, mask, L.src.p);
    }
    hipLaunchKernelGGL(k_csr_off<uint32_t>, dim3(go), dim3(256), 0, s, sorted, L.count, nc, bits, L.off.p);
  } else {
    const uint64_t* sorted = L.raw.p;
    if (L.count) {
      int r = radix_sort(c, L.raw.p, nullptr, L.tmp.p, nullptr, L.count, 2 * bits);
      sorted = r == 0 ? L.raw.p : L.tmp.p;
      hipLaunchKernelGGL(k_extract_src<uint64_t>, dim3(g), dim3(256), 0, s, sorted, L.count, mask, L.src.p);
    }
    hipLaunchKernelGGL(k_csr_off<uint64_t>, dim3(go), dim3(256), 0, s, sorted, L.count, nc, bits, L.off.p);
  }
  HIPCHK(hipGetLastError());
}

// beside: host work (launches on other streams) done once, right after the
// first batch of walk steps is enqueued and before the host waits for them
template <int KIND, int P>
static void run_walk(Ctx& c, CellList& acc, CellList& nearl, bool group,
                     const std::function<void()>& beside = {}) {
  hipStream_t s = c.stream;
  CellView v{};
  v.nch = c.c_nchild.p;
  v.c0 = c.c_child0.p;
  v.geo = c.c_geo.p;
  v.mass = c.c_mass.p;
  v.pkb = c.pkb.p;
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
  ensure(c.ws, c.counters, 512);
  int* ctr = c.counters.p + 256;
  int bits = list_bits(c.ncell);
  long long* h = c.hbuf;  // the counters, read back as 64-bit values
  auto H = [&](int off) { return h[off / 2]; };
  // A pair's step count is at most the sum of its cells' levels plus one, so
  // 2 depth + 2 steps drain the frontier; the host checks once at the end.
  int steps = 2 * c.depth + 2;
  long long nacc = 0, nnear = 0;
  auto fcap_of = [&](const dbuf<int2>& f) { return (int)std::min<size_t>(f.cap, (size_t)INT_MAX); };
  for (int attempt = 0;; attempt++) {
    int sblocks = (int)ceil_div(std::max(c.nsys, WC_INTS), 256);
    hipLaunchKernelGGL(k_seed, dim3((unsigned)sblocks), dim3(256), 0, s, c.front[0].p, c.nsys, ctr);
    int step = 0;
    bool done = false;
    while (!done) {
      for (int e = 0; e < steps; e++, step++)
        hipLaunchKernelGGL((k_walk<KIND, P>), dim3(WALK_BLOCKS), dim3(WALK_T), 0, s, v, step,
                           c.front[step & 1].p, fcap_of(c.front[step & 1]), c.front[1 - (step & 1)].p,
                           (long long)fcap_of(c.front[1 - (step & 1)]), ctr, acc.raw.p,
                           (long long)acc.raw.cap, nearl.raw.p, (long long)nearl.raw.cap, bits);
      HIPCHK(hipGetLastError());
      if (beside && attempt == 0 && step == steps) beside();
      HIPCHK(hipMemcpyAsync(h, ctr, WC_INTS * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      done = H(WC_FRONT + 32 * (step % 3)) == 0;  // frontier of the next step is empty
      if (H(WC_MAXF) > std::min(fcap_of(c.front[0]), fcap_of(c.front[1]))) break;  // overflowed: redo
    }
    nacc = H(WC_ACC);
    nnear = H(WC_NEAR);
    long long need_f = H(WC_MAXF);
    if (!walk_list_fits(nacc) || !walk_list_fits(nnear) || !walk_list_fits(need_f))
      throw unsupported_error{"interaction list or walk frontier longer than 2^31 - 64 entries"};
    bool again = false;
    if (need_f > std::min(fcap_of(c.front[0]), fcap_of(c.front[1]))) {
      ensure(c.ws, c.front[0], (size_t)need_f * 2);
      ensure(c.ws, c.front[1], (size_t)need_f * 2);
      again = true;
    }
    if ((size_t)nacc + 2 > acc.raw.cap) {
      ensure(c.ws, acc.raw, (size_t)nacc * 2 + 64);
      again = true;
    }
    if ((size_t)nnear + 2 > nearl.raw.cap) {
      ensure(c.ws, nearl.raw, (size_t)nnear * 2 + 64);
      again = true;
    }
    if (!again) break;
    if (attempt > 8) throw hip_error{hipErrorUnknown, "walk buffers did not converge"};
  }
  acc.count = nacc;
  nearl.count = nnear;
  if (group) {
    group_by_sink(c, acc);
    group_by_sink(c, nearl);
  }
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

// near_i = sum_{j near, j != i} m_j / d^2, partners in ascending id, bodies in
// sorted order, one running sum per body (k_fleaf adds the far part).
// One wavefront per sink leaf, a lane per sink body; each source leaf is
// staged in LDS (one coalesced load, the next one fetched while the current
// one is summed) and read by all lanes as broadcasts.
constexpr int NF_WAVES = 4;

__global__ void __launch_bounds__(64 * NF_WAVES) k_near_f(int nleaves, const int* __restrict__ leaves,
                                                          const int* __restrict__ cb,
                                                          const int* __restrict__ ce,
                                                          const int* __restrict__ off,
                                                          const int* __restrict__ src,
                                                          const double4* __restrict__ pm, double* f) {
  __shared__ double4 sbuf[NF_WAVES][64];
  int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int nblk = (nleaves + NF_WAVES - 1) / NF_WAVES;
  int blk = xcd_block();
  int li = blk * NF_WAVES + wv;
  if (blk >= nblk || li >= nleaves) return;
  int B = leaves[li];
  int b = cb[B], e = ce[B];
  int qb = off[B], qe = off[B + 1];
  for (int i0 = b; i0 < e; i0 += 64) {
    int i = i0 + lane;
    bool act = i < e;
    double4 me = act ? pm[i] : make_double4(0.0, 0.0, 0.0, 0.0);
    double near = 0.0;
    int q = qb, j0 = 0, je = 0;
    if (q < qe) {
      int A = src[q];
      j0 = cb[A];
      je = ce[A];
    }
    double4 cur = make_double4(0.0, 0.0, 0.0, 0.0);
    if (q < qe && lane < je - j0) cur = pm[j0 + lane];
    while (q < qe) {
      int na = min(64, je - j0);
      int nq = q, nj0 = j0 + 64, nje = je;
      if (nj0 >= je) {
        nq = q + 1;
        if (nq < qe) {
          int A = src[nq];
          nj0 = cb[A];
          nje = ce[A];
        }
      }
      __builtin_amdgcn_wave_barrier();
      sbuf[wv][lane] = cur;
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the staged chunk is visible to the wave
      cur = make_double4(0.0, 0.0, 0.0, 0.0);
      if (nq < qe && lane < nje - nj0) cur = pm[nj0 + lane];
      int tmax = act ? na : 0;
      for (int t = 0; t < tmax; t++) {
        double4 s = sbuf[wv][t];
        double dx = s.x - me.x, dy = s.y - me.y, dz = s.z - me.z;
        double d2 = (dx * dx + dy * dy) + dz * dz;
        if (j0 + t != i && d2 > 0.0) near = near + s.w / d2;
      }
      q = nq;
      j0 = nj0;
      je = nje;
    }
    if (act) f[i] = near;
    __builtin_amdgcn_wave_barrier();
  }
}

// f_i = (F summed from the root down to the leaf) + near_i, in that order, for
// the bodies of every leaf (f holds near_i on entry); one thread per leaf
__global__ void k_fleaf(int nleaves, const int* leaves, const int* cb, const int* ce, const int* parent,
                        const double* F, double* f) {
  int li = blockIdx.x * blockDim.x + threadIdx.x;
  if (li >= nleaves) return;
  int c = leaves[li];
  int path[FMM_MAX_LEVEL + 2];
  int len = 0;
  for (int q = c; q >= 0; q = parent[q]) path[len++] = q;
  double far = 0.0;
  for (int k = len - 1; k >= 0; k--) far = far + F[path[k]];
  for (int i = cb[c]; i < ce[c]; i++) f[i] = far + f[i];
}

// fmin_c = min of f over the cell's bodies (the same as the minimum over its
// children), a wavefront per chunk of CELL_CHUNK bodies; f >= 0, so the bit
// patterns order as the values and the chunks combine by an integer atomicMin
// (fmin starts at +inf)
constexpr int FM_T = 256;
__global__ void __launch_bounds__(FM_T) k_cell_min(const int* cb, const int* ce, const int* choff,
                                                   const long long* nchunks, int ncell, const double* f,
                                                   unsigned long long* fmin_bits) {
  int blk = blockIdx.x * (FM_T / 64) + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (blk >= (int)*nchunks) return;
  int lo = 0, hi = ncell - 1;  // cell owning this chunk: last c with choff[c] <= blk
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (choff[mid] <= blk)
      lo = mid;
    else
      hi = mid - 1;
  }
  int c = lo;
  int64_t b = cb[c] + (int64_t)(blk - choff[c]) * CELL_CHUNK;
  int64_t e = b + CELL_CHUNK < ce[c] ? b + CELL_CHUNK : ce[c];
  double m = INFINITY;
  for (int64_t i = b + lane; i < e; i += 64) m = f[i] < m ? f[i] : m;
  for (int o = 32; o > 0; o >>= 1) {
    double other = __shfl_xor(m, o, 64);
    m = other < m ? other : m;
  }
  if (lane == 0) atomicMin(&fmin_bits[c], (unsigned long long)__double_as_longlong(m));
}

__global__ void k_fill_inf(unsigned long long* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0x7ff0000000000000ull;
}

// The far sums F_B (list grouped on the second side stream, with the third
// set of sort scratch) run beside the near sums on the caller's stream; after
// the join the leaves add the two, then the cell minima are taken.
void estimate_walk(Ctx& c, const std::function<void()>& beside) {
  hipStream_t s = c.stream;
  int nc = (int)c.ncell;
  ensure(c.ws, c.fcell, nc);
  ensure(c.ws, c.fmin, nc);
  ensure(c.ws, c.fpart, (size_t)c.n);
  run_walk<0, 0>(c, c.est_far, c.est_near, false, beside);
  stream_wait(c.fork[6], s, c.side2);
  {
    OnStream on(c, c.side2);
    SideScratch alt(c, 3);
    group_by_sink(c, c.est_far);
    hipLaunchKernelGGL(k_fcell, dim3((nc + 255) / 256), dim3(256), 0, c.side2, nc, c.est_far.off.p,
                       c.est_far.src.p, c.c_mass.p, c.c_cx.p, c.c_cy.p, c.c_cz.p, c.fcell.p);
  }
  group_by_sink(c, c.est_near);
  {
    int nblk = (int)ceil_div(c.nleaf, NF_WAVES);
    unsigned grid = xcd_grid(nblk);
    hipLaunchKernelGGL(k_near_f, dim3(grid), dim3(64 * NF_WAVES), 0, s, (int)c.nleaf, c.leaves.p,
                       c.c_begin.p, c.c_end.p, c.est_near.off.p, c.est_near.src.p, c.pm.p, c.fpart.p);
  }
  stream_wait(c.fork[7], c.side2, s);
  hipLaunchKernelGGL(k_fleaf, dim3((unsigned)ceil_div(c.nleaf, 128)), dim3(128), 0, s, (int)c.nleaf, c.leaves.p,
                     c.c_begin.p, c.c_end.p, c.c_parent.p, c.fcell.p, c.fpart.p);
  unsigned long long* fmin_bits = (unsigned long long*)c.fmin.p;
  hipLaunchKernelGGL(k_fill_inf, dim3((nc + 255) / 256), dim3(256), 0, s, fmin_bits, nc);
  hipLaunchKernelGGL(k_cell_min, dim3(cell_chunk_blocks(c, FM_T / 64)), dim3(FM_T), 0, s, c.c_begin.p, c.c_end.p,
                     c.cell_choff.p, (const long long*)(c.counters.p + 4), nc, c.fpart.p, fmin_bits);
  HIPCHK(hipGetLastError());
}

template <int P>
static bool mac_dispatch(Ctx& c) {
  if constexpr (P > FMM_GPU_PMAX) {
    if (c.p > FMM_TABLE_PMAX) return false;
    run_walk<1, 0>(c, c.m2l, c.p2p, false);  // higher orders: run-time p
    return true;
  } else {
    if (c.p == P) {
      run_walk<1, P>(c, c.m2l, c.p2p, false);  // grouped by the caller (group_list)
      return true;
    }
    return mac_dispatch<P + 1>(c);
  }
}

// the acceptance walk's list grouped by sink (CSR, sources ascending)
void group_list(Ctx& c, CellList& L) { group_by_sink(c, L); }

void mac_walk(Ctx& c) {
  if (!mac_dispatch<1>(c)) throw hip_error{hipErrorInvalidValue, "walk order not compiled"};
}

}  // namespace fmm
