// Tree construction on gfx950: root box, 63-bit Morton keys, stable LSD radix
// sort, sorted SoA gather, breadth-first cells, masses, centres and radii.
//
// The paper builds an octree over the bodies (section 2.1, flowchart caption)
// and reuses the tree of its base code without describing it; the reading
// implemented here: cubic root box over the bodies' extent, 21 bits per axis,
// x most significant within each octal digit, a stable sort (ties keep the
// caller's order), cells = maximal runs of keys sharing a prefix, a cell with
// more than n_leaf bodies split into its non-empty octants (unless at level 21),
// ids breadth first (by level, then key order).  Expansion centre = centre of
// mass; size = largest distance of a body from it (section 2.3, "sizes").
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>

#include "fmm_device.h"

namespace fmm {

// ===================================================================== scan
constexpr int SCAN_T = 256, SCAN_I = 8, SCAN_TILE = SCAN_T * SCAN_I;

__device__ inline int block_excl_scan(int v, int* sh, int& total) {
  // sh: SCAN_T ints; returns exclusive prefix of v over the block
  int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int o = 1; o < SCAN_T; o <<= 1) {
    int a = t >= o ? sh[t - o] : 0;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  total = sh[SCAN_T - 1];
  int ex = sh[t] - v;
  __syncthreads();
  return ex;
}

__global__ void __launch_bounds__(SCAN_T) k_scan_reduce(const int* in, int64_t n, int* bsum) {
  __shared__ int sh[SCAN_T];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  int s = 0;
  for (int i = 0; i < SCAN_I; i++) {
    int64_t j = base + (int64_t)i * SCAN_T + threadIdx.x;
    if (j < n) s += in[j];
  }
  int tot;
  block_excl_scan(s, sh, tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// exclusive scan of one tile per block, plus a per-block offset
__global__ void __launch_bounds__(SCAN_T) k_scan_apply(const int* in, int* out, int64_t n,
                                                      const int* boff, long long* total,
                                                      int64_t nblocks) {
  __shared__ int sh[SCAN_T];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_I;
  int v[SCAN_I];
  int s = 0;
  for (int i = 0; i < SCAN_I; i++) {
    int64_t j = base + i;
    v[i] = j < n ? in[j] : 0;
    s += v[i];
  }
  int tot;
  int ex = block_excl_scan(s, sh, tot);
  int off = (boff ? boff[blockIdx.x] : 0) + ex;
  for (int i = 0; i < SCAN_I; i++) {
    int64_t j = base + i;
    if (j < n) out[j] = off;
    off += v[i];
  }
  if (total && blockIdx.x == nblocks - 1 && threadIdx.x == SCAN_T - 1)
    *total = (long long)(boff ? boff[blockIdx.x] : 0) + (long long)tot;
}

void exclusive_scan(Ctx& c, const int* in, int* out, int64_t n, long long* total_dev) {
  // recursive three-phase scan; scratch from c.scan_tmp
  int64_t sizes[16];  // block counts of the recursion levels (SCAN_TILE^16 exceeds any n)
  int nlev = 0;
  int64_t m = n;
  while (m > SCAN_TILE) {
    m = ceil_div(m, SCAN_TILE);
    sizes[nlev++] = m;
  }
  size_t need = 0;
  for (int l = 0; l < nlev; l++) need += 2 * (size_t)sizes[l] + 64;
  ensure(c.ws, c.scan_tmp, need + 64);
  if (n == 0) {
    if (total_dev) HIPCHK(hipMemsetAsync(total_dev, 0, sizeof(long long), c.stream));
    return;
  }
  if (nlev == 0) {
    hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(SCAN_T), 0, c.stream, in, out, n, nullptr,
                       total_dev, (int64_t)1);
    HIPCHK(hipGetLastError());
    return;
  }
  // level 0
  int* bsum = c.scan_tmp.p;
  int* boff = bsum + sizes[0] + 32;
  int64_t nb = sizes[0];
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(SCAN_T), 0, c.stream, in, n, bsum);
  HIPCHK(hipGetLastError());
  // scan of block sums (recursive via a nested context-free call)
  {
    // temporarily carve the remaining scratch for the recursion
    dbuf<int> saved = c.scan_tmp;
    c.scan_tmp.p = boff + nb + 32;
    c.scan_tmp.cap = saved.cap - (size_t)(c.scan_tmp.p - saved.p);
    exclusive_scan(c, bsum, boff, nb, nullptr);
    c.scan_tmp = saved;
  }
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(SCAN_T), 0, c.stream, in, out, n, boff,
                     total_dev, nb);
  HIPCHK(hipGetLastError());
}

long long read_total(Ctx& c, const long long* total_dev) {
  HIPCHK(hipMemcpyAsync(c.hbuf, total_dev, sizeof(long long), hipMemcpyDeviceToHost, c.stream));
  HIPCHK(hipStreamSynchronize(c.stream));
  return c.hbuf[0];
}

// ===================================================================== root box
constexpr int BB_T = 256;

__global__ void __launch_bounds__(BB_T) k_bbox_partial(const double* pos, int64_t n, double* part) {
  __shared__ double sh[6][BB_T];
  double lo[3], hi[3];
  int64_t i0 = (int64_t)blockIdx.x * BB_T + threadIdx.x;
  int64_t first = i0 < n ? i0 : 0;
  for (int d = 0; d < 3; d++) lo[d] = hi[d] = pos[3 * first + d];
  for (int64_t i = i0; i < n; i += (int64_t)gridDim.x * BB_T)
    for (int d = 0; d < 3; d++) {
      double v = pos[3 * i + d];
      if (v < lo[d]) lo[d] = v;
      if (v > hi[d]) hi[d] = v;
    }
  for (int d = 0; d < 3; d++) {
    sh[d][threadIdx.x] = lo[d];
    sh[3 + d][threadIdx.x] = hi[d];
  }
  __syncthreads();
  for (int o = BB_T / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int d = 0; d < 3; d++) {
        double a = sh[d][threadIdx.x + o], b = sh[3 + d][threadIdx.x + o];
        if (a < sh[d][threadIdx.x]) sh[d][threadIdx.x] = a;
        if (b > sh[3 + d][threadIdx.x]) sh[3 + d][threadIdx.x] = b;
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = sh[threadIdx.x][0];
}

// lo = min, L = largest extent (1 if zero), s = 2^21 / L  (rootbox = lo[3], L, s)
__global__ void __launch_bounds__(BB_T) k_bbox_final(const double* part, int nb, double* rootbox) {
  __shared__ double sh[6][BB_T];
  int t = threadIdx.x;
  double lo[3], hi[3];
  for (int d = 0; d < 3; d++) {
    lo[d] = part[d];
    hi[d] = part[3 + d];
  }
  for (int b = t; b < nb; b += BB_T)
    for (int d = 0; d < 3; d++) {
      if (part[6 * b + d] < lo[d]) lo[d] = part[6 * b + d];
      if (part[6 * b + 3 + d] > hi[d]) hi[d] = part[6 * b + 3 + d];
    }
  for (int d = 0; d < 3; d++) {
    sh[d][t] = lo[d];
    sh[3 + d][t] = hi[d];
  }
  __syncthreads();
  for (int o = BB_T / 2; o > 0; o >>= 1) {
    if (t < o)
      for (int d = 0; d < 3; d++) {
        if (sh[d][t + o] < sh[d][t]) sh[d][t] = sh[d][t + o];
        if (sh[3 + d][t + o] > sh[3 + d][t]) sh[3 + d][t] = sh[3 + d][t + o];
      }
    __syncthreads();
  }
  if (t != 0) return;
  double L = sh[3][0] - sh[0][0];
  if (sh[4][0] - sh[1][0] > L) L = sh[4][0] - sh[1][0];
  if (sh[5][0] - sh[2][0] > L) L = sh[5][0] - sh[2][0];
  if (L == 0.0) L = 1.0;
  rootbox[0] = sh[0][0];
  rootbox[1] = sh[1][0];
  rootbox[2] = sh[2][0];
  rootbox[3] = L;
  rootbox[4] = 2097152.0 / L;
}

// one workgroup per system (the systems of a batch): the same box over the
// bodies [off[s], off[s+1]) (min and max are exact in any order)
__global__ void __launch_bounds__(BB_T) k_bbox_sys(const double* pos, const int* off, double* rootbox) {
  __shared__ double sh[6][BB_T];
  int sys = blockIdx.x, t = threadIdx.x;
  int64_t b = off[sys], e = off[sys + 1];
  double lo[3], hi[3];
  for (int d = 0; d < 3; d++) lo[d] = hi[d] = pos[3 * b + d];
  for (int64_t i = b + t; i < e; i += BB_T)
    for (int d = 0; d < 3; d++) {
      double v = pos[3 * i + d];
      if (v < lo[d]) lo[d] = v;
      if (v > hi[d]) hi[d] = v;
    }
  for (int d = 0; d < 3; d++) {
    sh[d][t] = lo[d];
    sh[3 + d][t] = hi[d];
  }
  __syncthreads();
  for (int o = BB_T / 2; o > 0; o >>= 1) {
    if (t < o)
      for (int d = 0; d < 3; d++) {
        if (sh[d][t + o] < sh[d][t]) sh[d][t] = sh[d][t + o];
        if (sh[3 + d][t + o] > sh[3 + d][t]) sh[3 + d][t] = sh[3 + d][t + o];
      }
    __syncthreads();
  }
  if (t != 0) return;
  double L = sh[3][0] - sh[0][0];
  if (sh[4][0] - sh[1][0] > L) L = sh[4][0] - sh[1][0];
  if (sh[5][0] - sh[2][0] > L) L = sh[5][0] - sh[2][0];
  if (L == 0.0) L = 1.0;
  double* rb = rootbox + 8 * sys;
  rb[0] = sh[0][0];
  rb[1] = sh[1][0];
  rb[2] = sh[2][0];
  rb[3] = L;
  rb[4] = 2097152.0 / L;
}

// system of body i: the last s with off[s] <= i
__device__ __forceinline__ int system_of(const int* off, int nsys, int64_t i) {
  int lo = 0, hi = nsys - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// ===================================================================== keys
__device__ __forceinline__ uint64_t spread3(uint64_t x) {
  x &= 0x1fffffull;
  x = (x | (x << 32)) & 0x1f00000000ffffull;
  x = (x | (x << 16)) & 0x1f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

__device__ __forceinline__ uint64_t compact3(uint64_t x) {
  x &= 0x1249249249249249ull;
  x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
  x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
  x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
  x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
  x = (x ^ (x >> 32)) & 0x1fffffull;
  return x;
}

__global__ void k_keys(const double* pos, int64_t n, const double* rootbox_all, const int* sys_off,
                       int nsys, uint64_t* key, int* idx) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* rootbox = rootbox_all + (nsys > 1 ? 8 * system_of(sys_off, nsys, i) : 0);
  double s = rootbox[4];
  uint64_t q[3];
  for (int d = 0; d < 3; d++) {
    double t = floor((pos[3 * i + d] - rootbox[d]) * s);
    uint64_t v = (uint64_t)t;
    q[d] = v > 2097151ull ? 2097151ull : v;
  }
  key[i] = (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
  idx[i] = (int)i;
}

// ===================================================================== radix sort
// Stable LSD sort of (63-bit key, int payload), 8-bit digits.  Each block ranks a
// tile of RS_TILE keys: waves walk their sub-tile in 64-key chunks, computing
// for every key its rank among equal digits with 8 ballots, so the rank order
// equals the input order (stability).  Global digit offsets come from a
// per-digit scan of the digit-major block histograms (k_rs_rowscan).
constexpr int RS_T = 256, RS_W = RS_T / 64, RS_I = 16, RS_TILE = RS_T * RS_I;

template <class K>
__global__ void __launch_bounds__(RS_T) k_rs_hist(const K* key, int64_t n, int shift, int* hist,
                                                  int nblocks) {
  __shared__ int cnt[256];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int i = 0; i < RS_I; i++) {
    int64_t j = base + (int64_t)i * RS_T + threadIdx.x;
    if (j < n) atomicAdd(&cnt[(key[j] >> shift) & 255], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Per digit, the exclusive prefix of its tile counts over the tiles (one
// workgroup per digit, the row in runs of 8 x RS_T counts, each thread taking
// 8 consecutive ones), and the digit's total.  The scatter adds the totals of
// the smaller digits itself.
__global__ void __launch_bounds__(RS_T) k_rs_rowscan(const int* __restrict__ hist, int nblocks, int* offs,
                                                     int* rowtot) {
  __shared__ int wsum[2][RS_W];
  int d = blockIdx.x, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int* row = hist + (int64_t)d * nblocks;
  int* orow = offs + (int64_t)d * nblocks;
  int carry = 0;
  for (int base = 0, it = 0; base < nblocks; base += 8 * RS_T, it ^= 1) {
    int t0 = base + (int)threadIdx.x * 8;
    int v[8], sum = 0;
#pragma unroll
    for (int k = 0; k < 8; k++) {
      v[k] = t0 + k < nblocks ? row[t0 + k] : 0;
      sum += v[k];
    }
    int incl = sum;
    for (int o = 1; o < 64; o <<= 1) {
      int y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[it][w] = incl;  // alternate buffers: no second barrier per run
    __syncthreads();
    int before = 0, total = 0;
    for (int ww = 0; ww < RS_W; ww++) {
      if (ww < w) before += wsum[it][ww];
      total += wsum[it][ww];
    }
    int run = carry + before + incl - sum;
#pragma unroll
    for (int k = 0; k < 8; k++) {
      if (t0 + k < nblocks) orow[t0 + k] = run;
      run += v[k];
    }
    carry += total;
  }
  if (threadIdx.x == 0) rowtot[d] = carry;
}

// Ranks as above, then the tile is reordered by digit in LDS and written out
// with consecutive lanes on consecutive destinations (each digit's run of the
// tile is contiguous in the output), so the global writes coalesce.
template <bool VAL, class KI, class KO>
__global__ void __launch_bounds__(RS_T) k_rs_scatter(const KI* kin, const int* vin, KO* kout, int* vout,
                                                     int64_t n, int shift, const int* offs, const int* rowtot,
                                                     int nblocks) {
  __shared__ int wcnt[RS_W][256];
  __shared__ int goff[256], lofs[256], wsum[RS_W];
  __shared__ KO sk[RS_TILE];
  __shared__ int sv[VAL ? RS_TILE : 1];
  for (int t = threadIdx.x; t < RS_W * 256; t += RS_T) (&wcnt[0][0])[t] = 0;
  int w = threadIdx.x >> 6;
  int lane = threadIdx.x & 63;
  {
    // start of this digit in the output: the totals of the smaller digits
    // (an exclusive scan over the 256 digits, one per thread) plus the counts
    // of the earlier tiles
    int tot = rowtot[threadIdx.x];
    int incl = tot;
    for (int o = 1; o < 64; o <<= 1) {
      int y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int before = 0;
    for (int ww = 0; ww < w; ww++) before += wsum[ww];
    goff[threadIdx.x] = before + incl - tot + offs[(int64_t)threadIdx.x * nblocks + blockIdx.x];
    __syncthreads();
  }
  int64_t tile0 = (int64_t)blockIdx.x * RS_TILE;
  int64_t base = tile0 + (int64_t)w * (RS_TILE / RS_W);
  int tcount = (int)(n - tile0 < RS_TILE ? n - tile0 : RS_TILE);
  KI k[RS_I];
  int v[RS_I], rank[RS_I];
  uint64_t lt = lanemask_lt();
  for (int c = 0; c < RS_I; c++) {
    int64_t j = base + (int64_t)c * 64 + lane;
    bool valid = j < n;
    k[c] = valid ? kin[j] : 0;
    if (VAL) v[c] = valid ? vin[j] : 0;
    int d = (int)((k[c] >> shift) & 255);
    uint64_t peers = ballot(valid);
    for (int b = 0; b < 8; b++) {
      bool bit = (d >> b) & 1;
      uint64_t bb = ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    int before = __popcll(peers & lt);
    int cnt = wcnt[w][d];
    rank[c] = cnt + before;
    // the highest peer publishes the new running count for this digit
    if (valid && (peers >> lane) == 1ull) wcnt[w][d] = cnt + __popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // per digit: offsets of the waves within the tile's run, and the run length
  int d0 = threadIdx.x, tot = 0;
  for (int ww = 0; ww < RS_W; ww++) {
    int t = wcnt[ww][d0];
    wcnt[ww][d0] = tot;
    tot += t;
  }
  // exclusive scan of the run lengths over the 256 digits (one per thread)
  int incl = tot;
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int before_w = 0;
  for (int ww = 0; ww < w; ww++) before_w += wsum[ww];
  lofs[d0] = before_w + incl - tot;
  __syncthreads();
  for (int c = 0; c < RS_I; c++) {
    int64_t j = base + (int64_t)c * 64 + lane;
    if (j >= n) continue;
    int d = (int)((k[c] >> shift) & 255);
    int lp = lofs[d] + wcnt[w][d] + rank[c];
    sk[lp] = (KO)k[c];
    if (VAL) sv[lp] = v[c];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < tcount; t += RS_T) {
    KO key = sk[t];
    int d = (int)((key >> shift) & 255);
    int64_t dst = (int64_t)goff[d] + (t - lofs[d]);
    if (dst < n) {  // always true when the ranks are consistent with the histogram
      kout[dst] = key;
      if (VAL) vout[dst] = sv[t];
    }
  }
}

// Stable LSD sort of n keys over bits [0, nbits) (8 bits per pass), with an
// optional int payload.  Data ping-pongs between (k0, v0) and (k1, v1); the
// return value tells which buffer holds the result (0 or 1).
int radix_sort(Ctx& c, uint64_t* k0, int* v0, uint64_t* k1, int* v1, int64_t n, int nbits) {
  if (n <= 0) return 0;
  int nb = (int)ceil_div(n, RS_TILE);
  ensure(c.ws, c.sort_hist, (size_t)256 * nb * 2 + 256 + 64);
  int* hist = c.sort_hist.p;
  int* offs = hist + (size_t)256 * nb;
  int* rowtot = offs + (size_t)256 * nb;
  int src = 0;
  uint64_t* kk[2] = {k0, k1};
  int* vv[2] = {v0, v1};
  for (int shift = 0; shift < nbits; shift += 8) {
    hipLaunchKernelGGL(k_rs_hist<uint64_t>, dim3(nb), dim3(RS_T), 0, c.stream, kk[src], n, shift, hist, nb);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_rs_rowscan, dim3(256), dim3(RS_T), 0, c.stream, hist, nb, offs, rowtot);
    if (v0)
      hipLaunchKernelGGL((k_rs_scatter<true, uint64_t, uint64_t>), dim3(nb), dim3(RS_T), 0, c.stream,
                         kk[src], vv[src], kk[1 - src], vv[1 - src], n, shift, offs, rowtot, nb);
    else
      hipLaunchKernelGGL((k_rs_scatter<false, uint64_t, uint64_t>), dim3(nb), dim3(RS_T), 0, c.stream,
                         kk[src], nullptr, kk[1 - src], nullptr, n, shift, offs, rowtot, nb);
    HIPCHK(hipGetLastError());
    src = 1 - src;
  }
  return src;
}

// Stable LSD sort of n 64-bit keys whose values fit in nbits <= 32 bits: the
// first pass reads the 64-bit keys and writes 32-bit ones, later passes move
// 32-bit keys between b0 and b1.  Returns the buffer holding the result.
uint32_t* radix_sort_narrow(Ctx& c, const uint64_t* in, uint32_t* b0, uint32_t* b1, int64_t n, int nbits) {
  if (n <= 0) return b0;
  int nb = (int)ceil_div(n, RS_TILE);
  ensure(c.ws, c.sort_hist, (size_t)256 * nb * 2 + 256 + 64);
  int* hist = c.sort_hist.p;
  int* offs = hist + (size_t)256 * nb;
  int* rowtot = offs + (size_t)256 * nb;
  hipLaunchKernelGGL(k_rs_hist<uint64_t>, dim3(nb), dim3(RS_T), 0, c.stream, in, n, 0, hist, nb);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_rs_rowscan, dim3(256), dim3(RS_T), 0, c.stream, hist, nb, offs, rowtot);
  hipLaunchKernelGGL((k_rs_scatter<false, uint64_t, uint32_t>), dim3(nb), dim3(RS_T), 0, c.stream, in,
                     nullptr, b0, nullptr, n, 0, offs, rowtot, nb);
  HIPCHK(hipGetLastError());
  uint32_t* bb[2] = {b0, b1};
  int src = 0;
  for (int shift = 8; shift < nbits; shift += 8) {
    hipLaunchKernelGGL(k_rs_hist<uint32_t>, dim3(nb), dim3(RS_T), 0, c.stream, bb[src], n, shift, hist, nb);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_rs_rowscan, dim3(256), dim3(RS_T), 0, c.stream, hist, nb, offs, rowtot);
    hipLaunchKernelGGL((k_rs_scatter<false, uint32_t, uint32_t>), dim3(nb), dim3(RS_T), 0, c.stream,
                       bb[src], nullptr, bb[1 - src], nullptr, n, shift, offs, rowtot, nb);
    HIPCHK(hipGetLastError());
    src = 1 - src;
  }
  return bb[src];
}

// sorts c.key[0]/c.idx[0] (n entries) over bits [0, nbits); result in key[0]/idx[0]
void radix_sort_keys(Ctx& c, int64_t n, int nbits) {
  int r = radix_sort(c, c.key[0].p, c.idx[0].p, c.key[1].p, c.idx[1].p, n, nbits);
  if (r != 0) {
    std::swap(c.key[0], c.key[1]);
    std::swap(c.idx[0], c.idx[1]);
  }
}

// second key of a batch: the system of each body of the key-sorted order
// (from its caller index), payload = its position in that order
__global__ void k_sys_keys(const int* idx, int64_t n, const int* sys_off, int nsys, uint64_t* skey,
                           int* spos) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  skey[i] = (uint64_t)system_of(sys_off, nsys, idx[i]);
  spos[i] = (int)i;
}

__global__ void k_apply_pos(const int* spos, int64_t n, const uint64_t* kin, const int* vin,
                            uint64_t* kout, int* vout) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int j = spos[i];
  kout[i] = kin[j];
  vout[i] = vin[j];
}

__global__ void k_gather(const double* pos, const double* mass, const int* idx, int64_t n, double* sx,
                         double* sy, double* sz, double* sm, double4* pm) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int o = idx[i];
  double x = pos[3 * (int64_t)o], y = pos[3 * (int64_t)o + 1], z = pos[3 * (int64_t)o + 2], m = mass[o];
  sx[i] = x;
  sy[i] = y;
  sz[i] = z;
  sm[i] = m;
  pm[i] = make_double4(x, y, z, m);
}

// ===================================================================== cells
__device__ inline int octant_lower_bound(const uint64_t* key, int b, int e, int o, int shift) {
  // first index in [b, e) whose digit (at `shift`) is >= o; digits are non-decreasing
  int lo = b, hi = e;
  while (lo < hi) {
    int mid = lo + ((hi - lo) >> 1);
    int d = (int)((key[mid] >> shift) & 7);
    if (d < o)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// ---- the level loop on the device -----------------------------------------
// Level l's cells are [lvl[2l], lvl[2l] + lvl[2l+1]) (first id, count), kept on
// the device: every launch of a level reads its count there and the emit of
// level l writes level l + 1's entry, so the host enqueues a batch of levels
// without waiting and reads the table once at the end.  The cell arrays have
// a fixed capacity; a level whose children would not fit sets the overflow
// flag and ends the tree (the host grows the arrays and builds again).
constexpr int LV_T = 256, LV_NB = 256, LV_SPLIT_BLOCKS = 512;
constexpr int LV_TABLE = 128, LV_OVERFLOW = 180;  // int offsets in the device counters

__global__ void k_lv_init(int nsys, int* lvl, int* nleaf, int* overflow) {
  int t = threadIdx.x;
  if (t < 2 * (FMM_MAX_LEVEL + 2)) lvl[t] = t == 1 ? nsys : 0;
  if (t == 0) {
    *nleaf = 0;
    *overflow = 0;
  }
}

// Children of every cell of the level: eight lanes per cell, lane o finding
// the first body of octant o by its own binary search (the searches run side
// by side instead of one after another); cells that stay leaves are counted in
// *nleaf (one atomic per wavefront).  Grid-stride over the device count.
__global__ void __launch_bounds__(LV_T) k_split_lv(int level, const int* lvl, int n_leaf, const uint64_t* key,
                                                    const int* cb, const int* ce, int* split, int* nch,
                                                    int* nleaf) {
  int first = lvl[2 * level], count = lvl[2 * level + 1];
  int64_t total = (int64_t)count * 8;
  for (int64_t T0 = (int64_t)blockIdx.x * LV_T; T0 < total; T0 += (int64_t)gridDim.x * LV_T) {
    int64_t T = T0 + threadIdx.x;
    int t = (int)(T >> 3), o = (int)(T & 7);
    bool ok = t < count;  // the 8 lanes of a cell agree
    bool splits = false;
    int bound = 0, e = 0;
    if (ok) {
      int c = first + t;
      int b = cb[c];
      e = ce[c];
      splits = e - b > n_leaf && level < FMM_MAX_LEVEL;
      if (splits) {
        int shift = 3 * (FMM_MAX_LEVEL - (level + 1));
        bound = o == 0 ? b : octant_lower_bound(key, b, e, o, shift);
      }
    }
    int next = __shfl_down(bound, 1, 8);
    if (o == 7) next = e;
    int cnt = splits && next > bound ? 1 : 0;
    for (int m = 1; m < 8; m <<= 1) cnt += __shfl_xor(cnt, m, 8);
    if (ok && splits) {
      split[9 * (int64_t)t + o] = bound;
      if (o == 7) split[9 * (int64_t)t + 8] = e;
    }
    if (ok && o == 0) nch[t] = cnt;
    unsigned long long leaves = __ballot(ok && o == 0 && cnt == 0);
    if ((threadIdx.x & 63) == 0 && leaves) atomicAdd(nleaf, (int)__popcll(leaves));
  }
}

__device__ inline int block_sum(int v, int* sh) {
  int tot;
  block_excl_scan(v, sh, tot);
  return tot;
}

// children counts of a level summed over LV_NB contiguous ranges
__global__ void __launch_bounds__(LV_T) k_lv_bsum(int level, const int* lvl, const int* nch, int* bsum) {
  __shared__ int sh[SCAN_T];
  int count = lvl[2 * level + 1];
  int chunk = (count + LV_NB - 1) / LV_NB;
  int b0 = min(count, blockIdx.x * chunk), b1 = min(count, b0 + chunk);
  int v = 0;
  for (int t = b0 + threadIdx.x; t < b1; t += LV_T) v += nch[t];
  int tot = block_sum(v, sh);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// child ids by a scan of the counts (the range's offset from the block sums),
// then every cell's children, non-empty octants in octant order; block 0
// records the next level
__global__ void __launch_bounds__(LV_T) k_lv_emit(int level, int* lvl, const int* split, const int* nch,
                                                   const int* bsum, int cap, int* overflow, int* c_level,
                                                   int* c_begin, int* c_end, int* c_parent, int* c_child0,
                                                   int* c_nchild) {
  __shared__ int sh[SCAN_T];
  int first = lvl[2 * level], count = lvl[2 * level + 1];
  int next_first = first + count;
  int chunk = (count + LV_NB - 1) / LV_NB;
  int b0 = min(count, blockIdx.x * chunk), b1 = min(count, b0 + chunk);
  int pre = 0, all = 0;
  for (int k = threadIdx.x; k < LV_NB; k += LV_T) {
    int v = bsum[k];
    if (k < (int)blockIdx.x) pre += v;
    all += v;
  }
  pre = block_sum(pre, sh);
  all = block_sum(all, sh);
  bool over = (int64_t)next_first + all > cap;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int nxt = level + 1;
    if (nxt <= FMM_MAX_LEVEL + 1) {
      lvl[2 * nxt] = next_first;
      lvl[2 * nxt + 1] = over ? 0 : all;
    }
    if (over) *overflow = 1;
  }
  for (int base = b0; base < b1; base += LV_T) {
    int t = base + threadIdx.x;
    int k = t < b1 ? nch[t] : 0;
    int tile;
    int ex = block_excl_scan(k, sh, tile);
    if (t < b1) {
      int c = first + t;
      c_nchild[c] = over ? 0 : k;
      if (k == 0 || over) {
        c_child0[c] = -1;
      } else {
        int id = next_first + pre + ex;
        c_child0[c] = id;
        for (int o = 0; o < 8; o++) {
          int s0 = split[9 * (int64_t)t + o], s1 = split[9 * (int64_t)t + o + 1];
          if (s1 > s0) {
            c_level[id] = level + 1;
            c_begin[id] = s0;
            c_end[id] = s1;
            c_parent[id] = c;
            id++;
          }
        }
      }
    }
    pre += tile;
  }
}

// one root per system: cell s holds the bodies of system s
__global__ void k_roots(int nsys, const int* sys_off, int* c_level, int* c_begin, int* c_end,
                        int* c_parent) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsys) return;
  c_level[s] = 0;
  c_begin[s] = sys_off[s];
  c_end[s] = sys_off[s + 1];
  c_parent[s] = -1;
}

// mass, first moments and centre of mass, one level (deepest first); leaves sum
// their bodies in sorted order, internal cells their children in octant order
__global__ void k_mass_com(int first, int count, int level, const int* cb, const int* ce,
                           const int* c0, const int* nch, const double* sx, const double* sy,
                           const double* sz, const double* sm, const uint64_t* key,
                           const double* rootbox_all, const int* sys_off, int nsys, double* cm, double* csx, double* csy, double* csz,
                           double* cx, double* cy, double* cz) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  int c = first + t;
  double M = 0.0, X = 0.0, Y = 0.0, Z = 0.0;
  if (nch[c] == 0) {
    for (int i = cb[c]; i < ce[c]; i++) {
      double m = sm[i];
      M = M + m;
      X = X + m * sx[i];
      Y = Y + m * sy[i];
      Z = Z + m * sz[i];
    }
  } else {
    for (int k = c0[c]; k < c0[c] + nch[c]; k++) {
      M = M + cm[k];
      X = X + csx[k];
      Y = Y + csy[k];
      Z = Z + csz[k];
    }
  }
  cm[c] = M;
  csx[c] = X;
  csy[c] = Y;
  csz[c] = Z;
  if (M != 0.0) {
    cx[c] = X / M;
    cy[c] = Y / M;
    cz[c] = Z / M;
  } else {  // massless cell: centre of its cubic box
    const double* rootbox = rootbox_all + (nsys > 1 ? 8 * system_of(sys_off, nsys, cb[c]) : 0);
    uint64_t k0 = key[cb[c]];
    int sh = FMM_MAX_LEVEL - level;
    double h = ldexp(rootbox[3], -level);
    double q0 = (double)(compact3(k0 >> 2) >> sh), q1 = (double)(compact3(k0 >> 1) >> sh),
           q2 = (double)(compact3(k0) >> sh);
    cx[c] = rootbox[0] + (q0 + 0.5) * h;
    cy[c] = rootbox[1] + (q1 + 0.5) * h;
    cz[c] = rootbox[2] + (q2 + 0.5) * h;
  }
}

// radius: exact max over each cell's bodies of the squared distance to its
// centre (order independent), in chunks of RAD_CH bodies
constexpr int RAD_T = 256, RAD_CH = CELL_CHUNK;

__global__ void k_rad_chunks(const int* cb, const int* ce, int ncell, int* nchunk) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  nchunk[c] = (int)ceil_div(ce[c] - cb[c], RAD_CH);
}

// one wavefront per chunk (the count stays on the device, so the launch needs
// no host round trip; the grid covers an upper bound of it)
__global__ void __launch_bounds__(RAD_T) k_radius(const int* cb, const int* ce, const int* choff,
                                                 const long long* nchunks, int ncell, const double* sx,
                                                 const double* sy, const double* sz, const double* cx,
                                                 const double* cy, const double* cz,
                                                 unsigned long long* r2bits) {
  int blk = blockIdx.x * (RAD_T / 64) + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (blk >= (int)*nchunks) return;
  // cell owning this chunk: last c with choff[c] <= blk
  int lo = 0, hi = ncell - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (choff[mid] <= blk)
      lo = mid;
    else
      hi = mid - 1;
  }
  int c = lo;
  int64_t b = cb[c] + (int64_t)(blk - choff[c]) * RAD_CH;
  int64_t e = b + RAD_CH < ce[c] ? b + RAD_CH : ce[c];
  double x0 = cx[c], y0 = cy[c], z0 = cz[c];
  double best = 0.0;
  for (int64_t i = b + lane; i < e; i += 64) {
    double dx = sx[i] - x0, dy = sy[i] - y0, dz = sz[i] - z0;
    double d2 = (dx * dx + dy * dy) + dz * dz;
    if (d2 > best) best = d2;
  }
  for (int o = 32; o > 0; o >>= 1) {
    double other = __shfl_xor(best, o, 64);
    if (other > best) best = other;
  }
  if (lane == 0) atomicMax(&r2bits[c], (unsigned long long)__double_as_longlong(best));
}

// radius from the squared maximum; also the packed (centre, radius) record
// the walks read
__global__ void k_radius_final(const unsigned long long* r2bits, int ncell, const double* cx, const double* cy,
                               const double* cz, double* rad, double4* geo) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  double r = sqrt(__longlong_as_double((long long)r2bits[c]));
  rad[c] = r;
  geo[c] = make_double4(cx[c], cy[c], cz[c], r);
}

__global__ void k_leaf_of(const int* cb, const int* ce, const int* nch, int ncell, int* leaf_of) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell || nch[c] != 0) return;
  for (int i = cb[c]; i < ce[c]; i++) leaf_of[i] = c;
}

static inline dim3 grid1(int64_t n, int t = 256) { return dim3((unsigned)ceil_div(n, t)); }

// every body is in one cell per level: at most (depth + 1) n / CELL_CHUNK + ncell chunks
unsigned cell_chunk_blocks(const Ctx& c, int waves_per_block) {
  int64_t max_chunks = (int64_t)(c.depth + 1) * ceil_div(c.n, CELL_CHUNK) + c.ncell;
  return (unsigned)ceil_div(max_chunks, waves_per_block);
}

// mass, centre of mass and radius of every cell from the sorted bodies
void cell_moments(Ctx& c, bool with_radius) {
  hipStream_t s = c.stream;
  int nc = (int)c.ncell, nsys = c.nsys;
  long long* tot = (long long*)c.counters.p;
  ensure(c.ws, c.c_mass, nc);
  ensure(c.ws, c.c_sx, nc);
  ensure(c.ws, c.c_sy, nc);
  ensure(c.ws, c.c_sz, nc);
  ensure(c.ws, c.c_cx, nc);
  ensure(c.ws, c.c_cy, nc);
  ensure(c.ws, c.c_cz, nc);
  ensure(c.ws, c.c_rad, nc);
  ensure(c.ws, c.c_rad2bits, nc);
  for (int level = c.depth; level >= 0; level--) {
    int first = c.lvl_first[level], count = c.lvl_count[level];
    hipLaunchKernelGGL(k_mass_com, grid1(count, 128), dim3(128), 0, s, first, count, level,
                       c.c_begin.p, c.c_end.p, c.c_child0.p, c.c_nchild.p, c.sx.p, c.sy.p, c.sz.p,
                       c.sm.p, c.key[0].p, c.rootbox.p, c.sys_off.p, nsys, c.c_mass.p, c.c_sx.p, c.c_sy.p, c.c_sz.p,
                       c.c_cx.p, c.c_cy.p, c.c_cz.p);
    HIPCHK(hipGetLastError());
  }
  if (!with_radius) return;
  // radii
  ensure(c.ws, c.c_split, (size_t)nc + 64);
  ensure(c.ws, c.cell_choff, (size_t)nc + 64);
  int* nchunk = c.c_split.p;
  int* choff = c.cell_choff.p;
  long long* nchunks = (long long*)(c.counters.p + 4);
  hipLaunchKernelGGL(k_rad_chunks, grid1(nc), dim3(256), 0, s, c.c_begin.p, c.c_end.p, nc, nchunk);
  exclusive_scan(c, nchunk, choff, nc, nchunks);
  zero_fill(c, c.c_rad2bits.p, sizeof(unsigned long long) * nc);
  hipLaunchKernelGGL(k_radius, dim3(cell_chunk_blocks(c, RAD_T / 64)), dim3(RAD_T), 0, s, c.c_begin.p,
                     c.c_end.p, choff, nchunks, nc, c.sx.p, c.sy.p, c.sz.p, c.c_cx.p, c.c_cy.p, c.c_cz.p,
                     c.c_rad2bits.p);
  ensure(c.ws, c.c_geo, (size_t)nc);
  hipLaunchKernelGGL(k_radius_final, grid1(nc), dim3(256), 0, s, c.c_rad2bits.p, nc, c.c_cx.p, c.c_cy.p,
                     c.c_cz.p, c.c_rad.p, c.c_geo.p);
}

// Positions and masses changed, tree topology, order and lists kept: the
// sorted bodies, cell masses and centres are recomputed from the stored
// order.  The radii are not (they serve the acceptance test, which is not
// rerun, and the FP32 scaling, for which any positive size works), so the
// sequence needs no host round trip.
void refresh_frozen(Ctx& c, const double* pos, const double* mass) {
  hipLaunchKernelGGL(k_gather, grid1(c.n), dim3(256), 0, c.stream, pos, mass, c.idx[0].p, c.n, c.sx.p,
                     c.sy.p, c.sz.p, c.sm.p, c.pm.p);
  HIPCHK(hipGetLastError());
  cell_moments(c, false);
}

__global__ void k_list_leaves(const int* nch, int ncell, int* flag) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncell) flag[c] = nch[c] == 0 ? 1 : 0;
}

__global__ void k_compact_leaves(const int* flag, const int* off, int ncell, int* leaves) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncell && flag[c]) leaves[off[c]] = c;
}

void build_tree(Ctx& c, int64_t n, const double* pos, const double* mass) {
  hipStream_t s = c.stream;
  c.n = n;
  int nsys = c.nsys;
  for (int k = 0; k < 2; k++) {
    ensure(c.ws, c.key[k], n);
    ensure(c.ws, c.idx[k], n);
  }
  ensure(c.ws, c.sx, n);
  ensure(c.ws, c.sy, n);
  ensure(c.ws, c.sz, n);
  ensure(c.ws, c.sm, n);
  ensure(c.ws, c.leaf_of, n);
  ensure(c.ws, c.rootbox, (size_t)8 * nsys);
  {
    int* before = c.sys_off.p;
    ensure(c.ws, c.sys_off, (size_t)nsys + 1);
    if (c.sys_off.p != before) c.sys_off_uploaded.clear();
  }
  {
    // the device copy is reused while the split is unchanged (no host
    // allocation while it is: the comparison runs over the stored vectors)
    if (c.h_sys_off.empty()) c.h_sys_off.assign({0, n});
    bool same = c.sys_off_uploaded.size() == c.h_sys_off.size();
    for (size_t k = 0; same && k < c.h_sys_off.size(); k++) same = c.sys_off_uploaded[k] == (int)c.h_sys_off[k];
    if (!same) {
      c.sys_off_uploaded.assign(c.h_sys_off.begin(), c.h_sys_off.end());
      HIPCHK(hipMemcpyAsync(c.sys_off.p, c.sys_off_uploaded.data(), c.sys_off_uploaded.size() * sizeof(int),
                            hipMemcpyHostToDevice, s));
      HIPCHK(hipStreamSynchronize(s));
    }
  }
  if (nsys == 1) {
    int nbb = (int)std::min<int64_t>(1024, ceil_div(n, BB_T));
    ensure(c.ws, c.bbox_part, (size_t)6 * nbb);
    hipLaunchKernelGGL(k_bbox_partial, dim3(nbb), dim3(BB_T), 0, s, pos, n, c.bbox_part.p);
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(BB_T), 0, s, c.bbox_part.p, nbb, c.rootbox.p);
  } else {
    hipLaunchKernelGGL(k_bbox_sys, dim3(nsys), dim3(BB_T), 0, s, pos, c.sys_off.p, c.rootbox.p);
  }
  hipLaunchKernelGGL(k_keys, grid1(n), dim3(256), 0, s, pos, n, c.rootbox.p, c.sys_off.p, nsys,
                     c.key[0].p, c.idx[0].p);
  HIPCHK(hipGetLastError());
  if (c.have_events) HIPCHK(hipEventRecord(c.ev[15], s));
  radix_sort_keys(c, n, 64);
  if (nsys > 1) {
    // stable pass over the system id: (system, key, caller index) order
    for (int k = 0; k < 2; k++) {
      ensure(c.ws, c.skey[k], n);
      ensure(c.ws, c.spos[k], n);
    }
    hipLaunchKernelGGL(k_sys_keys, grid1(n), dim3(256), 0, s, c.idx[0].p, n, c.sys_off.p, nsys,
                       c.skey[0].p, c.spos[0].p);
    int bits = 1;
    while ((1 << bits) < nsys) bits++;
    int r = radix_sort(c, c.skey[0].p, c.spos[0].p, c.skey[1].p, c.spos[1].p, n, bits);
    hipLaunchKernelGGL(k_apply_pos, grid1(n), dim3(256), 0, s, c.spos[r].p, n, c.key[0].p, c.idx[0].p,
                       c.key[1].p, c.idx[1].p);
    HIPCHK(hipGetLastError());
    std::swap(c.key[0], c.key[1]);
    std::swap(c.idx[0], c.idx[1]);
  }
  ensure(c.ws, c.pm, n);
  if (c.have_events) HIPCHK(hipEventRecord(c.ev[16], s));
  hipLaunchKernelGGL(k_gather, grid1(n), dim3(256), 0, s, pos, mass, c.idx[0].p, n, c.sx.p, c.sy.p,
                     c.sz.p, c.sm.p, c.pm.p);
  HIPCHK(hipGetLastError());
  if (c.have_events) HIPCHK(hipEventRecord(c.ev[17], s));

  // breadth-first levels, built on the device (see k_lv_emit)
  size_t cap = (size_t)std::max<int64_t>(1024, 4 * n / std::max(1, c.prm.n_leaf) + 64 + 2 * nsys);
  cap = std::max(cap, c.c_level.cap);
  ensure(c.ws, c.counters, 512);  // the full size at once: counters[4..5] must outlive this call
  int* nleaf_dev = c.counters.p + 2;
  int* lvl = c.counters.p + LV_TABLE;
  int* overflow = c.counters.p + LV_OVERFLOW;
  constexpr int NLV = FMM_MAX_LEVEL + 2;  // table entries: levels 0..21 and the empty one after
  constexpr int FIRST_BATCH = 12;         // levels enqueued before the first read-back
  long long nleaf = 0;
  int depth = 0;
  for (int attempt = 0;; attempt++) {
    for (auto* b : {&c.c_level, &c.c_begin, &c.c_end, &c.c_parent, &c.c_child0, &c.c_nchild})
      ensure(c.ws, *b, cap);
    cap = std::min({c.c_level.cap, c.c_begin.cap, c.c_end.cap, c.c_parent.cap, c.c_child0.cap,
                    c.c_nchild.cap, (size_t)INT_MAX / 16});
    ensure(c.ws, c.c_split, 10 * cap + LV_NB + 64);
    int* split = c.c_split.p;  // 9 octant bounds per cell of the level
    int* nch = split + 9 * cap;
    int* bsum = nch + cap;
    hipLaunchKernelGGL(k_roots, grid1(nsys), dim3(256), 0, s, nsys, c.sys_off.p, c.c_level.p, c.c_begin.p,
                       c.c_end.p, c.c_parent.p);
    hipLaunchKernelGGL(k_lv_init, dim3(1), dim3(64), 0, s, nsys, lvl, nleaf_dev, overflow);
    int* h = (int*)c.hbuf;  // read-back: the table, then the leaf count and the overflow flag
    int level = 0;
    bool more = true;
    for (int batch_end = FIRST_BATCH; more; batch_end = NLV - 1) {
      for (; level < batch_end; level++) {
        hipLaunchKernelGGL(k_split_lv, dim3(LV_SPLIT_BLOCKS), dim3(LV_T), 0, s, level, lvl, c.prm.n_leaf,
                           c.key[0].p, c.c_begin.p, c.c_end.p, split, nch, nleaf_dev);
        hipLaunchKernelGGL(k_lv_bsum, dim3(LV_NB), dim3(LV_T), 0, s, level, lvl, nch, bsum);
        hipLaunchKernelGGL(k_lv_emit, dim3(LV_NB), dim3(LV_T), 0, s, level, lvl, split, nch, bsum, (int)cap,
                           overflow, c.c_level.p, c.c_begin.p, c.c_end.p, c.c_parent.p, c.c_child0.p,
                           c.c_nchild.p);
      }
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(h, lvl, 2 * NLV * sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(h + 2 * NLV, nleaf_dev, sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(h + 2 * NLV + 1, overflow, sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      more = level < NLV - 1 && h[2 * level + 1] > 0 && !h[2 * NLV + 1];
    }
    if (!h[2 * NLV + 1]) {
      c.lvl_first.clear();
      c.lvl_count.clear();
      for (int l = 0; l < NLV && h[2 * l + 1] > 0; l++) {
        c.lvl_first.push_back(h[2 * l]);
        c.lvl_count.push_back(h[2 * l + 1]);
      }
      nleaf = h[2 * NLV];
      depth = (int)c.lvl_first.size() - 1;
      break;
    }
    if (attempt > 8) throw hip_error{hipErrorUnknown, "cell arrays did not converge"};
    cap *= 2;  // a level did not fit: larger arrays, build again
  }
  c.ncell = (int64_t)c.lvl_first[depth] + c.lvl_count[depth];
  c.depth = depth;
  int nc = (int)c.ncell;

  cell_moments(c, true);
  hipLaunchKernelGGL(k_leaf_of, grid1(nc), dim3(256), 0, s, c.c_begin.p, c.c_end.p, c.c_nchild.p, nc,
                     c.leaf_of.p);
  HIPCHK(hipGetLastError());
  // the leaf cells in id order (built here, before any fork, so that every
  // stream sees the list)
  ensure(c.ws, c.c_split, (size_t)2 * nc + 64);
  ensure(c.ws, c.leaves, (size_t)nc);
  int* flag = c.c_split.p;
  int* off = flag + nc + 32;
  hipLaunchKernelGGL(k_list_leaves, grid1(nc), dim3(256), 0, s, c.c_nchild.p, nc, flag);
  exclusive_scan(c, flag, off, nc, nullptr);
  hipLaunchKernelGGL(k_compact_leaves, grid1(nc), dim3(256), 0, s, flag, off, nc, c.leaves.p);
  HIPCHK(hipGetLastError());
  c.nleaf = nleaf;
}

}  // namespace fmm
