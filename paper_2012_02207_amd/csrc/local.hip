// Downward pass and near field on gfx950 (section 2.1): L2L shifts each cell's
// local expansion to its children, L2P evaluates the leaf expansion at every
// body (potential and force), P2P adds the direct sum over the near-field leaf
// pairs, and the results are written in the caller's body order.  Also the
// plain O(N^2) direct sum used for checks.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fmm_device.h"

namespace fmm {

// L2L, one workgroup per parent: L_child(j, i) += sum_{k <= p-j} sum_{l=-k..k}
// L_parent(j+k, i+l) conj(Y_k^l(z_child - z_parent)).  The parent expansion
// and the conjugated harmonics of every child are laid out in LDS for both
// signs of the order (entry n(n+1) + m, m = -n..n), which makes every sum a
// branch-free loop; lanes evaluate harmonic columns, then (child,
// coefficient) sums.
constexpr int L2L_T = 256;

// G: children per pass (their harmonics share LDS with the parent's expansion;
// 8 = all at once, fewer at the orders where eight do not fit)
__global__ void __launch_bounds__(L2L_T) k_l2l(int p, int first, int count, const int* c0,
                                              const int* nch, const double* cx, const double* cy,
                                              const double* cz, double* loc, int G) {
  extern __shared__ double lds[];
  int P = first + blockIdx.x;
  if (blockIdx.x >= count || nch[P] == 0) return;
  int nc = ncoef(p), S = (p + 1) * (p + 1);
  int k0 = c0[P], kn = nch[P];
  double2* Lx = (double2*)lds;  // [S]
  double2* Yc = Lx + S;         // [child of the pass][S]
  int t = threadIdx.x;
  const double* Lp = loc + (size_t)P * nc * 2;
  for (int u = t; u < S; u += L2L_T) {
    int n = 0;
    while ((n + 1) * (n + 1) <= u) n++;
    int m = u - n * n - n, am = m < 0 ? -m : m;
    double a = Lp[2 * cidx(n, am)], b = Lp[2 * cidx(n, am) + 1];
    if (m < 0) {
      double sg = (am & 1) ? -1.0 : 1.0;
      a = sg * a;
      b = -sg * b;
    }
    Lx[u] = make_double2(a, b);
  }
  for (int j0 = 0; j0 < kn; j0 += G) {
    int gn = min(G, kn - j0);
    if (j0 > 0) __syncthreads();  // the previous pass has read its harmonics
    for (int u = t; u < gn * (p + 1); u += L2L_T) {  // column m of child j's harmonics
      int j = u / (p + 1), m = u - j * (p + 1);
      int ch = k0 + j0 + j;
      double x = cx[ch] - cx[P], y = cy[ch] - cy[P], z = cz[ch] - cz[P];
      double r2 = fma(x, x, fma(y, y, z * z));
      double pr = 1.0, pi = 0.0;
      for (int n = 1; n <= m; n++) {
        double inv = -1.0 / (double)(2 * n);
        double tr = fma(x, pr, -y * pi), ti = fma(x, pi, y * pr);
        pr = tr * inv;
        pi = ti * inv;
      }
      double2* Y = Yc + j * S;
      double sg = (m & 1) ? -1.0 : 1.0;
      // conj(Y_n^m) at +m; conj(Y_n^-m) = (-1)^m Y_n^m at -m
      Y[m * m + m + m] = make_double2(pr, -pi);
      if (m > 0) Y[m * m] = make_double2(sg * pr, sg * pi);
      double ar2 = 0.0, ai2 = 0.0, ar1 = pr, ai1 = pi;
      for (int n = m + 1; n <= p; n++) {
        double k = (double)(2 * n - 1) * z, inv = 1.0 / (double)((n + m) * (n - m));
        double vr = fma(k, ar1, -r2 * ar2) * inv, vi = fma(k, ai1, -r2 * ai2) * inv;
        Y[n * n + n + m] = make_double2(vr, -vi);
        if (m > 0) Y[n * n + n - m] = make_double2(sg * vr, sg * vi);
        ar2 = ar1;
        ai2 = ai1;
        ar1 = vr;
        ai1 = vi;
      }
    }
    __syncthreads();
    for (int u = t; u < gn * nc; u += L2L_T) {
      int j = u / nc, q = u - j * nc;
      int jn = 0;
      while (cidx(jn + 1, 0) <= q) jn++;
      int i = q - cidx(jn, 0);
      const double2* Y = Yc + j * S;
      double sr = 0.0, si = 0.0;
      for (int k = 0; k <= p - jn; k++) {
        int n = jn + k;
        const double2* Ln = Lx + n * n + n + i - k;
        const double2* Yk = Y + k * k;
#pragma unroll 4
        for (int r = 0; r <= 2 * k; r++) {  // l = r - k
          double2 a = Ln[r], b = Yk[r];
          sr = fma(a.x, b.x, fma(-a.y, b.y, sr));
          si = fma(a.x, b.y, fma(a.y, b.x, si));
        }
      }
      double* Lc = loc + (size_t)(k0 + j0 + j) * nc * 2;
      Lc[2 * q] += sr;
      Lc[2 * q + 1] += si;
    }
  }
}

// reciprocal square root to full FP64 accuracy: hardware estimate + 2 Newton steps
__device__ __forceinline__ double rsqrt_d(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

// L2P: the local expansion L shifted to offset (X, Y, Z) from its centre;
// harmonics built column by column and each used once.
__device__ __forceinline__ void l2p_eval(int p, const double* __restrict__ L, double X, double Y,
                                         double Z, double& ax, double& ay, double& az, double& ph) {
  double r2 = fma(X, X, fma(Y, Y, Z * Z));
  double s00 = 0.0, s10 = 0.0, s11r = 0.0, s11i = 0.0;
  double dr = 1.0, di = 0.0;  // Y_m^m
  for (int m = 0; m <= p; m++) {
    if (m > 0) {
      double inv = -1.0 / (double)(2 * m);
      double tr = fma(X, dr, -Y * di), ti = fma(X, di, Y * dr);
      dr = tr * inv;
      di = ti * inv;
    }
    double yr = dr, yi2 = di, pr2 = 0.0, pi2 = 0.0;
    for (int k = m; k <= p; k++) {
      if (k > m) {
        double kk = (double)(2 * k - 1) * Z, inv = 1.0 / (double)((k + m) * (k - m));
        double vr = fma(kk, yr, -r2 * pr2) * inv, vi = fma(kk, yi2, -r2 * pi2) * inv;
        pr2 = yr;
        pi2 = yi2;
        yr = vr;
        yi2 = vi;
      }
      // Y_k^m = (yr, yi2); contributions of the +m and -m terms
      double w = m == 0 ? 1.0 : 2.0;
      double Lr = L[2 * cidx(k, m)], Li = L[2 * cidx(k, m) + 1];
      s00 = fma(w, fma(Lr, yr, Li * yi2), s00);
      if (k + 1 <= p) {
        double Ur = L[2 * cidx(k + 1, m)], Ui = L[2 * cidx(k + 1, m) + 1];
        s10 = fma(w, fma(Ur, yr, Ui * yi2), s10);
        // + L_{k+1}^{m+1} conj(Y_k^m)
        double Vr = L[2 * cidx(k + 1, m + 1)], Vi = L[2 * cidx(k + 1, m + 1) + 1];
        s11r = fma(Vr, yr, fma(Vi, yi2, s11r));
        s11i = fma(Vi, yr, fma(-Vr, yi2, s11i));
        if (m >= 2) {  // the -m term: -conj(L_{k+1}^{m-1}) Y_k^m
          double Wr = L[2 * cidx(k + 1, m - 1)], Wi = L[2 * cidx(k + 1, m - 1) + 1];
          s11r = fma(-Wr, yr, fma(-Wi, yi2, s11r));
          s11i = fma(-Wr, yi2, fma(Wi, yr, s11i));
        } else if (m == 1) {  // the -1 term: -L_{k+1}^0 Y_k^1
          double Wr = L[2 * cidx(k + 1, 0)], Wi = L[2 * cidx(k + 1, 0) + 1];
          s11r = fma(-Wr, yr, fma(Wi, yi2, s11r));
          s11i = fma(-Wr, yi2, fma(-Wi, yr, s11i));
        }
      }
    }
  }
  ax = -s11r;
  ay = -s11i;
  az = s10;
  ph = -s00;
}

// P2P, one wavefront per sink leaf.  The n_B sink bodies are replicated over
// G = 64 / n_B lane groups, and group g takes every G-th body of each source
// leaf, so nearly every lane works even though leaves hold ~20 bodies.  Each
// source leaf is staged once in LDS with one coalesced load and read by the
// groups as broadcasts.  The G partial sums are combined in group order
// (deterministic) into the body's near-field (acc, pot), sorted order.
// MIXED: pair arithmetic in FP32 on the separation formed in FP64 and rounded
// once; FP32 partial sums are carried into FP64 after every source leaf
// (blocked compensation: the FP32 error grows with the leaf, not the list).
// one source body s (mass ms) acting on the sink me
__device__ __forceinline__ void pair32(const double4& s, float ms, const double4& me, float eps2f, float& fx,
                                       float& fy, float& fz, float& fp) {
  float dx = (float)(s.x - me.x), dy = (float)(s.y - me.y), dz = (float)(s.z - me.z);
  float d2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2f)));
  float rinv = __builtin_amdgcn_rsqf(d2);
  rinv = d2 > 0.f ? rinv : 0.f;
  float mr = ms * rinv;
  float mr3 = mr * rinv * rinv;
  fx = fmaf(mr3, dx, fx);
  fy = fmaf(mr3, dy, fy);
  fz = fmaf(mr3, dz, fz);
  fp -= mr;
}

__device__ __forceinline__ void pair64(const double4& s, double ms, const double4& me, double eps2, double& nx,
                                       double& ny, double& nz, double& np) {
  double dx = s.x - me.x, dy = s.y - me.y, dz = s.z - me.z;
  double d2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
  double rinv = rsqrt_d(d2);
  rinv = d2 > 0.0 ? rinv : 0.0;
  double mr = ms * rinv;
  double mr3 = mr * rinv * rinv;
  nx = fma(mr3, dx, nx);
  ny = fma(mr3, dy, ny);
  nz = fma(mr3, dz, nz);
  np -= mr;
}

// staged source record: FP64 position; in mixed mode the mass is rounded to
// FP32 once here and kept in the low word of .w
template <bool MIXED>
__device__ __forceinline__ double4 stage(double4 v) {
  if constexpr (MIXED) v.w = __longlong_as_double((long long)__float_as_uint((float)v.w));
  return v;
}

__device__ __forceinline__ float mass32(const double4& v) {
  return __uint_as_float((unsigned)__double_as_longlong(v.w));
}

// Occupancy: 6 waves per SIMD for the FP32 pair loop (<= 80 VGPRs), 5 for the
// FP64 one (measured best for each; the FP64 loop at 6 is slower), with the
// sink leaf's data wave-uniform (SGPRs).
constexpr int LG_WAVES = 4;

template <bool MIXED>
__global__ void __launch_bounds__(64 * LG_WAVES) __attribute__((amdgpu_waves_per_eu(MIXED ? 6 : 5))) k_leaf_group(const int* __restrict__ leaves,
                                                              NfPlan plan, const int* __restrict__ cb,
                                                              const int* __restrict__ ce,
                                                              const int* __restrict__ off,
                                                              const int* __restrict__ srcl,
                                                              const double4* __restrict__ pm,
                                                              double eps2, double4* nearbuf,
                                                              double4* __restrict__ part,
                                                              unsigned long long* npairs, int gmax) {
  __shared__ double4 sbuf[LG_WAVES][64];
  __shared__ double rbuf[LG_WAVES][4][64];
  int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  int nblk = (plan.max_items + LG_WAVES - 1) / LG_WAVES;
  int blk = xcd_block();
  int it = blk * LG_WAVES + wv;
  if (blk >= nblk || it >= plan.max_items) return;
  int li = it, seg = 0;
  if (it >= plan.nleaf) {  // a later segment of a long list
    int x = it - plan.nleaf;
    if (x >= *plan.nextra) return;
    int2 v = plan.extra[x];
    li = v.x;
    seg = v.y;
  }
  int B = leaves[li];
  int nseg = plan.cell_nseg[B];
  int b = cb[B], e = ce[B];
  int qb = off[B], qe = off[B + 1];
  if (nseg > 1) {  // one segment of a long list (the leaf's bodies fit one wavefront)
    qb += seg * plan.K;
    qe = min(qe, qb + plan.K);
  }
  // output: the near field itself (a whole list, or the first segment of a
  // long one), or the partial sums of a later segment
  bool to_part = seg > 0;
  int64_t pslot = to_part ? (int64_t)plan.cell_pbase[B] + (int64_t)(seg - 1) * (e - b) - b : 0;
  float eps2f = (float)eps2;
  long long pairs = 0;  // body pairs of this leaf (self pairs excluded), wave-uniform
  for (int i0 = b; i0 < e; i0 += 64) {
    int nB = min(64, e - i0);
    int G = 64 / nB;
    if (gmax > 0 && G > gmax) G = gmax;  // fewer groups: longer runs per lane, fewer partial sums
    int g = lane / nB, s = lane - g * nB;
    bool act = g < G;
    int i = i0 + s;
    double4 me = pm[i];
    double nx = 0.0, ny = 0.0, nz = 0.0, np = 0.0;
    float fx = 0.f, fy = 0.f, fz = 0.f, fp = 0.f;
    // source chunks (<= 64 bodies of one source leaf) in list order; the
    // next chunk is fetched into registers while the current one is summed
    int q = qb, j0 = 0, je = 0;
    if (q < qe) {
      int A = srcl[q];
      j0 = cb[A];
      je = ce[A];
    }
    double4 cur = make_double4(0.0, 0.0, 0.0, 0.0);
    if (q < qe && lane < je - j0) cur = stage<MIXED>(pm[j0 + lane]);
    while (q < qe) {
      int na = min(64, je - j0);
      pairs += (long long)nB * na - max(0, min(i0 + nB, j0 + na) - max(i0, j0));
      int nq = q, nj0 = j0 + 64, nje = je;
      if (nj0 >= je) {
        nq = q + 1;
        if (nq < qe) {
          int A = srcl[nq];
          nj0 = cb[A];
          nje = ce[A];
        }
      }
      __builtin_amdgcn_wave_barrier();
      sbuf[wv][lane] = cur;
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the staged chunk is visible to the wave
      cur = make_double4(0.0, 0.0, 0.0, 0.0);
      if (nq < qe && lane < nje - nj0) cur = stage<MIXED>(pm[nj0 + lane]);
      int tmax = act ? na : 0;
      // the sink's own leaf: its pair with itself gets mass 0 (with eps = 0
      // the d2 > 0 test also removes it); other chunks hold no sink body
      bool self = j0 < i0 + nB && i0 < j0 + na;
      if (self) {
        int ti = i - j0;
        for (int t = g; t < tmax; t += G) {
          double4 sb = sbuf[wv][t];
          if constexpr (MIXED)
            pair32(sb, t != ti ? mass32(sb) : 0.f, me, eps2f, fx, fy, fz, fp);
          else
            pair64(sb, t != ti ? sb.w : 0.0, me, eps2, nx, ny, nz, np);
        }
      } else {
        int t = g;
        if constexpr (MIXED) {
          for (; t + 3 * G < tmax; t += 4 * G) {
            double4 s0 = sbuf[wv][t], s1 = sbuf[wv][t + G], s2 = sbuf[wv][t + 2 * G], s3 = sbuf[wv][t + 3 * G];
            pair32(s0, mass32(s0), me, eps2f, fx, fy, fz, fp);
            pair32(s1, mass32(s1), me, eps2f, fx, fy, fz, fp);
            pair32(s2, mass32(s2), me, eps2f, fx, fy, fz, fp);
            pair32(s3, mass32(s3), me, eps2f, fx, fy, fz, fp);
          }
        }
        for (; t + G < tmax; t += 2 * G) {
          double4 s0 = sbuf[wv][t], s1 = sbuf[wv][t + G];
          if constexpr (MIXED) {
            pair32(s0, mass32(s0), me, eps2f, fx, fy, fz, fp);
            pair32(s1, mass32(s1), me, eps2f, fx, fy, fz, fp);
          } else {
            pair64(s0, s0.w, me, eps2, nx, ny, nz, np);
            pair64(s1, s1.w, me, eps2, nx, ny, nz, np);
          }
        }
        if (t < tmax) {
          double4 s0 = sbuf[wv][t];
          if constexpr (MIXED)
            pair32(s0, mass32(s0), me, eps2f, fx, fy, fz, fp);
          else
            pair64(s0, s0.w, me, eps2, nx, ny, nz, np);
        }
      }
      if constexpr (MIXED) {
        if (nq != q) {  // end of a source leaf: carry the FP32 block into FP64
          nx += (double)fx;
          ny += (double)fy;
          nz += (double)fz;
          np += (double)fp;
          fx = fy = fz = fp = 0.f;
        }
      }
      q = nq;
      j0 = nj0;
      je = nje;
    }
    // combine the groups in order
    __builtin_amdgcn_wave_barrier();
    rbuf[wv][0][lane] = nx;
    rbuf[wv][1][lane] = ny;
    rbuf[wv][2][lane] = nz;
    rbuf[wv][3][lane] = np;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);
    if (g == 0) {
      double tx = 0.0, ty = 0.0, tz = 0.0, tp = 0.0;
      for (int gg = 0; gg < G; gg++) {
        int l = gg * nB + s;
        tx += rbuf[wv][0][l];
        ty += rbuf[wv][1][l];
        tz += rbuf[wv][2][l];
        tp += rbuf[wv][3][l];
      }
      if (to_part)
        part[pslot + i] = make_double4(tx, ty, tz, tp);
      else
        nearbuf[i] = make_double4(tx, ty, tz, tp);
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (lane == 0 && pairs > 0) atomicAdd(npairs, (unsigned long long)pairs);
}

// Near-field work items (the plan above), one thread per leaf; ctr[0] counts
// the extra items and ctr[1] the partial slots (both zero on entry).
constexpr int NF_SEG_MIN = 256;    // list entries per segment, at least
constexpr int NF_SEG_DIV = 8192;   // and at least the list total / NF_SEG_DIV

__global__ void k_nf_plan(const int* __restrict__ leaves, int nleaf, const int* __restrict__ cb,
                          const int* __restrict__ ce, const int* __restrict__ off, int K, int* cell_nseg,
                          int* cell_pbase, int2* extra, int* ctr) {
  int li = blockIdx.x * blockDim.x + threadIdx.x;
  if (li >= nleaf) return;
  int B = leaves[li];
  int len = off[B + 1] - off[B], nB = ce[B] - cb[B];
  int ns = (nB <= 64 && len > K) ? (len + K - 1) / K : 1;
  cell_nseg[B] = ns;
  if (ns > 1) {
    int x = atomicAdd(ctr, ns - 1);
    for (int k = 1; k < ns; k++) extra[x + k - 1] = make_int2(li, k);
    cell_pbase[B] = atomicAdd(ctr + 1, (ns - 1) * nB);
  }
}

// the partial sums of segments 1..ns-1 of split leaves added, in segment
// order, to the first segment's sums
__global__ void k_nf_combine(int64_t n, const int* __restrict__ leaf_of, const int* __restrict__ cb,
                             const int* __restrict__ ce, const int* __restrict__ cell_nseg,
                             const int* __restrict__ cell_pbase, const double4* __restrict__ part,
                             double4* nearbuf) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int B = leaf_of[i];
  int ns = cell_nseg[B];
  if (ns <= 1) return;
  int nB = ce[B] - cb[B];
  const double4* pp = part + cell_pbase[B] + (i - cb[B]);
  double4 t = nearbuf[i];
  for (int k = 1; k < ns; k++) {
    double4 v = pp[(size_t)(k - 1) * nB];
    t.x += v.x;
    t.y += v.y;
    t.z += v.z;
    t.w += v.w;
  }
  nearbuf[i] = t;
}

// Builds c.nf for the current leaves and near-field list (on c.stream; the
// counters at c.counters[44..45] are cleared by the caller).
void plan_near_field(Ctx& c) {
  int nleaf = (int)c.nleaf;
  int64_t cnt = c.p2p.count;
  int K = (int)std::max<int64_t>(NF_SEG_MIN, ceil_div(cnt, NF_SEG_DIV));
  // a split leaf holds len > K entries in ceil(len / K) < 2 len / K items, so
  // extra items number fewer than cnt / K <= NF_SEG_DIV; its partial slots,
  // (ceil(len / K) - 1) n_B < 64 len / K, fewer than 64 cnt / K in all
  int64_t extra_max = std::min<int64_t>(NF_SEG_DIV, ceil_div(cnt, K));
  int64_t slot_max = std::min<int64_t>(64 * (int64_t)NF_SEG_DIV, ceil_div(64 * cnt, K));
  ensure(c.ws, c.nf_cell_nseg, (size_t)c.ncell);
  ensure(c.ws, c.nf_cell_pbase, (size_t)c.ncell);
  ensure(c.ws, c.nf_extra, (size_t)extra_max + 1);
  ensure(c.ws, c.nf_part, (size_t)slot_max + 1);
  int* ctr = c.counters.p + 44;
  hipLaunchKernelGGL(k_nf_plan, dim3((unsigned)ceil_div(nleaf, 256)), dim3(256), 0, c.stream, c.leaves.p, nleaf,
                     c.c_begin.p, c.c_end.p, c.p2p.off.p, K, c.nf_cell_nseg.p, c.nf_cell_pbase.p, c.nf_extra.p,
                     ctr);
  HIPCHK(hipGetLastError());
  c.nf = NfPlan{c.nf_cell_nseg.p, c.nf_cell_pbase.p, c.nf_extra.p, ctr, nleaf, K, (int)(nleaf + extra_max),
                (int)slot_max};
}

// Near field of every body into c.nearbuf (sorted order), on c.stream.
void launch_near_field(Ctx& c) {
  if (c.nleaf <= 0) return;
  ensure(c.ws, c.nearbuf, (size_t)c.n);
  const int* leaves = c.leaves.p;
  // body-pair count of the near field, read by fmm_stats
  // counters[40..41]: the body-pair count; [44], [45]: the plan's counts
  unsigned long long* npairs = (unsigned long long*)(c.counters.p + 40);
  zero_fill(c, npairs, 6 * sizeof(int));
  plan_near_field(c);
  int nblk = (c.nf.max_items + LG_WAVES - 1) / LG_WAVES;
  unsigned grid = xcd_grid(nblk);
  double e2 = c.eps_soft * c.eps_soft;
  int gmax = c.prm.p2p_groups;
  if (c.prm.precision == FMM_MIXED)
    hipLaunchKernelGGL(k_leaf_group<true>, dim3(grid), dim3(64 * LG_WAVES), 0, c.stream, leaves, c.nf,
                       c.c_begin.p, c.c_end.p, c.p2p.off.p, c.p2p.src.p, c.pm.p, e2, c.nearbuf.p,
                       c.nf_part.p, npairs, gmax);
  else
    hipLaunchKernelGGL(k_leaf_group<false>, dim3(grid), dim3(64 * LG_WAVES), 0, c.stream, leaves, c.nf,
                       c.c_begin.p, c.c_end.p, c.p2p.off.p, c.p2p.src.p, c.pm.p, e2, c.nearbuf.p,
                       c.nf_part.p, npairs, gmax);
  HIPCHK(hipGetLastError());
  if (c.nf.max_slots > 0) {
    hipLaunchKernelGGL(k_nf_combine, dim3((unsigned)ceil_div(c.n, 256)), dim3(256), 0, c.stream, c.n,
                       c.leaf_of.p, c.c_begin.p, c.c_end.p, c.nf_cell_nseg.p, c.nf_cell_pbase.p, c.nf_part.p,
                       c.nearbuf.p);
    HIPCHK(hipGetLastError());
  }
}

// Far field by L2P (the leaf's local expansion shifted to the body:
// Phi = -Re L'_0^0, a = (-Re L'_1^1, -Im L'_1^1, Re L'_1^0)) plus the near
// field, summed in FP64 and written in the caller's order; one thread per body.
__global__ void __launch_bounds__(256) k_far_final(int p, int64_t n, const int* __restrict__ leaf_of,
                                                   const double* __restrict__ cx, const double* __restrict__ cy,
                                                   const double* __restrict__ cz, const double* __restrict__ loc,
                                                   const double4* __restrict__ pm,
                                                   const double4* __restrict__ nearbuf,
                                                   const int* __restrict__ perm, double* acc, double* pot) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int B = leaf_of[i];
  double4 me = pm[i], nf = nearbuf[i];
  double ax, ay, az, ph;
  l2p_eval(p, loc + (size_t)B * ncoef(p) * 2, me.x - cx[B], me.y - cy[B], me.z - cz[B], ax, ay, az, ph);
  int64_t o = perm[i];
  acc[3 * o] = ax + nf.x;
  acc[3 * o + 1] = ay + nf.y;
  acc[3 * o + 2] = az + nf.z;
  pot[o] = ph + nf.w;
}

void launch_far_final(Ctx& c, double* acc, double* pot) {
  hipLaunchKernelGGL(k_far_final, dim3((unsigned)ceil_div(c.n, 256)), dim3(256), 0, c.stream, c.p, c.n,
                     c.leaf_of.p, c.c_cx.p, c.c_cy.p, c.c_cz.p, c.loc.p, c.pm.p, c.nearbuf.p, c.idx[0].p,
                     acc, pot);
  HIPCHK(hipGetLastError());
}

void launch_l2l(Ctx& c) { launch_l2l_buf(c, c.loc.p); }

void launch_l2l_buf(Ctx& c, double* loc) {
  size_t S = (size_t)(c.p + 1) * (c.p + 1);
  int G = sizeof(double2) * 9 * S <= 64 * 1024 ? 8 : 1;  // children per pass within 64 KB of LDS
  size_t lds = sizeof(double2) * (1 + G) * S;
  for (int level = 0; level < c.depth; level++) {  // parents at this level, children one below
    int first = c.lvl_first[level], count = c.lvl_count[level];
    hipLaunchKernelGGL(k_l2l, dim3(count), dim3(L2L_T), lds, c.stream, c.p, first, count, c.c_child0.p,
                       c.c_nchild.p, c.c_cx.p, c.c_cy.p, c.c_cz.p, loc, G);
  }
  HIPCHK(hipGetLastError());
}

// ---- plain direct sum (FP64, compensated accumulation), LDS source tiles
constexpr int DS_T = 256;

__device__ __forceinline__ void two_sum_acc(double& s, double& c, double v) {
  double t = s + v;
  double bp = t - s;
  c += (s - (t - bp)) + (v - bp);
  s = t;
}

__global__ void __launch_bounds__(DS_T) k_direct(int64_t n, const double* pos, const double* mass,
                                                 double eps2, int64_t nsink, const int32_t* sinks,
                                                 double* acc, double* pot) {
  __shared__ double tx[DS_T], ty[DS_T], tz[DS_T], tm[DS_T];
  int64_t s = (int64_t)blockIdx.x * DS_T + threadIdx.x;
  bool act = s < nsink;
  int64_t i = act ? (sinks ? sinks[s] : s) : 0;
  double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
  double ax = 0, cxx = 0, ay = 0, cyy = 0, az = 0, czz = 0, ph = 0, cph = 0;
  for (int64_t j0 = 0; j0 < n; j0 += DS_T) {
    int64_t j = j0 + threadIdx.x;
    if (j < n) {
      tx[threadIdx.x] = pos[3 * j];
      ty[threadIdx.x] = pos[3 * j + 1];
      tz[threadIdx.x] = pos[3 * j + 2];
      tm[threadIdx.x] = mass[j];
    }
    __syncthreads();
    int lim = (int)(n - j0 < DS_T ? n - j0 : DS_T);
    for (int t = 0; t < lim; t++) {
      double dx = tx[t] - xi, dy = ty[t] - yi, dz = tz[t] - zi;
      double d2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
      bool ok = (j0 + t != i) && d2 > 0.0;
      double rinv = ok ? 1.0 / sqrt(d2) : 0.0;
      double mr = tm[t] * rinv, mr3 = mr * rinv * rinv;
      two_sum_acc(ax, cxx, mr3 * dx);
      two_sum_acc(ay, cyy, mr3 * dy);
      two_sum_acc(az, czz, mr3 * dz);
      two_sum_acc(ph, cph, -mr);
    }
    __syncthreads();
  }
  if (act) {
    acc[3 * s] = ax + cxx;
    acc[3 * s + 1] = ay + cyy;
    acc[3 * s + 2] = az + czz;
    pot[s] = ph + cph;
  }
}

void direct_sum(int64_t n, const double* pos, const double* mass, double eps2, int64_t nsink,
                const int32_t* sinks, double* acc, double* pot, hipStream_t s) {
  hipLaunchKernelGGL(k_direct, dim3((unsigned)ceil_div(nsink, DS_T)), dim3(DS_T), 0, s, n, pos, mass,
                     eps2, nsink, sinks, acc, pot);
  HIPCHK(hipGetLastError());
}

// ---- input validation (optional): non-finite positions, negative / NaN masses
__global__ void k_check(const double* pos, const double* mass, int64_t n, int* bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool ok = isfinite(pos[3 * i]) && isfinite(pos[3 * i + 1]) && isfinite(pos[3 * i + 2]) &&
            isfinite(mass[i]) && mass[i] >= 0.0;
  if (!ok) atomicOr(bad, 1);
}

bool check_inputs_dev(Ctx& c, const double* pos, const double* mass, int64_t n) {
  ensure(c.ws, c.counters, 64);
  int* bad = c.counters.p + 32;
  HIPCHK(hipMemsetAsync(bad, 0, sizeof(int), c.stream));
  hipLaunchKernelGGL(k_check, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c.stream, pos, mass, n, bad);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(c.hbuf, bad, sizeof(int), hipMemcpyDeviceToHost, c.stream));
  HIPCHK(hipStreamSynchronize(c.stream));
  return ((int*)c.hbuf)[0] == 0;
}

}  // namespace fmm
