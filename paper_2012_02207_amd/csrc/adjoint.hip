// Adjoint of the force pass on gfx950: for a scalar L(acc, pot) with
// ga_k = dL/da_k and gp_k = dL/dpot_k, the gradients dL/dx_k and dL/dm_k.
//
// Differentiating the defining sums a_k = sum_j m_j u / s^3, pot_k =
// -sum_j m_j / s (u = x_j - x_k, s^2 = |u|^2 + eps^2) splits the gradient in
// two parts:
//   * sink side: the tidal tensor T_k = da_k/dx_k = -Hess Phi(x_k) applied to
//     ga_k, and -gp_k a_k;
//   * source side: body k moves the field every other body feels.  With
//     Psi(x) = sum_i [ga_i . (x - x_i) / s^3 - gp_i / s]  (the potential of
//     dipoles -ga_i and charges gp_i in the sign convention of the forward
//     pass), dL/dm_k = Psi(x_k) and the source part of dL/dx_k is m_k grad Psi(x_k).
// The far field of both uses the FMM of the forward pass on the same tree and
// interaction lists: Hess Phi from the forward local expansions shifted to the
// body (orders 2), and Psi by a second expansion pass whose multipoles hold
// the charges and dipoles (P2M of a dipole d is d . grad Y_n^m, from the ladder
// relations d/dz Y_n^m = Y_{n-1}^m, (d/dx + i d/dy) Y_n^m = Y_{n-1}^{m+1},
// (d/dx - i d/dy) Y_n^m = -Y_{n-1}^{m-1}), followed by the same M2M, M2L
// (FP64) and L2L.  The near field sums the softened pair terms directly.
//
// The jerk (da_k/dt along the motion, section 5) is the same operator:
// da_k/dt = T_k v_k + sum_j K(x_j - x_k) m_j v_j, the tidal tensor applied to
// the body's own velocity plus the field gradient of the dipoles m_j v_j.
#include <hip/hip_runtime.h>

#include "fmm_device.h"

namespace fmm {

// regular harmonics with fused multiply-adds into re/im at stride st
__device__ inline void regular_fma(int p, double x, double y, double z, double* re, double* im, int st) {
  double r2 = fma(x, x, fma(y, y, z * z));
  re[0] = 1.0;
  im[0] = 0.0;
  double pr = 1.0, pi = 0.0;
  for (int n = 1; n <= p; n++) {
    double inv = -1.0 / (double)(2 * n);
    double tr = fma(x, pr, -y * pi), ti = fma(x, pi, y * pr);
    pr = tr * inv;
    pi = ti * inv;
    re[cidx(n, n) * st] = pr;
    im[cidx(n, n) * st] = pi;
  }
  for (int m = 0; m < p; m++) {
    double ar2 = 0.0, ai2 = 0.0, ar1 = re[cidx(m, m) * st], ai1 = im[cidx(m, m) * st];
    for (int n = m + 1; n <= p; n++) {
      double k = (double)(2 * n - 1) * z, inv = 1.0 / (double)((n + m) * (n - m));
      double vr = fma(k, ar1, -r2 * ar2) * inv, vi = fma(k, ai1, -r2 * ai2) * inv;
      re[cidx(n, m) * st] = vr;
      im[cidx(n, m) * st] = vi;
      ar2 = ar1;
      ai2 = ai1;
      ar1 = vr;
      ai1 = vi;
    }
  }
}

// sorted copies: (ga, gp) and the forward acceleration
__global__ void k_adj_gather(int64_t n, const int* perm, const double* gacc, const double* gpot,
                             const double* acc, double4* gs, double4* as) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t o = perm[i];
  gs[i] = make_double4(gacc[3 * o], gacc[3 * o + 1], gacc[3 * o + 2], gpot ? gpot[o] : 0.0);
  as[i] = make_double4(acc[3 * o], acc[3 * o + 1], acc[3 * o + 2], 0.0);
}

// jerk: the tidal tensor acts on the body's velocity, the sources are the
// dipoles -m_j v_j (charge 0), so that grad Psi = sum_j K(x_j - x_k) m_j v_j
__global__ void k_jerk_gather(int64_t n, const int* perm, const double* vel, const double* mass,
                              double4* tv, double4* src) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t o = perm[i];
  double vx = vel[3 * o], vy = vel[3 * o + 1], vz = vel[3 * o + 2], m = mass[o];
  tv[i] = make_double4(vx, vy, vz, 0.0);
  src[i] = make_double4(m * vx, m * vy, m * vz, 0.0);
}

// P2M of charges q = gp and dipoles d = -ga at the leaf's centre:
// M_n^m = sum_i q_i Y_n^m + d_z Y_{n-1}^m + (d_x - i d_y)/2 Y_{n-1}^{m+1}
//                         - (d_x + i d_y)/2 Y_{n-1}^{m-1}     (at x_i - z)
constexpr int PA_T = 64, PA_LDS = 2048;  // doubles of harmonics per batch
constexpr int PA_PMAX = 30;                // highest order (swap tables exist up to 30)

__global__ void __launch_bounds__(PA_T) k_p2m_adj(int p, const int* leaves, int nleaves, const int* cb,
                                                  const int* ce, const double4* pm, const double4* gs,
                                                  const double* cx, const double* cy, const double* cz,
                                                  double* madj) {
  __shared__ double lds[PA_LDS];
  __shared__ double4 gsh[64];
  int li = blockIdx.x;
  if (li >= nleaves) return;
  int c = leaves[li];
  int nc = ncoef(p);
  int batch = min(64, PA_LDS / (2 * nc));
  double* yre = lds;
  double* yim = lds + nc * batch;
  int t = threadIdx.x;
  double x0 = cx[c], y0 = cy[c], z0 = cz[c];
  int b = cb[c], e = ce[c];
  constexpr int MAXK = (ncoef(PA_PMAX) + PA_T - 1) / PA_T;
  double acr[MAXK], aci[MAXK];
  for (int u = 0; u < MAXK; u++) acr[u] = aci[u] = 0.0;
  for (int i0 = b; i0 < e; i0 += batch) {
    int cnt = min(batch, e - i0);
    if (t < cnt) {
      double4 q = pm[i0 + t];
      regular_fma(p, q.x - x0, q.y - y0, q.z - z0, yre + t, yim + t, batch);
      gsh[t] = gs[i0 + t];
    }
    __syncthreads();
    for (int u = 0; u < MAXK; u++) {
      int k = t + PA_T * u;
      if (k >= nc) continue;
      int n = 0;
      while (cidx(n + 1, 0) <= k) n++;
      int m = k - cidx(n, 0);
      double sr = acr[u], si = aci[u];
      for (int j = 0; j < cnt; j++) {
        double4 g = gsh[j];
        double q = g.w, dx = -g.x, dy = -g.y, dz = -g.z;
        sr = fma(q, yre[k * batch + j], sr);
        si = fma(q, yim[k * batch + j], si);
        if (n >= 1) {
          if (m <= n - 1) {  // d_z Y_{n-1}^m
            sr = fma(dz, yre[cidx(n - 1, m) * batch + j], sr);
            si = fma(dz, yim[cidx(n - 1, m) * batch + j], si);
          }
          if (m + 1 <= n - 1) {  // (d_x - i d_y)/2 * Y_{n-1}^{m+1}
            double ar = yre[cidx(n - 1, m + 1) * batch + j], ai = yim[cidx(n - 1, m + 1) * batch + j];
            sr = fma(0.5 * dx, ar, fma(0.5 * dy, ai, sr));
            si = fma(0.5 * dx, ai, fma(-0.5 * dy, ar, si));
          }
          if (m - 1 <= n - 1) {  // -(d_x + i d_y)/2 * Y_{n-1}^{m-1}
            double ar, ai;
            if (m >= 1) {
              ar = yre[cidx(n - 1, m - 1) * batch + j];
              ai = yim[cidx(n - 1, m - 1) * batch + j];
            } else if (n - 1 >= 1) {  // Y^{-1} = -conj(Y^1)
              ar = -yre[cidx(n - 1, 1) * batch + j];
              ai = yim[cidx(n - 1, 1) * batch + j];
            } else {
              ar = ai = 0.0;
            }
            sr = fma(-0.5 * dx, ar, fma(0.5 * dy, ai, sr));
            si = fma(-0.5 * dx, ai, fma(-0.5 * dy, ar, si));
          }
        }
      }
      acr[u] = sr;
      aci[u] = si;
    }
    __syncthreads();
  }
  double* out = madj + (size_t)c * nc * 2;
  for (int u = 0; u < MAXK; u++) {
    int k = t + PA_T * u;
    if (k < nc) {
      out[2 * k] = acr[u];
      out[2 * k + 1] = aci[u];
    }
  }
}

// coefficient (n, q) of an expansion for either sign of q
__device__ __forceinline__ void lget(const double* L, int n, int q, double& a, double& b) {
  if (q >= 0) {
    a = L[2 * cidx(n, q)];
    b = L[2 * cidx(n, q) + 1];
  } else {
    double s = (q & 1) ? -1.0 : 1.0;
    a = s * L[2 * cidx(n, -q)];
    b = -s * L[2 * cidx(n, -q) + 1];
  }
}

// Low orders of the expansion L re-centred at offset (X, Y, Z):
// L'_j^i = sum_{k <= p-j} sum_l L_{j+k}^{i+l} conj(Y_k^l), for j in [J0, J1],
// i = 0..j, written to out[(j(j+1)/2 + i) - J0(J0+1)/2] (complex, re/im).
template <int J0, int J1>
__device__ inline void shift_low(int p, const double* L, double X, double Y, double Z, double* outr,
                                 double* outi) {
  constexpr int NT = (J1 + 1) * (J1 + 2) / 2 - J0 * (J0 + 1) / 2;
  for (int t = 0; t < NT; t++) outr[t] = outi[t] = 0.0;
  double r2 = fma(X, X, fma(Y, Y, Z * Z));
  double dr = 1.0, di = 0.0;  // Y_m^m
  for (int m = 0; m <= p; m++) {
    if (m > 0) {
      double inv = -1.0 / (double)(2 * m);
      double tr = fma(X, dr, -Y * di), ti = fma(X, di, Y * dr);
      dr = tr * inv;
      di = ti * inv;
    }
    double yr = dr, yi = di, pr = 0.0, pi = 0.0;
    double sg = (m & 1) ? -1.0 : 1.0;
    for (int k = m; k <= p - J0; k++) {
      if (k > m) {
        double kk = (double)(2 * k - 1) * Z, inv = 1.0 / (double)((k + m) * (k - m));
        double vr = fma(kk, yr, -r2 * pr) * inv, vi = fma(kk, yi, -r2 * pi) * inv;
        pr = yr;
        pi = yi;
        yr = vr;
        yi = vi;
      }
#pragma unroll
      for (int j = J0; j <= J1; j++) {
        if (j + k > p) continue;
#pragma unroll
        for (int i = 0; i <= j; i++) {
          int t = j * (j + 1) / 2 + i - J0 * (J0 + 1) / 2;
          double a, b;
          // l = +m: L_{j+k}^{i+m} conj(Y_k^m)
          lget(L, j + k, i + m, a, b);
          outr[t] = fma(a, yr, fma(b, yi, outr[t]));
          outi[t] = fma(b, yr, fma(-a, yi, outi[t]));
          if (m > 0) {  // l = -m: L_{j+k}^{i-m} (-1)^m Y_k^m
            lget(L, j + k, i - m, a, b);
            double cr = sg * yr, ci = sg * yi;
            outr[t] = fma(a, cr, fma(-b, ci, outr[t]));
            outi[t] = fma(a, ci, fma(b, cr, outi[t]));
          }
        }
      }
    }
  }
}

__device__ __forceinline__ double rsqrt_fp64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

// Near field of the gradient and jerk operators, one wavefront per work item of
// the forward near field's plan (a sink leaf, or one segment of a long list;
// the same layout as the forward near field): the leaf's bodies are replicated
// over G = 64 / n_B lane groups, group g takes every G-th body of each source
// leaf, whose positions and source records are staged in LDS by one coalesced
// load per chunk (the next chunk is fetched into registers while the current
// one is summed), and the G partial sums are combined in group order.
// Per sink k and source j (u = x_k - x_j, s^2 = |u|^2 + eps^2; the pair with
// itself and pairs with s = 0 contribute nothing):
//   Psi      += src_j.xyz . u / s^3 - src_j.w / s
//   grad Psi += src_j.xyz / s^3 + (src_j.w / s^3 - 3 (src_j.xyz . u) / s^5) u
//   tidal    += m_j [tv_k / s^3 - 3 (u . tv_k) u / s^5]
// written to out[2k] = (grad Psi, Psi) and out[2k+1] = (tidal, 0), or for a
// later segment of a split leaf to its partial slot (added by k_adj_combine).
constexpr int ADJ_WAVES = 4;

__device__ __forceinline__ void adj_pair(const double4& me, const double4& g, const double4& s,
                                         const double4& gj, bool use, double eps2, double& psi,
                                         double& px, double& py, double& pz, double& kx, double& ky,
                                         double& kz) {
  double ux = me.x - s.x, uy = me.y - s.y, uz = me.z - s.z;
  double s2 = fma(ux, ux, fma(uy, uy, fma(uz, uz, eps2)));
  double inv = rsqrt_fp64(s2);
  inv = (use && s2 > 0.0) ? inv : 0.0;
  double inv2 = inv * inv, inv3 = inv2 * inv, inv5 = inv3 * inv2;
  double ugj = fma(ux, gj.x, fma(uy, gj.y, uz * gj.z));
  psi = fma(ugj, inv3, fma(-gj.w, inv, psi));
  double c1 = -3.0 * ugj * inv5, c2 = gj.w * inv3;
  px = fma(gj.x, inv3, fma(c1 + c2, ux, px));
  py = fma(gj.y, inv3, fma(c1 + c2, uy, py));
  pz = fma(gj.z, inv3, fma(c1 + c2, uz, pz));
  double ug = fma(ux, g.x, fma(uy, g.y, uz * g.z));
  double w3 = s.w * inv3, w5 = -3.0 * s.w * ug * inv5;
  kx = fma(w3, g.x, fma(w5, ux, kx));
  ky = fma(w3, g.y, fma(w5, uy, ky));
  kz = fma(w3, g.z, fma(w5, uz, kz));
}

__global__ void __launch_bounds__(64 * ADJ_WAVES) k_adj_near(const int* __restrict__ leaves, NfPlan plan,
                                                           const int* __restrict__ cb, const int* __restrict__ ce,
                                                           const int* __restrict__ off,
                                                           const int* __restrict__ srcl,
                                                           const double4* __restrict__ pm,
                                                           const double4* __restrict__ tv,
                                                           const double4* __restrict__ src, double eps2,
                                                           double4* __restrict__ out,
                                                           double4* __restrict__ part) {
  __shared__ double4 spm[ADJ_WAVES][64];
  __shared__ double4 ssrc[ADJ_WAVES][64];
  __shared__ double rbuf[ADJ_WAVES][7][64];
  int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  int nblk = (plan.max_items + ADJ_WAVES - 1) / ADJ_WAVES;
  int blk = xcd_block();
  int it = blk * ADJ_WAVES + wv;
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
  bool to_part = seg > 0;  // later segments of a long list: partial slots
  int64_t pslot = to_part ? (int64_t)plan.cell_pbase[B] + (int64_t)(seg - 1) * (e - b) - b : 0;
  for (int i0 = b; i0 < e; i0 += 64) {
    int nB = min(64, e - i0);
    int G = 64 / nB;
    int g = lane / nB, sl = lane - g * nB;
    bool act = g < G;
    int i = i0 + sl;
    double4 me = pm[i], gk = tv[i];
    double psi = 0.0, px = 0.0, py = 0.0, pz = 0.0, kx = 0.0, ky = 0.0, kz = 0.0;
    int q = qb, j0 = 0, je = 0;
    if (q < qe) {
      int A = srcl[q];
      j0 = cb[A];
      je = ce[A];
    }
    double4 cpm = make_double4(0.0, 0.0, 0.0, 0.0), csrc = cpm;
    if (q < qe && lane < je - j0) {
      cpm = pm[j0 + lane];
      csrc = src[j0 + lane];
    }
    while (q < qe) {
      int na = min(64, je - j0);
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
      spm[wv][lane] = cpm;
      ssrc[wv][lane] = csrc;
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): the staged chunk is visible to the wave
      if (nq < qe && lane < nje - nj0) {
        cpm = pm[nj0 + lane];
        csrc = src[nj0 + lane];
      }
      int tmax = act ? na : 0;
      int ti = i - j0;  // the sink's own slot when this chunk holds it
      for (int t = g; t < tmax; t += G)
        adj_pair(me, gk, spm[wv][t], ssrc[wv][t], t != ti, eps2, psi, px, py, pz, kx, ky, kz);
      q = nq;
      j0 = nj0;
      je = nje;
    }
    __builtin_amdgcn_wave_barrier();
    rbuf[wv][0][lane] = px;
    rbuf[wv][1][lane] = py;
    rbuf[wv][2][lane] = pz;
    rbuf[wv][3][lane] = psi;
    rbuf[wv][4][lane] = kx;
    rbuf[wv][5][lane] = ky;
    rbuf[wv][6][lane] = kz;
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);
    if (g == 0) {
      double t[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      for (int gg = 0; gg < G; gg++) {
        int l = gg * nB + sl;
#pragma unroll
        for (int r = 0; r < 7; r++) t[r] += rbuf[wv][r][l];
      }
      double4* dst = to_part ? part + 2 * (pslot + i) : out + 2 * (int64_t)i;
      dst[0] = make_double4(t[0], t[1], t[2], t[3]);
      dst[1] = make_double4(t[4], t[5], t[6], 0.0);
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// the partial sums of segments 1..ns-1 of split leaves added, in segment
// order, to the first segment's sums
__global__ void k_adj_combine(int64_t n, const int* __restrict__ leaf_of, const int* __restrict__ cb,
                              const int* __restrict__ ce, const int* __restrict__ cell_nseg,
                              const int* __restrict__ cell_pbase, const double4* __restrict__ part,
                              double4* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int B = leaf_of[i];
  int ns = cell_nseg[B];
  if (ns <= 1) return;
  int nB = ce[B] - cb[B];
  const double4* pp = part + 2 * ((int64_t)cell_pbase[B] + (i - cb[B]));
  double4 a = out[2 * i], b = out[2 * i + 1];
  for (int k = 1; k < ns; k++) {
    const double4* q = pp + 2 * (int64_t)(k - 1) * nB;
    double4 u = q[0], v = q[1];
    a.x += u.x;
    a.y += u.y;
    a.z += u.z;
    a.w += u.w;
    b.x += v.x;
    b.y += v.y;
    b.z += v.z;
  }
  out[2 * i] = a;
  out[2 * i + 1] = b;
}

// One thread per body (sorted order); results in the caller's order.
// tv[i]: the vector the tidal tensor acts on (ga_i; in the jerk, v_i) and
// gp_i in .w; near[2i], near[2i+1]: the near sums of k_adj_near.
//   gradient: gpos = T ga - gp a + m grad Psi,  gmass = Psi;
//   jerk:     jerk = T v + grad Psi.
template <bool JERK>
__global__ void __launch_bounds__(256) k_adj_leaf(int p, int64_t n, const int* __restrict__ leaf_of,
                                                  const double* __restrict__ cx, const double* __restrict__ cy,
                                                  const double* __restrict__ cz,
                                                  const double* __restrict__ lfwd,
                                                  const double* __restrict__ ladj,
                                                  const double4* __restrict__ pm,
                                                  const double4* __restrict__ tv,
                                                  const double4* __restrict__ near,
                                                  const double4* __restrict__ as,
                                                  const int* __restrict__ perm, double* gpos,
                                                  double* gmass) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int B = leaf_of[i];
  int nc = ncoef(p);
  double4 me = pm[i], g = tv[i];
  double X = me.x - cx[B], Y = me.y - cy[B], Z = me.z - cz[B];
  // far field: Hess Phi from the forward expansion (order 2), Psi and grad Psi
  // from the adjoint expansion (orders 0, 1)
  double hr[3], hi[3], ar[3], ai[3];
  shift_low<2, 2>(p, lfwd + (size_t)B * nc * 2, X, Y, Z, hr, hi);
  shift_low<0, 1>(p, ladj + (size_t)B * nc * 2, X, Y, Z, ar, ai);
  // Phi_2 = -Re[conj(A) Y_2^0 + 2 conj(B) Y_2^1 + 2 conj(C) Y_2^2]
  double Hxx = 0.5 * hr[0] - 0.5 * hr[2], Hyy = 0.5 * hr[0] + 0.5 * hr[2], Hzz = -hr[0];
  double Hxy = -0.5 * hi[2], Hxz = hr[1], Hyz = hi[1];
  double gx = -(Hxx * g.x + Hxy * g.y + Hxz * g.z);
  double gy = -(Hxy * g.x + Hyy * g.y + Hyz * g.z);
  double gz = -(Hxz * g.x + Hyz * g.y + Hzz * g.z);
  double4 na = near[2 * i], nb = near[2 * i + 1];
  double psi = -ar[0] + na.w;
  double px = ar[2] + na.x, py = ai[2] + na.y, pz = -ar[1] + na.z;
  double kx = nb.x, ky = nb.y, kz = nb.z;
  int64_t o = perm[i];
  if constexpr (JERK) {
    gpos[3 * o] = gx - kx + px;
    gpos[3 * o + 1] = gy - ky + py;
    gpos[3 * o + 2] = gz - kz + pz;
  } else {
    double4 af = as[i];
    gpos[3 * o] = gx - kx - g.w * af.x + me.w * px;
    gpos[3 * o + 1] = gy - ky - g.w * af.y + me.w * py;
    gpos[3 * o + 2] = gz - kz - g.w * af.z + me.w * pz;
    gmass[o] = psi;
  }
}

// the expansion pass over the sources src (dipoles -xyz, charges w) and the
// leaf evaluation; the forward pass (tree, lists, local expansions) must be
// in place
template <bool JERK>
static void source_pass(Ctx& c, const double4* tv, const double4* src, const double4* as, double* out3,
                        double* out1) {
  hipStream_t s = c.stream;
  int64_t n = c.n;
  int nc = (int)c.ncell;
  size_t ne = (size_t)nc * ncoef(c.p) * 2;
  ensure(c.ws, c.madj, ne);
  ensure(c.ws, c.ladj, ne);
  unsigned g = (unsigned)ceil_div(n, 256);
  hipLaunchKernelGGL(k_p2m_adj, dim3((unsigned)c.nleaf), dim3(PA_T), 0, s, c.p, c.leaves.p, (int)c.nleaf,
                     c.c_begin.p, c.c_end.p, c.pm.p, src, c.c_cx.p, c.c_cy.p, c.c_cz.p, c.madj.p);
  HIPCHK(hipGetLastError());
  m2m_levels(c, c.madj.p);
  HIPCHK(hipMemsetAsync(c.ladj.p, 0, ne * sizeof(double), s));
  launch_m2l_fp64_buffers(c, nc, c.madj.p, c.ladj.p);
  launch_l2l_buf(c, c.ladj.p);
  // the work items of the forward near field of this evaluation
  ensure(c.ws, c.adjnear, 2 * (size_t)n);
  ensure(c.ws, c.adjpart, 2 * (size_t)c.nf.max_slots + 2);
  int nblk = (c.nf.max_items + ADJ_WAVES - 1) / ADJ_WAVES;
  hipLaunchKernelGGL(k_adj_near, dim3(xcd_grid(nblk)), dim3(64 * ADJ_WAVES), 0, s, c.leaves.p, c.nf,
                     c.c_begin.p, c.c_end.p, c.p2p.off.p, c.p2p.src.p, c.pm.p, tv, src,
                     c.eps_soft * c.eps_soft, c.adjnear.p, c.adjpart.p);
  HIPCHK(hipGetLastError());
  if (c.nf.max_slots > 0) {
    hipLaunchKernelGGL(k_adj_combine, dim3(g), dim3(256), 0, s, n, c.leaf_of.p, c.c_begin.p, c.c_end.p,
                       c.nf.cell_nseg, c.nf.cell_pbase, c.adjpart.p, c.adjnear.p);
    HIPCHK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_adj_leaf<JERK>, dim3(g), dim3(256), 0, s, c.p, n, c.leaf_of.p, c.c_cx.p, c.c_cy.p,
                     c.c_cz.p, c.loc.p, c.ladj.p, c.pm.p, tv, c.adjnear.p, as, c.idx[0].p, out3, out1);
  HIPCHK(hipGetLastError());
}

void adjoint_pass(Ctx& c, const double* gacc, const double* gpot, const double* acc_fwd, double* gpos,
                  double* gmass) {
  int64_t n = c.n;
  ensure(c.ws, c.gsort, (size_t)n);
  ensure(c.ws, c.asort, (size_t)n);
  hipLaunchKernelGGL(k_adj_gather, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c.stream, n, c.idx[0].p,
                     gacc, gpot, acc_fwd, c.gsort.p, c.asort.p);
  source_pass<false>(c, c.gsort.p, c.gsort.p, c.asort.p, gpos, gmass);
}

void jerk_pass(Ctx& c, const double* vel, const double* mass, double* jerk) {
  int64_t n = c.n;
  ensure(c.ws, c.gsort, (size_t)n);
  ensure(c.ws, c.asort, (size_t)n);
  hipLaunchKernelGGL(k_jerk_gather, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c.stream, n, c.idx[0].p,
                     vel, mass, c.gsort.p, c.asort.p);
  source_pass<true>(c, c.gsort.p, c.asort.p, nullptr, jerk, nullptr);
}

}  // namespace fmm
