/*
 * CPU oracle for the collisional FMM force evaluation -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain FP64 restatement, in the order the method runs, of the force pass of
 * Mukherjee et al. (2021), section 2 ("Taichi for Collisional Dynamics"):
 *   tree        -> octree over Morton-sorted bodies (section 2.1, Fig. 1 caption)
 *   upward      -> P2M and M2M in regular solid harmonics (section 2.2, eq. for M_n^m)
 *   estimate    -> scalar-force estimate f_i with a theta < 1 walk (section 2.3, eq. for f_i)
 *   walk        -> dual-tree walk with the error-controlled mutual MAC
 *                  (section 2.3, MAC equation, P_n and E_{A->B} equations)
 *   evaluation  -> rotation-accelerated M2L (section 2.4), L2L, L2P and direct P2P
 *                  for the near field (section 2.1)
 * plus the O(N^2) direct sum the method approximates (section 2.3, scalar-force
 * equation with its numerator; Plummer softening, appendix on softening).
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp (no fast-math).  Everything that
 * feeds the acceptance test is computed sequentially in a fixed order, so the
 * results do not depend on the OpenMP thread count: threads only split outputs.
 *
 * Readings where the paper is silent (tree construction, key layout, walk
 * split rule, harmonic normalisation, tie-breaks) are stated beside the code.
 */
#include "fmm_oracle.h"
#include "orc_tables.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NCOEF(p) (((p) + 1) * ((p) + 2) / 2)
#define CIDX(n, m) ((n) * ((n) + 1) / 2 + (m))
#define KEY_BITS 21
#define MAX_LEVEL 21

typedef struct {
  int64_t* a; /* flat (sink, source) */
  int64_t n;  /* number of pairs */
  int64_t cap;
} pairvec;

struct orc_ctx {
  int64_t n;
  int p, n_leaf, mac, m2l_kind;
  double err_tol, theta, theta_est, eps_soft;
  double rootbox[5];
  uint64_t* key;
  int64_t* perm;
  double* spos; /* sorted positions n x 3 */
  double* sm;   /* sorted masses */
  int64_t ncell, capcell;
  int32_t* level;
  int64_t *begin, *end, *parent, *child0;
  int32_t* nchild;
  double *mass, *com, *rad;
  double* mult; /* ncell x ncoef x 2 */
  double* pk;   /* ncell x (p+1) */
  double* fcell;
  double* fpart;
  double* fmin;
  double* loc;
  pairvec est_far, est_near, m2l, p2p;
};

static void pv_push(pairvec* v, int64_t sink, int64_t src) {
  if (v->n == v->cap) {
    v->cap = v->cap ? 2 * v->cap : 1024;
    v->a = (int64_t*)realloc(v->a, (size_t)v->cap * 2 * sizeof(int64_t));
  }
  v->a[2 * v->n] = sink;
  v->a[2 * v->n + 1] = src;
  v->n++;
}

static int cmp_pair(const void* x, const void* y) {
  const int64_t* a = (const int64_t*)x;
  const int64_t* b = (const int64_t*)y;
  if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
  if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;
  return 0;
}

/* sort directed pairs by (sink, source) and build CSR offsets over sinks */
static int64_t* pv_sort_csr(pairvec* v, int64_t ncell) {
  if (v->n) qsort(v->a, (size_t)v->n, 2 * sizeof(int64_t), cmp_pair);
  int64_t* off = (int64_t*)calloc((size_t)ncell + 1, sizeof(int64_t));
  for (int64_t k = 0; k < v->n; k++) off[v->a[2 * k] + 1]++;
  for (int64_t c = 0; c < ncell; c++) off[c + 1] += off[c];
  return off;
}

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

const double* orc_swap_table(int n) {
  if (n < 0 || n > ORC_PMAX) return NULL;
  int64_t off = (int64_t)n * (4 * (int64_t)n * n - 1) / 3;
  return orc_swap + off;
}
const double* orc_factorials(void) { return orc_fact; }

/* ------------------------------------------------------------------------ */
/* Solid harmonics (section 2.2).  Normalisation (reading of the cited
 * recurrences): Y_n^m = r^n P_n^m(cos t) e^{i m phi} / (n+m)!,
 * T_n^m = (n-m)! P_n^m(cos t) e^{i m phi} / r^{n+1}, Condon-Shortley phase,
 * Y_n^{-m} = (-1)^m conj(Y_n^m).  Under this choice 1/|x-y| = sum conj(Y(y)) T(x)
 * and the paper's P_n is rotation invariant.  The operation order below is
 * the canonical one (no contraction) because it feeds the acceptance test.   */
void orc_regular(int p, double x, double y, double z, double* re, double* im) {
  double r2 = (x * x + y * y) + z * z;
  re[0] = 1.0;
  im[0] = 0.0;
  for (int n = 1; n <= p; n++) {
    double pr = re[CIDX(n - 1, n - 1)], pi = im[CIDX(n - 1, n - 1)];
    double tr = x * pr - y * pi;
    double ti = x * pi + y * pr;
    double den = (double)(2 * n);
    re[CIDX(n, n)] = (-tr) / den;
    im[CIDX(n, n)] = (-ti) / den;
  }
  for (int m = 0; m < p; m++) {
    for (int n = m + 1; n <= p; n++) {
      double k = (double)(2 * n - 1) * z;
      double ar = k * re[CIDX(n - 1, m)];
      double ai = k * im[CIDX(n - 1, m)];
      double nr = ar, ni = ai;
      if (n - 2 >= m) {
        double br = r2 * re[CIDX(n - 2, m)];
        double bi = r2 * im[CIDX(n - 2, m)];
        nr = ar - br;
        ni = ai - bi;
      }
      double den = (double)((n + m) * (n - m));
      re[CIDX(n, m)] = nr / den;
      im[CIDX(n, m)] = ni / den;
    }
  }
}

void orc_irregular(int p, double x, double y, double z, double* re, double* im) {
  double r2 = (x * x + y * y) + z * z;
  re[0] = 1.0 / sqrt(r2);
  im[0] = 0.0;
  for (int n = 1; n <= p; n++) {
    double pr = re[CIDX(n - 1, n - 1)], pi = im[CIDX(n - 1, n - 1)];
    double tr = x * pr - y * pi;
    double ti = x * pi + y * pr;
    double k = -(double)(2 * n - 1) / r2;
    re[CIDX(n, n)] = k * tr;
    im[CIDX(n, n)] = k * ti;
  }
  for (int m = 0; m < p; m++) {
    for (int n = m + 1; n <= p; n++) {
      double k = (double)(2 * n - 1) * z;
      double nr = k * re[CIDX(n - 1, m)];
      double ni = k * im[CIDX(n - 1, m)];
      if (n - 2 >= m) {
        double c = (double)((n - 1) * (n - 1) - m * m);
        nr -= c * re[CIDX(n - 2, m)];
        ni -= c * im[CIDX(n - 2, m)];
      }
      re[CIDX(n, m)] = nr / r2;
      im[CIDX(n, m)] = ni / r2;
    }
  }
}

/* coefficient (n, m) for any sign of m from the m >= 0 storage */
static inline void cget(const double* re, const double* im, int n, int m, double* a, double* b) {
  if (m >= 0) {
    *a = re[CIDX(n, m)];
    *b = im[CIDX(n, m)];
  } else {
    double s = (m & 1) ? -1.0 : 1.0;
    *a = s * re[CIDX(n, -m)];
    *b = -s * im[CIDX(n, -m)];
  }
}

/* M2M (section 2.1): regular addition theorem, children shifted to the parent.
 * d = z_child - z_parent.  Loop order (n, m, k, l) with one running sum. */
static void m2m_accumulate(int p, const double* yre, const double* yim, const double* mre,
                           const double* mim, double* accre, double* accim) {
  for (int n = 0; n <= p; n++)
    for (int m = 0; m <= n; m++) {
      double sr = accre[CIDX(n, m)], si = accim[CIDX(n, m)];
      for (int k = 0; k <= n; k++)
        for (int l = -k; l <= k; l++) {
          int j = n - k, q = m - l;
          if (q > j || q < -j) continue;
          double ar, ai, br, bi;
          cget(yre, yim, k, l, &ar, &ai);
          cget(mre, mim, j, q, &br, &bi);
          double tr = ar * br - ai * bi;
          double ti = ar * bi + ai * br;
          sr = sr + tr;
          si = si + ti;
        }
      accre[CIDX(n, m)] = sr;
      accim[CIDX(n, m)] = si;
    }
}

void orc_m2m(int p, const double* mre, const double* mim, const double d[3], double* ore,
             double* oim) {
  int nc = NCOEF(p);
  double* yre = (double*)malloc(sizeof(double) * nc);
  double* yim = (double*)malloc(sizeof(double) * nc);
  orc_regular(p, d[0], d[1], d[2], yre, yim);
  for (int i = 0; i < nc; i++) ore[i] = oim[i] = 0.0;
  m2m_accumulate(p, yre, yim, mre, mim, ore, oim);
  free(yre);
  free(yim);
}

/* M2L, plain O(p^4) definition: the irregular addition theorem truncated at
 * total degree p,  L_n^m = (-1)^n sum_{k<=p-n} sum_l conj(M_k^l) T_{n+k}^{m+l}(R),
 * with the local field  Phi(x) = -sum conj(L_n^m) Y_n^m(x - z_B).  R = z_B - z_A. */
void orc_m2l_direct(int p, const double* mre, const double* mim, const double R[3],
                    double* lre, double* lim) {
  int nc2 = NCOEF(2 * p);
  double* tre = (double*)malloc(sizeof(double) * nc2);
  double* tim = (double*)malloc(sizeof(double) * nc2);
  orc_irregular(2 * p, R[0], R[1], R[2], tre, tim);
  for (int n = 0; n <= p; n++)
    for (int m = 0; m <= n; m++) {
      double sr = 0.0, si = 0.0;
      for (int k = 0; k <= p - n; k++)
        for (int l = -k; l <= k; l++) {
          double ar, ai, br, bi;
          cget(mre, mim, k, l, &ar, &ai);
          ai = -ai; /* conj(M) */
          cget(tre, tim, n + k, m + l, &br, &bi);
          sr += ar * br - ai * bi;
          si += ar * bi + ai * br;
        }
      double s = (n & 1) ? -1.0 : 1.0;
      lre[CIDX(n, m)] = s * sr;
      lim[CIDX(n, m)] = s * si;
    }
  free(tre);
  free(tim);
}

/* ---- rotation-accelerated M2L (section 2.4) ----------------------------- */
/* Real representation of order n: v[0] = Re c^0, v[2m-1] = Re c^m, v[2m] = Im c^m. */
static void zrot(int n, double* v, double ca, double sa) {
  double cm = 1.0, sm = 0.0;
  for (int m = 1; m <= n; m++) {
    double c2 = cm * ca - sm * sa;
    double s2 = sm * ca + cm * sa;
    cm = c2;
    sm = s2;
    double C = v[2 * m - 1], S = v[2 * m];
    v[2 * m - 1] = C * cm - S * sm;
    v[2 * m] = C * sm + S * cm;
  }
}

static void swap_apply(int n, double* v, double* tmp) {
  const double* W = orc_swap_table(n);
  int d = 2 * n + 1;
  for (int i = 0; i < d; i++) {
    double s = 0.0;
    for (int j = 0; j < d; j++) s += W[i * d + j] * v[j];
    tmp[i] = s;
  }
  memcpy(v, tmp, sizeof(double) * d);
}

/* The multipole is rotated by Q = S Rz(beta) S Rz(alpha) (S: swap x<->z) so that
 * R points along +z: alpha = pi/2 - phi, beta = -theta (phi, theta: azimuth and
 * polar angle of R).  Translation along z uses T_j^0(r z) = j!/r^{j+1} only.
 * Locals transform with the transpose of the multipole map; in the scaled basis
 * Lhat_n^m = L_n^m / ((n-m)!(n+m)!) that transpose is again S Rz S Rz with the
 * negated angles applied in reverse order. */
void orc_m2l_rotated(int p, const double* mre, const double* mim, const double R[3],
                     double* lre, double* lim) {
  int nr = (p + 1) * (p + 1);
  double* mu = (double*)calloc(nr, sizeof(double));  /* order n at offset n^2 */
  double* lam = (double*)calloc(nr, sizeof(double));
  double tmp[2 * ORC_PMAX + 1];
  double rho2 = R[0] * R[0] + R[1] * R[1];
  double r = sqrt(rho2 + R[2] * R[2]);
  double rho = sqrt(rho2);
  double ca, sa; /* alpha = pi/2 - phi */
  if (rho > 0.0) {
    ca = R[1] / rho;
    sa = R[0] / rho;
  } else {
    ca = 0.0;
    sa = 1.0;
  }
  double cb = R[2] / r, sb = -rho / r; /* beta = -theta */
  for (int n = 0; n <= p; n++) {
    double* v = mu + n * n;
    v[0] = mre[CIDX(n, 0)];
    for (int m = 1; m <= n; m++) {
      v[2 * m - 1] = mre[CIDX(n, m)];
      v[2 * m] = mim[CIDX(n, m)];
    }
    zrot(n, v, ca, sa);
    swap_apply(n, v, tmp);
    zrot(n, v, cb, sb);
    swap_apply(n, v, tmp);
  }
  /* translation along +z: L'_n^m = (-1)^(n+m) sum_{k=m}^{p-n} M'_k^m (n+k)!/r^(n+k+1) */
  double g[2 * ORC_PMAX + 2];
  double rinv = 1.0 / r, rp = rinv;
  for (int j = 0; j <= 2 * p; j++) {
    g[j] = orc_fact[j] * rp;
    rp *= rinv;
  }
  for (int n = 0; n <= p; n++) {
    double* w = lam + n * n;
    for (int m = 0; m <= n; m++) {
      double sr = 0.0, si = 0.0;
      for (int k = m; k <= p - n; k++) {
        double* v = mu + k * k;
        if (m == 0) {
          sr += v[0] * g[n + k];
        } else {
          sr += v[2 * m - 1] * g[n + k];
          si += v[2 * m] * g[n + k];
        }
      }
      double s = ((n + m) & 1) ? -1.0 : 1.0;
      double sc = 1.0 / (orc_fact[n - m] * orc_fact[n + m]);
      if (m == 0) {
        w[0] = s * sr * sc;
      } else {
        w[2 * m - 1] = s * sr * sc;
        w[2 * m] = s * si * sc;
      }
    }
    swap_apply(n, w, tmp);
    zrot(n, w, cb, -sb);
    swap_apply(n, w, tmp);
    zrot(n, w, ca, -sa);
    lre[CIDX(n, 0)] = w[0] * (orc_fact[n] * orc_fact[n]);
    lim[CIDX(n, 0)] = 0.0;
    for (int m = 1; m <= n; m++) {
      double f = orc_fact[n - m] * orc_fact[n + m];
      lre[CIDX(n, m)] = w[2 * m - 1] * f;
      lim[CIDX(n, m)] = w[2 * m] * f;
    }
  }
  free(mu);
  free(lam);
}

/* L2L (section 2.1): exact shift of the degree-p local polynomial,
 * L'_j^i = sum_{k<=p-j} sum_l L_{j+k}^{i+l} conj(Y_k^l(d)), d = z_child - z_parent. */
static void l2l_accumulate(int p, const double* lre, const double* lim, const double* yre,
                           const double* yim, double* ore, double* oim) {
  for (int j = 0; j <= p; j++)
    for (int i = 0; i <= j; i++) {
      double sr = 0.0, si = 0.0;
      for (int k = 0; k <= p - j; k++)
        for (int l = -k; l <= k; l++) {
          double ar, ai, br, bi;
          cget(lre, lim, j + k, i + l, &ar, &ai);
          cget(yre, yim, k, l, &br, &bi);
          bi = -bi;
          sr += ar * br - ai * bi;
          si += ar * bi + ai * br;
        }
      ore[CIDX(j, i)] += sr;
      oim[CIDX(j, i)] += si;
    }
}

void orc_l2l(int p, const double* lre, const double* lim, const double d[3], double* ore,
             double* oim) {
  int nc = NCOEF(p);
  double* yre = (double*)malloc(sizeof(double) * nc);
  double* yim = (double*)malloc(sizeof(double) * nc);
  orc_regular(p, d[0], d[1], d[2], yre, yim);
  for (int i = 0; i < nc; i++) ore[i] = oim[i] = 0.0;
  l2l_accumulate(p, lre, lim, yre, yim, ore, oim);
  free(yre);
  free(yim);
}

/* L2P (section 2.1): shift the local expansion to the body; the degree-0 term
 * is -Phi and the degree-1 terms give the gradient:
 * acc = (-Re L'_1^1, -Im L'_1^1, Re L'_1^0), Phi = -Re L'_0^0. */
static void l2p_eval(int p, const double* lre, const double* lim, const double* yre,
                     const double* yim, double* pot, double acc[3]) {
  double s00 = 0.0, s10 = 0.0, s11r = 0.0, s11i = 0.0;
  for (int k = 0; k <= p; k++)
    for (int l = -k; l <= k; l++) {
      double ar, ai, br, bi;
      cget(yre, yim, k, l, &br, &bi);
      bi = -bi;
      cget(lre, lim, k, l, &ar, &ai);
      s00 += ar * br - ai * bi;
      if (k + 1 <= p) {
        cget(lre, lim, k + 1, l, &ar, &ai);
        s10 += ar * br - ai * bi;
        cget(lre, lim, k + 1, l + 1, &ar, &ai);
        s11r += ar * br - ai * bi;
        s11i += ar * bi + ai * br;
      }
    }
  *pot = -s00;
  acc[0] = -s11r;
  acc[1] = -s11i;
  acc[2] = s10;
}

void orc_l2p(int p, const double* lre, const double* lim, const double X[3], double* pot,
             double acc[3]) {
  int nc = NCOEF(p);
  double* yre = (double*)malloc(sizeof(double) * nc);
  double* yim = (double*)malloc(sizeof(double) * nc);
  orc_regular(p, X[0], X[1], X[2], yre, yim);
  l2p_eval(p, lre, lim, yre, yim, pot, acc);
  free(yre);
  free(yim);
}

/* ------------------------------------------------------------------------ */
/* Direct summation (the plain definition the FMM approximates). */
static inline void neu_add(double* s, double* c, double v) {
  double t = *s + v;
  if (fabs(*s) >= fabs(v))
    *c += (*s - t) + v;
  else
    *c += (v - t) + *s;
  *s = t;
}

int orc_direct(int64_t n, const double* pos, const double* mass, double eps_soft, int64_t nsink,
               const int64_t* sinks, int compensated, double* acc, double* pot) {
  if (n < 1 || !pos || !mass || !acc || !pot || eps_soft < 0) return -1;
  if (!sinks) nsink = n;
  double e2 = eps_soft * eps_soft;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t s = 0; s < nsink; s++) {
    int64_t i = sinks ? sinks[s] : s;
    double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
    double sx[2] = {0, 0}, sy[2] = {0, 0}, sz[2] = {0, 0}, sp[2] = {0, 0};
    for (int64_t j = 0; j < n; j++) {
      if (j == i) continue;
      double dx = pos[3 * j] - xi, dy = pos[3 * j + 1] - yi, dz = pos[3 * j + 2] - zi;
      double r2 = ((dx * dx + dy * dy) + dz * dz) + e2;
      if (r2 == 0.0) continue;
      double rinv = 1.0 / sqrt(r2);
      double mr3 = mass[j] * rinv * rinv * rinv;
      if (compensated) {
        neu_add(&sx[0], &sx[1], mr3 * dx);
        neu_add(&sy[0], &sy[1], mr3 * dy);
        neu_add(&sz[0], &sz[1], mr3 * dz);
        neu_add(&sp[0], &sp[1], -mass[j] * rinv);
      } else {
        sx[0] += mr3 * dx;
        sy[0] += mr3 * dy;
        sz[0] += mr3 * dz;
        sp[0] -= mass[j] * rinv;
      }
    }
    acc[3 * s] = sx[0] + sx[1];
    acc[3 * s + 1] = sy[0] + sy[1];
    acc[3 * s + 2] = sz[0] + sz[1];
    pot[s] = sp[0] + sp[1];
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
orc_ctx* orc_new(void) { return (orc_ctx*)calloc(1, sizeof(orc_ctx)); }

static void ctx_clear(orc_ctx* c) {
  free(c->key); free(c->perm); free(c->spos); free(c->sm);
  free(c->level); free(c->begin); free(c->end); free(c->parent); free(c->child0); free(c->nchild);
  free(c->mass); free(c->com); free(c->rad); free(c->mult); free(c->pk);
  free(c->fcell); free(c->fpart); free(c->fmin); free(c->loc);
  free(c->est_far.a); free(c->est_near.a); free(c->m2l.a); free(c->p2p.a);
  memset(c, 0, sizeof(*c));
}

void orc_free(orc_ctx* c) {
  if (!c) return;
  ctx_clear(c);
  free(c);
}

int64_t orc_ncell(orc_ctx* c) { return c->ncell; }

/* ---- tree: root box, keys, sort, cells (reading: cubic root box over the
 * bodies' extent, 21 bits per axis, x most significant in each octal digit,
 * stable sort, cells = runs of keys sharing a prefix, split while a cell holds
 * more than n_leaf bodies and is above level 21; single-child chains kept). -- */
typedef struct { uint64_t k; int64_t i; } keyidx;
static int cmp_keyidx(const void* a, const void* b) {
  const keyidx* x = (const keyidx*)a;
  const keyidx* y = (const keyidx*)b;
  if (x->k != y->k) return x->k < y->k ? -1 : 1;
  return x->i < y->i ? -1 : (x->i > y->i);
}

static inline int digit_at(uint64_t key, int level) { /* octant index entering `level` */
  return (int)((key >> (3 * (MAX_LEVEL - level))) & 7u);
}

static int64_t add_cell(orc_ctx* c, int level, int64_t b, int64_t e, int64_t parent) {
  if (c->ncell == c->capcell) {
    c->capcell = c->capcell ? 2 * c->capcell : 1024;
    c->level = (int32_t*)realloc(c->level, sizeof(int32_t) * c->capcell);
    c->begin = (int64_t*)realloc(c->begin, sizeof(int64_t) * c->capcell);
    c->end = (int64_t*)realloc(c->end, sizeof(int64_t) * c->capcell);
    c->parent = (int64_t*)realloc(c->parent, sizeof(int64_t) * c->capcell);
    c->child0 = (int64_t*)realloc(c->child0, sizeof(int64_t) * c->capcell);
    c->nchild = (int32_t*)realloc(c->nchild, sizeof(int32_t) * c->capcell);
  }
  int64_t id = c->ncell++;
  c->level[id] = level;
  c->begin[id] = b;
  c->end[id] = e;
  c->parent[id] = parent;
  c->child0[id] = -1;
  c->nchild[id] = 0;
  return id;
}

static void build_tree(orc_ctx* c, const double* pos, const double* mass) {
  int64_t n = c->n;
  double lo[3], hi[3];
  for (int d = 0; d < 3; d++) lo[d] = hi[d] = pos[d];
  for (int64_t i = 1; i < n; i++)
    for (int d = 0; d < 3; d++) {
      double v = pos[3 * i + d];
      if (v < lo[d]) lo[d] = v;
      if (v > hi[d]) hi[d] = v;
    }
  double L = hi[0] - lo[0];
  if (hi[1] - lo[1] > L) L = hi[1] - lo[1];
  if (hi[2] - lo[2] > L) L = hi[2] - lo[2];
  if (L == 0.0) L = 1.0;
  double s = 2097152.0 / L; /* 2^21 / L */
  c->rootbox[0] = lo[0]; c->rootbox[1] = lo[1]; c->rootbox[2] = lo[2];
  c->rootbox[3] = L; c->rootbox[4] = s;
  keyidx* ki = (keyidx*)malloc(sizeof(keyidx) * n);
  for (int64_t i = 0; i < n; i++) {
    uint64_t q[3];
    for (int d = 0; d < 3; d++) {
      double t = floor((pos[3 * i + d] - lo[d]) * s);
      uint64_t v = (uint64_t)t;
      q[d] = v > 2097151u ? 2097151u : v;
    }
    uint64_t key = 0;
    for (int b = KEY_BITS - 1; b >= 0; b--)
      key = (key << 3) | (((q[0] >> b) & 1u) << 2) | (((q[1] >> b) & 1u) << 1) | ((q[2] >> b) & 1u);
    ki[i].k = key;
    ki[i].i = i;
  }
  qsort(ki, (size_t)n, sizeof(keyidx), cmp_keyidx); /* ties by index = stable */
  c->key = (uint64_t*)malloc(sizeof(uint64_t) * n);
  c->perm = (int64_t*)malloc(sizeof(int64_t) * n);
  c->spos = (double*)malloc(sizeof(double) * 3 * n);
  c->sm = (double*)malloc(sizeof(double) * n);
  for (int64_t i = 0; i < n; i++) {
    c->key[i] = ki[i].k;
    c->perm[i] = ki[i].i;
    for (int d = 0; d < 3; d++) c->spos[3 * i + d] = pos[3 * ki[i].i + d];
    c->sm[i] = mass[ki[i].i];
  }
  free(ki);
  /* breadth-first cell construction: ids by level, then key order */
  add_cell(c, 0, 0, n, -1);
  for (int64_t q = 0; q < c->ncell; q++) {
    int64_t b = c->begin[q], e = c->end[q];
    int lev = c->level[q];
    if (e - b <= c->n_leaf || lev >= MAX_LEVEL) continue;
    int64_t first = -1;
    int cnt = 0;
    int64_t i = b;
    while (i < e) {
      int dgt = digit_at(c->key[i], lev + 1);
      int64_t j = i;
      while (j < e && digit_at(c->key[j], lev + 1) == dgt) j++;
      int64_t id = add_cell(c, lev + 1, i, j, q);
      if (first < 0) first = id;
      cnt++;
      i = j;
    }
    c->child0[q] = first;
    c->nchild[q] = cnt;
  }
}

/* mass, centre of mass (expansion centre, reading) and exact radius */
static void cell_geometry(orc_ctx* c) {
  int64_t nc = c->ncell;
  c->mass = (double*)malloc(sizeof(double) * nc);
  c->com = (double*)malloc(sizeof(double) * 3 * nc);
  c->rad = (double*)malloc(sizeof(double) * nc);
  double* S = (double*)malloc(sizeof(double) * 3 * nc);
  for (int64_t q = nc - 1; q >= 0; q--) {
    double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    if (c->nchild[q] == 0) {
      for (int64_t i = c->begin[q]; i < c->end[q]; i++) {
        double m = c->sm[i];
        M = M + m;
        sx = sx + m * c->spos[3 * i];
        sy = sy + m * c->spos[3 * i + 1];
        sz = sz + m * c->spos[3 * i + 2];
      }
    } else {
      for (int64_t ch = c->child0[q]; ch < c->child0[q] + c->nchild[q]; ch++) {
        M = M + c->mass[ch];
        sx = sx + S[3 * ch];
        sy = sy + S[3 * ch + 1];
        sz = sz + S[3 * ch + 2];
      }
    }
    c->mass[q] = M;
    S[3 * q] = sx; S[3 * q + 1] = sy; S[3 * q + 2] = sz;
    if (M != 0.0) {
      c->com[3 * q] = sx / M;
      c->com[3 * q + 1] = sy / M;
      c->com[3 * q + 2] = sz / M;
    } else { /* massless cell: centre of its cubic box */
      int lev = c->level[q];
      uint64_t k = c->key[c->begin[q]];
      uint64_t cc[3] = {0, 0, 0};
      for (int l = 1; l <= lev; l++) {
        int dg = digit_at(k, l);
        cc[0] = (cc[0] << 1) | ((dg >> 2) & 1);
        cc[1] = (cc[1] << 1) | ((dg >> 1) & 1);
        cc[2] = (cc[2] << 1) | (dg & 1);
      }
      double h = ldexp(c->rootbox[3], -lev);
      for (int d = 0; d < 3; d++) c->com[3 * q + d] = c->rootbox[d] + ((double)cc[d] + 0.5) * h;
    }
  }
  free(S);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t q = 0; q < nc; q++) {
    double best = 0.0;
    for (int64_t i = c->begin[q]; i < c->end[q]; i++) {
      double dx = c->spos[3 * i] - c->com[3 * q];
      double dy = c->spos[3 * i + 1] - c->com[3 * q + 1];
      double dz = c->spos[3 * i + 2] - c->com[3 * q + 2];
      double d2 = (dx * dx + dy * dy) + dz * dz;
      if (d2 > best) best = d2;
    }
    c->rad[q] = sqrt(best);
  }
}

/* P2M (section 2.2, multipole-moment equation): M_n^m += m_i Y_n^m(x_i - z),
 * bodies in the given order; yre/yim are scratch of NCOEF(p). */
static void p2m_accumulate(int p, int64_t cnt, const double* pos, const double* mass,
                           const double* centre, double* yre, double* yim, double* mre,
                           double* mim) {
  int nc = NCOEF(p);
  for (int64_t i = 0; i < cnt; i++) {
    double dx = pos[3 * i] - centre[0];
    double dy = pos[3 * i + 1] - centre[1];
    double dz = pos[3 * i + 2] - centre[2];
    orc_regular(p, dx, dy, dz, yre, yim);
    double m = mass[i];
    for (int k = 0; k < nc; k++) {
      mre[k] = mre[k] + m * yre[k];
      mim[k] = mim[k] + m * yim[k];
    }
  }
}

void orc_p2m(int p, int64_t cnt, const double* pos, const double* mass, const double centre[3],
             double* mre, double* mim) {
  int nc = NCOEF(p);
  double* yre = (double*)malloc(sizeof(double) * nc);
  double* yim = (double*)malloc(sizeof(double) * nc);
  for (int k = 0; k < nc; k++) mre[k] = mim[k] = 0.0;
  p2m_accumulate(p, cnt, pos, mass, centre, yre, yim, mre, mim);
  free(yre);
  free(yim);
}

/* P_k of one multipole (section 2.3, P_n equation):
 * P_k^2 = sum_{m=-k..k} (k-m)!(k+m)! |M_k^m|^2, folded onto the stored m >= 0. */
void orc_pk(int p, const double* mre, const double* mim, double* out) {
  for (int k = 0; k <= p; k++) {
    double acc = 0.0;
    for (int m = 0; m <= k; m++) {
      double re = mre[CIDX(k, m)], im = mim[CIDX(k, m)];
      double w = (m == 0) ? (orc_fact[k] * orc_fact[k]) : (2.0 * (orc_fact[k - m] * orc_fact[k + m]));
      acc = acc + w * (re * re + im * im);
    }
    out[k] = sqrt(acc);
  }
}

/* P2M at leaves, M2M to the root, then P_k (section 2.3, P_n equation). */
static void upward(orc_ctx* c) {
  int p = c->p, nc = NCOEF(p);
  int64_t ncell = c->ncell;
  c->mult = (double*)calloc((size_t)ncell * nc * 2, sizeof(double));
  c->pk = (double*)malloc(sizeof(double) * ncell * (p + 1));
#pragma omp parallel
  {
    double* yre = (double*)malloc(sizeof(double) * nc);
    double* yim = (double*)malloc(sizeof(double) * nc);
#pragma omp for schedule(dynamic, 16)
    for (int64_t q = 0; q < ncell; q++) {
      if (c->nchild[q]) continue;
      double* mre = c->mult + (size_t)q * nc * 2;
      p2m_accumulate(p, c->end[q] - c->begin[q], c->spos + 3 * c->begin[q], c->sm + c->begin[q],
                     c->com + 3 * q, yre, yim, mre, mre + nc);
    }
    free(yre);
    free(yim);
  }
  /* M2M, deepest cells first (ids are breadth-first) */
  double* yre = (double*)malloc(sizeof(double) * nc);
  double* yim = (double*)malloc(sizeof(double) * nc);
  for (int64_t q = ncell - 1; q >= 0; q--) {
    if (!c->nchild[q]) continue;
    double* ore = c->mult + (size_t)q * nc * 2;
    double* oim = ore + nc;
    double* yr = (double*)malloc(sizeof(double) * nc * c->nchild[q]);
    double* yi = (double*)malloc(sizeof(double) * nc * c->nchild[q]);
    for (int ch = 0; ch < c->nchild[q]; ch++) {
      int64_t cc = c->child0[q] + ch;
      orc_regular(p, c->com[3 * cc] - c->com[3 * q], c->com[3 * cc + 1] - c->com[3 * q + 1],
                  c->com[3 * cc + 2] - c->com[3 * q + 2], yr + ch * nc, yi + ch * nc);
    }
    /* each child's shifted moments summed on their own (k, then l), then the
     * children added in octant order */
    for (int n = 0; n <= p; n++)
      for (int m = 0; m <= n; m++) {
        double sr = 0.0, si = 0.0;
        for (int ch = 0; ch < c->nchild[q]; ch++) {
          int64_t cc = c->child0[q] + ch;
          const double* mre = c->mult + (size_t)cc * nc * 2;
          const double* mim = mre + nc;
          double cr = 0.0, ci = 0.0;
          for (int k = 0; k <= n; k++)
            for (int l = -k; l <= k; l++) {
              int j = n - k, qq = m - l;
              if (qq > j || qq < -j) continue;
              double ar, ai, br, bi;
              cget(yr + ch * nc, yi + ch * nc, k, l, &ar, &ai);
              cget(mre, mim, j, qq, &br, &bi);
              double tr = ar * br - ai * bi;
              double ti = ar * bi + ai * br;
              cr = cr + tr;
              ci = ci + ti;
            }
          sr = sr + cr;
          si = si + ci;
        }
        ore[CIDX(n, m)] = sr;
        oim[CIDX(n, m)] = si;
      }
    free(yr);
    free(yi);
  }
  free(yre);
  free(yim);
  /* P_k^2 = sum_m (k-m)!(k+m)! |M_k^m|^2 over m = -k..k, folded onto m >= 0 */
  for (int64_t q = 0; q < ncell; q++) {
    const double* mre = c->mult + (size_t)q * nc * 2;
    orc_pk(p, mre, mre + nc, c->pk + q * (p + 1));
  }
}

/* ---- scalar-force estimate (section 2.3): a geometric walk with theta < 1;
 * accepted cell pairs add M/r^2 to each other's far sum; touching leaves are
 * summed body by body; f_i = (far sums along the root-to-leaf path) + near_i,
 * and each cell keeps the minimum of f over its bodies. ---------------------- */
static inline double com_r2(const orc_ctx* c, int64_t a, int64_t b) {
  double dx = c->com[3 * b] - c->com[3 * a];
  double dy = c->com[3 * b + 1] - c->com[3 * a + 1];
  double dz = c->com[3 * b + 2] - c->com[3 * a + 2];
  return (dx * dx + dy * dy) + dz * dz;
}

static void est_interact(orc_ctx* c, int64_t A, int64_t B) {
  int leafA = c->nchild[A] == 0, leafB = c->nchild[B] == 0;
  if (A == B) {
    if (leafA) {
      pv_push(&c->est_near, A, A);
      return;
    }
    int64_t c0 = c->child0[A];
    int nch = c->nchild[A];
    for (int i = 0; i < nch; i++)
      for (int j = i; j < nch; j++) est_interact(c, c0 + i, c0 + j);
    return;
  }
  double r = sqrt(com_r2(c, A, B));
  if ((c->rad[A] + c->rad[B]) < c->theta_est * r) {
    pv_push(&c->est_far, B, A);
    pv_push(&c->est_far, A, B);
    return;
  }
  if (leafA && leafB) {
    pv_push(&c->est_near, B, A);
    pv_push(&c->est_near, A, B);
    return;
  }
  int splitB = leafA || (c->rad[B] > c->rad[A] && !leafB);
  if (splitB) {
    for (int j = 0; j < c->nchild[B]; j++) est_interact(c, A, c->child0[B] + j);
  } else {
    for (int i = 0; i < c->nchild[A]; i++) est_interact(c, c->child0[A] + i, B);
  }
}

static void estimate(orc_ctx* c) {
  int64_t nc = c->ncell, n = c->n;
  est_interact(c, 0, 0);
  int64_t* offF = pv_sort_csr(&c->est_far, nc);
  int64_t* offN = pv_sort_csr(&c->est_near, nc);
  c->fcell = (double*)malloc(sizeof(double) * nc);
  c->fpart = (double*)malloc(sizeof(double) * n);
  c->fmin = (double*)malloc(sizeof(double) * nc);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t B = 0; B < nc; B++) {
    double F = 0.0;
    for (int64_t k = offF[B]; k < offF[B + 1]; k++) {
      int64_t A = c->est_far.a[2 * k + 1];
      F = F + c->mass[A] / com_r2(c, A, B);
    }
    c->fcell[B] = F;
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t B = 0; B < nc; B++) {
    if (c->nchild[B]) continue;
    /* far part: path sum from the root down to B */
    int64_t path[MAX_LEVEL + 2];
    int len = 0;
    for (int64_t q = B; q >= 0; q = c->parent[q]) path[len++] = q;
    double far = 0.0;
    for (int t = len - 1; t >= 0; t--) far = far + c->fcell[path[t]];
    for (int64_t i = c->begin[B]; i < c->end[B]; i++) {
      double xi = c->spos[3 * i], yi = c->spos[3 * i + 1], zi = c->spos[3 * i + 2];
      double near = 0.0;
      for (int64_t k = offN[B]; k < offN[B + 1]; k++) {
        int64_t A = c->est_near.a[2 * k + 1];
        for (int64_t j = c->begin[A]; j < c->end[A]; j++) {
          if (j == i) continue;
          double dx = c->spos[3 * j] - xi, dy = c->spos[3 * j + 1] - yi, dz = c->spos[3 * j + 2] - zi;
          double d2 = (dx * dx + dy * dy) + dz * dz;
          if (d2 > 0.0) near = near + c->sm[j] / d2;
        }
      }
      c->fpart[i] = far + near;
    }
  }
  for (int64_t q = nc - 1; q >= 0; q--) {
    double f;
    if (!c->nchild[q]) {
      f = INFINITY;
      for (int64_t i = c->begin[q]; i < c->end[q]; i++)
        if (c->fpart[i] < f) f = c->fpart[i];
    } else {
      f = c->fmin[c->child0[q]];
      for (int ch = 1; ch < c->nchild[q]; ch++)
        if (c->fmin[c->child0[q] + ch] < f) f = c->fmin[c->child0[q] + ch];
    }
    c->fmin[q] = f;
  }
  free(offF);
  free(offN);
}

/* ---- error-controlled mutual MAC (section 2.3):
 * theta < 1  and  E_{A->B} M_A/r^2 < eps f_B  and  E_{B->A} M_B/r^2 < eps f_A,
 * E_{A->B} = 8 max(rA,rB)/(rA+rB) / M_A * sum_k C(p,k) P_{k,A} rB^(p-k) / r^p.
 * M_A cancels.  theta = (rA + rB)/r (reading). */
static double mac_lhs(const orc_ctx* c, int64_t A, int64_t B, double r, double r2) {
  int p = c->p;
  double rA = c->rad[A], rB = c->rad[B];
  double rp = r;
  for (int i = 2; i <= p; i++) rp = rp * r;
  double mx = rA > rB ? rA : rB;
  double pref = (8.0 * mx) / (rA + rB);
  double powB = 1.0, SA = 0.0;
  double pw[ORC_PMAX + 1];
  pw[0] = 1.0;
  for (int j = 1; j <= p; j++) {
    powB = powB * rB;
    pw[j] = powB;
  }
  const double* PA = c->pk + A * (p + 1);
  for (int k = 0; k <= p; k++) SA = SA + (orc_binom[p][k] * PA[k]) * pw[p - k];
  return (pref * (SA / rp)) / r2;
}

static int mac_accept(const orc_ctx* c, int64_t A, int64_t B) {
  double r2 = com_r2(c, A, B);
  double r = sqrt(r2);
  double rA = c->rad[A], rB = c->rad[B];
  if (!((rA + rB) < c->theta * r)) return 0;
  if (c->mac == ORC_MAC_GEOMETRIC) return 1;
  if (rA + rB == 0.0) return 1;
  double lab = mac_lhs(c, A, B, r, r2);
  double lba = mac_lhs(c, B, A, r, r2);
  return (lab < c->err_tol * c->fmin[B]) && (lba < c->err_tol * c->fmin[A]);
}

/* dual-tree walk (section 2.1): mutual decisions, larger cell split (reading) */
static void interact(orc_ctx* c, int64_t A, int64_t B) {
  int leafA = c->nchild[A] == 0, leafB = c->nchild[B] == 0;
  if (A == B) {
    if (leafA) {
      pv_push(&c->p2p, A, A);
      return;
    }
    int64_t c0 = c->child0[A];
    int nch = c->nchild[A];
    for (int i = 0; i < nch; i++)
      for (int j = i; j < nch; j++) interact(c, c0 + i, c0 + j);
    return;
  }
  if (mac_accept(c, A, B)) {
    pv_push(&c->m2l, B, A);
    pv_push(&c->m2l, A, B);
    return;
  }
  if (leafA && leafB) {
    pv_push(&c->p2p, B, A);
    pv_push(&c->p2p, A, B);
    return;
  }
  int splitB = leafA || (c->rad[B] > c->rad[A] && !leafB);
  if (splitB) {
    for (int j = 0; j < c->nchild[B]; j++) interact(c, A, c->child0[B] + j);
  } else {
    for (int i = 0; i < c->nchild[A]; i++) interact(c, c->child0[A] + i, B);
  }
}

/* ---- evaluation: M2L, L2L, L2P, P2P, final sum ------------------------- */
static void evaluate(orc_ctx* c, const uint8_t* mask_caller, double* acc, double* pot) {
  int p = c->p, nc = NCOEF(p);
  int64_t ncell = c->ncell, n = c->n;
  int64_t* offM = pv_sort_csr(&c->m2l, ncell);
  int64_t* offP = pv_sort_csr(&c->p2p, ncell);
  uint8_t* need = (uint8_t*)calloc(ncell, 1);
  if (mask_caller) {
    for (int64_t q = 0; q < ncell; q++) {
      if (c->nchild[q]) continue;
      for (int64_t i = c->begin[q]; i < c->end[q]; i++)
        if (mask_caller[c->perm[i]]) { need[q] = 1; break; }
    }
    for (int64_t q = ncell - 1; q > 0; q--)
      if (need[q]) need[c->parent[q]] = 1;
  } else {
    memset(need, 1, ncell);
  }
  c->loc = (double*)calloc((size_t)ncell * nc * 2, sizeof(double));
#pragma omp parallel
  {
    double* tre = (double*)malloc(sizeof(double) * nc);
    double* tim = (double*)malloc(sizeof(double) * nc);
#pragma omp for schedule(dynamic, 4)
    for (int64_t B = 0; B < ncell; B++) {
      if (!need[B]) continue;
      double* lre = c->loc + (size_t)B * nc * 2;
      double* lim = lre + nc;
      for (int64_t k = offM[B]; k < offM[B + 1]; k++) {
        int64_t A = c->m2l.a[2 * k + 1];
        const double* mre = c->mult + (size_t)A * nc * 2;
        double R[3] = {c->com[3 * B] - c->com[3 * A], c->com[3 * B + 1] - c->com[3 * A + 1],
                       c->com[3 * B + 2] - c->com[3 * A + 2]};
        if (c->m2l_kind == ORC_M2L_DIRECT)
          orc_m2l_direct(p, mre, mre + nc, R, tre, tim);
        else
          orc_m2l_rotated(p, mre, mre + nc, R, tre, tim);
        for (int t = 0; t < nc; t++) {
          lre[t] += tre[t];
          lim[t] += tim[t];
        }
      }
    }
    free(tre);
    free(tim);
  }
  /* L2L, parents before children */
  {
    double* yre = (double*)malloc(sizeof(double) * nc);
    double* yim = (double*)malloc(sizeof(double) * nc);
    for (int64_t q = 1; q < ncell; q++) {
      if (!need[q]) continue;
      int64_t P = c->parent[q];
      orc_regular(p, c->com[3 * q] - c->com[3 * P], c->com[3 * q + 1] - c->com[3 * P + 1],
                  c->com[3 * q + 2] - c->com[3 * P + 2], yre, yim);
      const double* pl = c->loc + (size_t)P * nc * 2;
      double* ql = c->loc + (size_t)q * nc * 2;
      l2l_accumulate(p, pl, pl + nc, yre, yim, ql, ql + nc);
    }
    free(yre);
    free(yim);
  }
  double e2 = c->eps_soft * c->eps_soft;
  for (int64_t i = 0; i < n; i++) {
    acc[3 * i] = acc[3 * i + 1] = acc[3 * i + 2] = NAN;
    pot[i] = NAN;
  }
#pragma omp parallel
  {
    double* yre = (double*)malloc(sizeof(double) * nc);
    double* yim = (double*)malloc(sizeof(double) * nc);
#pragma omp for schedule(dynamic, 8)
    for (int64_t B = 0; B < ncell; B++) {
      if (c->nchild[B] || !need[B]) continue;
      const double* lre = c->loc + (size_t)B * nc * 2;
      for (int64_t i = c->begin[B]; i < c->end[B]; i++) {
        double xi = c->spos[3 * i], yi = c->spos[3 * i + 1], zi = c->spos[3 * i + 2];
        double fpot, fa[3];
        orc_regular(p, xi - c->com[3 * B], yi - c->com[3 * B + 1], zi - c->com[3 * B + 2], yre, yim);
        l2p_eval(p, lre, lre + nc, yre, yim, &fpot, fa);
        double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
        for (int64_t k = offP[B]; k < offP[B + 1]; k++) {
          int64_t A = c->p2p.a[2 * k + 1];
          for (int64_t j = c->begin[A]; j < c->end[A]; j++) {
            if (j == i) continue;
            double dx = c->spos[3 * j] - xi, dy = c->spos[3 * j + 1] - yi, dz = c->spos[3 * j + 2] - zi;
            double r2 = ((dx * dx + dy * dy) + dz * dz) + e2;
            if (r2 == 0.0) continue;
            double rinv = 1.0 / sqrt(r2);
            double mr3 = c->sm[j] * rinv * rinv * rinv;
            ax += mr3 * dx;
            ay += mr3 * dy;
            az += mr3 * dz;
            ph -= c->sm[j] * rinv;
          }
        }
        int64_t o = c->perm[i];
        acc[3 * o] = fa[0] + ax;
        acc[3 * o + 1] = fa[1] + ay;
        acc[3 * o + 2] = fa[2] + az;
        pot[o] = fpot + ph;
      }
    }
    free(yre);
    free(yim);
  }
  free(need);
  free(offM);
  free(offP);
}

int orc_run(orc_ctx* c, int64_t n, const double* pos, const double* mass, double eps_soft, int p,
            double err_tol, double theta, double theta_est, int n_leaf, int mac, int m2l_kind,
            int stage, const uint8_t* eval_mask, double* acc, double* pot) {
  if (!c || n < 1 || !pos || !mass) return -1;
  if (p < 1 || p > ORC_PMAX || !(err_tol > 0) || !(theta > 0) || !(theta_est > 0)) return -1;
  if (n_leaf < 1 || eps_soft < 0 || stage < ORC_STAGE_TREE || stage > ORC_STAGE_EVAL) return -1;
  if (stage == ORC_STAGE_EVAL && (!acc || !pot)) return -1;
  ctx_clear(c);
  c->n = n;
  c->p = p;
  c->n_leaf = n_leaf;
  c->mac = mac;
  c->m2l_kind = m2l_kind;
  c->err_tol = err_tol;
  c->theta = theta;
  c->theta_est = theta_est;
  c->eps_soft = eps_soft;
  build_tree(c, pos, mass);
  cell_geometry(c);
  if (stage < ORC_STAGE_UPWARD) return 0;
  upward(c);
  if (stage < ORC_STAGE_ESTIMATE) return 0;
  estimate(c);
  if (stage < ORC_STAGE_WALK) return 0;
  interact(c, 0, 0);
  if (stage < ORC_STAGE_EVAL) {
    int64_t* o1 = pv_sort_csr(&c->m2l, c->ncell);
    int64_t* o2 = pv_sort_csr(&c->p2p, c->ncell);
    free(o1);
    free(o2);
    return 0;
  }
  evaluate(c, eval_mask, acc, pot);
  return 0;
}

int64_t orc_get(orc_ctx* c, int what, const void** ptr) {
  int64_t nc = c->ncell;
  int ncoef = NCOEF(c->p);
  *ptr = NULL;
#define RET(P, N) do { if (!(P)) return 0; *ptr = (const void*)(P); return (N); } while (0)
  switch (what) {
    case ORC_KEYS: RET(c->key, c->n);
    case ORC_PERM: RET(c->perm, c->n);
    case ORC_CELL_LEVEL: RET(c->level, nc);
    case ORC_CELL_BEGIN: RET(c->begin, nc);
    case ORC_CELL_END: RET(c->end, nc);
    case ORC_CELL_PARENT: RET(c->parent, nc);
    case ORC_CELL_CHILD0: RET(c->child0, nc);
    case ORC_CELL_NCHILD: RET(c->nchild, nc);
    case ORC_CELL_MASS: RET(c->mass, nc);
    case ORC_CELL_COM: RET(c->com, 3 * nc);
    case ORC_CELL_RAD: RET(c->rad, nc);
    case ORC_MULT: RET(c->mult, nc * ncoef * 2);
    case ORC_PK: RET(c->pk, nc * (c->p + 1));
    case ORC_FCELL_EST: RET(c->fcell, nc);
    case ORC_F_PART: RET(c->fpart, c->n);
    case ORC_FMIN: RET(c->fmin, nc);
    case ORC_EST_FAR: RET(c->est_far.a, 2 * c->est_far.n);
    case ORC_EST_NEAR: RET(c->est_near.a, 2 * c->est_near.n);
    case ORC_M2L: RET(c->m2l.a, 2 * c->m2l.n);
    case ORC_P2P: RET(c->p2p.a, 2 * c->p2p.n);
    case ORC_LOCAL: RET(c->loc, nc * ncoef * 2);
    case ORC_ROOTBOX: RET(c->rootbox, 5);
    case ORC_SORTED_POS: RET(c->spos, 3 * c->n);
  }
#undef RET
  return 0;
}
