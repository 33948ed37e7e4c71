/*
 * CPU oracle for the collisional FMM force evaluation -- TEST INFRASTRUCTURE ONLY.
 *
 * This library is a plain, slow FP64 restatement of the force pass of
 * Mukherjee, Zhu, Trac & Rodriguez (2021), "Fast Multipole Methods for N-body
 * Simulations of Collisional Star Systems" (section 2 and its subsections),
 * plus the O(N^2) direct summation it approximates.  It exists to check the
 * GPU library.  Only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark may load it; the product path never does.
 *
 * Conventions: G = 1, acc = -grad(Phi), Phi_i = -sum_{j != i} m_j / sqrt(r_ij^2 + eps^2).
 * All arrays are host memory.  Positions are n x 3 row-major FP64.
 */
#ifndef FMM_ORACLE_H
#define FMM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_ctx orc_ctx;

/* which stages orc_run performs (cumulative: each implies the previous ones) */
enum { ORC_STAGE_TREE = 1, ORC_STAGE_UPWARD = 2, ORC_STAGE_ESTIMATE = 3,
       ORC_STAGE_WALK = 4, ORC_STAGE_EVAL = 5 };
enum { ORC_MAC_ERROR = 0, ORC_MAC_GEOMETRIC = 1 };
enum { ORC_M2L_ROTATION = 0, ORC_M2L_DIRECT = 1 };

/* exported arrays (orc_get) */
enum {
  ORC_KEYS = 0,        /* uint64[n]   sorted Morton keys                          */
  ORC_PERM = 1,        /* int64[n]    original index of sorted position           */
  ORC_CELL_LEVEL = 2,  /* int32[nc]                                               */
  ORC_CELL_BEGIN = 3,  /* int64[nc]   first sorted particle                       */
  ORC_CELL_END = 4,    /* int64[nc]   one past last                               */
  ORC_CELL_PARENT = 5, /* int64[nc]   -1 for the root                             */
  ORC_CELL_CHILD0 = 6, /* int64[nc]   first child id, -1 for leaves               */
  ORC_CELL_NCHILD = 7, /* int32[nc]   0 for leaves                                */
  ORC_CELL_MASS = 8,   /* double[nc]                                              */
  ORC_CELL_COM = 9,    /* double[nc*3]                                            */
  ORC_CELL_RAD = 10,   /* double[nc]                                              */
  ORC_MULT = 11,       /* double[nc*ncoef*2]  (re, im) per coefficient            */
  ORC_PK = 12,         /* double[nc*(p+1)]                                        */
  ORC_FCELL_EST = 13,  /* double[nc]  far-field scalar-force sums F_cell          */
  ORC_F_PART = 14,     /* double[n]   scalar force f_i, sorted order              */
  ORC_FMIN = 15,       /* double[nc]  min of f over the cell's particles          */
  ORC_EST_FAR = 16,    /* int64[2*k]  (sink, source) directed accepted pairs      */
  ORC_EST_NEAR = 17,   /* int64[2*k]  (sink, source) directed leaf pairs          */
  ORC_M2L = 18,        /* int64[2*k]  (sink, source) directed M2L pairs           */
  ORC_P2P = 19,        /* int64[2*k]  (sink, source) directed P2P leaf pairs      */
  ORC_LOCAL = 20,      /* double[nc*ncoef*2]  local expansions after L2L          */
  ORC_ROOTBOX = 21,    /* double[5]  lo_x, lo_y, lo_z, L, s                        */
  ORC_SORTED_POS = 22, /* double[n*3] positions in sorted order                   */
};

orc_ctx* orc_new(void);
void     orc_free(orc_ctx* c);

/* One force pass (or its first `stage` stages).  acc/pot (caller order) are
 * written only when stage == ORC_STAGE_EVAL and may be NULL otherwise.
 * eval_leaf_mask (may be NULL): per-particle flags in CALLER order; when given,
 * only leaves holding a flagged particle are evaluated and the other outputs
 * are set to NaN (exact same arithmetic for the evaluated ones).
 * Returns 0 on success, negative on bad arguments. */
int orc_run(orc_ctx* c, int64_t n, const double* pos, const double* mass,
            double eps_soft, int p, double err_tol, double theta, double theta_est,
            int n_leaf, int mac, int m2l_kind, int stage, const uint8_t* eval_mask,
            double* acc, double* pot);

/* pointer and element count (see enum) of an exported array; 0 if absent */
int64_t orc_get(orc_ctx* c, int what, const void** ptr);
int64_t orc_ncell(orc_ctx* c);

/* Plain O(N^2) direct summation for the sinks listed in `sinks` (or all when
 * sinks == NULL), sources = all particles.  compensated != 0 selects
 * Neumaier-compensated sums.  Outputs indexed like the sink list. */
int orc_direct(int64_t n, const double* pos, const double* mass, double eps_soft,
               int64_t nsink, const int64_t* sinks, int compensated,
               double* acc, double* pot);

/* Building blocks exposed for the pin tests. */
void orc_regular(int p, double x, double y, double z, double* re, double* im);
void orc_irregular(int p, double x, double y, double z, double* re, double* im);
/* M2L of one multipole (coefficients re/im, ncoef) across translation R = z_B - z_A */
void orc_m2l_direct(int p, const double* mre, const double* mim, const double R[3],
                    double* lre, double* lim);
void orc_m2l_rotated(int p, const double* mre, const double* mim, const double R[3],
                     double* lre, double* lim);
/* shift a local expansion by d = z_child - z_parent (exact polynomial shift) */
void orc_l2l(int p, const double* lre, const double* lim, const double d[3],
             double* ore, double* oim);
/* evaluate a local expansion at offset X from its centre: pot and acc */
void orc_l2p(int p, const double* lre, const double* lim, const double X[3],
             double* pot, double acc[3]);
/* shift a multipole from child centre to parent centre, d = z_child - z_parent */
void orc_m2m(int p, const double* mre, const double* mim, const double d[3],
             double* ore, double* oim);
/* P2M of cnt bodies about `centre`, and the per-order norms P_k of a multipole */
void orc_p2m(int p, int64_t cnt, const double* pos, const double* mass, const double centre[3],
             double* mre, double* mim);
void orc_pk(int p, const double* mre, const double* mim, double* out /* p+1 */);
const double* orc_swap_table(int n);   /* dense (2n+1)^2 row-major */
const double* orc_factorials(void);    /* 62 entries */
int orc_threads(void);                 /* OpenMP threads in use */

#ifdef __cplusplus
}
#endif
#endif
