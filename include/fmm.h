/*
 * fmm.h -- C ABI of the MI355X (gfx950) collisional FMM force pass.
 *
 * One call computes, for N point masses, the gravitational acceleration and
 * potential of every body with the fast multipole method of Mukherjee, Zhu,
 * Trac & Rodriguez (2021): an octree over Morton-sorted bodies, P2M/M2M in
 * regular solid harmonics (section 2.2), a scalar-force estimate and a
 * dual-tree walk with the error-controlled mutual acceptance criterion
 * (section 2.3), rotation-accelerated M2L (section 2.4), L2L, L2P and direct
 * P2P for the near field (section 2.1).
 *
 * Conventions: G = 1; acc_i = sum_{j != i} m_j (x_j - x_i) / (r_ij^2 + eps^2)^{3/2};
 * pot_i = -sum_{j != i} m_j / (r_ij^2 + eps^2)^{1/2}  (eps = Plummer softening,
 * applied to the direct near field only; the far field is unsoftened).
 * Pairs with r_ij^2 + eps^2 == 0 contribute nothing.
 *
 * Memory: unless stated otherwise every pointer argument is a HIP DEVICE
 * pointer on the context's device; positions are n x 3 row-major FP64,
 * masses FP64.  The caller owns inputs and outputs; the context owns all
 * scratch (tree, expansions, lists), grows it on demand and frees it in
 * fmm_destroy.  Work is enqueued on the given stream; functions that return
 * host-visible values synchronise that stream.  No function throws; every
 * status other than FMM_OK leaves outputs unspecified and the context usable.
 * A context must not be used from two host threads at once.
 */
#ifndef FMM_H
#define FMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FMM_OK = 0,
  FMM_EINVAL = -1,       /* bad argument (checked on the host before any launch) */
  FMM_ENOMEM = -2,       /* device allocation failed / workspace cap exceeded    */
  FMM_EHIP = -3,         /* a HIP runtime call failed (message in fmm_last_error) */
  FMM_ENOTBUILT = -4,    /* export asked for data no call has produced yet        */
  FMM_EDATA = -5,        /* non-finite position or negative/non-finite mass       */
  FMM_EUNSUPPORTED = -6  /* valid but not supported by the compiled library      */
} fmm_status;

typedef enum {
  FMM_FP64 = 0,   /* every stage in FP64                                            */
  FMM_MIXED = 1,  /* P2P and M2L below the root levels in FP32 (scaled, relative
                     coordinates, compensated sums); tree, acceptance test, P2M/M2M,
                     L2L, L2P and the final sum in FP64                              */
  FMM_DIRECT = 2  /* plain O(N^2) direct summation (FP64), for checks               */
} fmm_precision;

typedef enum {
  FMM_MAC_ERROR = 0,     /* error-controlled mutual criterion, section 2.3       */
  FMM_MAC_GEOMETRIC = 1  /* opening angle only: (r_A + r_B) < theta * r          */
} fmm_mac;

typedef struct {
  int p;            /* expansion order, 1..30 (swap tables exist for p <= 30, section 2.4) */
  double err_tol;   /* epsilon of the acceptance criterion, > 0 (section 2.3)             */
  double theta;     /* opening-angle cap, (0, 1], default 1 ("theta < 1", section 2.3)    */
  double theta_est; /* opening angle of the scalar-force estimate walk, default 1         */
  int n_leaf;       /* a cell with more bodies is split, 1..1024, default 64              */
  int precision;    /* fmm_precision                                                      */
  int mac;          /* fmm_mac                                                            */
  int check_inputs; /* 1: reject NaN/Inf positions, negative or NaN masses (FMM_EDATA)    */
  int root_levels;  /* mixed precision: M2L touching a cell above this level stays FP64 */
  int m2l_waves;    /* mixed precision: wavefronts per sink in the FP32 M2L, 1, 2 or 4 (default 1);
                       each takes a contiguous part of the sink's list, the parts added in order */
  int p2p_groups;   /* near field: at most this many lane groups share a sink leaf's sources
                       (0 = as many as the wavefront holds, the default; else 1..64) */
  int p2p_start;    /* after a tree build: 0 = the near field starts once its own list is
                       grouped (default); 1 = only after the M2L list is grouped as well, so
                       that a long near field does not hold the chip while that grouping waits */
} fmm_params;

/* counts and times of the last call (filled by fmm_stats); times in ms between
 * HIP events recorded on the call's stream */
typedef struct {
  int64_t n;              /* bodies                                       */
  int64_t ncell;          /* cells (root = 0, breadth-first ids)          */
  int64_t nleaf;          /* leaves                                       */
  int32_t depth;          /* deepest level                                */
  int64_t n_m2l;          /* directed M2L pairs                           */
  int64_t n_p2p_cells;    /* directed P2P leaf pairs (incl. self pairs)   */
  int64_t n_p2p_pairs;    /* directed body-body interactions in P2P       */
  int64_t n_est_far;      /* directed accepted pairs of the estimate walk */
  int64_t n_est_near;     /* directed leaf pairs of the estimate walk     */
  int64_t n_m2l_fp32;     /* M2L pairs evaluated in FP32 (mixed mode)     */
  /* stage times: tree (keys, sort, cells, radii, leaf list); upward (P2M, M2M,
   * P_k, on a side stream beside the estimate); estimate (its walk, list
   * grouping, far and near sums, cell minima); walk (acceptance walk and the
   * grouping of the M2L list); m2l (from there to the join: the M2L kernels
   * beside the near field); local (root-level add, L2L, final L2P and sum);
   * p2p (the near-field kernel on its side stream); total (the whole call) */
  double ms_tree, ms_upward, ms_estimate, ms_walk, ms_m2l, ms_local, ms_p2p, ms_total;
  size_t workspace_bytes; /* device memory held by the context            */
  int64_t nsys;           /* independent systems of the call (1 for fmm_forces) */
  double ms_m2l_kernel;   /* the main M2L kernel alone (FP32 kernel in mixed mode) */
  double ms_sort;         /* the stable radix sort of the bodies' Morton keys (tree stage) */
  double ms_gather;       /* the gather of positions and masses into sorted order (tree stage) */
  double ms_walk_steps;   /* the acceptance walk alone, before its lists are grouped (walk stage) */
  int64_t n_p2p_items;    /* near-field work items of the last evaluation: a sink leaf, or one
                             segment of a leaf's source list when the list is long */
} fmm_stats_t;

/* export selectors for fmm_export (host buffer, element counts from fmm_stats) */
typedef enum {
  FMM_X_KEYS = 0,       /* uint64[n]   sorted 63-bit Morton keys                    */
  FMM_X_PERM = 1,       /* int32[n]    caller index of each sorted body             */
  FMM_X_CELL_LEVEL = 2, /* int32[ncell]                                             */
  FMM_X_CELL_BEGIN = 3, /* int32[ncell] first sorted body                          */
  FMM_X_CELL_END = 4,   /* int32[ncell] one past the last                           */
  FMM_X_CELL_PARENT = 5,/* int32[ncell] -1 for the root                             */
  FMM_X_CELL_CHILD0 = 6,/* int32[ncell] first child, -1 for leaves                  */
  FMM_X_CELL_NCHILD = 7,/* int32[ncell]                                             */
  FMM_X_CELL_MASS = 8,  /* double[ncell]                                            */
  FMM_X_CELL_COM = 9,   /* double[ncell*3] centre of mass (expansion centre)        */
  FMM_X_CELL_RAD = 10,  /* double[ncell] max distance of a body from the centre     */
  FMM_X_MULT = 11,      /* double[ncell*ncoef*2] multipoles, (re, im) interleaved,
                           coefficient (n, m>=0) at n(n+1)/2 + m                    */
  FMM_X_PK = 12,        /* double[ncell*(p+1)] per-order norms P_k (section 2.3)    */
  FMM_X_FCELL = 13,     /* double[ncell] far-field scalar-force sums of the estimate */
  FMM_X_FPART = 14,     /* double[n] scalar force f_i in sorted order               */
  FMM_X_FMIN = 15,      /* double[ncell] min of f over the cell's bodies            */
  FMM_X_EST_FAR = 16,   /* int32[2*n_est_far] (sink, source) pairs, CSR by sink     */
  FMM_X_EST_NEAR = 17,  /* int32[2*n_est_near]                                      */
  FMM_X_M2L = 18,       /* int32[2*n_m2l]                                           */
  FMM_X_P2P = 19,       /* int32[2*n_p2p_cells]                                     */
  FMM_X_LOCAL = 20,     /* double[ncell*ncoef*2] local expansions after L2L         */
  FMM_X_ROOTBOX = 21    /* double[5*nsys] per system: lo_x, lo_y, lo_z, edge L,
                           key scale 2^21/L                                        */
} fmm_export_what;

typedef struct fmm_ctx fmm_ctx;

/* Defaults: p = 10, err_tol = 1e-7, theta = 1, theta_est = 1, n_leaf = 64,
 * precision = FMM_FP64, mac = FMM_MAC_ERROR, check_inputs = 0, root_levels = 3,
 * m2l_waves = 1, p2p_groups = 0, p2p_start = 0. */
void fmm_default_params(fmm_params* out /* host */);

/* Creates a context on the current HIP device.  prm (host) may be NULL for the
 * defaults.  *out receives the context (host pointer). */
fmm_status fmm_create(fmm_ctx** out, const fmm_params* prm);

/* Replaces the parameters used by later calls (validated as in fmm_create). */
fmm_status fmm_set_params(fmm_ctx* ctx, const fmm_params* prm);

/* Copies the context's current parameters (after fmm_autotune, the tuned
 * ones) into *out (host).  FMM_EINVAL for NULL arguments. */
fmm_status fmm_get_params(fmm_ctx* ctx, fmm_params* out);

/* Tree and upward pass only (keys, sort, cells, P2M, M2M, P_k): planning and
 * parity export.  Section 2.1 (octree, P2M at the leaves, M2M to the root),
 * section 2.2 (moment equation) and section 2.3 (the per-order norms P_n and
 * the cell sizes the acceptance test uses).  pos/mass: device, n >= 1.
 * FMM_EUNSUPPORTED if the context's p has no compiled kernel. */
fmm_status fmm_build(fmm_ctx* ctx, int64_t n, const double* pos, const double* mass,
                     void* stream /* hipStream_t, NULL = default stream */);

/* One full force evaluation: the flow of section 2.1 (tree, P2M, M2M, dual-tree
 * walk, M2L, L2L, L2P and the direct near field), the scalar-force estimate and
 * the error-controlled acceptance test of section 2.3, and the rotated M2L of
 * section 2.4.  Rebuilds the tree from pos.  p (1..30) and err_tol (> 0)
 * override the context's parameters for this call; eps_soft >= 0 softens the
 * near field.  acc (n x 3) and pot (n) are device buffers in the caller's body
 * order and are overwritten.  n == 1 gives acc = 0, pot = 0.  FMM_EINVAL for
 * bad arguments (before any launch); FMM_EUNSUPPORTED for an order without a
 * compiled kernel or for lists too long for the int32 CSR arrays. */
fmm_status fmm_forces(fmm_ctx* ctx, int64_t n, const double* pos, const double* mass,
                      double eps_soft, int p, double err_tol, double* acc, double* pot,
                      void* stream);

/* Force evaluation with the tree and interaction lists of the context's last
 * fmm_forces call kept (frozen): the bodies are taken in the stored order,
 * and cell centres, radii, P2M, M2M, M2L, L2L, L2P and P2P are recomputed from
 * pos and mass, the acceptance test is not.  The result is a smooth function
 * of pos and mass, which is what finite-difference checks of gradients need
 * (a change of the accepted pairs would make it jump).  n must equal the last
 * call's body count (FMM_ENOTBUILT if no evaluation was made, or another n);
 * p, err_tol and the system split are the last call's. */
fmm_status fmm_forces_frozen(fmm_ctx* ctx, int64_t n, const double* pos, const double* mass,
                             double eps_soft, double* acc, double* pot, void* stream);

/* fmm_forces_frozen replayed as a HIP graph, for step loops that keep the
 * tree: the first call (and any call with other buffers, eps_soft or stream,
 * or after the tree was rebuilt) runs the evaluation once eagerly, captures it
 * on the stream and instantiates the graph; later calls launch the graph.
 * pos, mass, acc and pot are baked into the graph, so the caller updates
 * pos/mass in place between calls.  The graph zeroes its buffers with kernels
 * (no memset nodes).  No stage times are recorded for replayed calls.
 * Errors as fmm_forces_frozen. */
fmm_status fmm_forces_frozen_graph(fmm_ctx* ctx, int64_t n, const double* pos, const double* mass,
                                   double eps_soft, double* acc, double* pot, void* stream);

/* Gradient of the force pass: for a scalar L(acc, pot) given gacc = dL/dacc
 * (n x 3) and gpot = dL/dpot (n, or NULL for zero), writes gpos = dL/dpos
 * (n x 3) and gmass = dL/dmass (n), all device buffers in the caller's body
 * order.  The forward pass at pos is recomputed first (tree, estimate, walk,
 * expansions; FP64 whatever the context's precision), and its interaction
 * lists serve the gradient too: the sink side applies the tidal tensor (the
 * Hessian of the potential from the order-2 local coefficients, plus the
 * softened near-field pair terms) to gacc; the source side runs a second
 * expansion pass (P2M, M2M, M2L, L2L on the same tree) over charges gpot and
 * dipoles -gacc.  The far field is the FMM approximation of the exact
 * gradient, accurate at the level of the forces (err_tol), not the exact
 * derivative of the approximate forces.  Errors as fmm_forces; p must have a
 * compiled kernel (FMM_EUNSUPPORTED otherwise). */
fmm_status fmm_adjoint(fmm_ctx* ctx, int64_t n, const double* pos, const double* mass, double eps_soft,
                       int p, double err_tol, const double* gacc, const double* gpot, double* gpos,
                       double* gmass, void* stream);

/* fmm_adjoint without its forward pass, for callers that keep the forward
 * evaluation (a rollout's backward pass): the same gradient at the positions
 * and masses of the context's last evaluation, whose tree, interaction lists,
 * local expansions and near-field work items are reused.  That evaluation
 * must be one system of n bodies in FP64 precision (fmm_forces,
 * fmm_forces_frozen, fmm_forces_frozen_graph, fmm_adjoint or fmm_jerk;
 * fmm_forces_noalloc leaves this state alone).  acc (n x 3, device, caller
 * order) is the acceleration that evaluation returned.  gacc, gpot, gpos and
 * gmass as in fmm_adjoint; the result equals fmm_adjoint's at the same inputs
 * bit for bit.  Errors: a null pointer or n < 1 -> FMM_EINVAL; no such
 * evaluation (none yet, another n, a batch, mixed or direct precision, or a
 * tree built since) -> FMM_ENOTBUILT. */
fmm_status fmm_adjoint_last(fmm_ctx* ctx, int64_t n, const double* acc, const double* gacc,
                            const double* gpot, double* gpos, double* gmass, void* stream);

/* Forces and their time derivative along the motion (the jerk, for
 * fourth-order Hermite integrators; section 5 of the paper):
 * jerk_k = sum_j m_j [w / s^3 - 3 (u . w) u / s^5], u = x_j - x_k,
 * w = v_j - v_k.  vel (n x 3) is a device buffer in the caller's order; acc,
 * pot and jerk are written like fmm_forces' outputs.  The far field is the
 * tidal tensor of the force pass applied to v_k plus the field gradient of
 * the dipoles m_j v_j, the second from an expansion pass on the same tree and
 * lists (the operator of fmm_adjoint).  FP64; errors as fmm_adjoint. */
fmm_status fmm_jerk(fmm_ctx* ctx, int64_t n, const double* pos, const double* vel, const double* mass,
                    double eps_soft, int p, double err_tol, double* acc, double* pot, double* jerk,
                    void* stream);

/* Limits of fmm_forces_noalloc: the largest body count, and the size of the
 * static device scratch it works in (one per device, held until the process
 * ends). */
#define FMM_NOALLOC_MAX_N 65536
#define FMM_NOALLOC_SCRATCH_BYTES (128u << 20)

/* fmm_forces for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Every
 * scratch buffer of the evaluation (sort state, cells, expansions, interaction
 * lists, partial sums, counters) is carved from the library's static device
 * array of FMM_NOALLOC_SCRATCH_BYTES instead of the context's workspace: the
 * call performs no hipMalloc, hipFree or other allocation.  fmm_create, on the
 * same device, set up everything it needs (the scratch's device address, the
 * kernels' constant tables, the context's streams, events and pinned host
 * words).  Arguments, outputs and results are those of fmm_forces with the
 * context's parameters.  Errors: n above FMM_NOALLOC_MAX_N, or another device
 * current than at fmm_create -> FMM_EINVAL; an input whose tree, expansions
 * and lists do not fit the scratch -> FMM_ENOMEM (fmm_last_error says so);
 * otherwise as fmm_forces.  All calls on one device share that device's
 * scratch, which keeps the last call's contents (each call initialises what
 * it reads): calls that overlap on one device, from any context or host
 * thread, race and must be serialised by the caller.  fmm_stats and
 * fmm_export describe the last call of the other entry points. */
fmm_status fmm_forces_noalloc(fmm_ctx* ctx, int64_t n, const double* pos, const double* mass,
                              double eps_soft, int p, double err_tol, double* acc, double* pot,
                              void* stream);

/* Largest number of systems one fmm_forces_batch call accepts. */
#define FMM_MAX_SYSTEMS 65536

/* Batched evaluation of nsys independent systems (an ensemble of clusters) in
 * one pass: system s is the bodies [offsets[s], offsets[s+1]) of pos/mass and
 * feels only its own bodies.  The result for each system is the one
 * fmm_forces gives for it alone (same per-system root box, Morton keys, tree,
 * estimate and interaction lists, section 2.1 and 2.3); the systems share
 * every launch: the sort orders bodies by (system, key), the tree is a forest
 * with one root per system (cells 0..nsys-1), and the walks start from every
 * (root, root) pair.  Cell ids are breadth first over the forest, so the cells
 * of one system appear in the order of that system's own tree.
 * offsets: HOST array of nsys + 1 values, offsets[0] = 0, strictly increasing
 * (every system holds at least one body), offsets[nsys] = total bodies; nsys
 * in 1..FMM_MAX_SYSTEMS, otherwise FMM_EINVAL.  Other arguments as fmm_forces;
 * acc and pot are in the caller's order over all systems. */
fmm_status fmm_forces_batch(fmm_ctx* ctx, int64_t nsys, const int64_t* offsets, const double* pos,
                            const double* mass, double eps_soft, int p, double err_tol,
                            double* acc, double* pot, void* stream);

/* Autotuner (for batched ensembles and single systems alike): picks, for this workload, when the
 * near field starts (p2p_start in {0, 1}, at the given n_leaf), the leaf
 * capacity n_leaf (the balance between the near field and the expansions),
 * then in mixed precision the FP32 M2L's wavefronts per sink (m2l_waves in
 * {1, 2, 4}), then the near field's lane groups per sink leaf (p2p_groups in
 * {0, 4, 2}), one parameter at a time at the best of the ones before, by
 * timing full evaluations of the systems given as for fmm_forces_batch (nsys =
 * 1, offsets = {0, n} for a single system): n_leaf in {16, 24, 32, 48, 64, 96,
 * 128}, one warm-up and two timed calls each, HIP events on the stream.  The
 * choices are set in the context's parameters (read them with fmm_get_params)
 * and n_leaf is also written to *chosen_n_leaf (host).  They are cached in the
 * process per (device, precision, p, err_tol, log2 of the body count, log2 of
 * the mean system size); a cached workload class returns at once without
 * running anything.  acc and pot receive the last evaluation.  Errors as
 * fmm_forces_batch; on error the parameters are unchanged. */
fmm_status fmm_autotune(fmm_ctx* ctx, int64_t nsys, const int64_t* offsets, const double* pos,
                        const double* mass, double eps_soft, int p, double err_tol, double* acc,
                        double* pot, void* stream, int* chosen_n_leaf);

/* Counts and per-stage times of the last call (synchronises its stream): the
 * cell and interaction-list sizes of the walk (section 2.1) and the interaction
 * counts behind the force-error/cost trade-off of section 4.1.  out: host.
 * FMM_EINVAL for NULL arguments. */
fmm_status fmm_stats(fmm_ctx* ctx, fmm_stats_t* out /* host */);

/* Copies an array of the last call into host memory (synchronises): the tree
 * and cells of section 2.1, the moments of section 2.2, the norms P_k, scalar
 * forces and interaction lists of section 2.3, the local expansions.  bytes
 * must be at least the size listed beside the selector (FMM_EINVAL otherwise);
 * FMM_ENOTBUILT if no call has produced the array yet. */
fmm_status fmm_export(fmm_ctx* ctx, int what, void* host_buf, size_t bytes);

/* Caps the context's device workspace (0 = no cap); exceeding it -> FMM_ENOMEM. */
fmm_status fmm_set_workspace_limit(fmm_ctx* ctx, size_t bytes);

/* Plain O(N^2) direct sum on the GPU for the sinks listed (device int32
 * indices, or all bodies when sinks == NULL), sources = all bodies.  Outputs
 * indexed like the sink list.  Used to measure force errors at large N. */
fmm_status fmm_direct(int64_t n, const double* pos, const double* mass, double eps_soft,
                      int64_t nsink, const int32_t* sinks, double* acc, double* pot,
                      void* stream);

const char* fmm_strerror(fmm_status s);
const char* fmm_last_error(fmm_ctx* ctx); /* detail of the last failure, "" if none */
void fmm_destroy(fmm_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* FMM_H */
