// Internal declarations of the gfx950 FMM library (not part of the C ABI).
//
// All translation units are compiled with -ffp-contract=off: every product and
// sum that feeds the acceptance test (centres, radii, P2M, M2M, P_k, the
// scalar-force estimate) is rounded exactly as written, in a fixed order, so
// the tree, the estimate and the interaction lists are reproducible bit for bit.
// Evaluation kernels (M2L, L2L, L2P, P2P) request fused multiply-adds
// explicitly with fma().
#pragma once

#include <hip/hip_runtime.h>

#include <functional>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fmm.h"
#include "fmm_limits.h"

#define FMM_MAX_LEVEL 21
#define FMM_GPU_PMAX 16  // orders with a register-resident (unrolled) M2L kernel; higher: m2l_hi.hip

namespace fmm {

constexpr int ncoef(int p) { return (p + 1) * (p + 2) / 2; }
__host__ __device__ constexpr int cidx(int n, int m) { return n * (n + 1) / 2 + m; }

// ------------------------------------------------------------------ buffers
struct hip_error {
  hipError_t code;
  std::string where;
};

void check(hipError_t e, const char* what);
#define HIPCHK(x) ::fmm::check((x), #x)

template <class T>
struct dbuf {
  T* p = nullptr;
  size_t cap = 0;      // elements
  unsigned epoch = 0;  // workspace epoch the allocation belongs to
};

struct Workspace;

// growable device allocation, tracked against the context's cap
void* ws_alloc(Workspace& w, size_t bytes);
void ws_free(Workspace& w, void* p, size_t bytes);

// Device workspace of a context.  Normally every buffer is its own hipMalloc.
// In arena mode (the allocation-free entry point) buffers are carved from a
// fixed region that the context does not own: nothing is allocated or freed,
// and each call starts a new epoch, so buffers of earlier calls count as
// absent and are carved again from the start of the region.
struct Workspace {
  size_t bytes = 0;
  size_t limit = 0;  // 0 = unlimited
  char* arena = nullptr;
  size_t arena_cap = 0, arena_used = 0;
  unsigned epoch = 0;
};

struct oom_error {};
// a valid request beyond what the data structures can index (FMM_EUNSUPPORTED)
struct unsupported_error {
  const char* what;
};

template <class T>
void ensure(Workspace& w, dbuf<T>& b, size_t n, bool keep = false, hipStream_t s = nullptr) {
  bool live = b.p && b.epoch == w.epoch;
  if (live && n <= b.cap) return;
  size_t ncap = n + n / 4 + 64;
  T* np = (T*)ws_alloc(w, ncap * sizeof(T));
  if (keep && live && b.cap) HIPCHK(hipMemcpyAsync(np, b.p, b.cap * sizeof(T), hipMemcpyDeviceToDevice, s));
  if (live) {
    if (keep) HIPCHK(hipStreamSynchronize(s));
    ws_free(w, b.p, b.cap * sizeof(T));
  }
  b.p = np;
  b.cap = ncap;
  b.epoch = w.epoch;
}

template <class T>
void release(Workspace& w, dbuf<T>& b) {
  if (b.p && b.epoch == w.epoch) ws_free(w, b.p, b.cap * sizeof(T));
  b.p = nullptr;
  b.cap = 0;
}

// ------------------------------------------------------------------ lists
// directed (sink, source) cell pairs grouped by sink: off[ncell+1], src[count]
struct CellList {
  dbuf<uint64_t> raw;  // emitted keys (sink << bits | source), any order
  dbuf<uint64_t> tmp;  // radix-sort ping-pong
  dbuf<int> off;       // CSR offsets by sink
  dbuf<int> src;       // sources, ascending within each sink
  int64_t count = 0;
};

// ------------------------------------------------------------------ near field
// Work items of the near-field kernels: item li < nleaf is leaf li of the leaf
// list (its whole source list, or the first segment of a long one); a leaf
// whose list is longer than K entries (and whose bodies fit one wavefront) is
// cut into ceil(len / K) contiguous segments, and segments 1.. are the extra
// items (leaf, segment) after the leaves, in any order.  The first segment
// writes the near field itself, segment k > 0 its partial sums to slots
// cell_pbase[B] + (k - 1) n_B + body; these are added in segment order
// afterwards, so the result does not depend on the order of the items.
struct NfPlan {
  const int* cell_nseg;   // segments of each leaf, by cell id
  const int* cell_pbase;  // first partial slot of each split leaf, by cell id
  const int2* extra;      // (leaf index, segment) of the extra items
  const int* nextra;      // extra item count (device)
  int nleaf;
  int K;                  // list entries per segment
  int max_items;          // host bound on the item count (grid size)
  int max_slots;          // host bound on the partial slots
};

// Work items of the FP64 M2L over whole lists: item B < ncell is sink B (its
// whole list, or the first K pairs of a long one), and a sink with more than
// K pairs appends its later segments (sink, segment) as extra items, which
// write partial expansions to slots pbase[B] + segment - 1; these are added
// to the sink's expansion in segment order afterwards.
struct M2lSeg {
  const int* nseg;    // segments of each sink (null: one item per sink)
  const int* pbase;   // first partial slot of each split sink
  const int2* extra;  // (sink, segment) of the extra items
  const int* nextra;  // extra item count (device)
  double* part;       // partial expansions, one slot each
  int K;              // pairs per segment
  int max_items;      // host bound on the item count (grid size)
};

// ------------------------------------------------------------------ context
struct Ctx {
  fmm_params prm{};
  int device = 0;
  std::string err;
  Workspace ws;
  hipStream_t stream = nullptr;

  int64_t n = 0;
  int p = 0;            // order of the last call
  double err_tol = 0;
  double eps_soft = 0;
  bool built = false, estimated = false, walked = false, evaluated = false;
  // the last evaluation was one FP64 system: its tree, lists, local
  // expansions and near-field plan serve fmm_adjoint_last
  bool adjoint_ready = false;

  // bodies (sorted order)
  dbuf<uint64_t> key[2];
  dbuf<int> idx[2];
  dbuf<double> sx, sy, sz, sm;
  dbuf<double4> pm;   // packed (x, y, z, m), sorted order
  dbuf<double> fpart;
  dbuf<int> leaf_of;  // leaf id of each sorted body
  dbuf<int> leaves;   // ids of the leaf cells, ascending (built by the upward pass)

  // radix sort scratch
  dbuf<int> sort_hist;

  // independent systems evaluated together (a forest: one root per system);
  // bodies of system s are [sys_off[s], sys_off[s+1]) in caller and sorted order
  int nsys = 1;
  std::vector<int64_t> h_sys_off;
  dbuf<int> sys_off;
  std::vector<int> sys_off_uploaded;  // host image of sys_off's current contents
  dbuf<uint64_t> skey[2];  // second sort pass (by system), ping-pong
  dbuf<int> spos[2];

  // bbox scratch: per-block min/max, then lo[3], L, s
  dbuf<double> bbox_part;
  dbuf<double> rootbox;  // per system: lo[3], L, s (stride 8 doubles)

  // cells (breadth-first ids)
  int64_t ncell = 0, nleaf = 0;
  int depth = 0;
  std::vector<int> lvl_first, lvl_count;
  dbuf<int> c_level, c_begin, c_end, c_parent, c_child0, c_nchild;
  dbuf<int> c_split;  // per-cell scratch for the level build (9 octant starts)
  dbuf<double> c_mass, c_sx, c_sy, c_sz;  // mass and first moments
  dbuf<double> c_cx, c_cy, c_cz, c_rad;   // centre of mass and radius
  dbuf<unsigned long long> c_rad2bits;
  dbuf<double> mult;  // ncell x ncoef x 2
  dbuf<double> pk;    // ncell x (p+1)
  dbuf<double> pkb;   // ncell x (p+1): C(p, k) * P_k, as the acceptance test forms it
  dbuf<double> fcell, fmin;
  // chunks of <= CELL_CHUNK sorted bodies per cell (the radius and the cell
  // minima of the estimate walk them): first chunk of each cell; the total
  // stays on the device at counters[4..5]
  dbuf<int> cell_choff;
  dbuf<double4> c_geo;  // (cx, cy, cz, rad) per cell, packed for the walks
  dbuf<double> loc;   // ncell x ncoef x 2
  dbuf<double> loc64; // mixed precision: FP64 M2L of the root-level pairs, added to loc
  dbuf<int> root_sinks;  // mixed precision: the sinks that have root-level pairs
  dbuf<double> scale; // mixed precision: expansion scale per cell
  dbuf<float> nmult;  // mixed precision: normalised FP32 moments, (p+1)^2 per cell

  // adjoint pass: expansions of the adjoint sources, sorted (ga, gp) and
  // forward acceleration, forward outputs of the recomputed pass
  dbuf<double> madj, ladj, fwd_acc, fwd_pot;
  dbuf<double4> gsort, asort;
  dbuf<double4> adjnear;  // adjoint near sums per sorted body: (grad Psi, Psi), (tidal term, 0)
  dbuf<double4> adjpart;  // their partial sums for split leaves (two records per slot)

  // walks
  dbuf<int2> front[2];
  // device counters (ints), by offset: [0..1] scan total (long long) of the
  // tree's level loop; [2] leaves counted by the level loop; [4..5] number of
  // body chunks of the cells (long long, read by the radius and cell-minimum
  // kernels); [32] input check; [40..41] near-field body pairs; [48..49]
  // FP32 M2L pairs (stats); [64] sinks with root-level pairs; [256..] walk
  // (64-bit counters at even int offsets)
  dbuf<int> counters;
  CellList est_far, est_near, m2l, p2p;
  int64_t n_p2p_pairs = 0;

  // scan scratch
  dbuf<int> scan_tmp;
  dbuf<long long> scan_tmp64;
  // second and third sets of sort and scan scratch for work on the side
  // streams that runs while the caller's stream sorts or scans (SideScratch)
  dbuf<int> sort_hist2, scan_tmp2, sort_hist3, scan_tmp3;

  // host pinned scratch for small read-backs
  long long* hbuf = nullptr;

  // timing
  // timing events: stage boundaries 0..8 on the caller's stream; 9, 10 around
  // the main M2L kernel; 11..13 the local stage around the join with the
  // near field; 14 the end of the upward pass on the side stream; 15..17 the
  // body sort (after the keys, after the sort, after the gather); 18 the end
  // of the acceptance walk (before its lists are grouped)
  hipEvent_t ev[19] = {};
  // second stream (default priority) for work independent of the caller's
  // stream: the upward pass beside the estimate walk, the near field beside
  // M2L and L2L; forked and joined with the events below
  hipStream_t side = nullptr, side2 = nullptr;  // side2: root-level FP64 M2L
  hipEvent_t fork[9] = {};
  dbuf<double4> nearbuf;  // near-field (acc, pot) per sorted body
  // near-field work items (plan_near_field) and the partial sums of split leaves
  dbuf<int> nf_cell_nseg, nf_cell_pbase;
  dbuf<int2> nf_extra;
  dbuf<double4> nf_part;
  NfPlan nf{};
  dbuf<int> m2l_nseg, m2l_pbase;
  dbuf<int2> m2l_extra;
  dbuf<double> m2l_part;

  // replay of the frozen-tree evaluation as a HIP graph (captured per set of
  // buffers; dropped whenever the tree is rebuilt)
  hipGraphExec_t gexec = nullptr;
  hipStream_t cap = nullptr;  // capture stream (the caller's may be the null stream)
  bool graph_valid = false;
  const void* gkey[5] = {};
  double gkey_eps = 0.0;
  bool have_events = false;
};

// Sorts and scans take their scratch from c.sort_hist and c.scan_tmp; within
// this scope they use the second (set = 2) or third (set = 3) set, so that
// sorts on the side streams may run concurrently with one on the caller's.
struct SideScratch {
  Ctx& c;
  dbuf<int>&h, &t;
  SideScratch(Ctx& cc, int set)
      : c(cc), h(set == 2 ? cc.sort_hist2 : cc.sort_hist3), t(set == 2 ? cc.scan_tmp2 : cc.scan_tmp3) {
    std::swap(c.sort_hist, h);
    std::swap(c.scan_tmp, t);
  }
  ~SideScratch() {
    std::swap(c.sort_hist, h);
    std::swap(c.scan_tmp, t);
  }
};

// launches of a scope go to another stream of the context
struct OnStream {
  Ctx& c;
  hipStream_t old;
  OnStream(Ctx& cc, hipStream_t s) : c(cc), old(cc.stream) { c.stream = s; }
  ~OnStream() { c.stream = old; }
};

// `to` waits (on the device) for the work enqueued so far on `from`
void stream_wait(hipEvent_t e, hipStream_t from, hipStream_t to);

// ------------------------------------------------------------------ stages
void exclusive_scan(Ctx& c, const int* in, int* out, int64_t n, long long* total_dev);
long long read_total(Ctx& c, const long long* total_dev);
int radix_sort(Ctx& c, uint64_t* k0, int* v0, uint64_t* k1, int* v1, int64_t n, int nbits);
uint32_t* radix_sort_narrow(Ctx& c, const uint64_t* in, uint32_t* b0, uint32_t* b1, int64_t n, int nbits);

void build_tree(Ctx& c, int64_t n, const double* pos, const double* mass);
void upward_pass(Ctx& c);
void expansions_up(Ctx& c);
void cell_moments(Ctx& c, bool with_radius);
constexpr int CELL_CHUNK = 1024;  // bodies per chunk of a cell (radius, cell minima)
// per-cell maximum (radius) or minimum (estimate) over the cells' bodies, a
// wavefront per chunk; grid for every chunk the tree can have
unsigned cell_chunk_blocks(const Ctx& c, int waves_per_block);
void zero_fill(Ctx& c, void* p, size_t bytes);
void refresh_frozen(Ctx& c, const double* pos, const double* mass);
// the scalar-force estimate; beside (if any) is called once while the walk
// runs on the device, to enqueue independent work on another stream
void estimate_walk(Ctx& c, const std::function<void()>& beside = {});
void mac_walk(Ctx& c);  // lists left ungrouped: see group_list
void group_list(Ctx& c, CellList& L);
void evaluate(Ctx& c, double* acc, double* pot, bool group);
void launch_normalize32(Ctx& c);
void direct_sum(int64_t n, const double* pos, const double* mass, double eps2, int64_t nsink,
                const int32_t* sinks, double* acc, double* pot, hipStream_t s);
bool check_inputs_dev(Ctx& c, const double* pos, const double* mass, int64_t n);

// M2L launchers (one per compiled order)
void launch_m2l_fp64(Ctx& c);
// constant tables of the kernels, uploaded once per device at context creation
void upload_up_tables();
void upload_m2l_tables();
void upload_hi_tables();
// generic-order FP64 M2L (any p <= 30; m2l_hi.hip), over every sink or the listed ones
void launch_m2l_hi(Ctx& c, int first_lo, const double* mult, double* loc, const int* sinks, const int* nsinks);
void launch_m2l_fp64_range(Ctx& c, int first_lo);
void launch_m2l_fp64_buffers(Ctx& c, int first_lo, const double* mult, double* loc);
void launch_m2l_fp64_sinks(Ctx& c, int first_lo, const double* mult, double* loc, const int* sinks,
                           const int* nsinks);
void m2m_levels(Ctx& c, double* mult);
void launch_l2l_buf(Ctx& c, double* loc);
void launch_near_field(Ctx& c);
void plan_near_field(Ctx& c);
void launch_far_final(Ctx& c, double* acc, double* pot);
void launch_m2l_mixed_lo(Ctx& c);
void launch_m2l_mixed_root(Ctx& c, double* loc64);
void add_root_locals(Ctx& c, double* loc, const double* loc64);
int mixed_first_lo(Ctx& c);
bool mixed_supported(int p);
void adjoint_pass(Ctx& c, const double* gacc, const double* gpot, const double* acc_fwd, double* gpos,
                  double* gmass);
void jerk_pass(Ctx& c, const double* vel, const double* mass, double* jerk);

}  // namespace fmm
