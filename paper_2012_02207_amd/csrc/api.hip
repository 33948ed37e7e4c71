// C ABI of the gfx950 FMM library (declared in include/fmm.h): argument
// validation, workspace ownership, stage orchestration, statistics and export.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>

#include "fmm_device.h"

struct fmm_ctx {
  fmm::Ctx c;
  fmm::Ctx* na = nullptr;  // state of fmm_forces_noalloc (buffers in the static scratch)
};

namespace fmm {

void check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw hip_error{e, what};
}

void* ws_alloc(Workspace& w, size_t bytes) {
  if (w.arena) {  // carve from the fixed region: no allocation
    size_t at = (w.arena_used + 255) & ~(size_t)255;
    if (at + bytes > w.arena_cap) throw oom_error{};
    w.arena_used = at + bytes;
    return w.arena + at;
  }
  if (w.limit && w.bytes + bytes > w.limit) throw oom_error{};
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes ? bytes : 1);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    (void)hipGetLastError();
    throw oom_error{};
  }
  check(e, "hipMalloc");
  w.bytes += bytes;
  return p;
}

void ws_free(Workspace& w, void* p, size_t bytes) {
  if (w.arena) return;  // the region outlives the call; its epoch ends with it
  (void)hipFree(p);
  w.bytes -= bytes;
}

// ---- device scratch of the allocation-free entry point ----------------------
// One static array per device, held until the process ends.  In host code the
// name `scratch` is a host-side stand-in, not a device address: its device
// address is taken once per device with hipGetSymbolAddress (with that device
// current) and only that address is ever handed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[FMM_NOALLOC_SCRATCH_BYTES];
static void* g_scratch_dev[64] = {};  // device address of `scratch`, per device
static std::mutex g_scratch_mu;

static void* scratch_address(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev < 0 || dev >= 64) throw unsupported_error{"device ordinal above 63"};
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_dev[dev] = ptr;
  }
  return g_scratch_dev[dev];
}

// zeroing by a kernel (not hipMemsetAsync), so the sequences stay capturable
__global__ void k_zero32(uint32_t* p, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

void zero_fill(Ctx& c, void* p, size_t bytes) {
  int64_t n = (int64_t)(bytes / 4);
  if (n <= 0) return;
  hipLaunchKernelGGL(k_zero32, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c.stream, (uint32_t*)p, n);
  HIPCHK(hipGetLastError());
}


// stream `to` waits for the work enqueued so far on `from` (event e)
void stream_wait(hipEvent_t e, hipStream_t from, hipStream_t to) {
  HIPCHK(hipEventRecord(e, from));
  HIPCHK(hipStreamWaitEvent(to, e, 0));
}
void launch_l2l(Ctx& c);


// M2L pairs with both cells at or below first_lo (the FP32 part of mixed mode)
__global__ void k_count_low_pairs(const int* off, const int* src, int ncell, int first_lo,
                                  unsigned long long* out) {
  int B = first_lo + blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long s = 0;
  if (B < ncell) {  // sources ascending: count those >= first_lo by a lower bound
    int lo = off[B], hi = off[B + 1], e = hi;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (src[mid] < first_lo)
        lo = mid + 1;
      else
        hi = mid;
    }
    s = (unsigned long long)(e - lo);
  }
  if (s) atomicAdd(out, s);
}

// The near field (and, in mixed precision, the FP64 M2L of the root-level
// pairs into a buffer of its own) on the side stream run beside the main M2L
// on the caller's stream (both ALU bound, with different occupancy limits);
// after the join the root-level part is added (for the sinks that have one),
// then L2L and the final L2P + sum.  loc gets exactly one contribution per
// kernel, so the order of the two M2L parts does not change the result.
// group: the lists come straight from the walk; the near-field list is
// grouped on the side stream (with its own sort scratch) while the M2L list is
// grouped on the caller's stream; with p2p_start = 1 the near field waits for
// both groupings.
void evaluate(Ctx& c, double* acc, double* pot, bool group) {
  hipStream_t s = c.stream;
  int nc = (int)c.ncell;
  size_t nl = (size_t)nc * ncoef(c.p) * 2;
  bool mixed = c.prm.precision == FMM_MIXED;
  bool root64 = mixed && mixed_first_lo(c) > 0;
  ensure(c.ws, c.loc, nl);
  ensure(c.ws, c.nearbuf, (size_t)c.n);
  if (root64) ensure(c.ws, c.loc64, nl);
  stream_wait(c.fork[2], s, c.side);
  // the (longer) M2L grouping is enqueued first, so that it runs while the
  // host enqueues the other
  if (group) group_list(c, c.m2l);
  {
    OnStream on(c, c.side);
    if (group) {
      SideScratch alt(c, 2);
      group_list(c, c.p2p);
      if (c.prm.p2p_start == 1) stream_wait(c.fork[8], s, c.side);
    }
    if (c.have_events) HIPCHK(hipEventRecord(c.ev[6], c.side));
    launch_near_field(c);
    if (c.have_events) HIPCHK(hipEventRecord(c.ev[7], c.side));
  }
  if (root64) {  // a few long interaction lists: a kernel of its own beside the others
    stream_wait(c.fork[5], s, c.side2);
    OnStream on(c, c.side2);
    launch_m2l_mixed_root(c, c.loc64.p);
  }
  if (c.have_events) HIPCHK(hipEventRecord(c.ev[4], s));
  // the M2L kernels write every sink they cover (zeros where there is no
  // pair); in mixed precision the root-level cells are not covered by the FP32
  // kernel and start at zero here
  if (mixed) zero_fill(c, c.loc.p, (size_t)mixed_first_lo(c) * ncoef(c.p) * 2 * sizeof(double));
  if (mixed)
    launch_m2l_mixed_lo(c);
  else
    launch_m2l_fp64(c);
  stream_wait(c.fork[3], c.side, s);
  if (root64) stream_wait(c.fork[4], c.side2, s);
  if (root64) add_root_locals(c, c.loc.p, c.loc64.p);
  if (c.have_events) HIPCHK(hipEventRecord(c.ev[5], s));
  launch_l2l(c);
  if (c.have_events) HIPCHK(hipEventRecord(c.ev[11], s));
  if (c.have_events) HIPCHK(hipEventRecord(c.ev[12], s));
  launch_far_final(c, acc, pot);
  if (c.have_events) HIPCHK(hipEventRecord(c.ev[13], s));
}

}  // namespace fmm

using namespace fmm;

static fmm_status validate_params(const fmm_params* p) {
  if (p->p < 1 || p->p > 30) return FMM_EINVAL;
  if (!(p->err_tol > 0) || !std::isfinite(p->err_tol)) return FMM_EINVAL;
  if (!(p->theta > 0) || p->theta > 1.0 || !(p->theta_est > 0) || p->theta_est > 1.0) return FMM_EINVAL;
  if (p->n_leaf < 1 || p->n_leaf > 1024) return FMM_EINVAL;
  if (p->precision < FMM_FP64 || p->precision > FMM_DIRECT) return FMM_EINVAL;
  if (p->mac != FMM_MAC_ERROR && p->mac != FMM_MAC_GEOMETRIC) return FMM_EINVAL;
  if (p->root_levels < 0 || p->root_levels > FMM_MAX_LEVEL + 1) return FMM_EINVAL;
  if (p->m2l_waves != 1 && p->m2l_waves != 2 && p->m2l_waves != 4) return FMM_EINVAL;
  if (p->p2p_groups < 0 || p->p2p_groups > 64) return FMM_EINVAL;
  if (p->p2p_start != 0 && p->p2p_start != 1) return FMM_EINVAL;
  return FMM_OK;
}

template <class F>
static fmm_status guarded(fmm_ctx* ctx, F&& f) {
  try {
    return f();
  } catch (const hip_error& e) {
    if (ctx) {
      ctx->c.err = std::string(e.where) + ": " + hipGetErrorString(e.code);
      (void)hipGetLastError();
    }
    return FMM_EHIP;
  } catch (const oom_error&) {
    if (ctx) ctx->c.err = "device workspace allocation failed or exceeded the cap";
    return FMM_ENOMEM;
  } catch (const unsupported_error& e) {
    if (ctx) ctx->c.err = e.what;
    return FMM_EUNSUPPORTED;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->c.err = "host allocation failed";
    return FMM_ENOMEM;
  }
}

extern "C" {

void fmm_default_params(fmm_params* out) {
  if (!out) return;
  out->p = 10;
  out->err_tol = 1e-7;
  out->theta = 1.0;
  out->theta_est = 1.0;
  out->n_leaf = 64;
  out->precision = FMM_FP64;
  out->mac = FMM_MAC_ERROR;
  out->check_inputs = 0;
  out->root_levels = 3;
  out->m2l_waves = 1;
  out->p2p_groups = 0;
  out->p2p_start = 0;
}

fmm_status fmm_create(fmm_ctx** out, const fmm_params* prm) {
  if (!out) return FMM_EINVAL;
  *out = nullptr;
  fmm_params p;
  fmm_default_params(&p);
  if (prm) p = *prm;
  fmm_status st = validate_params(&p);
  if (st != FMM_OK) return st;
  fmm_ctx* ctx = new (std::nothrow) fmm_ctx();
  if (!ctx) return FMM_ENOMEM;
  ctx->na = new (std::nothrow) Ctx();
  if (!ctx->na) {
    delete ctx;
    return FMM_ENOMEM;
  }
  ctx->c.prm = p;
  st = guarded(ctx, [&]() {
    for (Ctx* c : {&ctx->c, ctx->na}) {
      HIPCHK(hipGetDevice(&c->device));
      HIPCHK(hipHostMalloc((void**)&c->hbuf, 128 * sizeof(long long), hipHostMallocDefault));
      for (auto& e : c->ev) HIPCHK(hipEventCreate(&e));
      for (auto& e : c->fork) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      HIPCHK(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
      HIPCHK(hipStreamCreateWithFlags(&c->side2, hipStreamNonBlocking));
      HIPCHK(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    }
    // everything the allocation-free entry point needs is set up here: the
    // kernels' constant tables, the scratch address on this device, and host
    // containers sized so that its calls do not grow them
    upload_up_tables();
    upload_m2l_tables();
    upload_hi_tables();
    Ctx& na = *ctx->na;
    na.ws.arena = (char*)scratch_address(na.device);
    na.ws.arena_cap = FMM_NOALLOC_SCRATCH_BYTES;
    na.ws.epoch = 1;
    na.h_sys_off.reserve(4);
    na.sys_off_uploaded.reserve(4);
    na.lvl_first.reserve(FMM_MAX_LEVEL + 8);
    na.lvl_count.reserve(FMM_MAX_LEVEL + 8);
    ctx->c.err.reserve(256);
    return FMM_OK;
  });
  if (st != FMM_OK) {
    fmm_destroy(ctx);
    return st;
  }
  *out = ctx;
  return FMM_OK;
}

fmm_status fmm_set_params(fmm_ctx* ctx, const fmm_params* prm) {
  if (!ctx || !prm) return FMM_EINVAL;
  fmm_status st = validate_params(prm);
  if (st != FMM_OK) return st;
  ctx->c.prm = *prm;
  ctx->c.graph_valid = false;  // a captured graph holds the old precision and root split
  return FMM_OK;
}

static fmm_status common_checks(fmm_ctx* ctx, int64_t n, const double* pos, const double* mass) {
  if (!ctx || !pos || !mass || n < 1) return FMM_EINVAL;
  if (n > (int64_t)0x3fffffff) return FMM_EUNSUPPORTED;
  return FMM_OK;
}

static void run_build(Ctx& c, int64_t n, const double* pos, const double* mass) {
  c.built = c.estimated = c.walked = c.evaluated = false;
  c.adjoint_ready = false;
  c.graph_valid = false;
  build_tree(c, n, pos, mass);
  if (c.have_events) HIPCHK(hipEventRecord(c.ev[1], c.stream));
  upward_pass(c);
  if (c.have_events) HIPCHK(hipEventRecord(c.ev[2], c.stream));
  c.built = true;
}

// Tree, then the upward pass (P2M, M2M, P_k) on the side stream beside the
// scalar-force estimate on the caller's stream (the estimate needs the cells,
// not the multipoles); joined before the acceptance walk, which needs both.
static void build_and_estimate(Ctx& c, int64_t n, const double* pos, const double* mass) {
  c.built = c.estimated = c.walked = c.evaluated = false;
  c.graph_valid = false;
  build_tree(c, n, pos, mass);
  HIPCHK(hipEventRecord(c.ev[1], c.stream));
  stream_wait(c.fork[0], c.stream, c.side);
  HIPCHK(hipEventRecord(c.ev[2], c.stream));
  // the upward pass goes to the side stream while the estimate walk runs, so
  // that neither waits for the other's launches
  estimate_walk(c, [&]() {
    OnStream on(c, c.side);
    upward_pass(c);
    HIPCHK(hipEventRecord(c.ev[14], c.side));
  });
  c.built = true;
  c.estimated = true;
  stream_wait(c.fork[1], c.side, c.stream);
  HIPCHK(hipEventRecord(c.ev[3], c.stream));
}

fmm_status fmm_build(fmm_ctx* ctx, int64_t n, const double* pos, const double* mass, void* stream) {
  fmm_status st = common_checks(ctx, n, pos, mass);
  if (st != FMM_OK) return st;
  Ctx& c = ctx->c;
  return guarded(ctx, [&]() {
    c.stream = (hipStream_t)stream;
    c.err.clear();
    c.p = c.prm.p;
    c.err_tol = c.prm.err_tol;
    c.nsys = 1;
    c.h_sys_off.assign({0, n});
    if (c.prm.check_inputs && !check_inputs_dev(c, pos, mass, n)) return FMM_EDATA;
    c.have_events = true;
    HIPCHK(hipEventRecord(c.ev[0], c.stream));
    run_build(c, n, pos, mass);
    return FMM_OK;
  });
}

// one evaluation on the context state c (the caller's, or the allocation-free
// one); errors are reported through ctx
static fmm_status forces_on(fmm_ctx* ctx, Ctx& c, int64_t nsys, const int64_t* offsets, int64_t n,
                            const double* pos, const double* mass, double eps_soft, int p,
                            double err_tol, double* acc, double* pot, void* stream) {
  fmm_status st = common_checks(ctx, n, pos, mass);
  if (st != FMM_OK) return st;
  if (!acc || !pot) return FMM_EINVAL;
  if (!(eps_soft >= 0) || !std::isfinite(eps_soft)) return FMM_EINVAL;
  if (p < 1 || p > 30) return FMM_EINVAL;
  if (!(err_tol > 0) || !std::isfinite(err_tol)) return FMM_EINVAL;
  return guarded(ctx, [&]() {
    c.stream = (hipStream_t)stream;
    c.err.clear();
    c.adjoint_ready = false;
    c.p = p;
    c.err_tol = err_tol;
    c.eps_soft = eps_soft;
    c.nsys = (int)nsys;
    c.h_sys_off.assign(offsets, offsets + nsys + 1);
    if (c.prm.check_inputs && !check_inputs_dev(c, pos, mass, n)) return FMM_EDATA;
    if (c.prm.precision == FMM_DIRECT) {
      c.have_events = false;
      for (int64_t s = 0; s < nsys; s++) {
        int64_t b = offsets[s], m = offsets[s + 1] - b;
        direct_sum(m, pos + 3 * b, mass + b, eps_soft * eps_soft, m, nullptr, acc + 3 * b, pot + b,
                   c.stream);
      }
      return FMM_OK;
    }
    c.have_events = true;
    HIPCHK(hipEventRecord(c.ev[0], c.stream));
    build_and_estimate(c, n, pos, mass);
    mac_walk(c);
    HIPCHK(hipEventRecord(c.ev[18], c.stream));
    c.walked = true;
    evaluate(c, acc, pot, true);
    c.evaluated = true;
    c.adjoint_ready = c.prm.precision == FMM_FP64 && nsys == 1;
    HIPCHK(hipEventRecord(c.ev[8], c.stream));
    return FMM_OK;
  });
}

static fmm_status forces_impl(fmm_ctx* ctx, int64_t nsys, const int64_t* offsets, int64_t n,
                              const double* pos, const double* mass, double eps_soft, int p,
                              double err_tol, double* acc, double* pot, void* stream) {
  if (!ctx) return FMM_EINVAL;
  return forces_on(ctx, ctx->c, nsys, offsets, n, pos, mass, eps_soft, p, err_tol, acc, pot, stream);
}

fmm_status fmm_forces(fmm_ctx* ctx, int64_t n, const double* pos, const double* mass, double eps_soft,
                      int p, double err_tol, double* acc, double* pot, void* stream) {
  int64_t off[2] = {0, n};
  return forces_impl(ctx, 1, off, n, pos, mass, eps_soft, p, err_tol, acc, pot, stream);
}

fmm_status fmm_forces_noalloc(fmm_ctx* ctx, int64_t n, const double* pos, const double* mass,
                              double eps_soft, int p, double err_tol, double* acc, double* pot,
                              void* stream) {
  if (!ctx || !ctx->na) return FMM_EINVAL;
  if (n > FMM_NOALLOC_MAX_N) {
    ctx->c.err = "fmm_forces_noalloc: n exceeds FMM_NOALLOC_MAX_N";
    return FMM_EINVAL;
  }
  Ctx& a = *ctx->na;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != a.device) {
    (void)hipGetLastError();
    ctx->c.err = "fmm_forces_noalloc: called with another device current than at fmm_create";
    return FMM_EINVAL;
  }
  a.prm = ctx->c.prm;
  a.ws.arena_used = 0;  // a new epoch: the buffers of earlier calls are gone
  a.ws.epoch++;
  if (a.ws.epoch == 0) a.ws.epoch = 1;
  a.sys_off_uploaded.clear();
  a.graph_valid = false;
  int64_t off[2] = {0, n};
  fmm_status st = forces_on(ctx, a, 1, off, n, pos, mass, eps_soft, p, err_tol, acc, pot, stream);
  if (st == FMM_ENOMEM) ctx->c.err = "fmm_forces_noalloc: the static scratch is too small for this input";
  return st;
}

fmm_status fmm_forces_batch(fmm_ctx* ctx, int64_t nsys, const int64_t* offsets, const double* pos,
                            const double* mass, double eps_soft, int p, double err_tol, double* acc,
                            double* pot, void* stream) {
  if (!offsets || nsys < 1 || nsys > FMM_MAX_SYSTEMS) return FMM_EINVAL;
  if (offsets[0] != 0) return FMM_EINVAL;
  for (int64_t s = 0; s < nsys; s++)
    if (offsets[s + 1] <= offsets[s]) return FMM_EINVAL;  // every system holds a body
  return forces_impl(ctx, nsys, offsets, offsets[nsys], pos, mass, eps_soft, p, err_tol, acc, pot,
                     stream);
}

fmm_status fmm_stats(fmm_ctx* ctx, fmm_stats_t* out) {
  if (!ctx || !out) return FMM_EINVAL;
  Ctx& c = ctx->c;
  std::memset(out, 0, sizeof(*out));
  if (!c.built) return FMM_ENOTBUILT;
  return guarded(ctx, [&]() {
    HIPCHK(hipStreamSynchronize(c.stream));
    out->n = c.n;
    out->ncell = c.ncell;
    out->nleaf = c.nleaf;
    out->depth = c.depth;
    out->workspace_bytes = c.ws.bytes;
    out->nsys = c.nsys;
    if (c.walked) {
      out->n_m2l = c.m2l.count;
      out->n_p2p_cells = c.p2p.count;
      out->n_m2l_fp32 = 0;
      if (c.prm.precision == FMM_MIXED) {
        int first_lo = mixed_first_lo(c);
        unsigned long long* d = (unsigned long long*)(c.counters.p + 48);
        HIPCHK(hipMemsetAsync(d, 0, 8, c.stream));
        int cnt = (int)c.ncell - first_lo;
        if (cnt > 0)
          hipLaunchKernelGGL(k_count_low_pairs, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0,
                             c.stream, c.m2l.off.p, c.m2l.src.p, (int)c.ncell, first_lo, d);
        HIPCHK(hipMemcpyAsync(c.hbuf + 1, d, 8, hipMemcpyDeviceToHost, c.stream));
        HIPCHK(hipStreamSynchronize(c.stream));
        out->n_m2l_fp32 = c.hbuf[1];
      }
      // body-pair count of the near field
      if (c.evaluated) {  // counted by the leaf kernel of the last evaluation
        unsigned long long* d = (unsigned long long*)(c.counters.p + 40);
        HIPCHK(hipMemcpyAsync(c.hbuf, d, 8, hipMemcpyDeviceToHost, c.stream));
        HIPCHK(hipStreamSynchronize(c.stream));
        out->n_p2p_pairs = c.hbuf[0];
        // the near field's work items: the leaves and the extra segments
        HIPCHK(hipMemcpyAsync(c.hbuf, c.counters.p + 44, 4, hipMemcpyDeviceToHost, c.stream));
        HIPCHK(hipStreamSynchronize(c.stream));
        out->n_p2p_items = (int64_t)c.nleaf + *(const int*)c.hbuf;
      }
    }
    if (c.estimated) {
      out->n_est_far = c.est_far.count;
      out->n_est_near = c.est_near.count;
    }
    auto el = [&](int a, int b) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, c.ev[a], c.ev[b]) != hipSuccess) {
        (void)hipGetLastError();
        return 0.0;
      }
      return (double)ms;
    };
    if (c.have_events) {
      out->ms_tree = el(0, 1);
      if (c.evaluated) {
        // upward pass (side stream) and estimate (caller's stream) both start
        // at the end of the tree and overlap; so do the near field (side) and
        // M2L + L2L; ms_local is L2L plus the final L2P and sum
        out->ms_upward = el(1, 14);
        out->ms_estimate = el(2, 3);
        out->ms_walk = el(3, 4);
        out->ms_m2l = el(4, 5);
        out->ms_local = el(5, 11) + el(12, 13);
        out->ms_p2p = el(6, 7);
        out->ms_total = el(0, 8);
        out->ms_m2l_kernel = el(9, 10);
        out->ms_sort = el(15, 16);
        out->ms_gather = el(16, 17);
        out->ms_walk_steps = el(3, 18);
      } else {
        out->ms_upward = el(1, 2);
        out->ms_total = el(0, 2);
      }
    }
    return FMM_OK;
  });
}

fmm_status fmm_export(fmm_ctx* ctx, int what, void* host_buf, size_t bytes) {
  if (!ctx || !host_buf) return FMM_EINVAL;
  Ctx& c = ctx->c;
  if (!c.built) return FMM_ENOTBUILT;
  int64_t nc = c.ncell, n = c.n;
  size_t ncf = (size_t)ncoef(c.p) * 2;
  const void* src = nullptr;
  size_t need = 0;
  const CellList* lst = nullptr;
  switch (what) {
    case FMM_X_KEYS: src = c.key[0].p; need = n * 8; break;
    case FMM_X_PERM: src = c.idx[0].p; need = n * 4; break;
    case FMM_X_CELL_LEVEL: src = c.c_level.p; need = nc * 4; break;
    case FMM_X_CELL_BEGIN: src = c.c_begin.p; need = nc * 4; break;
    case FMM_X_CELL_END: src = c.c_end.p; need = nc * 4; break;
    case FMM_X_CELL_PARENT: src = c.c_parent.p; need = nc * 4; break;
    case FMM_X_CELL_CHILD0: src = c.c_child0.p; need = nc * 4; break;
    case FMM_X_CELL_NCHILD: src = c.c_nchild.p; need = nc * 4; break;
    case FMM_X_CELL_MASS: src = c.c_mass.p; need = nc * 8; break;
    case FMM_X_CELL_COM: break;
    case FMM_X_CELL_RAD: src = c.c_rad.p; need = nc * 8; break;
    case FMM_X_MULT: src = c.mult.p; need = nc * ncf * 8; break;
    case FMM_X_PK: src = c.pk.p; need = nc * (c.p + 1) * 8; break;
    case FMM_X_FCELL: if (!c.estimated) return FMM_ENOTBUILT; src = c.fcell.p; need = nc * 8; break;
    case FMM_X_FPART: if (!c.estimated) return FMM_ENOTBUILT; src = c.fpart.p; need = n * 8; break;
    case FMM_X_FMIN: if (!c.estimated) return FMM_ENOTBUILT; src = c.fmin.p; need = nc * 8; break;
    case FMM_X_EST_FAR: if (!c.estimated) return FMM_ENOTBUILT; lst = &c.est_far; break;
    case FMM_X_EST_NEAR: if (!c.estimated) return FMM_ENOTBUILT; lst = &c.est_near; break;
    case FMM_X_M2L: if (!c.walked) return FMM_ENOTBUILT; lst = &c.m2l; break;
    case FMM_X_P2P: if (!c.walked) return FMM_ENOTBUILT; lst = &c.p2p; break;
    case FMM_X_LOCAL: if (!c.evaluated) return FMM_ENOTBUILT; src = c.loc.p; need = nc * ncf * 8; break;
    case FMM_X_ROOTBOX: break;
    default: return FMM_EINVAL;
  }
  return guarded(ctx, [&]() {
    HIPCHK(hipStreamSynchronize(c.stream));
    if (what == FMM_X_ROOTBOX) {  // 5 values per system from the stride-8 device layout
      if (bytes < (size_t)c.nsys * 40) return FMM_EINVAL;
      std::vector<double> t((size_t)c.nsys * 8);
      HIPCHK(hipMemcpy(t.data(), c.rootbox.p, t.size() * 8, hipMemcpyDeviceToHost));
      double* o = (double*)host_buf;
      for (int s = 0; s < c.nsys; s++)
        for (int k = 0; k < 5; k++) o[5 * s + k] = t[8 * s + k];
      return FMM_OK;
    }
    if (what == FMM_X_CELL_COM) {
      if (bytes < (size_t)nc * 24) return FMM_EINVAL;
      std::vector<double> t((size_t)nc);
      double* o = (double*)host_buf;
      const double* parts[3] = {c.c_cx.p, c.c_cy.p, c.c_cz.p};
      for (int d = 0; d < 3; d++) {
        HIPCHK(hipMemcpy(t.data(), parts[d], nc * 8, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < nc; i++) o[3 * i + d] = t[i];
      }
      return FMM_OK;
    }
    if (lst) {
      size_t cnt = (size_t)lst->count;
      if (bytes < cnt * 8) return FMM_EINVAL;
      std::vector<int> off((size_t)nc + 1), srcv(cnt);
      HIPCHK(hipMemcpy(off.data(), lst->off.p, (nc + 1) * 4, hipMemcpyDeviceToHost));
      if (cnt) HIPCHK(hipMemcpy(srcv.data(), lst->src.p, cnt * 4, hipMemcpyDeviceToHost));
      int* o = (int*)host_buf;
      for (int64_t s = 0; s < nc; s++)
        for (int k = off[s]; k < off[s + 1]; k++) {
          o[2 * k] = (int)s;
          o[2 * k + 1] = srcv[k];
        }
      return FMM_OK;
    }
    if (bytes < need) return FMM_EINVAL;
    HIPCHK(hipMemcpy(host_buf, src, need, hipMemcpyDeviceToHost));
    return FMM_OK;
  });
}

// the frozen-tree evaluation: bodies and cell centres refreshed from the
// stored order, P2M, M2M, then M2L, near field, L2L and the final sum
static void run_frozen(Ctx& c, const double* pos, const double* mass, double* acc, double* pot) {
  if (c.have_events) HIPCHK(hipEventRecord(c.ev[0], c.stream));
  refresh_frozen(c, pos, mass);
  if (c.have_events) HIPCHK(hipEventRecord(c.ev[1], c.stream));
  expansions_up(c);
  if (c.have_events) {
    HIPCHK(hipEventRecord(c.ev[2], c.stream));
    HIPCHK(hipEventRecord(c.ev[14], c.stream));
    HIPCHK(hipEventRecord(c.ev[3], c.stream));  // no estimate, no walk
  }
  evaluate(c, acc, pot, false);
  if (c.have_events) HIPCHK(hipEventRecord(c.ev[8], c.stream));
}

static fmm_status frozen_checks(fmm_ctx* ctx, int64_t n, const double* pos, const double* mass,
                                double eps_soft, double* acc, double* pot) {
  fmm_status st = common_checks(ctx, n, pos, mass);
  if (st != FMM_OK) return st;
  if (!acc || !pot || !(eps_soft >= 0) || !std::isfinite(eps_soft)) return FMM_EINVAL;
  if (!ctx->c.evaluated || ctx->c.n != n) return FMM_ENOTBUILT;
  return FMM_OK;
}

fmm_status fmm_forces_frozen(fmm_ctx* ctx, int64_t n, const double* pos, const double* mass,
                             double eps_soft, double* acc, double* pot, void* stream) {
  fmm_status st = frozen_checks(ctx, n, pos, mass, eps_soft, acc, pot);
  if (st != FMM_OK) return st;
  Ctx& c = ctx->c;
  return guarded(ctx, [&]() {
    c.stream = (hipStream_t)stream;
    c.err.clear();
    c.eps_soft = eps_soft;
    c.have_events = true;
    run_frozen(c, pos, mass, acc, pot);
    c.adjoint_ready = c.prm.precision == FMM_FP64 && c.nsys == 1;
    return FMM_OK;
  });
}

fmm_status fmm_forces_frozen_graph(fmm_ctx* ctx, int64_t n, const double* pos, const double* mass,
                                   double eps_soft, double* acc, double* pot, void* stream) {
  fmm_status st = frozen_checks(ctx, n, pos, mass, eps_soft, acc, pot);
  if (st != FMM_OK) return st;
  Ctx& c = ctx->c;
  return guarded(ctx, [&]() {
    c.stream = (hipStream_t)stream;
    c.err.clear();
    c.eps_soft = eps_soft;
    c.have_events = false;  // no timing events inside the graph
    const void* key[5] = {pos, mass, acc, pot, stream};
    bool same = c.graph_valid && c.gkey_eps == eps_soft;
    for (int k = 0; k < 5 && same; k++) same = c.gkey[k] == key[k];
    if (!same) {
      if (c.gexec) {
        HIPCHK(hipGraphExecDestroy(c.gexec));
        c.gexec = nullptr;
      }
      c.graph_valid = false;
      run_frozen(c, pos, mass, acc, pot);  // eager once: every buffer is in place before capture
      hipGraph_t g = nullptr;
      {
        OnStream on(c, c.cap);  // captured on a stream of the context, launched on the caller's
        HIPCHK(hipStreamBeginCapture(c.cap, hipStreamCaptureModeRelaxed));
        try {
          run_frozen(c, pos, mass, acc, pot);
        } catch (...) {
          (void)hipStreamEndCapture(c.cap, &g);
          if (g) (void)hipGraphDestroy(g);
          throw;
        }
        HIPCHK(hipStreamEndCapture(c.cap, &g));
      }
      hipError_t e = hipGraphInstantiate(&c.gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      check(e, "hipGraphInstantiate");
      for (int k = 0; k < 5; k++) c.gkey[k] = key[k];
      c.gkey_eps = eps_soft;
      c.graph_valid = true;
    }
    HIPCHK(hipGraphLaunch(c.gexec, c.stream));
    c.adjoint_ready = c.prm.precision == FMM_FP64 && c.nsys == 1;
    return FMM_OK;
  });
}

fmm_status fmm_adjoint(fmm_ctx* ctx, int64_t n, const double* pos, const double* mass, double eps_soft,
                       int p, double err_tol, const double* gacc, const double* gpot, double* gpos,
                       double* gmass, void* stream) {
  if (!ctx || !gacc || !gpos || !gmass) return FMM_EINVAL;
  Ctx& c = ctx->c;
  if (p < 1 || p > 30) return FMM_EINVAL;
  fmm_params saved = c.prm;
  c.prm.precision = FMM_FP64;  // the gradient is formed in FP64
  fmm_status st = guarded(ctx, [&]() {
    ensure(c.ws, c.fwd_acc, (size_t)std::max<int64_t>(n, 1) * 3);
    ensure(c.ws, c.fwd_pot, (size_t)std::max<int64_t>(n, 1));
    return FMM_OK;
  });
  if (st == FMM_OK) {
    int64_t off[2] = {0, n};
    st = forces_impl(ctx, 1, off, n, pos, mass, eps_soft, p, err_tol, c.fwd_acc.p, c.fwd_pot.p, stream);
  }
  if (st == FMM_OK)
    st = guarded(ctx, [&]() {
      adjoint_pass(c, gacc, gpot, c.fwd_acc.p, gpos, gmass);
      return FMM_OK;
    });
  c.prm = saved;
  return st;
}

fmm_status fmm_adjoint_last(fmm_ctx* ctx, int64_t n, const double* acc, const double* gacc,
                            const double* gpot, double* gpos, double* gmass, void* stream) {
  if (!ctx || !acc || !gacc || !gpos || !gmass || n < 1) return FMM_EINVAL;
  Ctx& c = ctx->c;
  if (!c.evaluated || !c.adjoint_ready || c.n != n) {
    c.err = "fmm_adjoint_last: the last evaluation was not one FP64 system of this many bodies";
    return FMM_ENOTBUILT;
  }
  return guarded(ctx, [&]() {
    c.stream = (hipStream_t)stream;
    c.err.clear();
    adjoint_pass(c, gacc, gpot, acc, gpos, gmass);
    return FMM_OK;
  });
}

fmm_status fmm_jerk(fmm_ctx* ctx, int64_t n, const double* pos, const double* vel, const double* mass,
                    double eps_soft, int p, double err_tol, double* acc, double* pot, double* jerk,
                    void* stream) {
  if (!ctx || !vel || !jerk) return FMM_EINVAL;
  Ctx& c = ctx->c;
  if (p < 1 || p > 30) return FMM_EINVAL;
  fmm_params saved = c.prm;
  c.prm.precision = FMM_FP64;
  int64_t off[2] = {0, n};
  fmm_status st = forces_impl(ctx, 1, off, n, pos, mass, eps_soft, p, err_tol, acc, pot, stream);
  if (st == FMM_OK)
    st = guarded(ctx, [&]() {
      jerk_pass(c, vel, mass, jerk);
      return FMM_OK;
    });
  c.prm = saved;
  return st;
}

// ---- autotuner: near-field start, n_leaf, FP32 M2L wavefronts per sink and
// near-field lane groups per (device, precision, p, tolerance, size class) ----
namespace {
using TuneKey = std::tuple<int, int, int, double, int, int>;
struct TuneChoice {
  int n_leaf, m2l_waves, p2p_groups, p2p_start;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneChoice> g_tune_cache;

int size_class(int64_t v) {
  int c = 0;
  while (v > 1) {
    v >>= 1;
    c++;
  }
  return c;
}
}  // namespace

fmm_status fmm_autotune(fmm_ctx* ctx, int64_t nsys, const int64_t* offsets, const double* pos,
                        const double* mass, double eps_soft, int p, double err_tol, double* acc,
                        double* pot, void* stream, int* chosen_n_leaf) {
  if (!ctx || !chosen_n_leaf || !offsets) return FMM_EINVAL;
  if (nsys < 1 || nsys > FMM_MAX_SYSTEMS || offsets[0] != 0) return FMM_EINVAL;
  for (int64_t s = 0; s < nsys; s++)
    if (offsets[s + 1] <= offsets[s]) return FMM_EINVAL;
  Ctx& c = ctx->c;
  int64_t n = offsets[nsys];
  TuneKey key{c.device, c.prm.precision, p, err_tol, size_class(n), size_class(n / nsys)};
  auto apply = [&](const TuneChoice& t) {
    c.prm.n_leaf = t.n_leaf;
    c.prm.m2l_waves = t.m2l_waves;
    c.prm.p2p_groups = t.p2p_groups;
    c.prm.p2p_start = t.p2p_start;
    c.graph_valid = false;
    *chosen_n_leaf = t.n_leaf;
  };
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      apply(it->second);
      return FMM_OK;
    }
  }
  fmm_params saved = c.prm;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  fmm_status st = guarded(ctx, [&]() {
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    return FMM_OK;
  });
  if (st != FMM_OK) return st;
  // one warm-up and two timed evaluations of a configuration; ms < 0 on error
  auto timed = [&](const TuneChoice& t, float& ms) {
    c.prm.n_leaf = t.n_leaf;
    c.prm.m2l_waves = t.m2l_waves;
    c.prm.p2p_groups = t.p2p_groups;
    c.prm.p2p_start = t.p2p_start;
    fmm_status s1 = forces_impl(ctx, nsys, offsets, n, pos, mass, eps_soft, p, err_tol, acc, pot, stream);
    if (s1 != FMM_OK) return s1;
    s1 = guarded(ctx, [&]() {
      HIPCHK(hipEventRecord(e0, (hipStream_t)stream));
      return FMM_OK;
    });
    for (int r = 0; r < 2 && s1 == FMM_OK; r++)
      s1 = forces_impl(ctx, nsys, offsets, n, pos, mass, eps_soft, p, err_tol, acc, pot, stream);
    if (s1 != FMM_OK) return s1;
    return guarded(ctx, [&]() {
      HIPCHK(hipEventRecord(e1, (hipStream_t)stream));
      HIPCHK(hipEventSynchronize(e1));
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      return FMM_OK;
    });
  };
  // coordinate search: the near field's start (at the given leaf capacity,
  // so that the capacity is then chosen under the better schedule), the leaf
  // capacity (it sets the balance of near and far field), then the FP32 M2L's
  // wavefronts per sink (mixed precision only), then the near field's lane
  // groups
  TuneChoice best{saved.n_leaf, saved.m2l_waves, saved.p2p_groups, saved.p2p_start};
  float best_ms = 1e30f;
  static const int cand_start[] = {0, 1};
  static const int cand_leaf[] = {16, 24, 32, 48, 64, 96, 128};
  static const int cand_waves[] = {1, 2, 4};
  static const int cand_groups[] = {0, 4, 2};
  for (int ps : cand_start) {
    TuneChoice t = best;
    t.p2p_start = ps;
    float ms = 0;
    if ((st = timed(t, ms)) != FMM_OK) break;
    if (ms < best_ms) {
      best_ms = ms;
      best = t;
    }
  }
  for (int nl : cand_leaf) {
    if (st != FMM_OK) break;
    TuneChoice t = best;
    t.n_leaf = nl;
    float ms = 0;
    if ((st = timed(t, ms)) != FMM_OK) break;
    if (ms < best_ms) {
      best_ms = ms;
      best = t;
    }
  }
  if (st == FMM_OK && saved.precision == FMM_MIXED && mixed_supported(p)) {
    TuneChoice base = best;
    for (int w : cand_waves) {
      if (w == base.m2l_waves) continue;
      TuneChoice t = base;
      t.m2l_waves = w;
      float ms = 0;
      if ((st = timed(t, ms)) != FMM_OK) break;
      if (ms < best_ms) {
        best_ms = ms;
        best = t;
      }
    }
  }
  if (st == FMM_OK) {
    TuneChoice base = best;
    for (int g : cand_groups) {
      if (g == base.p2p_groups) continue;
      TuneChoice t = base;
      t.p2p_groups = g;
      float ms = 0;
      if ((st = timed(t, ms)) != FMM_OK) break;
      if (ms < best_ms) {
        best_ms = ms;
        best = t;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c.prm = saved;
  if (st != FMM_OK) return st;
  apply(best);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = best;
  return FMM_OK;
}

fmm_status fmm_get_params(fmm_ctx* ctx, fmm_params* out) {
  if (!ctx || !out) return FMM_EINVAL;
  *out = ctx->c.prm;
  return FMM_OK;
}

fmm_status fmm_set_workspace_limit(fmm_ctx* ctx, size_t bytes) {
  if (!ctx) return FMM_EINVAL;
  ctx->c.ws.limit = bytes;
  return FMM_OK;
}

fmm_status fmm_direct(int64_t n, const double* pos, const double* mass, double eps_soft, int64_t nsink,
                      const int32_t* sinks, double* acc, double* pot, void* stream) {
  if (n < 1 || !pos || !mass || !acc || !pot || nsink < 0) return FMM_EINVAL;
  if (!(eps_soft >= 0) || !std::isfinite(eps_soft)) return FMM_EINVAL;
  if (!sinks) nsink = n;
  if (nsink == 0) return FMM_OK;
  return guarded(nullptr, [&]() {
    direct_sum(n, pos, mass, eps_soft * eps_soft, nsink, sinks, acc, pot, (hipStream_t)stream);
    return FMM_OK;
  });
}

const char* fmm_strerror(fmm_status s) {
  switch (s) {
    case FMM_OK: return "ok";
    case FMM_EINVAL: return "invalid argument";
    case FMM_ENOMEM: return "out of device memory or workspace cap exceeded";
    case FMM_EHIP: return "HIP runtime error";
    case FMM_ENOTBUILT: return "requested data has not been produced yet";
    case FMM_EDATA: return "non-finite position or negative/non-finite mass";
    case FMM_EUNSUPPORTED: return "valid but not supported by the compiled library";
  }
  return "unknown status";
}

const char* fmm_last_error(fmm_ctx* ctx) { return ctx ? ctx->c.err.c_str() : ""; }

void fmm_destroy(fmm_ctx* ctx) {
  if (!ctx) return;
  Ctx& c = ctx->c;
  (void)hipDeviceSynchronize();
  auto rel = [&](auto& b) { release(c.ws, b); };
  for (int k = 0; k < 2; k++) {
    rel(c.key[k]);
    rel(c.idx[k]);
    rel(c.front[k]);
  }
  rel(c.sx); rel(c.sy); rel(c.sz); rel(c.sm); rel(c.pm); rel(c.pkb); rel(c.scale); rel(c.nmult); rel(c.fpart); rel(c.leaf_of); rel(c.leaves); rel(c.nearbuf); rel(c.loc64); rel(c.root_sinks); rel(c.madj); rel(c.ladj); rel(c.fwd_acc); rel(c.fwd_pot); rel(c.gsort); rel(c.asort); rel(c.sys_off); rel(c.skey[0]); rel(c.skey[1]); rel(c.spos[0]); rel(c.spos[1]); rel(c.sort_hist); rel(c.sort_hist2); rel(c.scan_tmp2); rel(c.sort_hist3); rel(c.scan_tmp3); rel(c.cell_choff); rel(c.c_geo);
  rel(c.bbox_part); rel(c.rootbox); rel(c.c_level); rel(c.c_begin); rel(c.c_end); rel(c.c_parent);
  rel(c.c_child0); rel(c.c_nchild); rel(c.c_split); rel(c.c_mass); rel(c.c_sx); rel(c.c_sy);
  rel(c.c_sz); rel(c.c_cx); rel(c.c_cy); rel(c.c_cz); rel(c.c_rad); rel(c.c_rad2bits); rel(c.mult);
  rel(c.pk); rel(c.fcell); rel(c.fmin); rel(c.loc); rel(c.counters); rel(c.scan_tmp);
  rel(c.scan_tmp64);
  rel(c.adjnear); rel(c.adjpart); rel(c.nf_cell_nseg); rel(c.nf_cell_pbase); rel(c.nf_extra);
  rel(c.nf_part); rel(c.m2l_nseg); rel(c.m2l_pbase); rel(c.m2l_extra); rel(c.m2l_part);
  for (CellList* L : {&c.est_far, &c.est_near, &c.m2l, &c.p2p}) {
    rel(L->raw); rel(L->tmp); rel(L->off); rel(L->src);
  }
  if (c.hbuf) (void)hipHostFree(c.hbuf);
  if (c.gexec) (void)hipGraphExecDestroy(c.gexec);
  for (hipStream_t* st : {&c.side, &c.side2, &c.cap})
    if (*st) {
      (void)hipStreamSynchronize(*st);
      (void)hipStreamDestroy(*st);
    }
  for (auto& e : c.ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : c.fork)
    if (e) (void)hipEventDestroy(e);
  if (Ctx* na = ctx->na) {  // its buffers live in the static scratch: nothing to free there
    if (na->hbuf) (void)hipHostFree(na->hbuf);
    for (hipStream_t* st : {&na->side, &na->side2, &na->cap})
      if (*st) {
        (void)hipStreamSynchronize(*st);
        (void)hipStreamDestroy(*st);
      }
    for (auto& e : na->ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& e : na->fork)
      if (e) (void)hipEventDestroy(e);
    delete na;
  }
  delete ctx;
}

}  // extern "C"
