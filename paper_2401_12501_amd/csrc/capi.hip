// C ABI: handles, argument checks, host/device staging and the apply/solve drivers.
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>

#include "pmx_internal.hpp"

namespace pmx {

static thread_local std::string g_last_error;
void set_last_error(const std::string& msg) { g_last_error = msg; }

double now_seconds() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

void apply_batch(const std::vector<ApplyJob>& jobs, int precision, int n_rhs, hipStream_t st) {
  if (jobs.empty()) return;
  Profiler* prof = jobs.size() == 1 ? &jobs[0].op->prof : nullptr;
  auto begin = [&](int ph) { return prof ? prof->begin(ph, st) : -1; };
  auto end = [&](int t) {
    if (prof) prof->end(t, st);
  };
  switch (precision) {
    case PMX_PREC_FP64_DIRECT: {
      int t = begin(PMX_PHASE_PREP);
      source_prep_batch(jobs, n_rhs, false, st);
      end(t);
      t = begin(PMX_PHASE_DIRECT64);
      far_direct64_batch(jobs, n_rhs, st);
      end(t);
      t = begin(PMX_PHASE_NEAR);
      near_combine_batch(jobs, n_rhs, st);
      end(t);
      break;
    }
    case PMX_PREC_FP32_DIRECT: {
      for (const ApplyJob& j : jobs) {
        pmx_operator* op = j.op;
        Profiler* pf = jobs.size() == 1 ? &op->prof : nullptr;
        int t = pf ? pf->begin(PMX_PHASE_PREP, st) : -1;
        source_prep(op, j.sigma, n_rhs, true, st);
        if (pf) pf->end(t, st);
        t = pf ? pf->begin(PMX_PHASE_DIRECT32, st) : -1;
        far_direct(op, false, n_rhs, st);
        if (pf) pf->end(t, st);
        t = pf ? pf->begin(PMX_PHASE_NEAR, st) : -1;
        near_combine(op, j.sigma, j.y, n_rhs, far_direct_chunks(op, false), false, st);
        if (pf) pf->end(t, st);
      }
      break;
    }
    case PMX_PREC_MIXED_FMM: {
      for (const ApplyJob& j : jobs) {
        if (!j.op->fmm) fmm_build(j.op, st);
        if (n_rhs >= 8) build_near_tiles(&j.op->s->ctx->c, j.op->s->g, j.op->nl, st);
      }
      pmx_operator* lead = jobs[0].op;
      if (lead->opts.overlap) side_stream(lead);
      hipStream_t side = lead->opts.overlap ? lead->side : st;
      int t = begin(PMX_PHASE_PREP);
      source_prep_batch(jobs, n_rhs, true, st);
      end(t);
      // the near correction (HBM-bound) writes y on the side stream, followed by the P2P
      // sums, while the M2L chain (MFMA) runs here; each L2P joins and adds the far field
      auto near_part = [&](hipStream_t side) {
        const int tn = prof ? prof->begin(PMX_PHASE_NEAR, side) : -1;
        near_only_batch(jobs, n_rhs, side);
        if (prof) prof->end(tn, side);
      };
      fmm_far_batch(jobs, n_rhs, st, side, lead->ev_fork, lead->ev_join, near_part);   // records its own phases
      break;
    }
    default:
      throw Error(PMX_ERR_INVALID, "unknown precision mode");
  }
}

void side_stream(pmx_operator* op) {
  if (op->side) return;
  PMX_HIP(hipStreamCreateWithFlags(&op->side, hipStreamNonBlocking));
  PMX_HIP(hipEventCreateWithFlags(&op->ev_fork, hipEventDisableTiming));
  PMX_HIP(hipEventCreateWithFlags(&op->ev_join, hipEventDisableTiming));
}

void apply_device(pmx_operator* op, int precision, int n_rhs, const double* sigma, double* y, hipStream_t st) {
  if (op->batcher) {
    batcher_apply(op->batcher, op, precision, n_rhs, sigma, y, st);
    return;
  }
  apply_batch({ApplyJob{op, sigma, y}}, precision, n_rhs, st);
}

void prepare_apply(pmx_operator* op, int precision, int n_rhs, hipStream_t st) {
  const int64_t N = op->s->g.N;
  Ctx* ctx = &op->s->ctx->c;
  const size_t nr = (size_t)n_rhs;
  const size_t nb = (size_t)((N + 255) / 256);
  if (op->qt64.n < nr * N) op->qt64.alloc(ctx, nr * N);
  if (op->qt32.n < nr * N) op->qt32.alloc(ctx, nr * N);
  if (op->ssum_part.n < nr * nb) op->ssum_part.alloc(ctx, nr * nb);
  if (op->ssum.n < nr) op->ssum.alloc(ctx, nr);
  if (precision == PMX_PREC_MIXED_FMM) {
    if (!op->fmm) fmm_build(op, st);
    fmm_reserve(op, n_rhs);
    if (n_rhs >= 8) build_near_tiles(ctx, op->s->g, op->nl, st);
    if (op->opts.overlap) side_stream(op);
  }
  // FP64 residuals of the refinement (and the FP64 path): chunk partials and packed rows
  const size_t part = (size_t)far_direct_chunks(op, true) * nr * N;
  if (op->part.n < part) op->part.alloc(ctx, part);
  const int g = n_rhs >= 16 ? 16 : (n_rhs >= 8 ? 8 : (n_rhs >= 4 ? 4 : (n_rhs >= 2 ? 2 : 1)));
  const size_t rl = (size_t)((3 + g + 1) / 2) * 2;
  if (op->rows64.n < rl * N) op->rows64.alloc(ctx, rl * N);
}

void represent_device(pmx_operator* op, int n_rhs, const double* sigma, double* u, hipStream_t st) {
  if (!op->nl.have_D) build_near_weights(&op->s->ctx->c, op->s->g, op->co, op->nl, op->opts, true, st);
  source_prep(op, sigma, n_rhs, false, st);
  const int t = op->prof.begin(PMX_PHASE_LOG, st);
  far_direct_log(op, n_rhs, st);
  op->prof.end(t, st);
  near_combine(op, sigma, u, n_rhs, far_direct_chunks(op, true), true, st);
  if (op->cplx()) near_cross(op, sigma, u, n_rhs, true, st);
  if (!op->co.has_c()) weighted_mean_remove(op, u, n_rhs, st);   // c = 0: the mean-zero solution
}

}  // namespace pmx

using namespace pmx;

namespace {

// ----------------------------------------------------------------------------- static scratch
// Scratch of the allocation-free apply: one array per GPU the library runs on, held until the
// process ends.  Host code never uses the array's name as an address (on the host it is only a
// stand-in for the symbol): its device address is looked up once per device, with that device
// current, when a context is created there, and kept in g_scratch.
constexpr size_t kScratchDoubles = (size_t)PMX_NOALLOC_SCRATCH_BYTES / sizeof(double);
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// Called with `device` current.  A failed lookup is kept and reported by the entry point, so
// that contexts still work for every other call.
void scratch_lookup(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess && ptr) {
    g_scratch[device] = static_cast<double*>(ptr);
    g_scratch_err[device] = hipSuccess;
  } else {
    g_scratch_err[device] = e != hipSuccess ? e : hipErrorInvalidSymbol;
    (void)hipGetLastError();   // do not leave the error for the next launch check
  }
}

double* scratch_ptr(int device) {
  PMX_REQUIRE(device >= 0 && device < kMaxDevices, PMX_ERR_INVALID, "device index out of range for the static scratch");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[device])
    throw Error(PMX_ERR_DEVICE, std::string("static scratch address unavailable: ") +
                                    hipGetErrorString(g_scratch_err[device] != hipSuccess ? g_scratch_err[device]
                                                                                          : hipErrorInvalidSymbol));
  return g_scratch[device];
}

// Requires p to be device memory (or managed memory) of `device`.
void require_device_array(const void* p, int device, const char* what) {
  hipPointerAttribute_t at;
  const hipError_t e = hipPointerGetAttributes(&at, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Error(PMX_ERR_INVALID, std::string(what) + " is not a device array");
  }
  PMX_REQUIRE(at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged, PMX_ERR_INVALID,
              std::string(what) + " is not a device array");
  PMX_REQUIRE(at.device == device, PMX_ERR_INVALID, std::string(what) + " lives on another device");
}

template <class F>
pmx_status guarded(F&& f) {
  try {
    f();
    g_last_error.clear();
    return PMX_OK;
  } catch (const pmx::Error& e) {
    set_last_error(e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return PMX_ERR_OOM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return PMX_ERR_DEVICE;
  }
}

// Device view of a caller array: the pointer itself (device) or a staged copy (host).
const double* stage_in(Ctx* ctx, DBuf<double>& buf, const double* p, size_t n, int mem_kind, hipStream_t st) {
  PMX_REQUIRE(p != nullptr, PMX_ERR_INVALID, "null input array");
  if (mem_kind == PMX_MEM_DEVICE) return p;
  PMX_REQUIRE(mem_kind == PMX_MEM_HOST, PMX_ERR_INVALID, "mem_kind must be PMX_MEM_HOST or PMX_MEM_DEVICE");
  buf.alloc(ctx, n);
  PMX_HIP(hipMemcpyAsync(buf.p, p, n * sizeof(double), hipMemcpyHostToDevice, st));
  return buf.p;
}

void check_opts(const pmx_options& o) {
  PMX_REQUIRE(o.eta_near > 0.0 && std::isfinite(o.eta_near), PMX_ERR_INVALID, "eta_near must be positive");
  PMX_REQUIRE(o.n_gl >= 2 && o.n_gl <= 16, PMX_ERR_INVALID, "n_gl must be in [2, 16]");
  PMX_REQUIRE(o.fmm_order >= 4 && o.fmm_order <= 6, PMX_ERR_INVALID, "fmm_order must be 4, 5 or 6");
  PMX_REQUIRE(o.fmm_leaf >= 8, PMX_ERR_INVALID, "fmm_leaf must be >= 8");
  PMX_REQUIRE(o.gmres_restart >= 1 && o.gmres_restart <= 500, PMX_ERR_INVALID, "gmres_restart must be in [1, 500]");
  PMX_REQUIRE(o.max_iter >= 1, PMX_ERR_INVALID, "max_iter must be >= 1");
  PMX_REQUIRE(o.gmres_tol > 0 && o.ir_tol > 0 && o.inner_tol > 0, PMX_ERR_INVALID, "tolerances must be positive");
  PMX_REQUIRE(o.precision >= 0 && o.precision <= 2, PMX_ERR_INVALID, "unknown precision mode");
  PMX_REQUIRE(o.overlap == 0 || o.overlap == 1, PMX_ERR_INVALID, "overlap must be 0 or 1");
}

}  // namespace

extern "C" {

const char* pmx_last_error(void) { return g_last_error.c_str(); }

void pmx_default_options(pmx_options* o) {
  if (!o) return;
  o->eta_near = 1.5;
  o->n_gl = 16;
  o->fmm_order = 6;
  o->fmm_leaf = 256;
  o->gmres_tol = 1e-10;
  o->gmres_restart = 60;
  o->max_iter = 400;
  o->ir_tol = 1e-8;
  o->inner_tol = 1e-4;
  o->max_ir = 20;
  o->precision = PMX_PREC_FP64_DIRECT;
  o->overlap = 1;
}

pmx_status pmx_ctx_create(int device, uint64_t hbm_budget_bytes, pmx_ctx** out) {
  return guarded([&] {
    PMX_REQUIRE(out != nullptr, PMX_ERR_INVALID, "out is null");
    *out = nullptr;
    int n = 0;
    PMX_HIP(hipGetDeviceCount(&n));
    PMX_REQUIRE(device >= 0 && device < n, PMX_ERR_INVALID, "no such device");
    PMX_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    PMX_HIP(hipGetDeviceProperties(&prop, device));
    scratch_lookup(device);
    auto* c = new pmx_ctx;
    c->c.device = device;
    c->c.budget = hbm_budget_bytes;
    c->c.n_cu = prop.multiProcessorCount;
    *out = c;
  });
}

void pmx_ctx_destroy(pmx_ctx* ctx) {
  if (ctx) ctx_release(ctx);
}

pmx_status pmx_surface_create(pmx_ctx* ctx, int n_patches, int q, const double* x, const double* xu,
                              const double* xv, const double* xuu, const double* xuv, const double* xvv, int mem_kind,
                              void* stream, pmx_surface** out) {
  return guarded([&] {
    PMX_REQUIRE(ctx && out, PMX_ERR_INVALID, "null handle");
    *out = nullptr;
    PMX_REQUIRE(n_patches >= 1 && q >= 2 && q <= 16, PMX_ERR_INVALID, "need n_patches >= 1 and 2 <= q <= 16");
    PMX_REQUIRE((int64_t)n_patches * q * q < ((int64_t)1 << 31), PMX_ERR_INVALID, "too many nodes");
    PMX_HIP(hipSetDevice(ctx->c.device));
    hipStream_t st = (hipStream_t)stream;
    auto* s = new pmx_surface;
    try {
      s->ctx = ctx;
      s->g.M = n_patches;
      s->g.q = q;
      s->g.N = (int64_t)n_patches * q * q;
      const size_t n3 = 3 * (size_t)s->g.N;
      DBuf<double> b[6];
      const double* d[6];
      const double* src[6] = {x, xu, xv, xuu, xuv, xvv};
      for (int k = 0; k < 6; ++k) d[k] = stage_in(&ctx->c, b[k], src[k], n3, mem_kind, st);
      build_geometry(&ctx->c, s->g, d[0], d[1], d[2], d[3], d[4], d[5], st);
      PMX_HIP(hipStreamSynchronize(st));
    } catch (...) {
      delete s;
      throw;
    }
    ctx_retain(ctx);
    *out = s;
  });
}

void pmx_surface_destroy(pmx_surface* s) {
  if (s) surface_release(s);
}

namespace {
pmx_status operator_create(pmx_surface* s, const double* a, const double* grad_a, const double* c, const double* b,
                           const pmx_options* opts, int mem_kind, void* stream, pmx_operator** out) {
  return guarded([&] {
    PMX_REQUIRE(s && out, PMX_ERR_INVALID, "null handle");
    *out = nullptr;
    PMX_HIP(hipSetDevice(s->ctx->c.device));
    hipStream_t st = (hipStream_t)stream;
    auto* op = new pmx_operator;
    try {
      op->s = s;
      if (opts) op->opts = *opts; else pmx_default_options(&op->opts);
      check_opts(op->opts);
      const double t0 = now_seconds();
      Ctx* ctx = &s->ctx->c;
      DBuf<double> ba, bg, bc, bb;
      const double* da = stage_in(ctx, ba, a, s->g.N, mem_kind, st);
      const double* dg = stage_in(ctx, bg, grad_a, 3 * (size_t)s->g.N, mem_kind, st);
      const double* dc = c ? stage_in(ctx, bc, c, s->g.N, mem_kind, st) : nullptr;
      const double* db = b ? stage_in(ctx, bb, b, 3 * (size_t)s->g.N, mem_kind, st) : nullptr;
      build_coeff(ctx, s->g, op->co, da, dg, dc, db, st);
      build_near_lists(ctx, s->g, op->opts.eta_near, op->nl, st);
      build_near_weights(ctx, s->g, op->co, op->nl, op->opts, false, st);
      PMX_HIP(hipStreamSynchronize(st));
      op->t_setup = now_seconds() - t0;
    } catch (...) {
      if (op->fmm) fmm_destroy(op->fmm);
      delete op;
      throw;
    }
    surface_retain(s);
    *out = op;
  });
}
}  // namespace

pmx_status pmx_operator_create(pmx_surface* s, const double* a, const double* grad_a, const pmx_options* opts,
                               int mem_kind, void* stream, pmx_operator** out) {
  return operator_create(s, a, grad_a, nullptr, nullptr, opts, mem_kind, stream, out);
}

pmx_status pmx_operator_create_c(pmx_surface* s, const double* a, const double* grad_a, const double* c,
                                 const double* b, const pmx_options* opts, int mem_kind, void* stream,
                                 pmx_operator** out) {
  if (!c) {
    set_last_error("c is null (use pmx_operator_create for c = 0, which takes no advection field)");
    if (out) *out = nullptr;
    return PMX_ERR_INVALID;
  }
  return operator_create(s, a, grad_a, c, b, opts, mem_kind, stream, out);
}

void pmx_operator_destroy(pmx_operator* op) {
  if (!op) return;
  if (op->fmm) fmm_destroy(op->fmm);
  if (op->ev_ready) (void)hipEventDestroy(op->ev_ready);
  if (op->ev_done) (void)hipEventDestroy(op->ev_done);
  if (op->ev_fork) (void)hipEventDestroy(op->ev_fork);
  if (op->ev_join) (void)hipEventDestroy(op->ev_join);
  if (op->side) (void)hipStreamDestroy(op->side);
  pmx_surface* s = op->s;
  delete op;
  surface_release(s);
}

pmx_status pmx_operator_get_stats(pmx_operator* op, pmx_operator_stats* out) {
  return guarded([&] {
    PMX_REQUIRE(op && out, PMX_ERR_INVALID, "null handle");
    std::memset(out, 0, sizeof(*out));
    out->n_nodes = op->s->g.N;
    out->n_patches = op->s->g.M;
    out->q = op->s->g.q;
    out->near_pairs = op->nl.nnz;
    uint64_t b = op->co.a.bytes() + op->co.gs.bytes() + op->co.tgt.bytes() + op->co.tg.bytes() + op->co.tf64.bytes() +
                 op->co.tgt32.bytes() + op->co.w_over_a.bytes() + op->nl.ptr.bytes() + op->nl.patch.bytes() +
                 op->nl.target.bytes() + op->nl.C.bytes() + op->nl.D.bytes() + op->nl.Ci.bytes() +
                 op->nl.Di.bytes() + op->part.bytes() +
                 op->qt64.bytes() + op->qt32.bytes();
    if (op->fmm) {
      fmm_stats(op->fmm, out);
      b += fmm_bytes(op->fmm);
    }
    out->device_bytes = b;
  });
}

pmx_status pmx_apply(pmx_operator* op, int precision, int n_rhs, const double* sigma, double* y, int mem_kind,
                     void* stream) {
  return guarded([&] {
    PMX_REQUIRE(op && sigma && y, PMX_ERR_INVALID, "null argument");
    PMX_REQUIRE(n_rhs >= 1 && n_rhs <= 1024, PMX_ERR_INVALID, "n_rhs must be in [1, 1024]");
    PMX_REQUIRE(!op->co.has_c() || precision == PMX_PREC_FP64_DIRECT, PMX_ERR_INVALID,
                "with c != 0 only the FP64 direct far field is available");
    PMX_HIP(hipSetDevice(op->s->ctx->c.device));
    hipStream_t st = (hipStream_t)stream;
    Ctx* ctx = &op->s->ctx->c;
    const size_t n = (size_t)op->cols(n_rhs) * op->s->g.N;   // c > 0: 2N reals per complex vector
    DBuf<double> bin, bout;
    const double* ds = stage_in(ctx, bin, sigma, n, mem_kind, st);
    double* dy = y;
    if (mem_kind == PMX_MEM_HOST) {
      bout.alloc(ctx, n);
      dy = bout.p;
    }
    apply_device(op, precision, op->cols(n_rhs), ds, dy, st);
    if (mem_kind == PMX_MEM_HOST) {
      PMX_HIP(hipMemcpyAsync(y, dy, n * sizeof(double), hipMemcpyDeviceToHost, st));
      PMX_HIP(hipStreamSynchronize(st));
    }
  });
}

pmx_status pmx_apply_noalloc(pmx_operator* op, int n_rhs, const double* sigma, double* y, void* stream) {
  return guarded([&] {
    PMX_REQUIRE(op && sigma && y, PMX_ERR_INVALID, "null argument");
    PMX_REQUIRE(n_rhs >= 1 && n_rhs <= 1024, PMX_ERR_INVALID, "n_rhs must be in [1, 1024]");
    const int dev = op->s->ctx->c.device;
    PMX_HIP(hipSetDevice(dev));
    const int64_t N = op->s->g.N;
    const int nc = op->cols(n_rhs);   // real columns (a complex operator: two per density)
    const size_t need = direct64_scratch_doubles(N, nc);
    if (need > kScratchDoubles)
      throw Error(PMX_ERR_TOO_LARGE, "the allocation-free apply needs " + std::to_string(need * sizeof(double)) +
                                         " bytes of scratch; the static scratch holds " +
                                         std::to_string((size_t)PMX_NOALLOC_SCRATCH_BYTES));
    require_device_array(sigma, dev, "sigma");
    require_device_array(y, dev, "y");
    double* base = scratch_ptr(dev);
    // carve the buffers in the order and rounding direct64_scratch_doubles counts them
    const size_t nr = (size_t)nc, nb = (size_t)((N + 255) / 256);
    auto up = [](size_t n) { return (n + 31) / 32 * 32; };
    ApplyScratch sc;
    size_t at = 0;
    sc.qt64 = base + at;
    at += up(nr * N);
    sc.spart = base + at;
    at += up(nr * nb);
    sc.ssum = base + at;
    at += up(nr);
    const int g = nc >= 16 ? 16 : (nc >= 8 ? 8 : (nc >= 4 ? 4 : (nc >= 2 ? 2 : 1)));
    sc.rows = base + at;
    at += up((size_t)((4 + g + 1) / 2) * 2 * N);
    sc.part = base + at;
    hipStream_t st = (hipStream_t)stream;
    const std::vector<ApplyJob> jobs{ApplyJob{op, sigma, y, &sc}};
    source_prep_batch(jobs, nc, false, st);
    far_direct64_batch(jobs, nc, st);
    near_combine_batch(jobs, nc, st);
  });
}

pmx_status pmx_solve(pmx_operator* op, const pmx_options* opts, int n_rhs, const double* f, double* sigma,
                     int sigma_in_is_guess, double* u, int mem_kind, void* stream, pmx_info* info) {
  pmx_status conv = PMX_OK;
  pmx_status st_ = guarded([&] {
    PMX_REQUIRE(op && f && sigma, PMX_ERR_INVALID, "null argument");
    PMX_REQUIRE(n_rhs >= 1 && n_rhs <= 1024, PMX_ERR_INVALID, "n_rhs must be in [1, 1024]");
    PMX_HIP(hipSetDevice(op->s->ctx->c.device));
    hipStream_t st = (hipStream_t)stream;
    pmx_options o = opts ? *opts : op->opts;
    check_opts(o);
    PMX_REQUIRE(!op->co.has_c() || o.precision == PMX_PREC_FP64_DIRECT, PMX_ERR_INVALID,
                "with c != 0 only the FP64 path (PMX_PREC_FP64_DIRECT) is available");
    Ctx* ctx = &op->s->ctx->c;
    const size_t n = (size_t)op->cols(n_rhs) * op->s->g.N;   // c > 0: 2N reals per complex vector
    const double t0 = now_seconds();
    DBuf<double> bf, bs, bu;
    const double* df = stage_in(ctx, bf, f, n, mem_kind, st);
    double* dsig = sigma;
    double* du = u;
    if (mem_kind == PMX_MEM_HOST) {
      bs.alloc(ctx, n);
      dsig = bs.p;
      if (sigma_in_is_guess) PMX_HIP(hipMemcpyAsync(dsig, sigma, n * sizeof(double), hipMemcpyHostToDevice, st));
      if (u) {
        bu.alloc(ctx, n);
        du = bu.p;
      }
    }
    std::vector<double> removed;
    SolveResult r = solve_device(op, o, n_rhs, df, dsig, sigma_in_is_guess != 0, st, removed);
    if (u) represent_device(op, op->cols(n_rhs), dsig, du, st);
    if (mem_kind == PMX_MEM_HOST) {
      PMX_HIP(hipMemcpyAsync(sigma, dsig, n * sizeof(double), hipMemcpyDeviceToHost, st));
      if (u) PMX_HIP(hipMemcpyAsync(u, du, n * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    PMX_HIP(hipStreamSynchronize(st));
    const double t1 = now_seconds();
    if (info) {
      for (int k = 0; k < n_rhs; ++k) {
        info[k].iters_total = r.iters[k];
        info[k].ir_steps = r.ir_steps;
        info[k].applies_fp64 = r.applies64;
        info[k].applies_low = r.applies_low;
        info[k].rel_residual = r.relres[k];
        info[k].removed_mean = removed[k];
        info[k].t_setup = op->t_setup;
        info[k].t_solve = t1 - t0;
      }
    }
    if (!r.converged) conv = PMX_ERR_NOT_CONVERGED;
  });
  if (st_ == PMX_OK && conv != PMX_OK) set_last_error("iteration limit reached before the tolerance");
  return st_ != PMX_OK ? st_ : conv;
}

pmx_status pmx_represent(pmx_operator* op, int n_rhs, const double* sigma, double* u, int mem_kind, void* stream) {
  return guarded([&] {
    PMX_REQUIRE(op && sigma && u, PMX_ERR_INVALID, "null argument");
    PMX_REQUIRE(n_rhs >= 1 && n_rhs <= 1024, PMX_ERR_INVALID, "n_rhs must be in [1, 1024]");
    PMX_HIP(hipSetDevice(op->s->ctx->c.device));
    hipStream_t st = (hipStream_t)stream;
    Ctx* ctx = &op->s->ctx->c;
    const size_t n = (size_t)op->cols(n_rhs) * op->s->g.N;   // c > 0: 2N reals per complex vector
    DBuf<double> bin, bout;
    const double* ds = stage_in(ctx, bin, sigma, n, mem_kind, st);
    double* du = u;
    if (mem_kind == PMX_MEM_HOST) {
      bout.alloc(ctx, n);
      du = bout.p;
    }
    represent_device(op, op->cols(n_rhs), ds, du, st);
    if (mem_kind == PMX_MEM_HOST) PMX_HIP(hipMemcpyAsync(u, du, n * sizeof(double), hipMemcpyDeviceToHost, st));
    PMX_HIP(hipStreamSynchronize(st));
  });
}

pmx_status pmx_operator_export_geometry(pmx_operator* op, double* n, double* H, double* w, double* grad_s_a) {
  return guarded([&] {
    PMX_REQUIRE(op, PMX_ERR_INVALID, "null handle");
    PMX_HIP(hipSetDevice(op->s->ctx->c.device));
    const int64_t N = op->s->g.N;
    std::vector<double> tmp(3 * N);
    auto aos = [&](const double* src, double* dst) {
      PMX_HIP(hipMemcpy(tmp.data(), src, 3 * N * sizeof(double), hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < N; ++i)
        for (int c = 0; c < 3; ++c) dst[3 * i + c] = tmp[c * N + i];
    };
    if (n) aos(op->s->g.n.p, n);
    if (grad_s_a) aos(op->co.gs.p, grad_s_a);
    if (H) PMX_HIP(hipMemcpy(H, op->s->g.H.p, N * sizeof(double), hipMemcpyDeviceToHost));
    if (w) PMX_HIP(hipMemcpy(w, op->s->g.w.p, N * sizeof(double), hipMemcpyDeviceToHost));
  });
}

pmx_status pmx_operator_export_near(pmx_operator* op, int64_t* ptr, int32_t* patch, double* C, double* D) {
  return guarded([&] {
    PMX_REQUIRE(op, PMX_ERR_INVALID, "null handle");
    PMX_HIP(hipSetDevice(op->s->ctx->c.device));
    const int64_t N = op->s->g.N, nnz = op->nl.nnz;
    const int q2 = op->s->g.q * op->s->g.q;
    if (ptr) PMX_HIP(hipMemcpy(ptr, op->nl.ptr.p, (N + 1) * sizeof(int64_t), hipMemcpyDeviceToHost));
    if (patch) PMX_HIP(hipMemcpy(patch, op->nl.patch.p, nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (C) PMX_HIP(hipMemcpy(C, op->nl.C.p, (size_t)nnz * q2 * sizeof(double), hipMemcpyDeviceToHost));
    if (D) {
      if (!op->nl.have_D) build_near_weights(&op->s->ctx->c, op->s->g, op->co, op->nl, op->opts, true, nullptr);
      PMX_HIP(hipMemcpy(D, op->nl.D.p, (size_t)nnz * q2 * sizeof(double), hipMemcpyDeviceToHost));
    }
  });
}

pmx_status pmx_operator_export_near_imag(pmx_operator* op, double* Ci, double* Di) {
  return guarded([&] {
    PMX_REQUIRE(op, PMX_ERR_INVALID, "null handle");
    PMX_REQUIRE(op->cplx(), PMX_ERR_INVALID, "the operator is real (c <= 0): its blocks have no imaginary part");
    PMX_HIP(hipSetDevice(op->s->ctx->c.device));
    const size_t n = (size_t)op->nl.nnz * op->s->g.q * op->s->g.q;
    if (Ci) PMX_HIP(hipMemcpy(Ci, op->nl.Ci.p, n * sizeof(double), hipMemcpyDeviceToHost));
    if (Di) {
      if (!op->nl.have_D) build_near_weights(&op->s->ctx->c, op->s->g, op->co, op->nl, op->opts, true, nullptr);
      PMX_HIP(hipMemcpy(Di, op->nl.Di.p, n * sizeof(double), hipMemcpyDeviceToHost));
    }
  });
}

pmx_status pmx_operator_is_complex(pmx_operator* op, int* out) {
  return guarded([&] {
    PMX_REQUIRE(op && out, PMX_ERR_INVALID, "null argument");
    *out = op->cplx() ? 1 : 0;
  });
}

pmx_status pmx_profile_enable(pmx_operator* op, int enable) {
  return guarded([&] {
    PMX_REQUIRE(op, PMX_ERR_INVALID, "null handle");
    op->prof.on = enable != 0;
  });
}

pmx_status pmx_profile_read(pmx_operator* op, double* ms, int64_t* count) {
  return guarded([&] {
    PMX_REQUIRE(op && ms && count, PMX_ERR_INVALID, "null argument");
    for (int k = 0; k < PMX_N_PHASES; ++k) {
      ms[k] = 0.0;
      count[k] = 0;
    }
    for (auto& r : op->prof.recs) {
      PMX_HIP(hipEventSynchronize(r.b));
      float t = 0.0f;
      PMX_HIP(hipEventElapsedTime(&t, r.a, r.b));
      ms[r.phase] += t;
      count[r.phase] += 1;
      op->prof.pool.push_back(r.a);
      op->prof.pool.push_back(r.b);
    }
    op->prof.recs.clear();
  });
}


// ----------------------------------------------------------------------------- edge operators
pmx_status pmx_edge_create(pmx_ctx* ctx, int n_curves, const int64_t* n_samples, const double* x, const double* xt,
                           const double* d, const double* a, const double* grad_a, int oversample, int mem_kind,
                           void* stream, pmx_edge** out) {
  return guarded([&] {
    PMX_REQUIRE(ctx && out && n_samples, PMX_ERR_INVALID, "null argument");
    *out = nullptr;
    PMX_REQUIRE(x && xt && d && a && grad_a, PMX_ERR_INVALID, "null input array");
    PMX_REQUIRE(n_curves >= 1 && n_curves <= 64, PMX_ERR_INVALID, "n_curves must be in [1, 64]");
    PMX_REQUIRE(oversample >= 1 && oversample <= 1024, PMX_ERR_INVALID, "oversample must be in [1, 1024]");
    PMX_REQUIRE(mem_kind == PMX_MEM_HOST || mem_kind == PMX_MEM_DEVICE, PMX_ERR_INVALID,
                "mem_kind must be PMX_MEM_HOST or PMX_MEM_DEVICE");
    std::vector<int64_t> off(n_curves + 1, 0);
    for (int k = 0; k < n_curves; ++k) {
      PMX_REQUIRE(n_samples[k] >= 3 && n_samples[k] < ((int64_t)1 << 31), PMX_ERR_INVALID,
                  "every curve needs at least 3 samples");
      off[k + 1] = off[k] + n_samples[k];
    }
    const int64_t M = off.back();
    PMX_REQUIRE(M * oversample < ((int64_t)1 << 31), PMX_ERR_INVALID, "too many fine points");
    PMX_HIP(hipSetDevice(ctx->c.device));
    hipStream_t st = (hipStream_t)stream;
    // the samples on the host (small): validated here, uploaded as 13 rows of M; device arrays are
    // read after the caller's stream has finished writing them
    if (mem_kind == PMX_MEM_DEVICE) PMX_HIP(hipStreamSynchronize(st));
    std::vector<double> h3[4], ha(M);
    const double* src3[4] = {x, xt, d, grad_a};
    for (int k = 0; k < 4; ++k) {
      h3[k].resize(3 * M);
      PMX_HIP(hipMemcpy(h3[k].data(), src3[k], 3 * M * sizeof(double),
                        mem_kind == PMX_MEM_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
    }
    PMX_HIP(hipMemcpy(ha.data(), a, M * sizeof(double),
                      mem_kind == PMX_MEM_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
    std::vector<double> soa(13 * M);
    for (int64_t j = 0; j < M; ++j) {
      const double* t = &h3[1][3 * j];
      const double* dd = &h3[2][3 * j];
      const double tl = std::sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
      const double dl = std::sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
      const double dt = tl > 0 ? (dd[0] * t[0] + dd[1] * t[1] + dd[2] * t[2]) / tl : 0.0;
      PMX_REQUIRE(tl > 0 && std::isfinite(tl), PMX_ERR_INVALID, "edge: a sample has a zero or non-finite xt");
      PMX_REQUIRE(std::isfinite(dl) && dl * dl - dt * dt > 1e-12 * dl * dl, PMX_ERR_INVALID,
                  "edge: a direction d is zero, non-finite or along the curve");
      PMX_REQUIRE(ha[j] > 0 && std::isfinite(ha[j]), PMX_ERR_INVALID, "edge: a must be positive and finite");
      for (int c = 0; c < 3; ++c) {
        PMX_REQUIRE(std::isfinite(h3[0][3 * j + c]) && std::isfinite(h3[3][3 * j + c]), PMX_ERR_INVALID,
                    "edge: non-finite position or grad_a");
        for (int k = 0; k < 3; ++k) soa[(3 * k + c) * M + j] = h3[k][3 * j + c];
        soa[(10 + c) * M + j] = h3[3][3 * j + c];
      }
      soa[9 * M + j] = ha[j];
    }
    // nu . grad a at the samples (nu = the part of d normal to xt, normalized), for D_gamma's condition
    double ga_max = 0.0, nga_max = 0.0;
    for (int64_t j = 0; j < M; ++j) {
      const double* t = &h3[1][3 * j];
      const double* dd = &h3[2][3 * j];
      const double* ga = &h3[3][3 * j];
      const double tl2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
      const double dt = (dd[0] * t[0] + dd[1] * t[1] + dd[2] * t[2]) / tl2;
      const double v[3] = {dd[0] - dt * t[0], dd[1] - dt * t[1], dd[2] - dt * t[2]};
      const double vl = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      nga_max = std::max(nga_max, std::fabs(v[0] * ga[0] + v[1] * ga[1] + v[2] * ga[2]) / vl);
      for (int c = 0; c < 3; ++c) ga_max = std::max(ga_max, std::fabs(ga[c]));
    }
    auto* e = new pmx_edge;
    try {
      e->ctx = ctx;
      e->e.ctx = &ctx->c;
      e->e.nu_grad_a_zero = nga_max <= 1e-14 * std::max(ga_max, 1.0);
      edge_build(&ctx->c, e->e, off, soa, oversample, st);
    } catch (...) {
      delete e;
      throw;
    }
    ctx_retain(ctx);
    *out = e;
  });
}

void pmx_edge_destroy(pmx_edge* e) {
  if (!e) return;
  pmx_ctx* c = e->ctx;
  delete e;
  ctx_release(c);
}

pmx_status pmx_edge_size(pmx_edge* e, int64_t* m_samples, int64_t* n_fine) {
  return guarded([&] {
    PMX_REQUIRE(e, PMX_ERR_INVALID, "null handle");
    if (m_samples) *m_samples = e->e.M;
    if (n_fine) *n_fine = e->e.Mf;
  });
}

pmx_status pmx_edge_export_points(pmx_edge* e, double* y, double* nu, double* w, double* a, double* nu_grad_a) {
  return guarded([&] {
    PMX_REQUIRE(e, PMX_ERR_INVALID, "null handle");
    PMX_HIP(hipSetDevice(e->ctx->c.device));
    const int64_t Mf = e->e.Mf;
    std::vector<double> P(10 * Mf);
    PMX_HIP(hipMemcpy(P.data(), e->e.pts.p, 10 * Mf * sizeof(double), hipMemcpyDeviceToHost));
    for (int64_t p = 0; p < Mf; ++p) {
      for (int c = 0; c < 3; ++c) {
        if (y) y[3 * p + c] = P[c * Mf + p];
        if (nu) nu[3 * p + c] = P[(3 + c) * Mf + p];
      }
      if (w) w[p] = P[8 * Mf + p];
      if (a) a[p] = P[9 * Mf + p];
      if (nu_grad_a) nu_grad_a[p] = P[6 * Mf + p] * P[9 * Mf + p];
    }
  });
}

pmx_status pmx_edge_apply(pmx_operator* op, pmx_edge* e, int kind, int n_rhs, const double* mu, double* y,
                          int mem_kind, void* stream) {
  return guarded([&] {
    PMX_REQUIRE(op && e && mu && y, PMX_ERR_INVALID, "null argument");
    PMX_REQUIRE(kind >= PMX_EDGE_K && kind <= PMX_EDGE_T, PMX_ERR_INVALID, "unknown edge operator");
    PMX_REQUIRE(n_rhs >= 1 && n_rhs <= 1024, PMX_ERR_INVALID, "n_rhs must be in [1, 1024]");
    PMX_REQUIRE(op->s->ctx->c.device == e->ctx->c.device, PMX_ERR_INVALID, "operator and edge on different devices");
    PMX_REQUIRE(!op->cplx() && !op->co.has_c() && !op->co.has_b, PMX_ERR_INVALID,
                "edge operators are provided for c = 0 without advection");
    PMX_HIP(hipSetDevice(e->ctx->c.device));
    hipStream_t st = (hipStream_t)stream;
    Ctx* ctx = &e->ctx->c;
    const size_t nin = (size_t)n_rhs * e->e.M, nout = (size_t)n_rhs * op->s->g.N;
    DBuf<double> bin, bout;
    const double* dmu = stage_in(ctx, bin, mu, nin, mem_kind, st);
    double* dy = y;
    if (mem_kind == PMX_MEM_HOST) {
      bout.alloc(ctx, nout);
      dy = bout.p;
    }
    edge_apply(op, e->e, kind, n_rhs, dmu, dy, st);
    if (mem_kind == PMX_MEM_HOST) PMX_HIP(hipMemcpyAsync(y, dy, nout * sizeof(double), hipMemcpyDeviceToHost, st));
    PMX_HIP(hipStreamSynchronize(st));
  });
}

pmx_status pmx_edge_apply_kprime(pmx_edge* e, int n_rhs, const double* mu, double* y, int mem_kind, void* stream) {
  return guarded([&] {
    PMX_REQUIRE(e && mu && y, PMX_ERR_INVALID, "null argument");
    PMX_REQUIRE(n_rhs >= 1 && n_rhs <= 1024, PMX_ERR_INVALID, "n_rhs must be in [1, 1024]");
    PMX_HIP(hipSetDevice(e->ctx->c.device));
    hipStream_t st = (hipStream_t)stream;
    Ctx* ctx = &e->ctx->c;
    const size_t n = (size_t)n_rhs * e->e.M;
    DBuf<double> bin, bout;
    const double* dmu = stage_in(ctx, bin, mu, n, mem_kind, st);
    double* dy = y;
    if (mem_kind == PMX_MEM_HOST) {
      bout.alloc(ctx, n);
      dy = bout.p;
    }
    edge_apply_on_curve(e->e, false, n_rhs, dmu, dy, st);
    if (mem_kind == PMX_MEM_HOST) PMX_HIP(hipMemcpyAsync(y, dy, n * sizeof(double), hipMemcpyDeviceToHost, st));
    PMX_HIP(hipStreamSynchronize(st));
  });
}

pmx_status pmx_edge_apply_dlayer(pmx_edge* e, int n_rhs, const double* mu, double* y, int mem_kind, void* stream) {
  return guarded([&] {
    PMX_REQUIRE(e && mu && y, PMX_ERR_INVALID, "null argument");
    PMX_REQUIRE(n_rhs >= 1 && n_rhs <= 1024, PMX_ERR_INVALID, "n_rhs must be in [1, 1024]");
    PMX_REQUIRE(e->e.nu_grad_a_zero, PMX_ERR_INVALID,
                "the on-curve double layer needs nu . grad a = 0 along the curves (else its kernel has a log term)");
    PMX_HIP(hipSetDevice(e->ctx->c.device));
    hipStream_t st = (hipStream_t)stream;
    Ctx* ctx = &e->ctx->c;
    const size_t n = (size_t)n_rhs * e->e.M;
    DBuf<double> bin, bout;
    const double* dmu = stage_in(ctx, bin, mu, n, mem_kind, st);
    double* dy = y;
    if (mem_kind == PMX_MEM_HOST) {
      bout.alloc(ctx, n);
      dy = bout.p;
    }
    edge_apply_on_curve(e->e, true, n_rhs, dmu, dy, st);
    if (mem_kind == PMX_MEM_HOST) PMX_HIP(hipMemcpyAsync(y, dy, n * sizeof(double), hipMemcpyDeviceToHost, st));
    PMX_HIP(hipStreamSynchronize(st));
  });
}

}  // extern "C"
