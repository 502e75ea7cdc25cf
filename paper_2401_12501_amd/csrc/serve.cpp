// Continuous-batching solve server.
//
// Requests (surface, coefficient, right-hand side) are submitted at any time and
// queue in arrival order.  pmx_server_step admits queued requests while an
// active slot is free and their estimated device footprint fits the context's
// HBM budget; each admitted request gets its own HIP stream and worker thread,
// which builds its surface and operator (geometry, near lists, correction
// blocks, FMM tree), keeps them and its Krylov state resident while it solves,
// then releases them.
//
// Operator applies of all solving requests are batched: a worker hands each
// apply (GMRES matvec or refinement residual) to the server's batcher and
// blocks until it is launched.  The batcher collects the applies that are
// pending (it waits until every solving request has one, or a short window has
// passed), makes its stream wait for each request's inputs, and runs every
// kernel of the apply path once for all of them (grouped launches, one argument
// record per request); the workers' streams then wait for that launch and carry
// on with their own Krylov updates.  Requests that arrive while others are on the
// GPU join the next batch once their setup is done.  Every kernel reduces in a
// fixed order and a grouped launch computes each request's data exactly as a
// single launch would, so a request's result does not depend on what else runs.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "pmx_internal.hpp"

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t id = 0;
  int n_patches = 0, q = 0;
  int64_t N = 0;
  std::vector<double> x, xu, xv, xuu, xuv, xvv, a, ga, f;
  bool want_u = false;
  bool held_for_memory = false;   // a slot was free but the budget kept it queued
  uint64_t est_bytes = 0;
  // results
  std::vector<double> sigma, u;
  pmx_info info{};
  pmx_status status = PMX_PENDING;
  std::string message;
  double t_submit = 0, t_admit = 0, t_done = 0;
  std::atomic<int> cancel{0};
  std::atomic<int> finished{0};
  std::thread worker;
};

}  // namespace

// Applies waiting for the next shared launch.
struct pmx_batcher {
  struct Pending {
    pmx_operator* op;
    int precision, n_rhs;
    const double* sigma;
    double* y;
    hipEvent_t ready, done;
    bool launched = false;
    pmx_status code = PMX_OK;
    std::string err;
  };
  int device = 0;
  hipStream_t st = nullptr;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::vector<Pending*> pending;
  int solving = 0;                 // requests between the start and the end of their solve
  bool stop = false;
  std::thread thr;
  double window_s = 500e-6;        // longest wait for the remaining solving requests
  // statistics
  uint64_t n_batches = 0, n_applies = 0, max_batch = 0;
};

struct pmx_server {
  pmx_ctx* ctx = nullptr;
  pmx_batcher* batcher = nullptr;
  pmx_options opts{};
  int max_active = 1;
  uint64_t next_id = 1;
  std::mutex mu;
  std::deque<std::shared_ptr<Request>> queue;
  std::map<uint64_t, std::shared_ptr<Request>> active, done;
  uint64_t reserved = 0;   // estimated bytes of the active requests
  uint64_t peak_reserved = 0;
  uint64_t n_held_for_memory = 0;   // requests that waited for memory with a slot free
};

namespace {

// Rough device footprint: geometry and factors, correction blocks (about six
// near patches per target), Krylov basis, FMM tree data and M2L slots.
uint64_t estimate_bytes(const pmx_options& o, int64_t N, int q, bool want_u) {
  const double per_node = 8.0 * 6 * q * q * (want_u ? 2 : 1) + 8.0 * (o.gmres_restart + 8) + 4000.0;
  return (uint64_t)(per_node * (double)N) + (16u << 20);
}

void batcher_loop(pmx_batcher* b) {
  (void)hipSetDevice(b->device);
  std::unique_lock<std::mutex> lk(b->mu);
  while (true) {
    b->cv_work.wait(lk, [&] { return b->stop || !b->pending.empty(); });
    if (b->stop && b->pending.empty()) break;
    // wait (bounded) until every solving request has an apply pending
    const auto t0 = std::chrono::steady_clock::now();
    const auto limit = t0 + std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                                std::chrono::duration<double>(b->window_s));
    b->cv_work.wait_until(lk, limit, [&] { return b->stop || (int)b->pending.size() >= b->solving; });
    std::vector<pmx_batcher::Pending*> batch;
    batch.swap(b->pending);
    lk.unlock();
    // group by precision and right-hand-side count; each group is one set of shared launches
    std::vector<bool> taken(batch.size(), false);
    for (size_t k = 0; k < batch.size(); ++k) {
      if (taken[k]) continue;
      std::vector<pmx_batcher::Pending*> grp;
      for (size_t m = k; m < batch.size(); ++m)
        if (!taken[m] && batch[m]->precision == batch[k]->precision && batch[m]->n_rhs == batch[k]->n_rhs) {
          taken[m] = true;
          grp.push_back(batch[m]);
        }
      std::vector<pmx::ApplyJob> jobs;
      pmx_status code = PMX_OK;
      std::string err;
      try {
        for (auto* p : grp) {
          PMX_HIP(hipStreamWaitEvent(b->st, p->ready, 0));
          jobs.push_back(pmx::ApplyJob{p->op, p->sigma, p->y});
        }
        pmx::apply_batch(jobs, grp[0]->precision, grp[0]->n_rhs, b->st);
      } catch (const pmx::Error& e) {
        code = e.code;
        err = e.what();
      } catch (const std::exception& e) {
        code = PMX_ERR_DEVICE;
        err = e.what();
      }
      for (auto* p : grp) {
        if (code == PMX_OK && hipEventRecord(p->done, b->st) != hipSuccess) {
          code = PMX_ERR_DEVICE;
          err = "cannot record the batch completion event";
        }
        p->code = code;
        p->err = err;
      }
    }
    lk.lock();
    b->n_batches++;
    b->n_applies += batch.size();
    if (batch.size() > b->max_batch) b->max_batch = batch.size();
    for (auto* p : batch) p->launched = true;
    b->cv_done.notify_all();
  }
}

void solving_delta(pmx_batcher* b, int d) {
  std::lock_guard<std::mutex> lk(b->mu);
  b->solving += d;
  b->cv_work.notify_all();
}

// The request's measured footprint so far replaces its estimate in the server's admission sum
// once it is larger (later admissions see the real size).
void account_footprint(pmx_server* sv, Request* r, const pmx::Ctx& rc) {
  const uint64_t used = rc.peak.load();
  std::lock_guard<std::mutex> lk(sv->mu);
  if (used > r->est_bytes) {
    sv->reserved += used - r->est_bytes;
    r->est_bytes = used;
    if (sv->reserved > sv->peak_reserved) sv->peak_reserved = sv->reserved;
  }
}

void run_request(pmx_server* sv, pmx_options opts, Request* r, pmx_batcher* batcher) {
  hipStream_t st = nullptr;
  pmx_surface* s = nullptr;
  pmx_operator* op = nullptr;
  pmx_ctx* sctx = sv->ctx;
  pmx_ctx rctx;   // the request's own accounting, charged to the server's context
  rctx.owned = false;
  rctx.c.device = sctx->c.device;
  rctx.c.n_cu = sctx->c.n_cu;
  rctx.c.parent = &sctx->c;
  pmx_ctx* ctx = &rctx;
  auto fail = [&](pmx_status code) {
    r->status = code;
    r->message = pmx_last_error();
  };
  if (hipSetDevice(ctx->c.device) != hipSuccess || hipStreamCreate(&st) != hipSuccess) {
    r->status = PMX_ERR_DEVICE;
    r->message = "cannot create a stream for the request";
    r->t_done = now_s();
    r->finished.store(1);
    return;
  }
  pmx_status rc = pmx_surface_create(ctx, r->n_patches, r->q, r->x.data(), r->xu.data(), r->xv.data(),
                                     r->xuu.data(), r->xuv.data(), r->xvv.data(), PMX_MEM_HOST, st, &s);
  if (rc == PMX_OK) rc = pmx_operator_create(s, r->a.data(), r->ga.data(), &opts, PMX_MEM_HOST, st, &op);
  if (rc == PMX_OK) {
    try {
      pmx::prepare_apply(op, opts.precision, 1, st);   // FMM tree and apply scratch, before joining batches
    } catch (const pmx::Error& e) {
      pmx::set_last_error(e.what());
      rc = e.code;
    }
    account_footprint(sv, r, rctx.c);
  }
  if (rc == PMX_OK) {
    op->cancel = &r->cancel;
    r->sigma.assign(r->N, 0.0);
    if (r->want_u) r->u.assign(r->N, 0.0);
    if (batcher) {
      op->batcher = batcher;
      solving_delta(batcher, +1);
    }
    rc = pmx_solve(op, &opts, 1, r->f.data(), r->sigma.data(), 0, r->want_u ? r->u.data() : nullptr, PMX_MEM_HOST,
                   st, &r->info);
    if (batcher) {
      solving_delta(batcher, -1);
      op->batcher = nullptr;
    }
  }
  if (rc != PMX_OK) fail(rc); else r->status = PMX_OK;
  account_footprint(sv, r, rctx.c);
  pmx_operator_destroy(op);
  pmx_surface_destroy(s);
  (void)hipStreamSynchronize(st);
  (void)hipStreamDestroy(st);
  r->t_done = now_s();
  // inputs are no longer needed
  std::vector<double>().swap(r->x); std::vector<double>().swap(r->xu); std::vector<double>().swap(r->xv);
  std::vector<double>().swap(r->xuu); std::vector<double>().swap(r->xuv); std::vector<double>().swap(r->xvv);
  std::vector<double>().swap(r->a); std::vector<double>().swap(r->ga); std::vector<double>().swap(r->f);
  r->finished.store(1);
}

// Move finished workers to the done map (caller holds the lock).
void reap(pmx_server* sv) {
  for (auto it = sv->active.begin(); it != sv->active.end();) {
    Request* r = it->second.get();
    if (r->finished.load()) {
      if (r->worker.joinable()) r->worker.join();
      sv->reserved -= r->est_bytes;
      sv->done[it->first] = it->second;
      it = sv->active.erase(it);
    } else {
      ++it;
    }
  }
}

}  // namespace

extern "C" {

pmx_status pmx_server_create(pmx_ctx* ctx, const pmx_options* opts, int max_active, pmx_server** out) {
  if (!ctx || !out || max_active < 1) {
    pmx::set_last_error("need a context, an output pointer and max_active >= 1");
    return PMX_ERR_INVALID;
  }
  auto* sv = new pmx_server;
  sv->ctx = ctx;
  if (opts) sv->opts = *opts; else { pmx_default_options(&sv->opts); sv->opts.precision = PMX_PREC_MIXED_FMM; }
  sv->max_active = max_active;
  auto* b = new pmx_batcher;
  b->device = ctx->c.device;
  if (hipSetDevice(b->device) != hipSuccess || hipStreamCreate(&b->st) != hipSuccess) {
    delete b;
    delete sv;
    pmx::set_last_error("cannot create the batch stream");
    return PMX_ERR_DEVICE;
  }
  b->thr = std::thread(batcher_loop, b);
  sv->batcher = b;
  ctx_retain(ctx);
  *out = sv;
  return PMX_OK;
}

pmx_status pmx_server_submit(pmx_server* sv, int n_patches, int q, const double* x, const double* xu,
                             const double* xv, const double* xuu, const double* xuv, const double* xvv,
                             const double* a, const double* grad_a, const double* f, int want_u,
                             uint64_t* ticket) {
  if (!sv || !ticket || !x || !xu || !xv || !xuu || !xuv || !xvv || !a || !grad_a || !f || n_patches < 1 ||
      q < 2 || q > 16) {
    pmx::set_last_error("invalid submit arguments");
    return PMX_ERR_INVALID;
  }
  auto r = std::make_shared<Request>();
  r->n_patches = n_patches;
  r->q = q;
  r->N = (int64_t)n_patches * q * q;
  r->want_u = want_u != 0;
  r->est_bytes = estimate_bytes(sv->opts, r->N, q, r->want_u);
  if (sv->ctx->c.budget && r->est_bytes > sv->ctx->c.budget) {
    pmx::set_last_error("request footprint exceeds the HBM budget");
    return PMX_ERR_TOO_LARGE;
  }
  const size_t n3 = 3 * (size_t)r->N;
  r->x.assign(x, x + n3); r->xu.assign(xu, xu + n3); r->xv.assign(xv, xv + n3);
  r->xuu.assign(xuu, xuu + n3); r->xuv.assign(xuv, xuv + n3); r->xvv.assign(xvv, xvv + n3);
  r->a.assign(a, a + r->N); r->ga.assign(grad_a, grad_a + n3); r->f.assign(f, f + r->N);
  r->t_submit = now_s();
  std::lock_guard<std::mutex> lk(sv->mu);
  r->id = sv->next_id++;
  *ticket = r->id;
  sv->queue.push_back(r);
  return PMX_OK;
}

pmx_status pmx_server_step(pmx_server* sv, int* n_active, int* n_queued) {
  if (!sv) {
    pmx::set_last_error("null server");
    return PMX_ERR_INVALID;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  reap(sv);
  const uint64_t budget = sv->ctx->c.budget;
  while (!sv->queue.empty() && (int)sv->active.size() < sv->max_active) {
    auto r = sv->queue.front();
    if (budget && !sv->active.empty() && sv->reserved + r->est_bytes > budget) {   // wait for memory
      if (!r->held_for_memory) {
        r->held_for_memory = true;
        ++sv->n_held_for_memory;
      }
      break;
    }
    sv->queue.pop_front();
    if (r->cancel.load()) {
      r->status = PMX_ERR_CANCELLED;
      r->t_done = now_s();
      r->finished.store(1);
      sv->done[r->id] = r;
      continue;
    }
    r->t_admit = now_s();
    sv->reserved += r->est_bytes;
    if (sv->reserved > sv->peak_reserved) sv->peak_reserved = sv->reserved;
    sv->active[r->id] = r;
    r->worker = std::thread(run_request, sv, sv->opts, r.get(), sv->batcher);
  }
  if (n_active) *n_active = (int)sv->active.size();
  if (n_queued) *n_queued = (int)sv->queue.size();
  return PMX_OK;
}

pmx_status pmx_server_poll(pmx_server* sv, uint64_t ticket, double* sigma, double* u, pmx_info* info,
                           double* times) {
  if (!sv) {
    pmx::set_last_error("null server");
    return PMX_ERR_INVALID;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  reap(sv);
  auto it = sv->done.find(ticket);
  if (it == sv->done.end()) {
    for (auto& q : sv->queue)
      if (q->id == ticket) return PMX_PENDING;
    if (sv->active.count(ticket)) return PMX_PENDING;
    pmx::set_last_error("unknown ticket (never submitted or already collected)");
    return PMX_ERR_INVALID;
  }
  Request* r = it->second.get();
  if (sigma && !r->sigma.empty()) std::memcpy(sigma, r->sigma.data(), r->N * sizeof(double));
  if (u && !r->u.empty()) std::memcpy(u, r->u.data(), r->N * sizeof(double));
  if (info) *info = r->info;
  if (times) {   // seconds: queued (submit -> admit), service (admit -> done), total (submit -> done)
    const double adm = r->t_admit > 0 ? r->t_admit : r->t_done;
    times[0] = adm - r->t_submit;
    times[1] = r->t_done - adm;
    times[2] = r->t_done - r->t_submit;
  }
  const pmx_status st = r->status;
  if (st != PMX_OK) pmx::set_last_error(r->message.empty() ? "request failed" : r->message);
  sv->done.erase(it);
  return st;
}

pmx_status pmx_server_cancel(pmx_server* sv, uint64_t ticket) {
  if (!sv) {
    pmx::set_last_error("null server");
    return PMX_ERR_INVALID;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  for (auto& q : sv->queue)
    if (q->id == ticket) {
      q->cancel.store(1);
      return PMX_OK;
    }
  auto it = sv->active.find(ticket);
  if (it != sv->active.end()) {
    it->second->cancel.store(1);
    return PMX_OK;
  }
  pmx::set_last_error("ticket is not queued or active");
  return PMX_ERR_INVALID;
}

pmx_status pmx_server_get_stats(pmx_server* sv, uint64_t* n_batches, uint64_t* n_applies, uint64_t* max_batch,
                                uint64_t* n_held_for_memory, uint64_t* peak_reserved_bytes) {
  if (!sv || !sv->batcher) {
    pmx::set_last_error("null server");
    return PMX_ERR_INVALID;
  }
  {
    std::lock_guard<std::mutex> lk(sv->batcher->mu);
    if (n_batches) *n_batches = sv->batcher->n_batches;
    if (n_applies) *n_applies = sv->batcher->n_applies;
    if (max_batch) *max_batch = sv->batcher->max_batch;
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  if (n_held_for_memory) *n_held_for_memory = sv->n_held_for_memory;
  if (peak_reserved_bytes) *peak_reserved_bytes = sv->peak_reserved;
  return PMX_OK;
}

void pmx_server_destroy(pmx_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    for (auto& kv : sv->active) kv.second->cancel.store(1);
  }
  for (auto& kv : sv->active)
    if (kv.second->worker.joinable()) kv.second->worker.join();
  if (pmx_batcher* b = sv->batcher) {
    {
      std::lock_guard<std::mutex> lk(b->mu);
      b->stop = true;
      b->cv_work.notify_all();
    }
    if (b->thr.joinable()) b->thr.join();
    (void)hipStreamSynchronize(b->st);
    (void)hipStreamDestroy(b->st);
    delete b;
  }
  pmx_ctx* ctx = sv->ctx;
  delete sv;
  ctx_release(ctx);
}

}  // extern "C"

namespace pmx {

void batcher_apply(pmx_batcher* b, pmx_operator* op, int precision, int n_rhs, const double* sigma, double* y,
                   hipStream_t st) {
  pmx_batcher::Pending p;
  p.op = op;
  p.precision = precision;
  p.n_rhs = n_rhs;
  p.sigma = sigma;
  p.y = y;
  // the operator's two events are reused: it has at most one apply in flight, and each
  // record happens after the other stream's wait on the previous record was enqueued
  if (!op->ev_ready) PMX_HIP(hipEventCreateWithFlags(&op->ev_ready, hipEventDisableTiming));
  if (!op->ev_done) PMX_HIP(hipEventCreateWithFlags(&op->ev_done, hipEventDisableTiming));
  p.ready = op->ev_ready;
  p.done = op->ev_done;
  pmx_status code = PMX_OK;
  std::string err;
  if (hipEventRecord(p.ready, st) != hipSuccess) {
    code = PMX_ERR_DEVICE;
    err = "cannot record the apply input event";
  } else {
    std::unique_lock<std::mutex> lk(b->mu);
    b->pending.push_back(&p);
    b->cv_work.notify_all();
    b->cv_done.wait(lk, [&] { return p.launched; });
    code = p.code;
    err = p.err;
  }
  if (code == PMX_OK && hipStreamWaitEvent(st, p.done, 0) != hipSuccess) {
    code = PMX_ERR_DEVICE;
    err = "cannot wait for the batched apply";
  }
  if (code != PMX_OK) throw Error(code, err);
}

}  // namespace pmx
