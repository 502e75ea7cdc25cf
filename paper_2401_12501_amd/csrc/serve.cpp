// Continuous-batching solve server.
//
// Requests (surface, coefficient, right-hand side) are submitted at any time and
// queue in arrival order.  pmx_server_step admits queued requests while an
// active slot is free and their estimated device footprint fits the context's
// HBM budget; each admitted request gets its own HIP stream and worker thread,
// which builds its surface and operator (geometry, near lists, correction
// blocks, FMM tree), keeps them and its Krylov state resident while it solves,
// then releases them.  Work of all active requests is in flight on the device
// at once, so a request that arrives while others run starts as soon as a slot
// and memory are free.  Every kernel of the path reduces in a fixed order, so a
// request's result does not depend on what else runs beside it.
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

struct pmx_server {
  pmx_ctx* ctx = nullptr;
  pmx_options opts{};
  int max_active = 1;
  uint64_t next_id = 1;
  std::mutex mu;
  std::deque<std::shared_ptr<Request>> queue;
  std::map<uint64_t, std::shared_ptr<Request>> active, done;
  uint64_t reserved = 0;   // estimated bytes of the active requests
};

namespace {

// Rough device footprint: geometry and factors, correction blocks (about six
// near patches per target), Krylov basis, FMM tree data and M2L slots.
uint64_t estimate_bytes(const pmx_options& o, int64_t N, int q, bool want_u) {
  const double per_node = 8.0 * 6 * q * q * (want_u ? 2 : 1) + 8.0 * (o.gmres_restart + 8) + 4000.0;
  return (uint64_t)(per_node * (double)N) + (16u << 20);
}

void run_request(pmx_ctx* ctx, pmx_options opts, Request* r) {
  hipStream_t st = nullptr;
  pmx_surface* s = nullptr;
  pmx_operator* op = nullptr;
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
    op->cancel = &r->cancel;
    r->sigma.assign(r->N, 0.0);
    if (r->want_u) r->u.assign(r->N, 0.0);
    rc = pmx_solve(op, &opts, 1, r->f.data(), r->sigma.data(), 0, r->want_u ? r->u.data() : nullptr, PMX_MEM_HOST,
                   st, &r->info);
  }
  if (rc != PMX_OK) fail(rc); else r->status = PMX_OK;
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
    if (budget && !sv->active.empty() && sv->reserved + r->est_bytes > budget) break;   // wait for memory
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
    sv->active[r->id] = r;
    r->worker = std::thread(run_request, sv->ctx, sv->opts, r.get());
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

void pmx_server_destroy(pmx_server* sv) {
  if (!sv) return;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    for (auto& kv : sv->active) kv.second->cancel.store(1);
  }
  for (auto& kv : sv->active)
    if (kv.second->worker.joinable()) kv.second->worker.join();
  delete sv;
}

}  // extern "C"
