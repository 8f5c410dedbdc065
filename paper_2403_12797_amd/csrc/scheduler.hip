// Served path: gp_submit / gp_poll with continuous batching.
//
// A scheduler thread per context admits queued requests as soon as a stream
// slot is free and the request's device footprint fits what the context's
// HBM budget has left, enqueues its fit and/or predict on that slot's stream
// (so the work of admitted requests overlaps on the GPU; the enqueue runs
// without the context lock), and retires requests whose completion event
// has fired.  The number of slots follows the budget (slot_count).  Admission scans the queue in
// arrival order and takes the first request that fits; a request that does
// not fit is passed over at most kMaxBypass times, after which admission
// waits for it (no request starves behind a stream of smaller ones).
// Fitted models are lean (w, the tables and the variance factor) and stay
// device-resident; a model handed to the caller keeps its bytes charged to
// the budget until it is freed.
#include <algorithm>
#include <chrono>
#include <stdlib.h>
#include <string.h>

#include "runtime.h"

namespace mgp {

// Stream slots: MGP_SLOTS if set (1..16), else one per 32 GiB of the HBM
// budget, between 4 and 8.
constexpr int kMinSlots = 4, kMaxSlots = 8;
static int slot_count(size_t budget) {
  if (const char* v = getenv("MGP_SLOTS")) {
    const int k = atoi(v);
    if (k >= 1 && k <= 16) return k;
  }
  const int64_t k = (int64_t)(budget >> 35);
  return (int)std::max<int64_t>(kMinSlots, std::min<int64_t>(kMaxSlots, k));
}
constexpr int kMaxBypass = 32;

static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

bool fault_take(gp_ctx* ctx, const char* name) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  std::string& f = ctx->faults;
  const std::string key = std::string(name) + ",";
  const size_t pos = f.find(key);
  if (pos == std::string::npos) return false;
  f.erase(pos, key.size());
  return true;
}

// Release a finished request's transient resources (mu held).
static void finish(gp_ctx* ctx, Request* r, gp_status st) {
  r->status = st;
  r->t_done = now_s();
  hipStream_t s = r->slot >= 0 ? ctx->slots[r->slot].stream : nullptr;
  if (r->ws) {
    hipFreeAsync(r->ws, s);
    r->ws = nullptr;
  }
  ctx->in_flight_bytes -= r->footprint;
  if (st != GP_OK && r->model) {
    model_release(r->model, s, false);
    r->model = nullptr;
  }
  if (st == GP_OK && r->model) {
    // the model outlives the request: its bytes stay charged until it is freed
    r->model->charged = true;
    ctx->resident_bytes.fetch_add(r->model->bytes);
  }
}

// Allocate and enqueue one admitted request on slot k.  Called with lk
// held; the slot is reserved for r, and the allocations and the (many)
// kernel launches of the request are made with the lock released, so
// gp_submit and gp_poll are not held up meanwhile (only this thread touches
// the slots).
static void launch(gp_ctx* ctx, Request* r, int k, std::unique_lock<std::mutex>& lk) {
  Slot& sl = ctx->slots[k];
  const gp_request& d = r->desc;
  r->slot = k;
  sl.req = r;
  lk.unlock();
  gp_status st = GP_OK;
  hipError_t e = hipMallocAsync(&r->ws, r->ws_bytes ? r->ws_bytes : 256, sl.stream);
  if (e != hipSuccess) {
    r->ws = nullptr;
    st = GP_ENOMEM;
  }
  const gp_model* pm = d.model;
  if (st == GP_OK && d.kind != GP_REQ_PREDICT) {
    gp_params prm = d.params;
    prm.eps = r->eps;
    prm.alpha = r->alpha;
    int64_t M = 0;
    validate_params(&prm, &M);
    st = model_alloc(ctx, &prm, M, true, sl.stream, &r->model);
    if (st == GP_OK) {
      enqueue_fit(r->model, d.x, d.y, d.N, r->layout, r->ws, sl.stream);
      hipMemcpyAsync(sl.flags_host, r->model->flags, 2 * sizeof(int), hipMemcpyDeviceToHost, sl.stream);
      pm = r->model;
    }
  } else if (st == GP_OK) {
    sl.flags_host[0] = sl.flags_host[1] = 0;
  }
  if (st == GP_OK && d.kind != GP_REQ_FIT && d.Ns > 0 && (d.mean || d.var)) {
    // predict workspace follows the fit workspace in the same block
    enqueue_predict(pm, d.xs, d.Ns, d.mean, d.var, (char*)r->ws + r->fit_ws_bytes, sl.stream);
  }
  if (st == GP_OK) hipEventRecord(sl.done, sl.stream);
  lk.lock();
  if (st != GP_OK) {
    sl.req = nullptr;
    finish(ctx, r, st);
    return;
  }
  r->t_admit = now_s();
}

static void scheduler_loop(gp_ctx* ctx) {
  hipSetDevice(ctx->device);
  std::unique_lock<std::mutex> lk(ctx->mu);
  while (true) {
    // retire finished slots
    bool retired = false;
    int active = 0;
    for (int k = 0; k < (int)ctx->slots.size(); ++k) {
      Slot& sl = ctx->slots[k];
      if (!sl.req) continue;
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipErrorNotReady) {
        ++active;
        continue;
      }
      Request* r = sl.req;
      sl.req = nullptr;
      gp_status st = GP_OK;
      if (q != hipSuccess)
        st = GP_EDEVICE;
      else if (sl.flags_host[1])
        st = GP_EINVAL;
      else if (sl.flags_host[0] || r->inject_chol)
        st = GP_ENOTSPD;
      finish(ctx, r, st);
      retired = true;
    }
    if (retired) ctx->cv_done.notify_all();
    if (ctx->stop && ctx->queue.empty() && active == 0) break;
    // admit the first queued request that fits while a slot is free
    auto it = ctx->queue.begin();
    while (it != ctx->queue.end()) {
      Request* r = *it;
      if (ctx->stop) {
        it = ctx->queue.erase(it);
        r->status = GP_ECANCELED;
        ctx->cv_done.notify_all();
        continue;
      }
      int free_slot = -1;
      for (int k = 0; k < (int)ctx->slots.size(); ++k)
        if (!ctx->slots[k].req) {
          free_slot = k;
          break;
        }
      if (free_slot < 0) break;
      const size_t used = ctx->in_flight_bytes + ctx->resident_bytes.load();
      if (used + r->footprint <= ctx->budget) {
        if (it != ctx->queue.begin()) ctx->queue.front()->bypassed += 1;
        it = ctx->queue.erase(it);
        ctx->in_flight_bytes += r->footprint;
        launch(ctx, r, free_slot, lk);
        if (r->status != GP_PENDING) ctx->cv_done.notify_all();
        else ++active;
        // gp_submit may have appended while the lock was released, which
        // invalidates deque iterators: rescan from the head
        it = ctx->queue.begin();
        continue;
      }
      // r waits for memory; later requests may pass it until the head has
      // been passed over kMaxBypass times
      if (ctx->queue.front()->bypassed >= kMaxBypass) break;
      ++it;
    }
    if (active > 0)
      ctx->cv_work.wait_for(lk, std::chrono::microseconds(50));
    else if (!ctx->queue.empty())
      // waiting for memory held by models the caller has not freed yet
      // (their release notifies without the lock, so also wake up on time)
      ctx->cv_work.wait_for(lk, std::chrono::milliseconds(1));
    else if (!ctx->stop)
      ctx->cv_work.wait(lk);
  }
}

gp_status scheduler_start(gp_ctx* ctx) {
  ctx->slots.resize(slot_count(ctx->budget));
  for (auto& sl : ctx->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void**)&sl.flags_host, 16, hipHostMallocDefault) != hipSuccess)
      return fail(GP_EDEVICE, "scheduler: stream/event/pinned allocation failed");
  }
  if (const char* f = getenv("MGP_FAULT")) {
    ctx->faults = f;
    if (!ctx->faults.empty() && ctx->faults.back() != ',') ctx->faults += ",";
  }
  ctx->thread = std::thread(scheduler_loop, ctx);
  return GP_OK;
}

void scheduler_stop(gp_ctx* ctx) {
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->stop = true;
  }
  ctx->cv_work.notify_all();
  if (ctx->thread.joinable()) ctx->thread.join();
  hipDeviceSynchronize();
  for (auto& kv : ctx->requests) {
    Request* r = kv.second;
    if (r->model) model_release(r->model, nullptr, false);
    delete r;
  }
  hipStreamSynchronize(nullptr);
  ctx->requests.clear();
  for (auto& sl : ctx->slots) {
    if (sl.stream) hipStreamDestroy(sl.stream);
    if (sl.done) hipEventDestroy(sl.done);
    if (sl.flags_host) hipHostFree(sl.flags_host);
  }
  ctx->slots.clear();
}

}  // namespace mgp

using namespace mgp;

extern "C" {

}  // extern "C"

namespace mgp {
// Validate a request and fill r's descriptor copy, layout and sizes
// (no device work, no ctx lock).
static gp_status prepare_request(gp_ctx* ctx, const gp_request* req, Request* r) {
  r->desc = *req;
  int64_t M = 0;
  int prec = 0;
  if (req->kind == GP_REQ_FIT || req->kind == GP_REQ_FIT_PREDICT) {
    gp_status st = validate_params(&req->params, &M);
    if (st != GP_OK) return st;
    if (req->N < 1 || !req->x || !req->y) return fail(GP_EINVAL, "FIT request needs x, y and N >= 1");
    for (int j = 0; j < req->params.p; ++j) {
      r->eps[j] = req->params.eps[j];
      r->alpha[j] = req->params.alpha[j];
    }
    prec = req->params.precision;
  } else if (req->kind == GP_REQ_PREDICT) {
    if (!req->model) return fail(GP_EINVAL, "PREDICT request needs a model");
    M = req->model->M;
    prec = req->model->precision;
  } else {
    return fail(GP_EINVAL, "unknown request kind %d", req->kind);
  }
  if (req->kind != GP_REQ_FIT && req->Ns > 0 && (req->mean || req->var) && !req->xs)
    return fail(GP_EINVAL, "predict part needs xs");
  if (req->Ns < 0) return fail(GP_EINVAL, "Ns must be >= 0");
  size_t ws = 0, foot = 0;
  if (req->kind != GP_REQ_PREDICT) {
    // the layout (and the Gram chunk in it) is fixed here, once
    r->layout = fit_layout(req->N, req->params.p, req->params.n, M, prec,
                           tuned_chunk(ctx, req->params.p, req->params.n, req->N), false, true);
    ws += (r->layout.total + 255) & ~(size_t)255;
    r->model_bytes = model_bytes(M, prec, true);
    foot += r->model_bytes;
  }
  r->fit_ws_bytes = ws;
  if (req->kind != GP_REQ_FIT) ws += predict_workspace_bytes(req->Ns, M, prec);
  foot += ws;
  r->ws_bytes = ws;
  r->footprint = foot;
  return GP_OK;
}
}  // namespace mgp

extern "C" {

gp_status gp_request_footprint(gp_ctx* ctx, const gp_request* req, size_t* model_bytes_out,
                               size_t* transient_bytes_out) {
  if (!ctx || !req) return fail(GP_EINVAL, "ctx/req is NULL");
  Request r;
  const gp_status st = prepare_request(ctx, req, &r);
  if (st != GP_OK) return st;
  if (model_bytes_out) *model_bytes_out = r.model_bytes;
  if (transient_bytes_out) *transient_bytes_out = r.ws_bytes;
  return GP_OK;
}

gp_status gp_ctx_memory(gp_ctx* ctx, size_t* budget, size_t* in_flight, size_t* resident) {
  if (!ctx) return fail(GP_EINVAL, "ctx is NULL");
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (budget) *budget = ctx->budget;
  if (in_flight) *in_flight = ctx->in_flight_bytes;
  if (resident) *resident = ctx->resident_bytes.load();
  return GP_OK;
}

gp_status gp_submit(gp_ctx* ctx, const gp_request* req, int64_t* req_id) {
  if (!ctx || !req || !req_id) return fail(GP_EINVAL, "ctx/req/req_id is NULL");
  *req_id = 0;
  Request* r = new Request();
  const gp_status pst = prepare_request(ctx, req, r);
  if (pst != GP_OK) {
    delete r;
    return pst;
  }
  const size_t foot = r->footprint;
  if (foot > ctx->budget) {
    const size_t budget = ctx->budget;
    delete r;
    return fail(GP_ENOMEM, "request needs %zu device bytes, budget is %zu", foot, budget);
  }
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->stop) {
      delete r;
      return fail(GP_ECANCELED, "context is shutting down");
    }
    const std::string key = "chol,";
    const size_t pos = ctx->faults.find(key);
    if (pos != std::string::npos && req->kind != GP_REQ_PREDICT) {
      ctx->faults.erase(pos, key.size());
      r->inject_chol = true;
    }
    r->id = ctx->next_id++;
    r->t_submit = now_s();
    ctx->requests[r->id] = r;
    ctx->queue.push_back(r);
    *req_id = r->id;
  }
  ctx->cv_work.notify_one();
  return GP_OK;
}

gp_status gp_poll(gp_ctx* ctx, int64_t req_id, int32_t wait_us, gp_model** model_out) {
  if (!ctx) return fail(GP_EINVAL, "ctx is NULL");
  if (model_out) *model_out = nullptr;
  std::unique_lock<std::mutex> lk(ctx->mu);
  auto it = ctx->requests.find(req_id);
  if (it == ctx->requests.end()) return fail(GP_ENOTFOUND, "unknown request id %lld", (long long)req_id);
  Request* r = it->second;
  if (r->status == GP_PENDING && wait_us != 0) {
    auto done = [&] { return r->status != GP_PENDING; };
    if (wait_us < 0)
      ctx->cv_done.wait(lk, done);
    else
      ctx->cv_done.wait_for(lk, std::chrono::microseconds(wait_us), done);
  }
  if (r->status == GP_PENDING) return GP_PENDING;
  const gp_status st = r->status;
  if (r->model) {
    if (model_out && st == GP_OK) {
      *model_out = r->model;
    } else {
      model_release(r->model, nullptr, false);
    }
    r->model = nullptr;
  }
  ctx->requests.erase(it);
  delete r;
  if (st < 0) return fail(st, "request %lld failed with status %d", (long long)req_id, (int)st);
  return st;
}

}  // extern "C"
