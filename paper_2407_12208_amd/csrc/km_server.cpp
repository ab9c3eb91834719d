// km_server.cpp -- continuous-batching k-means server.
//
// A scheduler thread owns a device arena of a fixed byte budget, a private
// library context and two HIP streams (compute, copy).  Each scheduler round:
//   1. enqueue one Lloyd round (assignment pass + centre update) for every
//      running request, and the final assignment pass for the requests whose
//      rounds are over, as batched launches on the compute stream;
//   2. while that runs, admit waiting requests in arrival order whose device
//      footprint fits the free arena (copy their data in on the copy stream);
//   3. wait for the round, read every running request's result record,
//      retire finished / failed / cancelled requests (copy results to the
//      caller's host buffers, free their arena range, wake pollers).
// A request's arithmetic is that of kmeans_lloyd on it alone: kernels treat
// the problems of a batched launch independently.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "km_context.hpp"

namespace km {

// First-fit allocator over one device allocation.
class RangeAlloc {
 public:
  bool init(size_t bytes) {
    if (hipMalloc(reinterpret_cast<void**>(&base_), bytes) != hipSuccess) {
      base_ = nullptr;
      return false;
    }
    cap_ = bytes;
    free_[0] = bytes;
    return true;
  }
  void destroy() {
    if (base_) (void)hipFree(base_);
    base_ = nullptr;
  }
  // offset or SIZE_MAX
  size_t alloc(size_t bytes) {
    bytes = Arena::align(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        used_ += bytes;
        return off;
      }
    }
    return SIZE_MAX;
  }
  void release(size_t off, size_t bytes) {
    bytes = Arena::align(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  char* base() const { return base_; }
  size_t cap() const { return cap_; }

 private:
  char* base_ = nullptr;
  size_t cap_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;
};

// Queued: in the arrival queue.  Admitting: taken off the queue by the
// scheduler, its data being copied in (the lock is not held meanwhile).
// Active: in the running set.  Done: finished, failed or cancelled.
enum class ReqState { Queued, Admitting, Active, Done };

struct Request {
  uint64_t ticket;
  km_problem host;       // caller's host pointers
  km_precision prec;
  AssignPlan plan;
  size_t footprint = 0;
  size_t off = SIZE_MAX;
  // device-side problem and batch state
  km_problem dev{};
  BatchState bs{};
  ReqState state = ReqState::Queued;
  int32_t status = KM_PENDING;  // final status once Done
  std::atomic<bool> cancel{false};  // set by kmeans_cancel, read by the scheduler
  bool final_enqueued = false;
};

static size_t request_footprint(const km_problem& q, const AssignPlan& a) {
  Plan pl;
  pl.add<float>((size_t)q.n * q.d);             // X
  pl.add<float>((size_t)q.k * q.d);             // C (ping)
  pl.add<float>((size_t)q.k * q.d);             // C (pong)
  pl.add<int32_t>((size_t)q.n);                 // labels
  if (q.mindist) pl.add<float>((size_t)q.n);
  pl.add<double>((size_t)q.max_iter + 1);       // SSE history (always kept)
  plan_pass(pl, a);
  plan_update(pl, q.n, q.d, q.k);
  return pl.bytes;
}

}  // namespace km

struct km_server {
  km_context* ctx = nullptr;        // private context of the scheduler thread
  km::RangeAlloc arena;
  int32_t max_active = 0;
  hipStream_t compute = nullptr, copy = nullptr;
  std::mutex mu;
  std::condition_variable cv_work;  // scheduler waits for requests
  std::condition_variable cv_done;  // pollers wait for completion
  std::deque<km::Request*> queued;
  std::vector<km::Request*> active;
  std::map<uint64_t, std::unique_ptr<km::Request>> all;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread thr;
  void loop();
  bool admit_one(km::Request* r);
  void retire(km::Request* r, int32_t status, bool copy_results, const km::KResult* res);
};

using namespace km;

// Carve a request's device range and copy its inputs in (copy stream).
bool km_server::admit_one(Request* r) {
  const size_t off = arena.alloc(r->footprint);
  if (off == SIZE_MAX) return false;
  r->off = off;
  Arena a;
  a.base = arena.base() + off;
  a.cap = r->footprint;
  a.used = 0;
  const km_problem& h = r->host;
  km_problem& d = r->dev;
  d = h;
  float* X = a.take<float>((size_t)h.n * h.d);
  float* C0 = a.take<float>((size_t)h.k * h.d);
  float* C1 = a.take<float>((size_t)h.k * h.d);
  d.X = X;
  d.C_inout = C0;
  d.labels = a.take<int32_t>((size_t)h.n);
  d.mindist = h.mindist ? a.take<float>((size_t)h.n) : nullptr;
  d.sse_hist = a.take<double>((size_t)h.max_iter + 1);
  d.stats = nullptr;
  BatchState& s = r->bs;
  s.prob = &r->dev;
  s.plan = r->plan;
  s.bufs = carve_pass(a, r->plan);
  s.upd = carve_update(a, h.n, h.d, h.k);
  s.upd.X = X;
  s.upd.labels = d.labels;
  s.upd.result = s.bufs.result;
  s.upd.status = s.bufs.status;
  s.cur = C0;
  s.nxt = C1;
  s.it = 0;
  s.done = h.max_iter == 0;
  if (hipMemcpyAsync(X, h.X, sizeof(float) * (size_t)h.n * h.d, hipMemcpyHostToDevice, copy) != hipSuccess ||
      hipMemcpyAsync(C0, h.C_inout, sizeof(float) * (size_t)h.k * h.d, hipMemcpyHostToDevice, copy) != hipSuccess ||
      hipMemsetAsync(s.bufs.status, 0, sizeof(int), copy) != hipSuccess ||
      hipMemsetAsync(s.bufs.result, 0, sizeof(KResult), copy) != hipSuccess) {
    arena.release(off, r->footprint);
    r->off = SIZE_MAX;
    return false;
  }
  return true;
}

void km_server::retire(Request* r, int32_t status, bool copy_results, const KResult* res_in) {
  // results: compute stream is idle here (the round was synchronised)
  if (copy_results) {
    const km_problem& h = r->host;
    const km_problem& d = r->dev;
    bool ok = hipMemcpy(h.C_inout, r->bs.cur, sizeof(float) * (size_t)h.k * h.d, hipMemcpyDeviceToHost) ==
                  hipSuccess &&
              hipMemcpy(h.labels, d.labels, sizeof(int32_t) * (size_t)h.n, hipMemcpyDeviceToHost) == hipSuccess;
    if (ok && h.mindist)
      ok = hipMemcpy(h.mindist, d.mindist, sizeof(float) * (size_t)h.n, hipMemcpyDeviceToHost) == hipSuccess;
    if (ok && h.sse_hist)
      ok = hipMemcpy(h.sse_hist, d.sse_hist, sizeof(double) * (size_t)(r->bs.it + 1), hipMemcpyDeviceToHost) ==
           hipSuccess;
    if (!ok) status = KM_ERR_DEVICE;
  }
  if (r->host.stats) {
    KResult res{};
    if (res_in) res = *res_in;
    else (void)hipMemcpy(&res, r->bs.bufs.result, sizeof(KResult), hipMemcpyDeviceToHost);
    km_stats* o = r->host.stats;
    o->n_corrected = r->plan.route == Route::Direct64Exact ? 0 : res.n_corrected;
    o->n_pairs = res.n_pairs;
    o->iters = r->bs.it;
    o->data_status = status_from_bits(res.status);
    o->sse_last = res.sse;
    o->shift_last = res.shift;
    o->alpha_used = r->plan.alpha_used;
  }
  arena.release(r->off, r->footprint);
  r->off = SIZE_MAX;
  std::lock_guard<std::mutex> g(mu);
  r->status = status;
  r->state = ReqState::Done;
  cv_done.notify_all();
}

void km_server::loop() {
  (void)hipSetDevice(ctx->device);
  for (;;) {
    // ---- wait for work
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stop || !queued.empty() || !active.empty(); });
      if (stop && queued.empty() && active.empty()) break;
      if (stop) {  // cancel everything not yet admitted
        for (Request* r : queued) {
          r->status = KM_ERR_CANCELLED;
          r->state = ReqState::Done;
        }
        queued.clear();
        cv_done.notify_all();
      }
    }
    // ---- 1. enqueue one round for the running requests
    std::vector<BatchState*> iter, fin;
    for (Request* r : active) {
      if (r->cancel) continue;
      if (!r->bs.done) iter.push_back(&r->bs);
      else if (!r->final_enqueued) fin.push_back(&r->bs);
    }
    hipError_t e = enqueue_batch_round(ctx, iter, compute);
    if (e == hipSuccess && !fin.empty()) e = enqueue_batch_pass(ctx, fin, true, compute);
    for (Request* r : active)
      if (!r->cancel && r->bs.done && std::find(fin.begin(), fin.end(), &r->bs) != fin.end())
        r->final_enqueued = true;
    // ---- 2. admission while the round runs.  The head request leaves the
    // queue (state Admitting) before the lock is released for its copies,
    // so a concurrent cancel only flags it; a request that does not fit goes
    // back to the head of the queue (FIFO: no overtaking).
    std::vector<Request*> admitted;
    {
      std::unique_lock<std::mutex> lk(mu);
      while (!queued.empty() && (int)(active.size() + admitted.size()) < max_active) {
        Request* r = queued.front();
        queued.pop_front();
        r->state = ReqState::Admitting;
        lk.unlock();
        const bool ok = admit_one(r);
        lk.lock();
        if (!ok) {
          if (r->cancel.load()) {
            r->status = KM_ERR_CANCELLED;
            r->state = ReqState::Done;
            cv_done.notify_all();
            continue;
          }
          r->state = ReqState::Queued;
          queued.push_front(r);
          break;
        }
        r->state = ReqState::Active;
        admitted.push_back(r);
      }
    }
    if (!admitted.empty()) (void)hipStreamSynchronize(copy);
    for (size_t i = 0; i < admitted.size();) {  // cancelled while admitted
      Request* r = admitted[i];
      if (r->cancel.load()) {
        retire(r, KM_ERR_CANCELLED, false, nullptr);
        admitted.erase(admitted.begin() + (long)i);
      } else {
        ++i;
      }
    }
    // ---- 3. wait for the round, read every running request's result
    // record with one gather and one copy, retire
    hipError_t es = hipStreamSynchronize(compute);
    std::vector<KResult> res(active.size());
    if (e == hipSuccess && es == hipSuccess && !active.empty()) {
      std::vector<const KResult*> src(active.size());
      for (size_t i = 0; i < active.size(); ++i) src[i] = active[i]->bs.bufs.result;
      es = read_results(ctx, src, res.data(), compute);
    }
    std::vector<Request*> keep;
    for (size_t i = 0; i < active.size(); ++i) {
      Request* r = active[i];
      if (r->cancel.load()) {
        retire(r, KM_ERR_CANCELLED, false, nullptr);
        continue;
      }
      if (e != hipSuccess || es != hipSuccess) {
        retire(r, KM_ERR_DEVICE, false, nullptr);
        continue;
      }
      const int32_t ds = status_from_bits(res[i].status);
      if (ds != KM_OK) {
        retire(r, ds, false, &res[i]);
        continue;
      }
      if (r->final_enqueued) {
        retire(r, KM_OK, true, &res[i]);
        continue;
      }
      if (!r->bs.done && r->host.tol > 0.0 && r->bs.it > 0 && res[i].shift < r->host.tol) r->bs.done = true;
      keep.push_back(r);
    }
    active.swap(keep);
    for (Request* r : admitted) active.push_back(r);
  }
}

extern "C" {

int32_t kmeans_server_create(km_context* ctx, size_t hbm_budget_bytes, int32_t max_active, km_server** out) {
  if (!out) return KM_ERR_ARG;
  *out = nullptr;
  if (!ctx || hbm_budget_bytes < (1u << 20) || max_active < 1) return KM_ERR_ARG;
  km_server* s = new (std::nothrow) km_server();
  if (!s) return KM_ERR_OOM;
  int32_t rc = kmeans_context_create(ctx->device, &s->ctx);
  if (rc != KM_OK) {
    delete s;
    return rc;
  }
  if (!s->arena.init(hbm_budget_bytes)) {
    kmeans_context_destroy(s->ctx);
    delete s;
    return KM_ERR_OOM;
  }
  if (hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking) != hipSuccess) {
    s->arena.destroy();
    kmeans_context_destroy(s->ctx);
    delete s;
    return KM_ERR_DEVICE;
  }
  s->max_active = max_active;
  s->thr = std::thread([s] { s->loop(); });
  *out = s;
  return KM_OK;
}

int32_t kmeans_submit(km_server* s, const km_problem* q, const km_precision* prec, uint64_t* ticket) {
  if (!s || !q || !ticket) return KM_ERR_ARG;
  km_precision p = precision_or_default(prec);
  int32_t v = validate_precision(p);
  if (v != KM_OK) return v;
  if (!q->X || !q->C_inout || !q->labels || q->max_iter < 0) return KM_ERR_ARG;
  v = check_shape(q->n, q->d, q->k, p);
  if (v != KM_OK) return v;
  auto r = std::make_unique<Request>();
  r->host = *q;
  r->prec = p;
  r->plan = plan_assign(p, q->n, q->d, q->k);
  r->footprint = request_footprint(*q, r->plan);
  if (r->footprint > s->arena.cap()) return KM_ERR_OOM;  // can never fit
  std::lock_guard<std::mutex> g(s->mu);
  if (s->stop) return KM_ERR_CANCELLED;
  r->ticket = s->next_ticket++;
  *ticket = r->ticket;
  s->queued.push_back(r.get());
  s->all[r->ticket] = std::move(r);
  s->cv_work.notify_one();
  return KM_OK;
}

int32_t kmeans_poll(km_server* s, uint64_t ticket, int32_t timeout_ms) {
  if (!s) return KM_ERR_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return KM_ERR_NOTFOUND;
  Request* r = it->second.get();
  auto done = [&] { return r->state == ReqState::Done; };
  if (timeout_ms < 0) s->cv_done.wait(lk, done);
  else if (timeout_ms > 0) s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done);
  return r->state == ReqState::Done ? r->status : KM_PENDING;
}

int32_t kmeans_cancel(km_server* s, uint64_t ticket) {
  if (!s) return KM_ERR_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return KM_ERR_NOTFOUND;
  Request* r = it->second.get();
  if (r->state == ReqState::Done) return KM_OK;
  if (r->state == ReqState::Queued) {
    s->queued.erase(std::remove(s->queued.begin(), s->queued.end(), r), s->queued.end());
    r->status = KM_ERR_CANCELLED;
    r->state = ReqState::Done;
    s->cv_done.notify_all();
  } else {
    r->cancel.store(true);  // Admitting or Active: retired by the scheduler
  }
  return KM_OK;
}

int32_t kmeans_server_destroy(km_server* s) {
  if (!s) return KM_ERR_ARG;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->thr.joinable()) s->thr.join();
  (void)hipStreamDestroy(s->compute);
  (void)hipStreamDestroy(s->copy);
  s->arena.destroy();
  kmeans_context_destroy(s->ctx);
  delete s;
  return KM_OK;
}

}  // extern "C"
