// Serving: continuous batching of contact queries from many clients.
//
// cm_submit copies a request (host queries, optional cotangents) into the
// pending queue.  A scheduler thread, started on the first submit, keeps up to
// kSlots batches in flight on their own streams: whenever a slot is free it
// admits pending requests in arrival order (sized at submit from the objects'
// counts) while the device memory the slots
// hold stays within the context's budget (each request's plan scratch and
// buffers estimated as the plan lays them out; a slot's buffer is sized to its
// batch, and idle slots give theirs back when a batch needs the room), packs
// their queries into one batch, runs the forward pass over the forward-only
// requests and the gradient pass (one forward sweep that also writes the
// records, and the adjoint) over those that asked for a gradient, and copies
// the results back into pinned staging.  Batches on
// different streams overlap; each slot's batch is planned and launched by the
// slot's own worker thread (planners share the object registry under a
// reader lock), so batches are planned concurrently while others run.
// Completion is detected with events; results are scattered to the callers'
// buffers and the tickets are marked done.  A query's results depend only on
// that query (fixed-order reductions), so they are the same alone and mixed.
#include <chrono>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "runtime.h"

namespace cm {

namespace {

constexpr int kSlots = 3;
constexpr int64_t kMaxBatchQueries = 16384;
constexpr size_t kQueueLimit = 1 << 20;
// a batch's layout can exceed the sum of its requests' layouts by a tape tile
// and a few aligned arrays per request (rounding of the merged sizes)
constexpr size_t kSlackPerRequest = size_t(16) << 10;
constexpr size_t kDevGranule = size_t(1) << 20;  // slot buffers are sized in MiB

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Req {
  cm_ticket id = 0;
  std::vector<cm_query> q;
  bool grad = false;
  std::vector<float> cot;  // AoS [G][12]
  float* out_groups = nullptr;
  float* out_grad = nullptr;
  int64_t G = 0;
  size_t bytes = 0;
  double t_submit = 0;
};

// Device and pinned buffers of one in-flight batch, grown on demand.
struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  void* dmem = nullptr;
  size_t dcap = 0;
  char* pinned = nullptr;
  size_t pcap = 0;
  bool busy = false;     // admitted requests: being planned or on the device
  bool running = false;  // launched: the scheduler polls its event
  std::thread worker;    // plans and launches the slot's batches
  std::condition_variable wcv;
  std::vector<Req*> reqs;
  std::unique_ptr<cm_plan> pf, pg;  // forward plan (forward-only requests), adjoint plan (gradient requests)
  size_t bytes = 0;
  // offsets into dmem / pinned
  size_t d_q = 0, d_qg = 0, d_out = 0, d_outg = 0, d_cot = 0, d_grad = 0, d_pf = 0, d_pg = 0;
  size_t h_q = 0, h_qg = 0, h_out = 0, h_outg = 0, h_cot = 0, h_grad = 0;
  int64_t n = 0, ng = 0, G = 0, Gg = 0;
};

}  // namespace

struct Serving {
  cm_context* ctx = nullptr;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::deque<Req*> pending;
  std::unordered_map<cm_ticket, cm_status> finished;
  std::unordered_map<cm_ticket, int> live;  // submitted, not yet finished
  size_t inflight = 0;            // estimated bytes of the admitted requests
  size_t held = 0, peak_held = 0;  // device bytes the slots' buffers hold (never above the budget)
  bool stop = false;
  bool quit_workers = false;
  cm_ticket next = 1;
  int64_t n_submitted = 0, n_completed = 0, n_batches = 0, n_queries = 0;
  std::vector<double> latencies;  // seconds from submit to results written, in completion order
  Slot slots[kSlots];
};

namespace {

// Device bytes a request needs inside a batch: its share of the plan scratch
// (entries, bitmask, partials, ...) plus its input and output buffers.  A
// forward request joins the forward plan (no tape); a gradient request joins
// the adjoint plan (a tape of float values), whose forward sweep also writes
// its records, and brings cotangents and a gradient buffer.
size_t request_bytes(cm_context* ctx, const PlanSizes& z, bool grad) {
  cm_plan probe;  // laid out for the request's sizes (no tables are built)
  probe.ctx = ctx;
  probe.reserved = true;
  probe.cap = z;
  probe.tape_kind = grad ? 1 : 0;
  size_t b = plan_layout(&probe, nullptr) + 64 * size_t(z.n) + 48 * size_t(z.G);  // plan, queries, records
  if (grad) b += 48 * size_t(z.G) + 48 * size_t(z.n);                             // cotangents, gradient
  return b + kSlackPerRequest;
}

// Device bytes slot t holds, or, once admitted, will hold for its batch (its
// worker sizes the buffer after admission).  Called with S->mu held.
size_t claim(const Slot& t) { return t.busy ? std::max(t.dcap, align_up(t.bytes, kDevGranule)) : t.dcap; }
size_t claims_except(const Serving* S, const Slot* s) {
  size_t c = 0;
  for (const Slot& t : S->slots)
    if (&t != s) c += claim(t);
  return c;
}

// Frees the buffers of idle slots other than `keep` (their last batch has
// completed).  Called with S->mu held.
void release_idle(Serving* S, const Slot* keep) {
  for (Slot& t : S->slots) {
    if (&t == keep || t.busy || !t.dmem) continue;
    (void)hipStreamSynchronize(t.stream);
    (void)hipFree(t.dmem);
    S->held -= t.dcap;
    t.dmem = nullptr;
    t.dcap = 0;
  }
}

// Sizes the slot's device buffer for a batch of `bytes` (exactly, in MiB
// granules; a larger buffer is kept) so that what the slots hold and have
// been admitted to hold never exceeds the budget.
bool ensure_device(Serving* S, Slot& s, size_t bytes) {
  if (s.dcap >= bytes) return true;
  const size_t want = align_up(bytes, kDevGranule);
  std::lock_guard<std::mutex> lk(S->mu);
  if (claims_except(S, &s) + want > S->ctx->budget) release_idle(S, &s);
  if (claims_except(S, &s) + want > S->ctx->budget) return false;
  if (s.dmem) {
    (void)hipStreamSynchronize(s.stream);
    (void)hipFree(s.dmem);
    S->held -= s.dcap;
    s.dmem = nullptr;
    s.dcap = 0;
  }
  if (hipMalloc(&s.dmem, want) != hipSuccess) { s.dmem = nullptr; return false; }
  s.dcap = want;
  S->held += want;
  S->peak_held = std::max(S->peak_held, S->held);
  return true;
}

bool ensure_pinned(Slot& s, size_t bytes) {
  if (s.pcap >= bytes) return true;
  if (s.pinned) (void)hipHostFree(s.pinned);
  s.pcap = std::max(bytes, 2 * s.pcap);
  if (hipHostMalloc(reinterpret_cast<void**>(&s.pinned), s.pcap, 0) != hipSuccess) {
    s.pinned = nullptr; s.pcap = 0; return false;
  }
  return true;
}

// Builds the batch's plans and buffers and enqueues its work on the slot's stream.
cm_status launch_batch(Serving* S, cm_context* ctx, Slot& s) {
  std::vector<cm_query> qa, qg;
  std::vector<const Req*> gr;
  for (const Req* r : s.reqs) {
    if (r->grad) { qg.insert(qg.end(), r->q.begin(), r->q.end()); gr.push_back(r); }
    else qa.insert(qa.end(), r->q.begin(), r->q.end());
  }
  s.n = int64_t(qa.size());
  s.ng = int64_t(qg.size());
  // the slot's plans are reused batch after batch (their host tables keep
  // their capacity); the slot is free only once its previous batch completed
  size_t bf = 0, bg = 0;
  cm_status st = CM_OK;
  if (s.n) {
    if (!s.pf) s.pf.reset(new cm_plan);
    s.pf->tape_kind = 0;  // forward only
    st = plan_host(ctx, qa.data(), int32_t(s.n), s.pf.get(), &bf);
    if (st != CM_OK) return st;
  }
  if (s.ng) {
    if (!s.pg) s.pg.reset(new cm_plan);
    s.pg->tape_kind = 1;  // float adjoint only
    st = plan_host(ctx, qg.data(), int32_t(s.ng), s.pg.get(), &bg);
    if (st != CM_OK) return st;
  }
  s.G = s.n ? s.pf->G : 0;
  s.Gg = s.ng ? s.pg->G : 0;
  size_t off = 0;
  auto take = [&](size_t b) { size_t r = off; off = align_up(off + b, 256); return r; };
  s.d_pf = take(bf);
  s.d_pg = take(bg);
  s.d_q = take(64 * size_t(s.n));
  s.d_qg = take(64 * size_t(s.ng));
  s.d_out = take(48 * size_t(s.G));
  s.d_outg = take(48 * size_t(s.Gg));
  s.d_cot = take(48 * size_t(s.Gg));
  s.d_grad = take(48 * size_t(s.ng));
  if (!ensure_device(S, s, off)) return fail(ctx, CM_E_OOM, "serving: device allocation within the budget failed");
  size_t hoff = 0;
  auto htake = [&](size_t b) { size_t r = hoff; hoff = align_up(hoff + b, 256); return r; };
  s.h_q = htake(64 * size_t(s.n));
  s.h_qg = htake(64 * size_t(s.ng));
  s.h_out = htake(48 * size_t(s.G));
  s.h_outg = htake(48 * size_t(s.Gg));
  s.h_cot = htake(48 * size_t(s.Gg));
  s.h_grad = htake(48 * size_t(s.ng));
  if (!ensure_pinned(s, hoff)) return fail(ctx, CM_E_OOM, "serving: pinned allocation failed");
  char* d = static_cast<char*>(s.dmem);
  std::memcpy(s.pinned + s.h_q, qa.data(), 64 * size_t(s.n));
  if (s.ng) {
    std::memcpy(s.pinned + s.h_qg, qg.data(), 64 * size_t(s.ng));
    // cotangents AoS [G][12] per request -> SoA [12][Gg] for the adjoint plan
    float* c = reinterpret_cast<float*>(s.pinned + s.h_cot);
    int64_t g0 = 0;
    for (const Req* r : gr) {
      for (int64_t g = 0; g < r->G; ++g)
        for (int k = 0; k < 12; ++k) c[k * s.Gg + g0 + g] = r->cot[size_t(12 * g + k)];
      g0 += r->G;
    }
  }
  hipStream_t st_ = s.stream;
  if (s.n) {
    if (hipMemcpyAsync(d + s.d_q, s.pinned + s.h_q, 64 * size_t(s.n), hipMemcpyHostToDevice, st_) != hipSuccess)
      return fail(ctx, CM_E_HIP, "serving: upload failed");
    if ((st = plan_bind(s.pf.get(), d + s.d_pf, st_)) != CM_OK) return st;
    float* out = reinterpret_cast<float*>(d + s.d_out);
    const int64_t G = s.G;
    cm_groups og{out, out + 3 * G, out + 6 * G, out + 7 * G, out + 10 * G, out + 11 * G};
    FwdArgs a = fwd_args(ctx, s.pf.get(), reinterpret_cast<const cm_query*>(d + s.d_q), og, nullptr);
    if (launch_forward(a, st_) != hipSuccess) return fail(ctx, CM_E_HIP, "serving: forward launch failed");
    if (hipMemcpyAsync(s.pinned + s.h_out, d + s.d_out, 48 * size_t(s.G), hipMemcpyDeviceToHost, st_) != hipSuccess)
      return fail(ctx, CM_E_HIP, "serving: download failed");
  }
  if (s.ng) {
    if (hipMemcpyAsync(d + s.d_qg, s.pinned + s.h_qg, 64 * size_t(s.ng), hipMemcpyHostToDevice, st_) != hipSuccess ||
        hipMemcpyAsync(d + s.d_cot, s.pinned + s.h_cot, 48 * size_t(s.Gg), hipMemcpyHostToDevice, st_) != hipSuccess)
      return fail(ctx, CM_E_HIP, "serving: upload failed");
    if ((st = plan_bind(s.pg.get(), d + s.d_pg, st_)) != CM_OK) return st;
    float* c = reinterpret_cast<float*>(d + s.d_cot);
    float* og_ = reinterpret_cast<float*>(d + s.d_outg);
    const int64_t Gg = s.Gg;
    // records and gradient from one forward sweep and one adjoint
    cm_groups ogg{og_, og_ + 3 * Gg, og_ + 6 * Gg, og_ + 7 * Gg, og_ + 10 * Gg, og_ + 11 * Gg};
    FwdArgs b = fwd_args(ctx, s.pg.get(), reinterpret_cast<const cm_query*>(d + s.d_qg), ogg, nullptr);
    b.cot = OutPtrs{c, c + 3 * Gg, c + 6 * Gg, c + 7 * Gg, c + 10 * Gg, c + 11 * Gg};
    b.grad = reinterpret_cast<float*>(d + s.d_grad);
    if (launch_backward(b, st_, true) != hipSuccess) return fail(ctx, CM_E_HIP, "serving: adjoint launch failed");
    if (hipMemcpyAsync(s.pinned + s.h_grad, d + s.d_grad, 48 * size_t(s.ng), hipMemcpyDeviceToHost, st_) != hipSuccess ||
        hipMemcpyAsync(s.pinned + s.h_outg, d + s.d_outg, 48 * size_t(s.Gg), hipMemcpyDeviceToHost, st_) != hipSuccess)
      return fail(ctx, CM_E_HIP, "serving: download failed");
  }
  if (hipEventRecord(s.done, st_) != hipSuccess) return fail(ctx, CM_E_HIP, "serving: event record failed");
  return CM_OK;
}

// Scatters a finished batch's results to the callers' buffers.
void scatter(Slot& s) {
  const float* out = reinterpret_cast<const float*>(s.pinned + s.h_out);
  const float* outg = reinterpret_cast<const float*>(s.pinned + s.h_outg);
  const float* grad = reinterpret_cast<const float*>(s.pinned + s.h_grad);
  int64_t g0 = 0, gg0 = 0, qg0 = 0;
  for (Req* r : s.reqs) {
    if (r->grad) {
      for (int64_t g = 0; g < r->G; ++g)
        for (int k = 0; k < 12; ++k) r->out_groups[12 * g + k] = outg[k * s.Gg + gg0 + g];
      gg0 += r->G;
      std::memcpy(r->out_grad, grad + 12 * qg0, 48 * r->q.size());
      qg0 += int64_t(r->q.size());
    } else {
      for (int64_t g = 0; g < r->G; ++g)
        for (int k = 0; k < 12; ++k) r->out_groups[12 * g + k] = out[k * s.G + g0 + g];
      g0 += r->G;
    }
  }
}

// Marks the slot's requests done with `st` and frees the slot.  Called with S->mu held.
void finish_slot(Serving* S, Slot& s, cm_status st, double t_done, bool record) {
  for (Req* r : s.reqs) {
    S->finished[r->id] = st;
    S->live.erase(r->id);
    S->n_completed++;
    if (record) {
      S->n_queries += int64_t(r->q.size());
      if (S->latencies.size() < (size_t(1) << 24)) S->latencies.push_back(t_done - r->t_submit);
    }
    delete r;
  }
  s.reqs.clear();
  S->inflight -= s.bytes;
  s.bytes = 0;
  s.busy = false;
  s.running = false;
  S->done_cv.notify_all();
}

// A slot's worker: plans and launches each batch the scheduler admits into
// the slot, then hands it back for completion polling.
void worker(Serving* S, Slot* s) {
  (void)hipSetDevice(S->ctx->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    s->wcv.wait(lk, [&] { return (s->busy && !s->running) || S->quit_workers; });
    if (!(s->busy && !s->running)) break;
    lk.unlock();
    const cm_status st = launch_batch(S, S->ctx, *s);
    lk.lock();
    if (st == CM_OK) s->running = true;
    else finish_slot(S, *s, st, 0.0, false);
    S->cv.notify_all();
  }
}

void scheduler(Serving* S) {
  cm_context* ctx = S->ctx;
  (void)hipSetDevice(ctx->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    bool progressed = false;
    // completions
    for (Slot& s : S->slots) {
      if (!s.running) continue;
      hipError_t q = hipEventQuery(s.done);
      if (q == hipErrorNotReady) continue;
      const cm_status st = q == hipSuccess ? CM_OK : CM_E_HIP;
      lk.unlock();
      if (st == CM_OK) scatter(s);
      const double t_done = now_s();
      lk.lock();
      finish_slot(S, s, st, t_done, true);
      progressed = true;
    }
    // admission into free slots: a batch may use the budget less what the
    // other slots hold (idle slots give their buffers back when it is short)
    for (Slot& s : S->slots) {
      if (s.busy || S->pending.empty()) continue;
      size_t bytes = 0;
      int64_t nq = 0;
      while (!S->pending.empty()) {
        Req* r = S->pending.front();
        // what the other slots hold or were admitted to hold (batches still
        // being planned by their workers included)
        auto room = [&]() {
          const size_t o = claims_except(S, &s);
          return ctx->budget > o ? ctx->budget - o : size_t(0);
        };
        bool fits = align_up(bytes + r->bytes, kDevGranule) <= room();
        if (!fits && s.reqs.empty()) {
          release_idle(S, &s);
          fits = align_up(r->bytes, kDevGranule) <= room();
        }
        if (!s.reqs.empty() && (!fits || nq + int64_t(r->q.size()) > kMaxBatchQueries)) break;
        if (s.reqs.empty() && !fits) break;  // wait for busy slots to finish
        S->pending.pop_front();
        s.reqs.push_back(r);
        bytes += r->bytes;
        nq += int64_t(r->q.size());
      }
      if (s.reqs.empty()) continue;
      s.busy = true;
      s.bytes = bytes;
      S->inflight += bytes;
      S->n_batches++;
      s.wcv.notify_one();  // the slot's worker plans and launches it
      progressed = true;
    }
    bool any_busy = false;
    for (Slot& s : S->slots) any_busy = any_busy || s.busy;
    if (S->stop && !any_busy) break;
    if (!progressed) {
      if (any_busy) S->cv.wait_for(lk, std::chrono::microseconds(50));
      else if (S->pending.empty()) S->cv.wait_for(lk, std::chrono::milliseconds(50));
    }
  }
}

Serving* start(cm_context* ctx) {
  auto* S = new Serving;
  S->ctx = ctx;
  for (Slot& s : S->slots) {
    if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) {
      delete S;
      return nullptr;
    }
  }
  for (Slot& s : S->slots) s.worker = std::thread(worker, S, &s);
  S->th = std::thread(scheduler, S);
  return S;
}

}  // namespace

void serving_stop(cm_context* ctx) {
  Serving* S = ctx->serving;
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    // requests not yet admitted fail
    for (Req* r : S->pending) {
      S->finished[r->id] = CM_E_BUSY;
      S->live.erase(r->id);
      delete r;
    }
    S->pending.clear();
  }
  S->cv.notify_all();
  S->th.join();  // (returns once no slot is busy: the workers are waiting)
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->quit_workers = true;
  }
  for (Slot& s : S->slots) {
    s.wcv.notify_all();
    if (s.worker.joinable()) s.worker.join();
  }
  for (Slot& s : S->slots) {
    if (s.dmem) (void)hipFree(s.dmem);
    if (s.pinned) (void)hipHostFree(s.pinned);
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.stream) (void)hipStreamDestroy(s.stream);
  }
  delete S;
  ctx->serving = nullptr;
}

}  // namespace cm

using namespace cm;

extern "C" {

cm_status cm_submit(cm_context* ctx, const cm_request* req, cm_ticket* ticket) {
  if (!ctx || !req || !ticket || !req->q || req->n <= 0 || !req->out_groups)
    return fail(ctx, CM_E_INVALID, "bad request");
  if (ctx->device < 0) return fail(ctx, CM_E_INVALID, "host-only context cannot serve");
  if (req->want_grad && (!req->cotangent || !req->out_grad)) return fail(ctx, CM_E_INVALID, "gradient request needs cotangent and out_grad");
  if (req->want_grad && ctx->prm.st_iters > 4) return fail(ctx, CM_E_INVALID, "the adjoint supports st_iters <= 4");
  for (int32_t i = 0; i < req->n; ++i) {
    const cm_query& q = req->q[i];
    const float na = q.qa[0] * q.qa[0] + q.qa[1] * q.qa[1] + q.qa[2] * q.qa[2] + q.qa[3] * q.qa[3];
    const float nb = q.qb[0] * q.qb[0] + q.qb[1] * q.qb[1] + q.qb[2] * q.qb[2] + q.qb[3] * q.qb[3];
    if (!(std::sqrt(na) >= 1e-12f) || !(std::sqrt(nb) >= 1e-12f)) return fail(ctx, CM_E_INVALID, "degenerate quaternion");
  }
  auto* r = new Req;
  r->q.assign(req->q, req->q + req->n);
  r->grad = req->want_grad != 0;
  r->out_groups = req->out_groups;
  r->out_grad = req->out_grad;
  r->t_submit = now_s();
  {
    PlanSizes z;
    cm_status st = plan_sizes(ctx, r->q.data(), req->n, &z);
    if (st != CM_OK) { delete r; return st; }
    r->G = z.G;
    r->bytes = request_bytes(ctx, z, r->grad);
  }
  if (r->bytes > ctx->budget) { delete r; return fail(ctx, CM_E_OOM, "request exceeds the memory budget on its own"); }
  if (r->grad) r->cot.assign(req->cotangent, req->cotangent + 12 * r->G);
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!ctx->serving) {
      ctx->serving = start(ctx);
      if (!ctx->serving) { delete r; ctx->err = "serving: stream creation failed"; return CM_E_HIP; }
    }
  }
  Serving* S = ctx->serving;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->pending.size() >= kQueueLimit) { delete r; return CM_E_BUSY; }
    r->id = S->next++;
    *ticket = r->id;
    S->live[r->id] = 1;
    S->pending.push_back(r);
    S->n_submitted++;
  }
  S->cv.notify_one();
  return CM_OK;
}

cm_status cm_poll(cm_context* ctx, cm_ticket t, int32_t* done, cm_status* result) {
  if (!ctx || !done) return CM_E_INVALID;
  Serving* S = ctx->serving;
  if (!S) return fail(ctx, CM_E_NOTFOUND, "unknown ticket");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->finished.find(t);
  if (it != S->finished.end()) {
    *done = 1;
    if (result) *result = it->second;
    S->finished.erase(it);
    return CM_OK;
  }
  if (S->live.count(t)) { *done = 0; return CM_OK; }
  return CM_E_NOTFOUND;
}

cm_status cm_wait(cm_context* ctx, cm_ticket t, int32_t timeout_ms, cm_status* result) {
  if (!ctx) return CM_E_INVALID;
  Serving* S = ctx->serving;
  if (!S) return fail(ctx, CM_E_NOTFOUND, "unknown ticket");
  std::unique_lock<std::mutex> lk(S->mu);
  const auto deadline = std::chrono::steady_clock::now() + std::chrono::milliseconds(timeout_ms);
  for (;;) {
    auto it = S->finished.find(t);
    if (it != S->finished.end()) {
      if (result) *result = it->second;
      S->finished.erase(it);
      return CM_OK;
    }
    if (!S->live.count(t)) return CM_E_NOTFOUND;
    if (S->done_cv.wait_until(lk, deadline) == std::cv_status::timeout) return CM_E_BUSY;
  }
}

cm_status cm_serve_latencies(cm_context* ctx, double* out, int64_t cap, int64_t* n) {
  if (!ctx || !n) return CM_E_INVALID;
  *n = 0;
  Serving* S = ctx->serving;
  if (!S) return CM_OK;
  std::lock_guard<std::mutex> lk(S->mu);
  const int64_t m = std::min<int64_t>(cap, int64_t(S->latencies.size()));
  if (out) std::copy(S->latencies.begin(), S->latencies.begin() + m, out);
  S->latencies.erase(S->latencies.begin(), S->latencies.begin() + m);
  *n = m;
  return CM_OK;
}

cm_status cm_serve_stats(cm_context* ctx, int64_t* st) {
  if (!ctx || !st) return CM_E_INVALID;
  Serving* S = ctx->serving;
  for (int i = 0; i < 7; ++i) st[i] = 0;
  if (!S) return CM_OK;
  std::lock_guard<std::mutex> lk(S->mu);
  int64_t busy = 0;
  for (Slot& s : S->slots) busy += s.busy ? int64_t(s.reqs.size()) : 0;
  st[0] = S->n_submitted;
  st[1] = S->n_completed;
  st[2] = S->n_batches;
  st[3] = int64_t(S->pending.size());
  st[4] = busy;
  st[5] = int64_t(S->peak_held);
  st[6] = S->n_queries;
  return CM_OK;
}

}  // extern "C"
