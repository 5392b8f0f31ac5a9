// Serving loop over resident H^2 operators (declarations in include/h2.h).
//
// Requests enter a FIFO queue.  Each carries an event recorded on the
// submitter's stream at submission, so the input it names is read only after
// the work that produced it.  A scheduler thread repeatedly (1) retires
// finished calls (event query), releasing their slot and budget, and (2)
// admits new calls: the oldest waiting request picks the operator and
// precision, every other waiting request for the same pair joins it while
// the fused vector count stays within max_fuse_nv, and the call starts when
// a slot is free and the budget -- a region of free HBM taken at creation --
// holds its fused input/output buffers.  Each call waits for its requests'
// events, gathers their input columns into one buffer (device copies), runs
// one multi-vector product on the slot's stream with the slot's workspace,
// and scatters the output columns back.  Calls are enqueued without the
// server lock held, so submitters never wait for a launch sequence; calls on
// different slots run concurrently.  Reduced precisions must be prepared on
// the operator before requests use them (nothing in the loop allocates or
// synchronizes the device).
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "h2_internal.h"

namespace h2 {
namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  int64_t id, op, nv;
  int prec;
  const double* X;
  double* Y;
  hipEvent_t ready = nullptr;  // recorded on the submitter's stream
  Clock::time_point t_submit, t_done;
  bool done = false;
};

// What a call needs of each of its requests, copied out of the queue so the
// call can be enqueued without the server lock.
struct Part {
  const double* X;
  double* Y;
  int64_t nv;
  hipEvent_t ready;
};

struct Call {
  std::vector<int64_t> reqs;  // request ids, in column order
  std::vector<Part> parts;    // the same requests' pointers and events
  int64_t op = 0, nv = 0;
  int prec = H2_PREC_FP64;
  int64_t buf_off = 0, buf_len = 0;  // doubles in the budget pool
};

struct Slot {
  Workspace ws;
  hipStream_t stream = nullptr;
  hipEvent_t done_ev = nullptr;
  bool busy = false;
  Call call;
};

// First-fit allocator over one device region (units: doubles).
struct Pool {
  double* base = nullptr;
  int64_t size = 0;
  std::map<int64_t, int64_t> used;  // offset -> length
  bool alloc(int64_t len, int64_t* off) {
    int64_t pos = 0;
    for (const auto& kv : used) {
      if (kv.first - pos >= len) break;
      pos = kv.first + kv.second;
    }
    if (pos + len > size) return false;
    used[pos] = len;
    *off = pos;
    return true;
  }
  void release(int64_t off) { used.erase(off); }
};

}  // namespace
}  // namespace h2

struct h2_server_s {
  std::vector<h2_op_s*> ops;
  int device = 0;
  int64_t max_fuse = 64;
  std::vector<h2::Slot> slots;
  h2::Pool pool;
  std::mutex mu;
  std::condition_variable cv_done;
  std::deque<int64_t> waiting;
  std::map<int64_t, h2::Request> reqs;
  std::vector<hipEvent_t> free_events;  // request events for reuse
  int64_t next_id = 1;
  bool stop = false;
  std::string thread_error;
  h2_server_stats_t st{};
  std::thread worker;
};

namespace h2 {
namespace {

int fail_s(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? H2_ENOMEM : H2_EHIP;
}

// Enqueue one fused call on slot `sl` (server lock not held: it reads only
// the call, the slot and the operator).  Returns an error message or "".
std::string start_call(h2_server_s* S, Slot& sl, const Call& c) {
  h2_op_s* h = S->ops[c.op];
  const int64_t n = h->n;
  double* Xb = S->pool.base + c.buf_off;
  double* Yb = Xb + n * c.nv;
  int64_t col = 0;
  for (const Part& p : c.parts) {
    hipError_t e = hipStreamWaitEvent(sl.stream, p.ready, 0);
    if (e == hipSuccess)
      e = hipMemcpyAsync(Xb + n * col, p.X, sizeof(double) * n * p.nv, hipMemcpyDeviceToDevice, sl.stream);
    if (e != hipSuccess) return std::string("gather: ") + hipGetErrorString(e);
    col += p.nv;
  }
  if (gemv_ws(h, sl.ws, false, 1.0, Xb, n, c.nv, 0.0, Yb, n, c.prec, sl.stream) != H2_OK)
    return std::string("product: ") + h2_last_error();
  col = 0;
  for (const Part& p : c.parts) {
    const hipError_t e =
        hipMemcpyAsync(p.Y, Yb + n * col, sizeof(double) * n * p.nv, hipMemcpyDeviceToDevice, sl.stream);
    if (e != hipSuccess) return std::string("scatter: ") + hipGetErrorString(e);
    col += p.nv;
  }
  const hipError_t e = hipEventRecord(sl.done_ev, sl.stream);
  return e == hipSuccess ? std::string() : std::string("hipEventRecord: ") + hipGetErrorString(e);
}

// Algorithmic work of one product of `h` with nv vectors at a precision:
// the low-rank data at that precision's width, the dense blocks and every
// vector in FP64 (x^ and y^ written and read once each).
void call_work(const h2_op_s* h, int64_t nv, int prec, double* bytes, double* flops) {
  const h2_stats_t& st = h->stats;
  const double lowrank =
      (double)(st.entries_U + st.entries_V + st.entries_E + st.entries_F + st.entries_S);
  const double dense = (double)st.entries_D;
  const double w = prec == H2_PREC_FP32 ? 4.0 : prec == H2_PREC_BF16 ? 2.0 : 8.0;
  *bytes = w * lowrank + 8.0 * dense + 8.0 * (double)nv * (2.0 * st.n + 4.0 * st.tree_rows);
  *flops = 2.0 * (double)nv * (lowrank + dense) + (double)nv * st.n;
}

void scheduler(h2_server_s* S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    bool progressed = false;
    // (1) retire finished calls
    int64_t running = 0;
    for (Slot& sl : S->slots) {
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.done_ev);
      if (q == hipErrorNotReady) { ++running; continue; }
      if (q != hipSuccess && S->thread_error.empty()) S->thread_error = hipGetErrorString(q);
      const auto now = Clock::now();
      for (int64_t id : sl.call.reqs) {
        Request& r = S->reqs.at(id);
        r.done = true;
        r.t_done = now;
        if (r.ready) S->free_events.push_back(r.ready);
        r.ready = nullptr;
        ++S->st.completed;
      }
      S->pool.release(sl.call.buf_off);
      sl.busy = false;
      progressed = true;
      S->cv_done.notify_all();
    }
    // (2) admit new calls while a slot is free and the budget has room
    while (!S->waiting.empty()) {
      Slot* free_slot = nullptr;
      for (Slot& sl : S->slots)
        if (!sl.busy) { free_slot = &sl; break; }
      if (!free_slot) break;
      const Request& head = S->reqs.at(S->waiting.front());
      Call c;
      c.op = head.op;
      c.prec = head.prec;
      std::deque<int64_t> rest;
      for (int64_t id : S->waiting) {
        const Request& r = S->reqs.at(id);
        if (r.op == head.op && r.prec == head.prec && c.nv + r.nv <= S->max_fuse) {
          c.reqs.push_back(id);
          c.parts.push_back(Part{r.X, r.Y, r.nv, r.ready});
          c.nv += r.nv;
        } else {
          rest.push_back(id);
        }
      }
      const int64_t n = S->ops[c.op]->n;
      c.buf_len = 2 * n * c.nv;
      if (!S->pool.alloc(c.buf_len, &c.buf_off)) break;  // wait for memory to free up
      S->waiting.swap(rest);
      free_slot->call = std::move(c);
      free_slot->busy = true;
      ++S->st.calls;
      S->st.vectors += free_slot->call.nv;
      double cb = 0.0, cf = 0.0;
      call_work(S->ops[free_slot->call.op], free_slot->call.nv, free_slot->call.prec, &cb, &cf);
      S->st.alg_bytes += cb;
      S->st.alg_flops += cf;
      ++running;
      progressed = true;
      // enqueue without the lock: submitters and waiters proceed meanwhile
      lk.unlock();
      const std::string err = start_call(S, *free_slot, free_slot->call);
      lk.lock();
      if (!err.empty() && S->thread_error.empty()) S->thread_error = err;
    }
    if (running > S->st.max_inflight_calls) S->st.max_inflight_calls = running;
    if (S->stop && S->waiting.empty() && running == 0) break;
    if (!progressed) {
      // poll finished calls every 20 us; wake at once on new submissions
      S->cv_done.wait_for(lk, std::chrono::microseconds(20));
    }
  }
}

}  // namespace
}  // namespace h2

using namespace h2;

extern "C" {

int h2_server_create(const h2_handle* ops, int64_t nops, int64_t slots, int64_t budget_bytes,
                     int64_t max_fuse_nv, h2_server* out) {
  if (!out || !ops || nops < 1 || slots < 1 || max_fuse_nv < 1 ||
      max_fuse_nv > kPassVectorsMfma) {
    set_error("h2_server_create: bad arguments");
    return H2_EINVAL;
  }
  *out = nullptr;
  h2_server_s* S = new (std::nothrow) h2_server_s();
  if (!S) { set_error("out of host memory"); return H2_ENOMEM; }
  int64_t nmax = 0, Hmax = 0;
  for (int64_t i = 0; i < nops; ++i) {
    if (!ops[i]) { delete S; set_error("null operator"); return H2_EINVAL; }
    S->ops.push_back(ops[i]);
    nmax = std::max(nmax, ops[i]->n);
    Hmax = std::max(Hmax, ops[i]->H);
  }
  S->device = ops[0]->device;
  for (int64_t i = 1; i < nops; ++i)
    if (ops[i]->device != S->device) { delete S; set_error("operators on different devices"); return H2_EINVAL; }
  S->max_fuse = max_fuse_nv;
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(S->device);
  int rc = H2_OK;
  hipError_t e = hipSuccess;
  S->slots.resize(slots);
  for (Slot& sl : S->slots) {
    if ((rc = ws_create(&sl.ws, nmax, Hmax, kPassVectorsMfma)) != H2_OK) break;
    if ((e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&sl.done_ev, hipEventDisableTiming)) != hipSuccess) {
      rc = fail_s(e, "server slot");
      break;
    }
  }
  size_t free_b = 0, total_b = 0;
  if (rc == H2_OK && (e = hipMemGetInfo(&free_b, &total_b)) != hipSuccess) rc = fail_s(e, "hipMemGetInfo");
  if (rc == H2_OK) {
    // the budget is taken out of the HBM that is free now (after the slots'
    // workspaces): a quarter of it by default, and never more than 90%
    const int64_t cap = (int64_t)(0.9 * (double)free_b);
    if (budget_bytes <= 0) budget_bytes = (int64_t)free_b / 4;
    if (budget_bytes > cap) {
      set_error("h2_server_create: budget of " + std::to_string(budget_bytes) + " bytes exceeds 90% of the " +
                std::to_string(free_b) + " bytes of free HBM");
      rc = H2_ENOMEM;
    }
  }
  if (rc == H2_OK) {
    S->pool.size = budget_bytes / (int64_t)sizeof(double);
    if ((e = hipMalloc(reinterpret_cast<void**>(&S->pool.base), sizeof(double) * S->pool.size)) != hipSuccess)
      rc = fail_s(e, "hipMalloc(server budget)");
  }
  if (rc == H2_OK && 2 * nmax * 1 > S->pool.size) {
    set_error("h2_server_create: budget smaller than one single-vector call");
    rc = H2_EINVAL;
  }
  if (rc != H2_OK) {
    for (Slot& sl : S->slots) {
      ws_destroy(&sl.ws);
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
      if (sl.done_ev) (void)hipEventDestroy(sl.done_ev);
    }
    if (S->pool.base) (void)hipFree(S->pool.base);
    delete S;
    if (prev >= 0) (void)hipSetDevice(prev);
    return rc;
  }
  S->st.slots = slots;
  S->st.budget_bytes = budget_bytes;
  S->st.hbm_free_at_create = (int64_t)free_b;
  if (prev >= 0) (void)hipSetDevice(prev);
  S->worker = std::thread(scheduler, S);
  *out = S;
  return H2_OK;
}

int h2_server_submit(h2_server S, int64_t op, int prec, int64_t nv, const double* X, double* Y, void* stream,
                     int64_t* id) {
  if (!S || !id || op < 0 || op >= (int64_t)S->ops.size() || nv < 1 || nv > S->max_fuse || !X || !Y ||
      (prec != H2_PREC_FP64 && prec != H2_PREC_FP32 && prec != H2_PREC_BF16)) {
    set_error("h2_server_submit: bad arguments");
    return H2_EINVAL;
  }
  if (2 * S->ops[op]->n * nv > S->pool.size) {
    set_error("h2_server_submit: request larger than the budget");
    return H2_EINVAL;
  }
  if (!prepared(S->ops[op], prec)) {
    set_error("h2_server_submit: precision not prepared on this operator (call h2_prepare first)");
    return H2_EINVAL;
  }
  {
    std::lock_guard<std::mutex> g(S->mu);
    if (!S->thread_error.empty()) {
      set_error("server: " + S->thread_error);
      return H2_EHIP;
    }
    hipEvent_t ev = nullptr;
    if (!S->free_events.empty()) {
      ev = S->free_events.back();
      S->free_events.pop_back();
    } else {
      int prev = -1;
      (void)hipGetDevice(&prev);
      (void)hipSetDevice(S->device);
      const hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (prev >= 0) (void)hipSetDevice(prev);
      if (e != hipSuccess) return fail_s(e, "hipEventCreate(request)");
    }
    // the input is read after the work queued on the submitter's stream so far
    const hipError_t e = hipEventRecord(ev, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
      S->free_events.push_back(ev);
      return fail_s(e, "hipEventRecord(request)");
    }
    Request r;
    r.ready = ev;
    r.id = S->next_id++;
    r.op = op;
    r.nv = nv;
    r.prec = prec;
    r.X = X;
    r.Y = Y;
    r.t_submit = Clock::now();
    S->reqs[r.id] = r;
    S->waiting.push_back(r.id);
    ++S->st.submitted;
    *id = r.id;
  }
  S->cv_done.notify_all();
  return H2_OK;
}

int h2_server_wait(h2_server S, int64_t id, double* latency_ms) {
  if (!S) { set_error("null server"); return H2_EINVAL; }
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) { set_error("unknown request"); return H2_EINVAL; }
  S->cv_done.wait(lk, [&] { return it->second.done || !S->thread_error.empty(); });
  if (!it->second.done) {
    set_error("server: " + S->thread_error);
    return H2_EHIP;
  }
  if (latency_ms)
    *latency_ms = std::chrono::duration<double, std::milli>(it->second.t_done - it->second.t_submit).count();
  S->reqs.erase(it);
  return S->thread_error.empty() ? H2_OK : H2_EHIP;
}

int h2_server_stats(h2_server S, h2_server_stats_t* st) {
  if (!S || !st) { set_error("null server or output"); return H2_EINVAL; }
  std::lock_guard<std::mutex> g(S->mu);
  *st = S->st;
  return H2_OK;
}

int h2_server_free(h2_server S) {
  if (!S) return H2_OK;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv_done.notify_all();
  if (S->worker.joinable()) S->worker.join();
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(S->device);
  (void)hipDeviceSynchronize();
  for (Slot& sl : S->slots) {
    ws_destroy(&sl.ws);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.done_ev) (void)hipEventDestroy(sl.done_ev);
  }
  for (hipEvent_t ev : S->free_events) (void)hipEventDestroy(ev);
  for (auto& kv : S->reqs)
    if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
  if (S->pool.base) (void)hipFree(S->pool.base);
  if (prev >= 0) (void)hipSetDevice(prev);
  delete S;
  return H2_OK;
}

}  // extern "C"
