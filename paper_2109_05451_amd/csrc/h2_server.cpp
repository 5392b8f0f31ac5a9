// Serving loop over resident H^2 operators (declarations in include/h2.h).
//
// Requests enter a FIFO queue.  A scheduler thread repeatedly (1) retires
// finished calls (event query), releasing their slot and budget, and (2)
// admits new calls: the oldest waiting request picks the operator and
// precision, every other waiting request for the same pair joins it while
// the fused vector count stays within max_fuse_nv, and the call starts when
// a slot is free and the budget holds its fused input/output buffers.  Each
// call gathers its requests' input columns into one buffer (device copies),
// runs one multi-vector product on the slot's stream with the slot's
// workspace, and scatters the output columns back.  Calls on different slots
// run concurrently.
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
  Clock::time_point t_submit, t_done;
  bool done = false;
};

struct Call {
  std::vector<int64_t> reqs;  // request ids, in column order
  int64_t op = 0, nv = 0;
  int64_t buf_off = 0, buf_len = 0;  // doubles in the budget pool
  hipEvent_t done_ev = nullptr;
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

// Start one fused call on slot `sl` (lock held).
hipError_t start_call(h2_server_s* S, Slot& sl, Call& c) {
  h2_op_s* h = S->ops[c.op];
  const int64_t n = h->n;
  double* Xb = S->pool.base + c.buf_off;
  double* Yb = Xb + n * c.nv;
  int64_t col = 0;
  const Request& first = S->reqs.at(c.reqs.front());
  for (int64_t id : c.reqs) {
    const Request& r = S->reqs.at(id);
    hipError_t e = hipMemcpyAsync(Xb + n * col, r.X, sizeof(double) * n * r.nv, hipMemcpyDeviceToDevice, sl.stream);
    if (e != hipSuccess) return e;
    col += r.nv;
  }
  const int rc = gemv_ws(h, sl.ws, false, 1.0, Xb, n, c.nv, 0.0, Yb, n, first.prec, sl.stream);
  if (rc != H2_OK) return hipErrorLaunchFailure;
  col = 0;
  for (int64_t id : c.reqs) {
    const Request& r = S->reqs.at(id);
    hipError_t e = hipMemcpyAsync(r.Y, Yb + n * col, sizeof(double) * n * r.nv, hipMemcpyDeviceToDevice, sl.stream);
    if (e != hipSuccess) return e;
    col += r.nv;
  }
  return hipEventRecord(sl.done_ev, sl.stream);
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
      std::deque<int64_t> rest;
      for (int64_t id : S->waiting) {
        const Request& r = S->reqs.at(id);
        if (r.op == head.op && r.prec == head.prec && c.nv + r.nv <= S->max_fuse) {
          c.reqs.push_back(id);
          c.nv += r.nv;
        } else {
          rest.push_back(id);
        }
      }
      const int64_t n = S->ops[c.op]->n;
      c.buf_len = 2 * n * c.nv;
      if (!S->pool.alloc(c.buf_len, &c.buf_off)) break;  // wait for memory to free up
      S->waiting.swap(rest);
      free_slot->call = c;
      free_slot->busy = true;
      const hipError_t e = start_call(S, *free_slot, free_slot->call);
      if (e != hipSuccess && S->thread_error.empty()) S->thread_error = hipGetErrorString(e);
      ++S->st.calls;
      S->st.vectors += c.nv;
      ++running;
      progressed = true;
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
  if (!out || !ops || nops < 1 || slots < 1 || budget_bytes <= 0 || max_fuse_nv < 1 ||
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
  if (prev >= 0) (void)hipSetDevice(prev);
  S->worker = std::thread(scheduler, S);
  *out = S;
  return H2_OK;
}

int h2_server_submit(h2_server S, int64_t op, int prec, int64_t nv, const double* X, double* Y, int64_t* id) {
  if (!S || !id || op < 0 || op >= (int64_t)S->ops.size() || nv < 1 || nv > S->max_fuse || !X || !Y ||
      (prec != H2_PREC_FP64 && prec != H2_PREC_FP32 && prec != H2_PREC_BF16)) {
    set_error("h2_server_submit: bad arguments");
    return H2_EINVAL;
  }
  if (2 * S->ops[op]->n * nv > S->pool.size) {
    set_error("h2_server_submit: request larger than the budget");
    return H2_EINVAL;
  }
  {
    std::lock_guard<std::mutex> g(S->mu);
    if (!S->thread_error.empty()) {
      set_error("server: " + S->thread_error);
      return H2_EHIP;
    }
    Request r;
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
  if (S->pool.base) (void)hipFree(S->pool.base);
  if (prev >= 0) (void)hipSetDevice(prev);
  delete S;
  return H2_OK;
}

}  // extern "C"
