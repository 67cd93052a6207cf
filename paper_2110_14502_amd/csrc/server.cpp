// Serving loop: continuous batching of amplitude requests.
//
// A worker thread owns the device work.  Requests wait in arrival order;
// the worker admits, oldest first, those whose plan is resident or built, as
// in-flight slots and device memory free up (plans stay resident between
// requests and are evicted least-recently used), merges waiting requests
// that share a plan into one batched contraction (the bitstrings become the
// batch dimension of every step), launches each call directly (no graph
// capture on the request's path) on one of several HIP streams so that calls
// overlap on the device, and completes a request when its call's event
// fires, without synchronising the shared streams.  Plans of new circuits are
// searched on host threads of their own, so that a request whose plan is
// being searched does not hold up the requests behind it; they are bound on
// a stream of their own.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <future>
#include <list>
#include <map>
#include <thread>
#include <unordered_map>

#include "executor.h"

namespace rqc {

namespace {

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

struct Req {
  uint64_t ticket = 0;
  int n_qubits = 0;
  std::vector<rqc_gate> gates;
  std::vector<int32_t> open;
  std::vector<uint8_t> bits;
  int prec = RQC_F32;
  int max_log2 = 0;
  uint64_t plan_key = 0;
  uint64_t seed = 0;
  uint64_t key = 0;  // effective plan key
  double t_submit = 0;
};

// First-fit allocator over the caller's device pool.
class Pool {
 public:
  void init(char* base, uint64_t bytes) {
    base_ = base;
    size_ = bytes;
  }
  char* alloc(uint64_t sz) {
    sz = (sz + 255) & ~uint64_t(255);
    uint64_t at = 0;
    auto it = used_.begin();
    for (; it != used_.end(); ++it) {
      if (it->first >= at + sz) break;
      at = std::max(at, it->first + it->second);
    }
    if (at + sz > size_) return nullptr;
    used_.insert(it, {at, sz});
    in_use_ += sz;
    peak_ = std::max(peak_, in_use_);
    return base_ + at;
  }
  void free(char* p) {
    const uint64_t at = (uint64_t)(p - base_);
    for (auto it = used_.begin(); it != used_.end(); ++it)
      if (it->first == at) {
        in_use_ -= it->second;
        used_.erase(it);
        return;
      }
  }
  uint64_t peak() const { return peak_; }

 private:
  char* base_ = nullptr;
  uint64_t size_ = 0, in_use_ = 0, peak_ = 0;
  std::list<std::pair<uint64_t, uint64_t>> used_;
};

struct PlanEntry {
  rqc_plan* plan = nullptr;
  char* res = nullptr;
  int uses = 0;  // in-flight calls
  double last = 0;
};

struct Call {
  std::vector<Req> reqs;
  PlanEntry* pe = nullptr;
  char* ws = nullptr;
  double* out = nullptr;
  int stream = 0;
  hipEvent_t ev = nullptr;
  PendingRun run;
  double t_start = 0;
};

// A plan searched on a host thread.
struct Built {
  rqc_plan* plan = nullptr;
  rqc_status st = RQC_OK;
};

Built build_plan(Req r) {
  Built b;
  rqc_circuit* c = nullptr;
  rqc_network* n = nullptr;
  b.st = rqc_circuit_create(r.n_qubits, r.gates.data(), r.gates.size(), &c);
  if (b.st == RQC_OK) b.st = rqc_network_create(c, r.open.data(), (int32_t)r.open.size(), &n);
  if (b.st == RQC_OK) {
    rqc_plan_opts o;
    rqc_plan_opts_default(&o);
    o.max_log2_elems = r.max_log2 > 0 ? r.max_log2 : 26;
    // The first request of a circuit waits for this search: a short one.
    o.path_trials = 32;
    o.reconf_rounds = 1;
    o.seed = r.seed;
    b.st = rqc_plan_create(n, &o, &b.plan);
  }
  rqc_network_destroy(n);
  rqc_circuit_destroy(c);
  return b;
}

uint64_t fnv(const void* p, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  return h;
}

}  // namespace
}  // namespace rqc

struct rqc_server {
  rqc_server_opts opts;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::deque<rqc::Req> queue;
  std::vector<rqc_result> finished;
  std::unordered_map<uint64_t, std::vector<double>> held;  // ticket -> amplitudes
  std::list<rqc::Call> calls;
  std::unordered_map<uint64_t, rqc::PlanEntry> plans;
  rqc::Pool pool;
  std::vector<hipStream_t> streams;
  hipStream_t bind_stream = nullptr;
  std::unordered_map<uint64_t, std::future<rqc::Built>> building;  // worker thread only
  uint64_t next_ticket = 1;
  uint64_t outstanding = 0;
  bool stop = false;
  int next_stream = 0;
  rqc_server_stats stats;
  std::thread worker;
  void loop();
  bool admit_one();
  void complete(rqc::Call& c, rqc_status st);
  void fail(const rqc::Req& r, rqc_status st);
};

void rqc_server::fail(const rqc::Req& r, rqc_status st) {
  rqc_result res;
  std::memset(&res, 0, sizeof res);
  res.ticket = r.ticket;
  res.status = st;
  res.n_open = (int32_t)r.open.size();
  res.t_submit = r.t_submit;
  res.t_start = res.t_done = rqc::now_s(t0);
  std::lock_guard<std::mutex> g(mu);
  finished.push_back(res);
  stats.rejected++;
  outstanding--;
  done_cv.notify_all();
}

// Admit the oldest waiting request whose plan is resident or built (plus the
// waiting requests sharing that plan); start the search of plans not seen
// yet.  Returns false when nothing could be admitted now.
bool rqc_server::admit_one() {
  std::vector<rqc::Req> batch;
  uint64_t key = 0;
  int prec = 0;
  {
    std::lock_guard<std::mutex> g(mu);
    if (queue.empty()) return false;
    if ((int)calls.size() >= opts.max_inflight) return false;
    bool found = false;
    for (const rqc::Req& r : queue) {
      if (plans.count(r.key)) {
        found = true;
      } else {
        auto b = building.find(r.key);
        if (b == building.end()) {
          building.emplace(r.key, std::async(std::launch::async, rqc::build_plan, r));
        } else if (b->second.wait_for(std::chrono::seconds(0)) == std::future_status::ready) {
          found = true;
        }
      }
      if (found) {
        key = r.key;
        prec = r.prec;
        break;
      }
    }
    if (!found) return false;
    for (auto it = queue.begin(); it != queue.end() && (int)batch.size() < opts.max_batch;) {
      if (it->key == key && it->prec == prec) {
        batch.push_back(std::move(*it));
        it = queue.erase(it);
      } else {
        ++it;
      }
    }
  }
  const rqc::Req& r0 = batch.front();
  auto requeue = [&]() {
    std::lock_guard<std::mutex> g(mu);
    for (auto it = batch.rbegin(); it != batch.rend(); ++it) queue.push_front(std::move(*it));
  };
  // Plan: resident, or searched and now bound on the bind stream.
  rqc::PlanEntry* pe = nullptr;
  auto pit = plans.find(key);
  if (pit != plans.end()) {
    pe = &pit->second;
    stats.plans_reused++;
  } else {
    auto bit = building.find(key);
    rqc::Built b = bit->second.get();
    building.erase(bit);
    if (b.st != RQC_OK) {
      rqc_plan_destroy(b.plan);
      for (auto& r : batch) fail(r, b.st);
      return true;
    }
    rqc_plan* p = b.plan;
    size_t rb = 0;
    rqc_plan_resident_bytes(p, &rb);
    char* res = pool.alloc(rb);
    // Evict idle plans (least recently used first) until the plan fits.
    while (!res) {
      auto victim = plans.end();
      for (auto it = plans.begin(); it != plans.end(); ++it)
        if (it->second.uses == 0 && (victim == plans.end() || it->second.last < victim->second.last))
          victim = it;
      if (victim == plans.end()) break;
      pool.free(victim->second.res);
      rqc_plan_destroy(victim->second.plan);
      plans.erase(victim);
      res = pool.alloc(rb);
    }
    if (!res) {
      if (calls.empty()) {
        rqc_plan_destroy(p);
        for (auto& r : batch) fail(r, RQC_EHBM);
        return true;
      }
      // Keep the searched plan for when memory frees up.
      std::promise<rqc::Built> keep;
      keep.set_value(b);
      building.emplace(key, keep.get_future());
      requeue();
      return false;
    }
    if (rqc_plan_bind_memory(p, res, rb, bind_stream) != RQC_OK) {
      pool.free(res);
      rqc_plan_destroy(p);
      for (auto& r : batch) fail(r, RQC_EDEVICE);
      return true;
    }
    pe = &plans[key];
    pe->plan = p;
    pe->res = res;
    stats.plans_built++;
  }
  // Workspace + output for this call.
  const uint64_t nb = batch.size();
  size_t min_ws = 0, pref_ws = 0;
  if (rqc_contract_workspace(pe->plan, 0, nb, r0.prec, &min_ws, &pref_ws) != RQC_OK) {
    for (auto& r : batch) fail(r, RQC_EINVAL);
    return true;
  }
  const uint64_t out_bytes = 16ull * nb << r0.open.size();
  char* out = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = pref_ws;
  // Output and workspace; idle resident plans other than this one are
  // evicted (least recently used first) before giving up.
  while (true) {
    out = pool.alloc(out_bytes);
    ws_bytes = pref_ws;
    ws = out ? pool.alloc(ws_bytes) : nullptr;
    if (out && !ws) {
      ws_bytes = min_ws;
      ws = pool.alloc(ws_bytes);
    }
    if (out && ws) break;
    if (out) pool.free(out);
    out = nullptr;
    auto victim = plans.end();
    for (auto it = plans.begin(); it != plans.end(); ++it)
      if (&it->second != pe && it->second.uses == 0 &&
          (victim == plans.end() || it->second.last < victim->second.last))
        victim = it;
    if (victim == plans.end()) break;
    pool.free(victim->second.res);
    rqc_plan_destroy(victim->second.plan);
    plans.erase(victim);
  }
  if (!out || !ws) {
    if (out) pool.free(out);
    if (calls.empty() && pe->uses == 0) {
      for (auto& r : batch) fail(r, RQC_EHBM);
      return true;
    }
    requeue();
    return false;
  }
  std::vector<uint8_t> bits;
  for (auto& r : batch) bits.insert(bits.end(), r.bits.begin(), r.bits.end());
  rqc::Call call;
  call.pe = pe;
  call.ws = ws;
  call.out = reinterpret_cast<double*>(out);
  call.stream = next_stream;
  next_stream = (next_stream + 1) % (int)streams.size();
  call.t_start = rqc::now_s(t0);
  hipStream_t s = streams[call.stream];
  try {
    rqc::contract(pe->plan, nullptr, 0, bits.data(), nb, r0.prec, ws, ws_bytes, call.out, nullptr, s,
                  call.run, /*direct=*/true);
    rqc::hip_check(hipEventCreateWithFlags(&call.ev, hipEventDisableTiming), "event");
    rqc::hip_check(hipEventRecord(call.ev, s), "event record");
  } catch (const rqc::Error& e) {
    pool.free(ws);
    pool.free(out);
    for (auto& r : batch) fail(r, e.code);
    return true;
  }
  pe->uses++;
  pe->last = call.t_start;
  call.reqs = std::move(batch);
  {
    std::lock_guard<std::mutex> g(mu);
    calls.push_back(std::move(call));
    stats.max_inflight_seen = std::max<uint64_t>(stats.max_inflight_seen, calls.size());
  }
  return true;
}

void rqc_server::complete(rqc::Call& c, rqc_status st) {
  rqc_run_report rep;
  std::memset(&rep, 0, sizeof rep);
  hipStream_t s = streams[c.stream];
  if (st == RQC_OK) {
    try {
      rqc::report(c.pe->plan, c.run, s, &rep, /*sync=*/false);
    } catch (const rqc::Error& e) {
      st = e.code;
    }
  }
  const size_t ne = size_t(1) << c.reqs.front().open.size();
  std::vector<double> host(2 * ne * c.reqs.size(), 0.0);
  if (st == RQC_OK && hipMemcpy(host.data(), c.out, 8 * host.size(), hipMemcpyDeviceToHost) != hipSuccess)
    st = RQC_EDEVICE;
  const double t_done = rqc::now_s(t0);
  (void)hipEventDestroy(c.ev);
  pool.free(c.ws);
  pool.free(reinterpret_cast<char*>(c.out));
  c.pe->uses--;
  std::lock_guard<std::mutex> g(mu);
  for (size_t i = 0; i < c.reqs.size(); ++i) {
    rqc_result res;
    std::memset(&res, 0, sizeof res);
    res.ticket = c.reqs[i].ticket;
    res.status = st;
    res.n_open = (int32_t)c.reqs[i].open.size();
    auto& h = held[res.ticket];
    h.assign(host.begin() + 2 * ne * i, host.begin() + 2 * ne * (i + 1));
    res.amplitudes = h.data();
    res.t_submit = c.reqs[i].t_submit;
    res.t_start = c.t_start;
    res.t_done = t_done;
    res.fp32_reruns = rep.fp32_reruns;
    finished.push_back(res);
    stats.completed++;
    outstanding--;
  }
  done_cv.notify_all();
}

void rqc_server::loop() {
  (void)hipSetDevice(opts.device);
  while (true) {
    bool progressed = false;
    // Completions first: they free slots and memory.
    std::vector<std::list<rqc::Call>::iterator> ready;
    {
      std::lock_guard<std::mutex> g(mu);
      for (auto it = calls.begin(); it != calls.end(); ++it) {
        const hipError_t q = hipEventQuery(it->ev);
        if (q == hipSuccess || q != hipErrorNotReady) ready.push_back(it);
      }
    }
    for (auto it : ready) {
      const hipError_t q = hipEventQuery(it->ev);
      complete(*it, q == hipSuccess ? RQC_OK : RQC_EDEVICE);
      std::lock_guard<std::mutex> g(mu);
      calls.erase(it);
      progressed = true;
    }
    while (admit_one()) progressed = true;
    std::unique_lock<std::mutex> lk(mu);
    if (stop && queue.empty() && calls.empty()) break;
    if (!progressed) {
      // Idle: wait for a request; with calls in flight or plans being
      // searched, poll their events and futures.
      if (calls.empty() && building.empty()) cv.wait(lk, [&] { return stop || !queue.empty(); });
      else cv.wait_for(lk, std::chrono::microseconds(200));
    }
  }
}

extern "C" {

rqc_status rqc_server_create(const rqc_server_opts* o, rqc_server** out) {
  if (!o || !out || !o->device_pool || o->hbm_budget_bytes == 0) {
    rqc::set_error("server needs a device pool and its size");
    return RQC_EINVAL;
  }
  if ((reinterpret_cast<uintptr_t>(o->device_pool) & 255) != 0) {
    rqc::set_error("device pool not 256-byte aligned");
    return RQC_EINVAL;
  }
  auto* s = new (std::nothrow) rqc_server;
  if (!s) return RQC_ENOMEM;
  s->opts = *o;
  if (s->opts.max_inflight <= 0) s->opts.max_inflight = 8;
  if (s->opts.n_streams <= 0) s->opts.n_streams = 4;
  if (s->opts.max_batch <= 0) s->opts.max_batch = 64;
  std::memset(&s->stats, 0, sizeof s->stats);
  s->t0 = std::chrono::steady_clock::now();
  s->pool.init(static_cast<char*>(o->device_pool), o->hbm_budget_bytes);
  if (const hipError_t e = hipSetDevice(o->device); e != hipSuccess) {
    delete s;
    rqc::set_error(std::string("hipSetDevice failed: ") + hipGetErrorName(e));
    return RQC_EDEVICE;
  }
  for (int i = 0; i <= s->opts.n_streams; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (auto x : s->streams) (void)hipStreamDestroy(x);
      if (s->bind_stream) (void)hipStreamDestroy(s->bind_stream);
      delete s;
      rqc::set_error("stream creation failed");
      return RQC_EDEVICE;
    }
    if (i == s->opts.n_streams) s->bind_stream = st;
    else s->streams.push_back(st);
  }
  s->worker = std::thread([s] { s->loop(); });
  *out = s;
  return RQC_OK;
}

rqc_status rqc_server_submit(rqc_server* s, const rqc_request* r, uint64_t* ticket) {
  if (!s || !r || !ticket) return RQC_EINVAL;
  if (r->n_qubits <= 0 || r->n_open < 0 || r->n_open > r->n_qubits || r->n_open > 20 ||
      (r->n_gates && !r->gates) || (r->n_open && !r->open_qubits) ||
      (r->n_qubits > r->n_open && !r->closed_bits) ||
      (r->prec != RQC_F32 && r->prec != RQC_F16 && r->prec != RQC_BF16)) {
    rqc::set_error("invalid request");
    return RQC_EINVAL;
  }
  rqc::Req q;
  q.n_qubits = r->n_qubits;
  q.gates.assign(r->gates, r->gates + r->n_gates);
  q.open.assign(r->open_qubits, r->open_qubits + r->n_open);
  q.bits.assign(r->closed_bits, r->closed_bits + (r->n_qubits - r->n_open));
  q.prec = r->prec;
  q.max_log2 = r->max_log2_elems;
  q.plan_key = r->plan_key;
  q.seed = r->seed;
  if (r->plan_key) {
    q.key = rqc::fnv(&r->plan_key, 8, 0x12345);
  } else {
    uint64_t h = rqc::fnv(&q.n_qubits, sizeof q.n_qubits);
    h = rqc::fnv(q.gates.data(), q.gates.size() * sizeof(rqc_gate), h);
    h = rqc::fnv(q.open.data(), q.open.size() * 4, h);
    h = rqc::fnv(&q.max_log2, 4, h);
    q.key = h;
  }
  std::lock_guard<std::mutex> g(s->mu);
  q.ticket = s->next_ticket++;
  q.t_submit = rqc::now_s(s->t0);
  *ticket = q.ticket;
  s->queue.push_back(std::move(q));
  s->stats.submitted++;
  s->outstanding++;
  s->cv.notify_all();
  return RQC_OK;
}

rqc_status rqc_server_poll(rqc_server* s, rqc_result* out, size_t cap, size_t* n) {
  if (!s || !n || (cap && !out)) return RQC_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  const size_t k = std::min(cap, s->finished.size());
  for (size_t i = 0; i < k; ++i) out[i] = s->finished[i];
  s->finished.erase(s->finished.begin(), s->finished.begin() + k);
  *n = k;
  return RQC_OK;
}

rqc_status rqc_server_release(rqc_server* s, uint64_t ticket) {
  if (!s) return RQC_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  s->held.erase(ticket);
  return RQC_OK;
}

rqc_status rqc_server_drain(rqc_server* s) {
  if (!s) return RQC_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->done_cv.wait(lk, [&] { return s->outstanding == 0; });
  return RQC_OK;
}

rqc_status rqc_server_get_stats(rqc_server* s, rqc_server_stats* out) {
  if (!s || !out) return RQC_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  *out = s->stats;
  out->peak_bytes = s->pool.peak();
  return RQC_OK;
}

void rqc_server_destroy(rqc_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  for (auto& kv : s->building) {
    rqc::Built b = kv.second.get();
    rqc_plan_destroy(b.plan);
  }
  for (auto& kv : s->plans) rqc_plan_destroy(kv.second.plan);
  for (auto x : s->streams) (void)hipStreamDestroy(x);
  if (s->bind_stream) (void)hipStreamDestroy(s->bind_stream);
  delete s;
}

}  // extern "C"
