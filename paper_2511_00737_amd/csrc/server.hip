// Serving loop: device-resident tenants (encrypted models, Galois keys), requests admitted by
// their device-memory footprint, and continuous batching -- a scheduler thread turns the
// requests waiting at each moment into a batch on one of several streams, so requests that
// arrive while others run are admitted as soon as a stream and memory free up, and their
// work overlaps on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "batch.hpp"
#include "session.hpp"

using namespace ephdc;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over one device block; blocks are returned in any order and merged.
class Arena {
 public:
  void init(char* base, size_t bytes) {
    base_ = base;
    free_.clear();
    free_[0] = bytes;
    used_ = 0;
  }
  bool ready() const { return base_ != nullptr; }
  char* base() const { return base_; }
  // offset of a block of `bytes`, or SIZE_MAX when no free range is large enough
  size_t get(size_t bytes) {
    bytes = align_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > bytes) free_[off + bytes] = len - bytes;
        used_ += bytes;
        return off;
      }
    }
    return SIZE_MAX;
  }
  void put(size_t off, size_t bytes) {
    bytes = align_up(bytes);
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
  size_t used() const { return used_; }

 private:
  char* base_ = nullptr;
  std::map<size_t, size_t> free_;
  size_t used_ = 0;
};

struct Tenant {
  ephdc_session* s;
  const int8_t* d_base;
};

struct Req {
  uint64_t ticket;
  uint32_t tenant, Q;
  const uint8_t* d_x;
  uint32_t* d_out;
  size_t hv_bytes;
  hipEvent_t ready = nullptr;      // recorded on the caller's stream at submission
  uint32_t q_first = 0, n_ct = 0;  // where the request's queries sit in its output
  double t_submit = 0, t_admit = 0, t_done = 0;
  int state = 0;  // 0 waiting, 1 in flight, 2 done, < 0 failed (negated status)
};

// Submit-to-done latencies in a fixed histogram: bins of 1 % relative width from 1 us to
// about 1000 s; percentiles are read to within that 1 %.
class LatencyHist {
 public:
  static constexpr double kLo = 1e-6, kRatio = 1.01;
  static constexpr int kBins = 2100;
  void add(double s) {
    int i = s <= kLo ? 0 : (int)(std::log(s / kLo) / std::log(kRatio));
    bins_[std::min(std::max(i, 0), kBins - 1)] += 1;
    ++n_;
  }
  // seconds at fraction p of the recorded latencies (the geometric centre of its bin)
  double percentile(double p) const {
    if (!n_) return 0.0;
    const uint64_t want = std::min<uint64_t>(n_ - 1, (uint64_t)(p * (double)(n_ - 1) + 0.5));
    uint64_t run = 0;
    for (int i = 0; i < kBins; ++i) {
      run += bins_[i];
      if (run > want) return kLo * std::pow(kRatio, i + 0.5);
    }
    return kLo * std::pow(kRatio, kBins - 0.5);
  }

 private:
  uint64_t bins_[kBins] = {};
  uint64_t n_ = 0;
};

// Finished tickets (done, failed or rejected) kept for ephdc_server_query / _result until
// released; past this many, the oldest are forgotten.
constexpr size_t kKeepFinished = 1 << 16;

struct Inflight {
  ephdc_batch* batch = nullptr;
  int stream = -1;
  hipEvent_t done = nullptr;
  size_t off = 0, bytes = 0;
  std::vector<uint64_t> tickets;
};

}  // namespace

struct ephdc_server {
  // configuration
  size_t budget = 0;
  uint32_t nstreams = 2, max_batch = 64;
  bool pack = false;  // requests of one tenant share ciphertexts within a batch
  size_t pt_bytes = (size_t)256 << 20;
  // state (guarded by mu)
  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::vector<Tenant> tenants;
  std::map<uint64_t, Req> reqs;
  std::deque<uint64_t> waiting;
  uint64_t next_ticket = 1;
  bool stop = false;
  // device side (scheduler thread)
  int device = -1;
  void* mem = nullptr;
  Arena arena;
  std::vector<hipStream_t> streams;
  std::vector<bool> stream_busy;
  std::list<Inflight> inflight;
  std::thread worker;
  std::string worker_error;
  bool broken = false;  // the scheduler could not start: every request fails
  uint32_t planning = 0;  // batches taken from the queue and being planned outside the lock
  std::deque<uint64_t> finished;  // finished tickets, oldest first (may hold released ones)
  // statistics
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  uint64_t submitted = 0, completed = 0, rejected = 0, failed = 0, batches = 0, batched_requests = 0;
  size_t peak_bytes = 0;
  LatencyHist latencies;  // completed requests
};

namespace {

double now_s(const ephdc_server* sv) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - sv->t0).count();
}

// Device memory of one request outside the batch block: its query hypervectors.
size_t hv_bytes(const ephdc_session* s, uint32_t Q) { return (size_t)s->P.D * s->P.G(Q) * s->P.B(); }

// A request reaches a final state: its submission event is released, and the oldest
// finished tickets beyond kKeepFinished are forgotten (callers that never release them
// keep the server's memory bounded).
void finish(ephdc_server* sv, Req& r, int state) {
  r.state = state;
  r.t_done = now_s(sv);
  if (r.ready) {
    (void)hipEventDestroy(r.ready);
    r.ready = nullptr;
  }
  sv->finished.push_back(r.ticket);
  while (sv->finished.size() > kKeepFinished) {
    auto it = sv->reqs.find(sv->finished.front());
    if (it != sv->reqs.end() && (it->second.state == 2 || it->second.state < 0)) sv->reqs.erase(it);
    sv->finished.pop_front();
  }
}

// Completes every in-flight batch whose event has fired; returns whether any did.
bool reap(ephdc_server* sv, std::unique_lock<std::mutex>&) {
  bool any = false;
  for (auto it = sv->inflight.begin(); it != sv->inflight.end();) {
    const hipError_t q = hipEventQuery(it->done);
    if (q == hipErrorNotReady) {
      ++it;
      continue;
    }
    for (uint64_t tk : it->tickets) {
      Req& r = sv->reqs[tk];
      if (q == hipSuccess) {
        finish(sv, r, 2);
        sv->latencies.add(r.t_done - r.t_submit);
        ++sv->completed;
      } else {
        finish(sv, r, -EPHDC_ERR_HIP);
        ++sv->failed;
      }
    }
    batch_free(it->batch);
    (void)hipEventDestroy(it->done);
    sv->arena.put(it->off, it->bytes);
    sv->stream_busy[it->stream] = false;
    it = sv->inflight.erase(it);
    any = true;
  }
  if (any) sv->done_cv.notify_all();
  return any;
}

// Forms and launches one batch from the head of the waiting queue on stream `si`: requests
// are taken in arrival order while the batch's footprint fits the free device memory.  The
// selection and the memory reservation happen under the lock; planning, uploading the work
// lists and enqueueing the launches do not, so submissions and queries proceed meanwhile.
// Returns false when nothing could be admitted.
bool admit(ephdc_server* sv, int si, std::unique_lock<std::mutex>& lk) {
  std::vector<uint64_t> take;
  std::vector<ephdc_request> rq;
  std::vector<size_t> hvb;
  std::vector<hipEvent_t> ready;
  size_t hv_total = 0, need = 0;
  const size_t free_bytes = sv->budget - sv->arena.used();
  // footprint of a candidate list: with packing the batch holds the packed hypervectors
  // itself, else every request's hypervectors come on top of the batch block
  auto footprint = [&](const std::vector<ephdc_request>& l, size_t hv) {
    return batch_bytes(l.data(), (uint32_t)l.size(), sv->pt_bytes, 2, 128, sv->pack) + (sv->pack ? 0 : hv);
  };
  while (!sv->waiting.empty() && take.size() < sv->max_batch) {
    Req& r = sv->reqs[sv->waiting.front()];
    const Tenant& t = sv->tenants[r.tenant];
    ephdc_request e{};
    e.session = t.s;
    e.d_x = r.d_x;
    e.d_base = t.d_base;
    e.d_hv = reinterpret_cast<int8_t*>(0x1000);  // placeholder: placed after measuring
    e.Q = r.Q;
    e.d_score_ct = r.d_out;
    rq.push_back(e);
    const size_t hv = align_up(r.hv_bytes);
    const size_t total = footprint(rq, hv_total + hv);
    if (total > free_bytes) {
      rq.pop_back();
      if (take.empty() && footprint({e}, hv) > sv->budget) {
        // larger than the whole budget: can never be admitted
        ++sv->rejected;
        sv->waiting.pop_front();
        finish(sv, r, -EPHDC_ERR_OOM);
        sv->done_cv.notify_all();
        continue;
      }
      break;
    }
    hv_total += hv;
    need = total;
    take.push_back(r.ticket);
    hvb.push_back(r.hv_bytes);
    ready.push_back(r.ready);
    sv->waiting.pop_front();
  }
  if (take.empty()) return false;
  const size_t off = sv->arena.get(need);
  if (off == SIZE_MAX) {  // fragmented: put the requests back and wait for a completion
    for (auto it = take.rbegin(); it != take.rend(); ++it) sv->waiting.push_front(*it);
    return false;
  }
  const double t_admit = now_s(sv);
  for (uint64_t tk : take) {
    sv->reqs[tk].state = 1;
    sv->reqs[tk].t_admit = t_admit;
  }
  sv->stream_busy[si] = true;
  sv->peak_bytes = std::max(sv->peak_bytes, sv->arena.used());
  ++sv->planning;  // neither waiting nor in flight until published: waits must still see it
  const bool pack = sv->pack;
  const size_t pt_bytes = sv->pt_bytes;
  hipStream_t hs = sv->streams[si];
  char* base = sv->arena.base() + off;

  lk.unlock();  // ---- plan and launch without the lock
  size_t hv_off = 0;
  if (!pack) {
    for (size_t i = 0; i < take.size(); ++i) {
      rq[i].d_hv = reinterpret_cast<int8_t*>(base + hv_off);
      hv_off += align_up(hvb[i]);
    }
  }
  hipError_t e = hipSuccess;
  for (hipEvent_t ev : ready)  // the requests' inputs are written on the callers' streams
    if (e == hipSuccess && ev) e = hipStreamWaitEvent(hs, ev, 0);
  ephdc_batch* b = nullptr;
  ephdc_status st = e == hipSuccess ? batch_new(rq.data(), (uint32_t)rq.size(), pt_bytes, 2, 128, pack,
                                                base + hv_off, need - hv_off, hs, &b)
                                    : EPHDC_ERR_HIP;
  if (st == EPHDC_OK) e = batch_enqueue(b, hs);
  std::vector<std::pair<uint32_t, uint32_t>> where(take.size());
  if (st == EPHDC_OK) {
    for (size_t i = 0; i < take.size(); ++i) {
      if (pack) {
        uint32_t qoff = 0;
        batch_packing(b, (uint32_t)i, &qoff, &where[i].first, &where[i].second);
      } else {
        where[i] = {0u, rq[i].session->P.G(rq[i].Q)};
      }
    }
  }
  hipEvent_t ev = nullptr;
  if (st == EPHDC_OK && e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (st == EPHDC_OK && e == hipSuccess) e = hipEventRecord(ev, hs);
  const bool ok = st == EPHDC_OK && e == hipSuccess;
  if (!ok) {
    // the launch failed: release the memory once this stream is idle
    (void)hipStreamSynchronize(hs);
    if (b) batch_free(b);
    if (ev) (void)hipEventDestroy(ev);
  }
  lk.lock();  // ---- publish
  --sv->planning;
  if (!ok) {
    sv->arena.put(off, need);
    sv->stream_busy[si] = false;
    for (uint64_t tk : take) {
      finish(sv, sv->reqs[tk], st != EPHDC_OK ? -(int)st : -EPHDC_ERR_HIP);
      ++sv->failed;
    }
    sv->done_cv.notify_all();
    return true;
  }
  for (size_t i = 0; i < take.size(); ++i) {
    Req& r = sv->reqs[take[i]];
    r.q_first = where[i].first;
    r.n_ct = where[i].second;
  }
  Inflight f;
  f.batch = b;
  f.stream = si;
  f.done = ev;
  f.off = off;
  f.bytes = need;
  f.tickets = std::move(take);
  sv->inflight.push_back(std::move(f));
  ++sv->batches;
  sv->batched_requests += sv->inflight.back().tickets.size();
  return true;
}

void worker_main(ephdc_server* sv) {
  std::unique_lock<std::mutex> lk(sv->mu);
  if (hipSetDevice(sv->device) != hipSuccess) {
    // no scheduler: fail what waits now and (through `broken`) every later submission
    sv->worker_error = "hipSetDevice failed in the scheduler thread";
    sv->broken = true;
    while (!sv->waiting.empty()) {
      finish(sv, sv->reqs[sv->waiting.front()], -EPHDC_ERR_HIP);
      ++sv->failed;
      sv->waiting.pop_front();
    }
    sv->done_cv.notify_all();
    return;
  }
  while (true) {
    reap(sv, lk);
    if (sv->stop && sv->waiting.empty() && sv->inflight.empty()) break;
    bool progressed = false;
    for (int si = 0; si < (int)sv->streams.size() && !sv->waiting.empty(); ++si)
      if (!sv->stream_busy[si] && admit(sv, si, lk)) progressed = true;
    if (progressed) continue;
    // wait for a submission, or poll the in-flight batches
    if (sv->inflight.empty())
      sv->cv.wait(lk, [&] { return sv->stop || !sv->waiting.empty(); });
    else
      sv->cv.wait_for(lk, std::chrono::microseconds(100));
  }
}

// Allocates the device block and streams and starts the scheduler (on the first tenant).
ephdc_status start(ephdc_server* sv, int device) {
  sv->device = device;
  HIP_TRY(hipSetDevice(device), "set device");
  if (hipMalloc(&sv->mem, sv->budget) != hipSuccess) {
    sv->mem = nullptr;
    (void)hipGetLastError();
    return fail(EPHDC_ERR_OOM, "hipMalloc failed for the server's request memory");
  }
  sv->arena.init((char*)sv->mem, sv->budget);
  for (uint32_t i = 0; i < sv->nstreams; ++i) {
    hipStream_t s = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "stream");
    sv->streams.push_back(s);
    sv->stream_busy.push_back(false);
  }
  sv->worker = std::thread(worker_main, sv);
  return EPHDC_OK;
}

}  // namespace

extern "C" {

ephdc_status ephdc_server_create(size_t budget_bytes, uint32_t streams, uint32_t max_batch, ephdc_server** out) {
  if (!out) return fail(EPHDC_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (budget_bytes < ((size_t)64 << 20)) return fail(EPHDC_ERR_ARG, "budget must be at least 64 MiB");
  if (streams < 1 || streams > 8) return fail(EPHDC_ERR_ARG, "streams must be in [1, 8]");
  ephdc_server* sv = new ephdc_server();
  sv->budget = budget_bytes;
  sv->nstreams = streams;
  sv->max_batch = max_batch ? max_batch : 64;
  sv->pt_bytes = std::min<size_t>((size_t)256 << 20, budget_bytes / 8);
  *out = sv;
  return EPHDC_OK;
}

ephdc_status ephdc_server_set_packing(ephdc_server* sv, int enable) {
  if (!sv) return fail(EPHDC_ERR_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->submitted) return fail(EPHDC_ERR_ARG, "packing must be set before the first request");
  sv->pack = enable != 0;
  return EPHDC_OK;
}

ephdc_status ephdc_server_result(ephdc_server* sv, uint64_t ticket, uint32_t* q_first, uint32_t* n_ct) {
  if (!sv || !q_first || !n_ct) return fail(EPHDC_ERR_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return fail(EPHDC_ERR_ARG, "unknown ticket");
  if (it->second.state != 2) return fail(EPHDC_ERR_ARG, "request not done");
  *q_first = it->second.q_first;
  *n_ct = it->second.n_ct;
  return EPHDC_OK;
}

ephdc_status ephdc_server_add_tenant(ephdc_server* sv, ephdc_session* s, const int8_t* d_base, uint32_t* tenant) {
  if (!sv || !s || !tenant) return fail(EPHDC_ERR_ARG, "NULL argument");
  std::unique_lock<std::mutex> lk(sv->mu);
  if (sv->stop) return fail(EPHDC_ERR_ARG, "server is shutting down");
  if (!sv->tenants.empty() && s->device != sv->device)
    return fail(EPHDC_ERR_UNSUPPORTED, "every tenant of a server lives on one device");
  if (sv->tenants.empty()) {
    lk.unlock();
    ephdc_status st = start(sv, s->device);
    if (st != EPHDC_OK) return st;
    lk.lock();
  }
  *tenant = (uint32_t)sv->tenants.size();
  sv->tenants.push_back(Tenant{s, d_base});
  return EPHDC_OK;
}

ephdc_status ephdc_server_submit(ephdc_server* sv, uint32_t tenant, const uint8_t* d_x, uint32_t Q, uint32_t* d_score_ct,
                                 void* stream, uint64_t* ticket) {
  if (!sv || !d_x || !d_score_ct || !ticket) return fail(EPHDC_ERR_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->stop) return fail(EPHDC_ERR_ARG, "server is shutting down");
  if (sv->broken) return fail(EPHDC_ERR_HIP, sv->worker_error);
  if (tenant >= sv->tenants.size()) return fail(EPHDC_ERR_ARG, "unknown tenant");
  const Tenant& t = sv->tenants[tenant];
  if (!t.d_base) return fail(EPHDC_ERR_ARG, "tenant has no base hypervectors");
  const ParamSet& P = t.s->P;
  if (Q == 0 || Q > t.s->max_Q) return fail(EPHDC_ERR_ARG, "Q must be in [1, the tenant session's max_Q]");
  if (P.F % 16 != 0 || P.D % 64 != 0) return fail(EPHDC_ERR_UNSUPPORTED, "encoding needs F % 16 == 0 and D % 64 == 0");
  if ((uint64_t)P.F * P.D >= (1ull << 31) || (uint64_t)Q * P.F >= (1ull << 31))
    return fail(EPHDC_ERR_UNSUPPORTED, "encoding needs F * D and Q * F below 2^31");
  if ((uintptr_t)d_x & 15) return fail(EPHDC_ERR_ARG, "x must be 16-byte aligned");
  Req r;
  r.ticket = sv->next_ticket++;
  r.tenant = tenant;
  r.Q = Q;
  r.d_x = d_x;
  r.d_out = d_score_ct;
  r.hv_bytes = hv_bytes(t.s, Q);
  // the batch that takes this request waits for the work the caller queued so far on `stream`
  HIP_TRY(hipEventCreateWithFlags(&r.ready, hipEventDisableTiming), "submission event");
  if (hipError_t e = hipEventRecord(r.ready, (hipStream_t)stream); e != hipSuccess) {
    (void)hipEventDestroy(r.ready);
    return hip_fail(e, "submission event");
  }
  r.t_submit = now_s(sv);
  sv->reqs.emplace(r.ticket, r);
  sv->waiting.push_back(r.ticket);
  ++sv->submitted;
  *ticket = r.ticket;
  sv->cv.notify_all();
  return EPHDC_OK;
}

ephdc_status ephdc_server_query(ephdc_server* sv, uint64_t ticket, int32_t* state, double times[3]) {
  if (!sv || !state) return fail(EPHDC_ERR_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return fail(EPHDC_ERR_ARG, "unknown ticket");
  *state = it->second.state;
  if (times) {
    times[0] = it->second.t_submit;
    times[1] = it->second.t_admit;
    times[2] = it->second.t_done;
  }
  return EPHDC_OK;
}

ephdc_status ephdc_server_wait(ephdc_server* sv, uint64_t ticket, double timeout_s) {
  if (!sv) return fail(EPHDC_ERR_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto finished = [&] {
    if (ticket == 0) return sv->waiting.empty() && sv->inflight.empty() && sv->planning == 0;
    auto it = sv->reqs.find(ticket);
    return it == sv->reqs.end() || it->second.state >= 2 || it->second.state < 0;
  };
  if (ticket != 0 && sv->reqs.find(ticket) == sv->reqs.end()) return fail(EPHDC_ERR_ARG, "unknown ticket");
  const auto deadline = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
  while (!finished()) {
    if (timeout_s > 0 && std::chrono::steady_clock::now() >= deadline)
      return fail(EPHDC_ERR_TIMEOUT, "wait timed out");
    sv->done_cv.wait_for(lk, std::chrono::milliseconds(1));
  }
  if (ticket != 0) {
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return fail(EPHDC_ERR_ARG, "ticket released or forgotten");
    if (it->second.state < 0) return fail((ephdc_status)(-it->second.state), "request failed");
  }
  return EPHDC_OK;
}

ephdc_status ephdc_server_release(ephdc_server* sv, uint64_t ticket) {
  if (!sv) return fail(EPHDC_ERR_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return fail(EPHDC_ERR_ARG, "unknown ticket");
  if (it->second.state != 2 && it->second.state >= 0) return fail(EPHDC_ERR_ARG, "request not finished");
  sv->reqs.erase(it);
  return EPHDC_OK;
}

ephdc_status ephdc_server_stats(ephdc_server* sv, double out[14]) {
  if (!sv || !out) return fail(EPHDC_ERR_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto pct = [&](double p) { return sv->latencies.percentile(p) * 1e3; };
  out[0] = (double)sv->submitted;
  out[1] = (double)sv->completed;
  out[2] = (double)sv->rejected;
  out[3] = (double)sv->waiting.size();
  out[4] = (double)(sv->inflight.size() + sv->planning);
  out[5] = (double)sv->batches;
  out[6] = sv->batches ? (double)sv->batched_requests / (double)sv->batches : 0.0;
  out[7] = pct(0.50);
  out[8] = pct(0.99);
  out[9] = (double)sv->peak_bytes;
  out[10] = (double)sv->budget;
  out[11] = now_s(sv);
  out[12] = (double)sv->failed;
  out[13] = (double)sv->reqs.size();
  return EPHDC_OK;
}

ephdc_status ephdc_server_destroy(ephdc_server* sv) {
  if (!sv) return fail(EPHDC_ERR_ARG, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    sv->cv.notify_all();
  }
  if (sv->worker.joinable()) sv->worker.join();
  for (auto& kv : sv->reqs)
    if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
  for (hipStream_t s : sv->streams) (void)hipStreamDestroy(s);
  if (sv->mem) (void)hipFree(sv->mem);
  delete sv;
  return EPHDC_OK;
}

}  // extern "C"
