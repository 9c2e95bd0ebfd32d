// Request queue with continuous batching.
//
// Callers submit factorization requests (bcgs_problem: device X, Q, R and
// info) from any thread; submit never blocks on the device.  One scheduler
// thread per queue owns a fixed set of device streams ("slots", at most
// max_inflight) and admits a waiting request as soon as a slot is free and
// the request's HBM footprint (X + Q + R + its workspace) fits in what the
// running requests leave of the budget.  Which request: the oldest
// (arrival order), or the one with the least estimated work net of its
// waiting time (shortest first with aging: the estimate, in seconds, is
// the streamed bytes over 3 TB/s plus 25 us per synchronization point, and
// every second spent waiting takes one second off it, so a large request
// waits at most about its own estimate for smaller ones).  An
// admitted request runs its whole schedule on its slot's stream, exactly as
// bcgs_qr_ex would (same kernels, same tuned choices, same bits), so
// requests that arrive while others run overlap with them on the device.
// Completion is detected by an event per slot; the device info record is
// copied to pinned host memory behind the schedule, and the request's
// times (host steady clock, seconds since the queue was created) are kept
// until the caller collects them with poll or wait.
//
// Optionally a request whose Cholesky factorization breaks down is run
// once more, at the head of the queue, with a more stable variant (e.g.
// BCGSI+P-1S -> BCGSI+P-2S, whose Table 1 assumption is u kappa <= 1
// instead of u kappa^2 <= 1), into the same outputs.
//
// A request may leave Q and R to the queue (both pointers NULL): they are
// then carved at admission out of the queue's output arena (one device
// allocation made when the queue is created; first-fit over 256-byte
// units with coalescing, all on the host), so a long backlog holds no
// output memory and admission also waits for arena space.  The caller gets
// them with the result and returns them with bcgs_queue_free_output, which
// is ordered on the caller's stream: the range is reused only after an
// event recorded there has completed.
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "common.h"

namespace bcgs {
namespace {

constexpr int kMaxSlots = 16;
constexpr size_t kMaxWaiting = 1 << 20;

struct Request {
  bcgs_problem prob;
  Plan plan;
  size_t footprint = 0;
  bool own = false;        // Q and R allocated by the queue at admission
  bool placed = false;     // queue-allocated outputs already assigned
  bool done = false;
  bool first = false;      // a retry: admitted before everything else
  double est = 0;          // estimated device seconds (admission order)
  hipEvent_t ready = nullptr;  // recorded on the submitter's stream
  bcgs_request_stats stats{};
};

// First-fit allocator over [0, bytes) in 256-byte units (host side).
class Arena {
 public:
  void init(size_t bytes) {
    bytes_ = bytes & ~size_t(255);
    free_.clear();
    if (bytes_) free_[0] = bytes_;
  }
  // offset of a block of `n` bytes, or SIZE_MAX when none is free
  size_t alloc(size_t n) {
    n = (n + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t off = it->first, left = it->second - n;
      free_.erase(it);
      if (left) free_[off + n] = left;
      used_[off] = n;
      return off;
    }
    return SIZE_MAX;
  }
  bool owns(size_t off) const { return used_.count(off) != 0; }
  void release(size_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return;
    size_t n = u->second;
    used_.erase(u);
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + n == next->first) {
      n += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += n;
        return;
      }
    }
    free_[off] = n;
  }

 private:
  size_t bytes_ = 0;
  std::map<size_t, size_t> free_;   // offset -> size
  std::map<size_t, size_t> used_;
};

struct PendingFree {
  size_t off;
  hipEvent_t ev;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bcgs_info* host_info = nullptr;    // pinned
  uint64_t ticket = 0;               // 0 = idle
};

}  // namespace
}  // namespace bcgs

struct bcgs_queue {
  bcgs::Slot slots[bcgs::kMaxSlots];
  char* out_base = nullptr;          // output arena (device)
  size_t out_bytes = 0;
  bcgs::Arena out;                   // guarded by mu
  std::vector<bcgs::PendingFree> pending_free;
  std::vector<hipEvent_t> spare_events;
  int nslots = 0;
  int device = 0;
  size_t budget = 0;
  size_t in_use = 0;
  int retry = 0;                     // rerun breakdowns with retry_variant
  int retry_variant = 0;
  int admission = BCGS_ADMIT_ARRIVAL;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work;   // scheduler: new request / stop
  std::condition_variable cv_done;   // waiters: a request finished
  std::deque<uint64_t> waiting;
  std::map<uint64_t, bcgs::Request> reqs;
  uint64_t next_ticket = 1;
  int running = 0;
  bool stop = false;
  bcgs_status fault = BCGS_OK;       // sticky runtime failure
  std::thread thread;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() -
                                         t0).count();
  }
  void run();
  std::deque<uint64_t>::iterator pick();
};

namespace bcgs {
namespace {

size_t q_bytes(const bcgs_problem& p) {
  return (size_t)p.m * p.n * (p.precision == BCGS_FP32_BULK ? 4 : 8);
}
size_t r_bytes(const bcgs_problem& p) { return (size_t)p.n * p.n * 8; }

size_t footprint_of(const bcgs_problem& p, const Plan& plan) {
  const size_t esz = p.precision == BCGS_FP32_BULK ? 4 : 8;
  const size_t x = (size_t)((p.n - 1) * p.ldx + p.m) * esz;
  const size_t q = (size_t)((p.n - 1) * p.ldq + p.m) * esz;
  const size_t r = (size_t)((p.n - 1) * p.ldr + p.n) * 8;
  return x + q + r + plan.bytes;
}

// Estimated device time of a request in seconds, for the shortest-first
// admission order only: P-1S-like schedules read Q_{1:k} once per block
// column (n q / 2 columns over the run), BCGSI+ twice; plus X, U and Q
// once each, and a fixed cost per synchronization point.
double estimate_seconds(const bcgs_problem& p) {
  const double esz = p.precision == BCGS_FP32_BULK ? 4.0 : 8.0;
  const double q = (double)(p.n / p.s);
  const double reads = p.variant == BCGS_I_PLUS ? 2.0 : 1.0;
  const double cols = reads * (double)p.n * q / 2.0 + 3.0 * (double)p.n;
  const double syncs =
      (double)bcgs_sync_count(p.m, p.n, p.s, (bcgs_variant)p.variant);
  return (double)p.m * esz * cols / 3e12 + 25e-6 * syncs;
}

// Start request `t` on slot `sl` (scheduler thread, lock not held).
bcgs_status start_on(Slot& sl, Request& rq) {
  if (sl.ws_bytes < rq.plan.bytes) {
    if (sl.ws) {
      if (hipStreamSynchronize(sl.stream) != hipSuccess) return BCGS_ERR_HIP;
      (void)hipFree(sl.ws);
      sl.ws = nullptr;
      sl.ws_bytes = 0;
    }
    if (hipMalloc(&sl.ws, rq.plan.bytes) != hipSuccess) {
      sl.ws = nullptr;
      return BCGS_ERR_NOMEM;
    }
    sl.ws_bytes = rq.plan.bytes;
  }
  const bcgs_problem& p = rq.prob;
  // the submitter's work on X (and on its own outputs) comes first
  if (rq.ready && hipStreamWaitEvent(sl.stream, rq.ready, 0) != hipSuccess)
    return BCGS_ERR_HIP;
  bcgs_status st = run_problem(rq.plan, p.X, p.ldx, p.Q, p.ldq, p.R, p.ldr,
                               sl.ws, p.d_info, sl.stream);
  if (st != BCGS_OK) return st;
  if (hipMemcpyAsync(sl.host_info, p.d_info, sizeof(bcgs_info),
                     hipMemcpyDeviceToHost, sl.stream) != hipSuccess ||
      hipEventRecord(sl.done, sl.stream) != hipSuccess)
    return BCGS_ERR_HIP;
  return BCGS_OK;
}

}  // namespace
}  // namespace bcgs

using namespace bcgs;

void bcgs_queue::run() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lock(mu);
  for (;;) {
    // 1. retire finished slots
    for (int i = 0; i < nslots; ++i) {
      Slot& sl = slots[i];
      if (!sl.ticket) continue;
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipErrorNotReady) continue;
      const uint64_t tk = sl.ticket;
      Request& rq = reqs[tk];
      rq.stats.t_done = now();
      if (q == hipSuccess) {
        rq.stats.info = *sl.host_info;
        rq.stats.status = rq.stats.info.status == BCGS_OK
                              ? BCGS_OK : BCGS_ERR_BREAKDOWN;
      } else {
        rq.stats.status = BCGS_ERR_HIP;
        fault = BCGS_ERR_HIP;
      }
      in_use -= rq.footprint;
      --running;
      sl.ticket = 0;
      Plan again;
      if (rq.stats.status == BCGS_ERR_BREAKDOWN && retry &&
          rq.stats.attempts == 1 && rq.prob.variant != retry_variant &&
          check_problem(rq.prob.X, rq.prob.ldx, rq.prob.m, rq.prob.n,
                        rq.prob.s, retry_variant, rq.prob.precision,
                        rq.prob.Q, rq.prob.ldq, rq.prob.R, rq.prob.ldr,
                        rq.prob.d_info, &again) == BCGS_OK) {
        // run it once more, first in line, with the stable variant
        rq.prob.variant = retry_variant;
        rq.plan = again;
        rq.footprint = footprint_of(rq.prob, again);
        rq.stats.variant = retry_variant;
        rq.stats.status = BCGS_PENDING;
        rq.first = true;
        waiting.push_front(tk);
        continue;
      }
      rq.done = true;
      cv_done.notify_all();
    }
    // 2. admit in arrival order while a slot and the memory are free
    for (size_t i = 0; i < pending_free.size();) {
      if (hipEventQuery(pending_free[i].ev) == hipErrorNotReady) {
        ++i;
        continue;
      }
      out.release(pending_free[i].off);
      spare_events.push_back(pending_free[i].ev);
      pending_free[i] = pending_free.back();
      pending_free.pop_back();
    }
    bool blocked = false;
    while (!waiting.empty() && running < nslots) {
      const auto at = pick();
      Request& rq = reqs[*at];
      if (running > 0 && in_use + rq.footprint > budget) break;
      if (rq.own && !rq.placed) {
        // outputs from the arena: Q then R, both or neither
        const size_t oq = out.alloc(q_bytes(rq.prob));
        const size_t orr = oq == SIZE_MAX ? SIZE_MAX : out.alloc(r_bytes(rq.prob));
        if (orr == SIZE_MAX) {
          if (oq != SIZE_MAX) out.release(oq);
          if (!stop || running > 0 || !pending_free.empty()) {
            blocked = true;              // wait for arena space
            break;
          }
          // being destroyed and nothing can free space: give up on it
          waiting.erase(at);
          rq.stats.status = BCGS_ERR_NOMEM;
          rq.stats.t_start = rq.stats.t_done = now();
          rq.done = true;
          cv_done.notify_all();
          continue;
        }
        rq.prob.Q = out_base + oq;
        rq.prob.R = reinterpret_cast<double*>(out_base + orr);
        rq.stats.Q = rq.prob.Q;
        rq.stats.R = rq.prob.R;
        rq.placed = true;
      }
      ++rq.stats.attempts;
      int k = 0;
      while (slots[k].ticket) ++k;
      const uint64_t t = *at;
      waiting.erase(at);
      in_use += rq.footprint;
      ++running;
      slots[k].ticket = t;
      rq.stats.t_start = now();
      lock.unlock();
      const bcgs_status st = start_on(slots[k], rq);
      lock.lock();
      if (st != BCGS_OK) {   // nothing of it is in flight: finish it here
        (void)hipStreamSynchronize(slots[k].stream);
        if (rq.own && rq.stats.Q) {
          out.release(static_cast<char*>(rq.stats.Q) - out_base);
          out.release(reinterpret_cast<char*>(rq.stats.R) - out_base);
          rq.stats.Q = nullptr;
          rq.stats.R = nullptr;
        }
        rq.stats.status = st;
        rq.stats.t_done = now();
        rq.done = true;
        in_use -= rq.footprint;
        --running;
        slots[k].ticket = 0;
        cv_done.notify_all();
      }
    }
    if (stop && waiting.empty() && running == 0) break;
    // 3. wait for work: poll the device while requests run or returned
    //    outputs are pending, else sleep until a submission, a returned
    //    output or the stop request
    if (running > 0 || !pending_free.empty()) {
      lock.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lock.lock();
    } else {
      const size_t nfree = pending_free.size();
      cv_work.wait(lock, [&] {
        return stop || pending_free.size() != nfree ||
               (!waiting.empty() && !blocked);
      });
    }
  }
}

// The waiting request to admit next (lock held, waiting not empty).
std::deque<uint64_t>::iterator bcgs_queue::pick() {
  if (admission == BCGS_ADMIT_ARRIVAL) return waiting.begin();
  const double t = now();
  auto best = waiting.begin();
  double key_best = 0;
  for (auto it = waiting.begin(); it != waiting.end(); ++it) {
    const Request& rq = reqs[*it];
    if (rq.first) return it;
    const double key = rq.est - (t - rq.stats.t_submit);
    if (it == waiting.begin() || key < key_best) {
      best = it;
      key_best = key;
    }
  }
  return best;
}

extern "C" {

bcgs_status bcgs_queue_create(const bcgs_queue_config* cfg,
                              bcgs_queue_t* out) {
  if (!cfg || !out) return BCGS_ERR_ARG;
  if (cfg->max_inflight < 1 || cfg->max_inflight > kMaxSlots ||
      cfg->hbm_budget_bytes == 0)
    return BCGS_ERR_ARG;
  if (cfg->retry_on_breakdown &&
      (cfg->retry_variant < BCGS_I_PLUS || cfg->retry_variant > BCGS_I_PLUS_1S))
    return BCGS_ERR_ARG;
  if (cfg->admission != BCGS_ADMIT_ARRIVAL &&
      cfg->admission != BCGS_ADMIT_SHORTEST)
    return BCGS_ERR_ARG;
  const size_t arena = cfg->output_arena_bytes & ~size_t(255);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess) return BCGS_ERR_HIP;
  if (cfg->device < 0 || cfg->device >= ndev) return BCGS_ERR_ARG;
  bcgs_queue* q = new bcgs_queue();
  q->device = cfg->device;
  q->budget = cfg->hbm_budget_bytes;
  q->nslots = cfg->max_inflight;
  q->retry = cfg->retry_on_breakdown != 0;
  q->retry_variant = cfg->retry_variant;
  q->admission = cfg->admission;
  q->t0 = std::chrono::steady_clock::now();
  int prev = 0;
  (void)hipGetDevice(&prev);
  bcgs_status st = BCGS_OK;
  if (hipSetDevice(cfg->device) != hipSuccess) st = BCGS_ERR_HIP;
  if (st == BCGS_OK && arena) {
    if (hipMalloc((void**)&q->out_base, arena) != hipSuccess) {
      q->out_base = nullptr;
      st = BCGS_ERR_NOMEM;
    } else {
      q->out_bytes = arena;
      q->out.init(arena);
    }
  }
  for (int i = 0; st == BCGS_OK && i < q->nslots; ++i) {
    Slot& sl = q->slots[i];
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) !=
            hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) !=
            hipSuccess ||
        hipHostMalloc((void**)&sl.host_info, sizeof(bcgs_info),
                      hipHostMallocDefault) != hipSuccess)
      st = BCGS_ERR_HIP;
  }
  (void)hipSetDevice(prev);
  if (st != BCGS_OK) {
    for (int i = 0; i < q->nslots; ++i) {
      Slot& sl = q->slots[i];
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
      if (sl.done) (void)hipEventDestroy(sl.done);
      if (sl.host_info) (void)hipHostFree(sl.host_info);
    }
    if (q->out_base) (void)hipFree(q->out_base);
    delete q;
    return st;
  }
  q->thread = std::thread([q] { q->run(); });
  *out = q;
  return BCGS_OK;
}

bcgs_status bcgs_queue_submit(bcgs_queue_t q, const bcgs_problem* p,
                              hipStream_t stream, uint64_t* ticket) {
  if (!q || !p || !ticket) return BCGS_ERR_ARG;
  Request rq;
  rq.prob = *p;
  rq.own = !p->Q && !p->R;
  if (rq.own && !q->out_bytes) return BCGS_ERR_ARG;   // no output arena
  if (rq.own && q_bytes(*p) + r_bytes(*p) + 512 > q->out_bytes)
    return BCGS_ERR_NOMEM;
  if (rq.own) {
    // outputs come later: check against a placeholder layout (ld = m, n)
    // that cannot overlap X
    rq.prob.ldq = p->m;
    rq.prob.ldr = p->n;
  }
  const bcgs_problem& c = rq.prob;
  const char* x_end = static_cast<const char*>(c.X) +
                      (size_t)((c.n - 1) * c.ldx + c.m) * 8;
  const bcgs_status st = check_problem(
      c.X, c.ldx, c.m, c.n, c.s, c.variant, c.precision,
      rq.own ? x_end : c.Q, c.ldq,
      rq.own ? reinterpret_cast<const double*>(x_end + (size_t)c.m * c.n * 8)
             : c.R,
      c.ldr, c.d_info, &rq.plan);
  if (st != BCGS_OK) return st;
  rq.footprint = footprint_of(c, rq.plan);
  rq.est = estimate_seconds(c);
  {
    std::lock_guard<std::mutex> lock(q->mu);
    if (q->stop) return BCGS_ERR_ARG;
    if (q->fault != BCGS_OK) return q->fault;
    if (q->waiting.size() >= kMaxWaiting) return BCGS_ERR_QUEUE_FULL;
    if (!q->spare_events.empty()) {
      rq.ready = q->spare_events.back();
      q->spare_events.pop_back();
    }
  }
  if (!rq.ready && hipEventCreateWithFlags(&rq.ready, hipEventDisableTiming) !=
                       hipSuccess)
    return BCGS_ERR_HIP;
  if (hipEventRecord(rq.ready, stream) != hipSuccess) {
    (void)hipEventDestroy(rq.ready);
    return BCGS_ERR_HIP;
  }
  std::lock_guard<std::mutex> lock(q->mu);
  rq.stats.status = BCGS_PENDING;
  rq.stats.variant = p->variant;
  rq.stats.attempts = 0;
  rq.stats.t_submit = q->now();
  const uint64_t t = q->next_ticket++;
  q->reqs.emplace(t, rq);
  q->waiting.push_back(t);
  *ticket = t;
  q->cv_work.notify_one();
  return BCGS_OK;
}

bcgs_status bcgs_queue_poll(bcgs_queue_t q, uint64_t ticket,
                            bcgs_request_stats* out) {
  if (!q || !out) return BCGS_ERR_ARG;
  std::lock_guard<std::mutex> lock(q->mu);
  auto it = q->reqs.find(ticket);
  if (it == q->reqs.end()) return BCGS_ERR_ARG;
  *out = it->second.stats;
  if (!it->second.done) {
    out->status = BCGS_PENDING;
    return BCGS_PENDING;
  }
  const bcgs_status st = it->second.stats.status;
  if (it->second.ready) q->spare_events.push_back(it->second.ready);
  q->reqs.erase(it);
  return st;
}

bcgs_status bcgs_queue_wait(bcgs_queue_t q, uint64_t ticket,
                            bcgs_request_stats* out) {
  if (!q || !out) return BCGS_ERR_ARG;
  std::unique_lock<std::mutex> lock(q->mu);
  auto it = q->reqs.find(ticket);
  if (it == q->reqs.end()) return BCGS_ERR_ARG;
  q->cv_done.wait(lock, [&] { return it->second.done; });
  *out = it->second.stats;
  const bcgs_status st = it->second.stats.status;
  if (it->second.ready) q->spare_events.push_back(it->second.ready);
  q->reqs.erase(it);
  return st;
}

bcgs_status bcgs_queue_free_output(bcgs_queue_t q, void* ptr,
                                   hipStream_t stream) {
  if (!q) return BCGS_ERR_ARG;
  if (!ptr) return BCGS_OK;
  char* c = static_cast<char*>(ptr);
  if (!q->out_base || c < q->out_base || c >= q->out_base + q->out_bytes)
    return BCGS_ERR_ARG;
  const size_t off = (size_t)(c - q->out_base);
  hipEvent_t ev = nullptr;
  {
    std::lock_guard<std::mutex> lock(q->mu);
    if (!q->out.owns(off)) return BCGS_ERR_ARG;
    if (!q->spare_events.empty()) {
      ev = q->spare_events.back();
      q->spare_events.pop_back();
    }
  }
  if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
    return BCGS_ERR_HIP;
  if (hipEventRecord(ev, stream) != hipSuccess) {
    (void)hipEventDestroy(ev);
    return BCGS_ERR_HIP;
  }
  std::lock_guard<std::mutex> lock(q->mu);
  q->pending_free.push_back({off, ev});
  q->cv_work.notify_one();
  return BCGS_OK;
}

bcgs_status bcgs_queue_destroy(bcgs_queue_t q) {
  if (!q) return BCGS_ERR_ARG;
  {
    std::lock_guard<std::mutex> lock(q->mu);
    q->stop = true;
    q->cv_work.notify_all();
  }
  if (q->thread.joinable()) q->thread.join();
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(q->device);
  for (int i = 0; i < q->nslots; ++i) {
    Slot& sl = q->slots[i];
    (void)hipStreamSynchronize(sl.stream);
    if (sl.ws) (void)hipFree(sl.ws);
    (void)hipStreamDestroy(sl.stream);
    (void)hipEventDestroy(sl.done);
    (void)hipHostFree(sl.host_info);
  }
  for (auto& pf : q->pending_free) {
    (void)hipEventSynchronize(pf.ev);
    (void)hipEventDestroy(pf.ev);
  }
  for (hipEvent_t ev : q->spare_events) (void)hipEventDestroy(ev);
  for (auto& kv : q->reqs)
    if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
  if (q->out_base) (void)hipFree(q->out_base);
  (void)hipSetDevice(prev);
  delete q;
  return BCGS_OK;
}

}  // extern "C"
