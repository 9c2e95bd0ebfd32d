// Many independent factorizations in one launch, and the autotuner that
// picks their launch choices.
//
// Batched launch.  Every problem keeps its own schedule (the passes,
// reductions and epilogues of its variant), so a problem's kernels and
// their order are exactly those of a lone bcgs_qr_ex call with the same
// tuned choices, and its results are bitwise the same.  The schedules are
// captured once into a HIP graph: the caller's stream forks into a fixed
// set of branch streams, each problem goes to the branch with the least
// modelled work so far (largest problems first), and the branches join
// back.  Replaying the instantiated graph is one launch from the host, and
// independent problems on different branches overlap on the device.  The
// executable graph is cached per stream and reused while the problem list
// (pointers, shapes, choices) is unchanged.
//
// Autotuner.  Choices are kept per problem class (floor(log2 m), n, s,
// variant, precision): the largest number of workgroups of a streaming pass
// (fewer, longer row ranges cut the partial-sum traffic of small problems)
// and the tile shape of the s <= 16 pass.  bcgs_autotune times every
// candidate on the caller's own problem with HIP events and keeps the
// fastest; bcgs_qr, bcgs_qr_ex, bcgs_qr_batched and the request queue all
// read the same table.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "common.h"

namespace bcgs {

// ------------------------------------------------------------- tuning ---
namespace {

typedef std::tuple<int, int64_t, int, int, int> TuneKey;

std::mutex g_tune_mu;
std::map<TuneKey, Tuning> g_tune;

int log2_floor(int64_t m) {
  int b = 0;
  while ((int64_t(1) << (b + 1)) <= m) ++b;
  return b;
}

TuneKey tune_key(int64_t m, int64_t n, int s, int variant, int precision) {
  return TuneKey(log2_floor(m), n, s, variant, precision);
}

}  // namespace

bool tuned_choice(int64_t m, int64_t n, int s, int variant, int precision,
                  Tuning* out) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune.find(tune_key(m, n, s, variant, precision));
  if (it == g_tune.end()) return false;
  *out = it->second;
  return true;
}

static void set_choice(int64_t m, int64_t n, int s, int variant,
                       int precision, const Tuning& t) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune[tune_key(m, n, s, variant, precision)] = t;
}

static bool erase_choice(int64_t m, int64_t n, int s, int variant,
                         int precision, Tuning* old) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune.find(tune_key(m, n, s, variant, precision));
  if (it == g_tune.end()) return false;
  *old = it->second;
  g_tune.erase(it);
  return true;
}

// Modelled bytes of one factorization (the per-variant pass count of the
// schedules in driver.hip: P-1S reads about q^2/2 + 4.5 q blocks, P-2S
// q^2 + 6 q, BCGSI+ 2 q^2 + 6 q).
static double model_cost(const bcgs_problem& p) {
  const double q = (double)(p.n / p.s);
  const double blk = (double)p.m * (double)p.s *
                     (p.precision == BCGS_FP32_BULK ? 4.0 : 8.0);
  switch (p.variant) {
    case BCGS_P_1S: return blk * (q * q / 2 + 4.5 * q);
    case BCGS_P_2S: return blk * (q * q + 6 * q);
    default: return blk * (2 * q * q + 6 * q);
  }
}

// --------------------------------------------------------- batch state ---
namespace {

constexpr int kBranches = 16;          // streams created per caller stream

// branches used by a batch: BCGS_BATCH_BRANCHES (1..16), default 8
int branches_used() {
  static const int n = [] {
    const char* e = getenv("BCGS_BATCH_BRANCHES");
    const int v = e ? atoi(e) : 8;
    return v < 1 ? 1 : (v > kBranches ? kBranches : v);
  }();
  return n;
}

struct BatchState {
  int device = -1;
  void* arena = nullptr;
  size_t arena_bytes = 0;
  hipStream_t cap = nullptr;     // the graph is captured on and launched
  hipEvent_t in_ev = nullptr;    // into this library stream, ordered after
  hipEvent_t out_ev = nullptr;   // and before the caller's stream by events
  hipStream_t branch[kBranches] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kBranches] = {};
  std::vector<char> key;
  hipGraphExec_t exec = nullptr;
};

std::mutex g_batch_mu;
std::map<hipStream_t, BatchState> g_batch;

void drop_graph(BatchState& b) {
  if (b.exec) (void)hipGraphExecDestroy(b.exec);
  b.exec = nullptr;
  b.key.clear();
}

bool ensure_streams(BatchState& b) {
  if (b.fork) return true;
  if (hipStreamCreateWithFlags(&b.cap, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&b.in_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&b.out_ev, hipEventDisableTiming) !=
          hipSuccess ||
      hipEventCreateWithFlags(&b.fork, hipEventDisableTiming) != hipSuccess)
    return false;
  for (int i = 0; i < kBranches; ++i) {
    if (hipStreamCreateWithFlags(&b.branch[i], hipStreamNonBlocking) !=
            hipSuccess ||
        hipEventCreateWithFlags(&b.join[i], hipEventDisableTiming) !=
            hipSuccess)
      return false;
  }
  return true;
}

// Enqueue every problem's schedule on the branch streams, forked from and
// joined back into `st` (captured when `st` is capturing).
bcgs_status enqueue_branches(BatchState& b, const std::vector<Plan>& plans,
                             const bcgs_problem* probs,
                             const std::vector<size_t>& offs,
                             const std::vector<int>& order,
                             const std::vector<int>& branch_of,
                             hipStream_t st) {
  int used = 0;
  for (int i : order) used = std::max(used, branch_of[i] + 1);
  if (hipEventRecord(b.fork, st) != hipSuccess) return BCGS_ERR_HIP;
  for (int k = 0; k < used; ++k)
    if (hipStreamWaitEvent(b.branch[k], b.fork, 0) != hipSuccess)
      return BCGS_ERR_HIP;
  bcgs_status res = BCGS_OK;
  for (int i : order) {
    const bcgs_problem& p = probs[i];
    const bcgs_status r = run_problem(
        plans[i], p.X, p.ldx, p.Q, p.ldq, p.R, p.ldr,
        static_cast<char*>(b.arena) + offs[i], p.d_info,
        b.branch[branch_of[i]]);
    if (r != BCGS_OK && res == BCGS_OK) res = r;
  }
  for (int k = 0; k < used; ++k) {
    if (hipEventRecord(b.join[k], b.branch[k]) != hipSuccess ||
        hipStreamWaitEvent(st, b.join[k], 0) != hipSuccess)
      return BCGS_ERR_HIP;
  }
  return res;
}

}  // namespace

}  // namespace bcgs

using namespace bcgs;

extern "C" {

bcgs_status bcgs_qr_batched(const bcgs_problem* probs, int32_t count,
                            hipStream_t stream) {
  if (count < 0 || (count > 0 && !probs)) return BCGS_ERR_ARG;
  if (count == 0) return BCGS_OK;
  // 1. check every problem before anything is enqueued
  std::vector<Plan> plans(count);
  std::vector<size_t> offs(count);
  size_t total = 0;
  for (int i = 0; i < count; ++i) {
    const bcgs_problem& p = probs[i];
    const bcgs_status st =
        check_problem(p.X, p.ldx, p.m, p.n, p.s, p.variant, p.precision, p.Q,
                      p.ldq, p.R, p.ldr, p.d_info, &plans[i]);
    if (st != BCGS_OK) return st;
    offs[i] = total;
    total += (plans[i].bytes + 255) & ~size_t(255);
  }
  // 2. largest problems first, each to the least loaded branch
  std::vector<int> order(count), branch_of(count, 0);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return model_cost(probs[a]) > model_cost(probs[b]);
  });
  {
    double load[kBranches] = {};
    const int nb = branches_used();
    for (int i : order) {
      int k = 0;
      for (int j = 1; j < nb; ++j)
        if (load[j] < load[k]) k = j;
      branch_of[i] = k;
      load[k] += model_cost(probs[i]);
    }
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return BCGS_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_batch_mu);
  BatchState& b = g_batch[stream];
  if (b.device != -1 && b.device != dev) return BCGS_ERR_ARG;
  b.device = dev;
  if (!ensure_streams(b)) return BCGS_ERR_HIP;
  // 3. workspace arena (one region per problem)
  if (b.arena_bytes < total) {
    if (b.arena) {
      if (hipStreamSynchronize(stream) != hipSuccess ||
          hipStreamSynchronize(b.cap) != hipSuccess)
        return BCGS_ERR_HIP;
      for (int k = 0; k < kBranches; ++k)
        if (hipStreamSynchronize(b.branch[k]) != hipSuccess)
          return BCGS_ERR_HIP;
      (void)hipFree(b.arena);
      b.arena = nullptr;
      b.arena_bytes = 0;
    }
    drop_graph(b);
    if (hipMalloc(&b.arena, total) != hipSuccess) {
      b.arena = nullptr;
      return BCGS_ERR_NOMEM;
    }
    b.arena_bytes = total;
  }
  // 4. reuse the executable graph while nothing that shapes it changed
  std::vector<char> key(sizeof(bcgs_problem) * count +
                        sizeof(Tuning) * count + sizeof(void*));
  {
    char* k = key.data();
    memcpy(k, probs, sizeof(bcgs_problem) * count);
    k += sizeof(bcgs_problem) * count;
    for (int i = 0; i < count; ++i, k += sizeof(Tuning))
      memcpy(k, &plans[i].tune, sizeof(Tuning));
    memcpy(k, &b.arena, sizeof(void*));
  }
  const char* mode = getenv("BCGS_BATCH_MODE");
  if (mode && strcmp(mode, "persistent") == 0) {
    // one persistent launch when every problem's steps have a body there
    bool used = false;
    const bcgs_status r =
        persist_run(plans, probs, offs, b.arena, key, stream, &used);
    if (used || r != BCGS_OK) return r;
    return BCGS_ERR_UNSUPPORTED;
  }
  if (mode && strcmp(mode, "streams") == 0) {
    // same schedule on the branch streams without a graph (comparison)
    return enqueue_branches(b, plans, probs, offs, order, branch_of, stream);
  }
  if (!b.exec || b.key != key) {
    drop_graph(b);
    if (hipStreamBeginCapture(b.cap, hipStreamCaptureModeRelaxed) !=
        hipSuccess)
      return BCGS_ERR_HIP;
    const bcgs_status r =
        enqueue_branches(b, plans, probs, offs, order, branch_of, b.cap);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(b.cap, &graph);
    if (r != BCGS_OK || ec != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      return r != BCGS_OK ? r : BCGS_ERR_HIP;
    }
    const hipError_t ei = hipGraphInstantiate(&b.exec, graph, nullptr,
                                              nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      b.exec = nullptr;
      return BCGS_ERR_HIP;
    }
    b.key = key;
  }
  if (hipEventRecord(b.in_ev, stream) != hipSuccess ||
      hipStreamWaitEvent(b.cap, b.in_ev, 0) != hipSuccess ||
      hipGraphLaunch(b.exec, b.cap) != hipSuccess ||
      hipEventRecord(b.out_ev, b.cap) != hipSuccess ||
      hipStreamWaitEvent(stream, b.out_ev, 0) != hipSuccess)
    return BCGS_ERR_HIP;
  return BCGS_OK;
}

bcgs_status bcgs_autotune(const bcgs_problem* probs, int32_t count,
                          hipStream_t stream) {
  if (count < 0 || (count > 0 && !probs)) return BCGS_ERR_ARG;
  for (int i = 0; i < count; ++i) {
    const bcgs_problem& p = probs[i];
    Plan chk;
    const bcgs_status st =
        check_problem(p.X, p.ldx, p.m, p.n, p.s, p.variant, p.precision, p.Q,
                      p.ldq, p.R, p.ldr, p.d_info, &chk);
    if (st != BCGS_OK) return st;
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return BCGS_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return BCGS_ERR_HIP;
  }
  bcgs_status res = BCGS_OK;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  for (int i = 0; i < count && res == BCGS_OK; ++i) {
    const bcgs_problem& p = probs[i];
    const int s = (int)p.s;
    Tuning have;
    if (tuned_choice(p.m, p.n, s, p.variant, p.precision, &have)) continue;
    // candidates: workgroup caps, then tile shapes under the best cap
    std::vector<Tuning> cands;
    for (int wg = 512; wg >= 16; wg /= 2) {
      if (wg < 512 && cdiv(p.m, 64) <= wg) continue;   // same split as 512
      Tuning t;
      t.max_wg = wg;
      cands.push_back(t);
    }
    auto time_one = [&](const Tuning& t, float* best_ms) -> bcgs_status {
      Plan pl;
      if (!make_plan(p.m, p.n, p.s, p.variant, p.precision, &pl, &t))
        return BCGS_ERR_ARG;
      if (ws_bytes < pl.bytes) {
        if (ws) {
          if (hipStreamSynchronize(stream) != hipSuccess) return BCGS_ERR_HIP;
          (void)hipFree(ws);
          ws = nullptr;
          ws_bytes = 0;
        }
        if (hipMalloc(&ws, pl.bytes) != hipSuccess) {
          ws = nullptr;
          return BCGS_ERR_NOMEM;
        }
        ws_bytes = pl.bytes;
      }
      float ms = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {   // first run warms up
        if (hipEventRecord(e0, stream) != hipSuccess) return BCGS_ERR_HIP;
        const bcgs_status r = run_problem(pl, p.X, p.ldx, p.Q, p.ldq, p.R,
                                          p.ldr, ws, p.d_info, stream);
        if (r != BCGS_OK) return r;
        if (hipEventRecord(e1, stream) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess)
          return BCGS_ERR_HIP;
        float t_ms = 0.f;
        if (hipEventElapsedTime(&t_ms, e0, e1) != hipSuccess)
          return BCGS_ERR_HIP;
        if (rep > 0) ms = std::min(ms, t_ms);
      }
      *best_ms = ms;
      return BCGS_OK;
    };
    Tuning best;
    float best_ms = 1e30f;
    for (const Tuning& t : cands) {
      float ms;
      res = time_one(t, &ms);
      if (res != BCGS_OK) break;
      if (ms < best_ms) { best_ms = ms; best = t; }
    }
    if (res == BCGS_OK && (p.precision == BCGS_FP64 && s <= 16)) {
      const Tuning base = best;
      for (int sh = 0; sh < pass16_shape_count(); ++sh) {
        // small problems: four-wave shapes only (as the automatic choice)
        if (p.m <= pass16_small_rows() && !pass16_shape_four_waves(sh))
          continue;
        Tuning t = base;
        t.shape = sh;
        float ms;
        res = time_one(t, &ms);
        if (res != BCGS_OK) break;
        if (ms < best_ms * 0.98f) { best_ms = ms; best = t; }
      }
    }
    if (res == BCGS_OK) set_choice(p.m, p.n, s, p.variant, p.precision, best);
  }
  if (ws) {
    (void)hipStreamSynchronize(stream);
    (void)hipFree(ws);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return res;
}

bcgs_status bcgs_tuning_get(int64_t m, int64_t n, int64_t s,
                            bcgs_variant variant, bcgs_precision precision,
                            bcgs_tuning* out) {
  if (!out || s < 1 || s > kMaxS) return BCGS_ERR_ARG;
  Tuning t;
  if (!tuned_choice(m, n, (int)s, variant, precision, &t)) {
    out->max_wg = Tuning().max_wg;
    out->shape = -1;
    return BCGS_PENDING;
  }
  out->max_wg = t.max_wg;
  out->shape = t.shape;
  return BCGS_OK;
}

bcgs_status bcgs_tuning_set(int64_t m, int64_t n, int64_t s,
                            bcgs_variant variant, bcgs_precision precision,
                            const bcgs_tuning* choice) {
  if (s < 1 || s > kMaxS || n < 1 || m < n) return BCGS_ERR_ARG;
  if (variant < BCGS_I_PLUS || variant > BCGS_I_PLUS_1S) return BCGS_ERR_ARG;
  if (precision != BCGS_FP64 && precision != BCGS_FP32_BULK)
    return BCGS_ERR_ARG;
  if (!choice) {
    Tuning old;
    (void)erase_choice(m, n, (int)s, variant, precision, &old);
    return BCGS_OK;
  }
  if (choice->max_wg < 1 || choice->max_wg > 512) return BCGS_ERR_ARG;
  if (choice->shape < -1 || choice->shape >= pass16_shape_count())
    return BCGS_ERR_ARG;
  Tuning t;
  t.max_wg = choice->max_wg;
  t.shape = choice->shape;
  set_choice(m, n, (int)s, variant, precision, t);
  return BCGS_OK;
}

void bcgs_tuning_clear(void) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune.clear();
}

}  // extern "C"

namespace bcgs {

void batch_release() {
  persist_release();
  std::lock_guard<std::mutex> lock(g_batch_mu);
  for (auto& kv : g_batch) {
    BatchState& b = kv.second;
    (void)hipStreamSynchronize(kv.first);
    if (b.cap) (void)hipStreamSynchronize(b.cap);
    drop_graph(b);
    if (b.arena) (void)hipFree(b.arena);
    for (int i = 0; i < kBranches; ++i) {
      if (b.branch[i]) {
        (void)hipStreamSynchronize(b.branch[i]);
        (void)hipStreamDestroy(b.branch[i]);
      }
      if (b.join[i]) (void)hipEventDestroy(b.join[i]);
    }
    if (b.fork) (void)hipEventDestroy(b.fork);
    if (b.cap) {
      (void)hipStreamSynchronize(b.cap);
      (void)hipStreamDestroy(b.cap);
    }
    if (b.in_ev) (void)hipEventDestroy(b.in_ev);
    if (b.out_ev) (void)hipEventDestroy(b.out_ev);
  }
  g_batch.clear();
}

}  // namespace bcgs
