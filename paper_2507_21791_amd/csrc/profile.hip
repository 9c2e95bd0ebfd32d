// Launch profiling: optional HIP events around every kernel the library
// enqueues on a stream, each tagged with the launch's algorithmic HBM bytes
// and flops (the work the method itself requires, not what the kernel
// happens to move), so callers can compute achieved rates per kernel.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "common.h"

namespace bcgs {

struct ProfRec {
  int kind, tag;
  hipEvent_t a, b;
  double bytes, flops;
  const char* name;      // interned (see prof_name), or null
};

struct Prof {
  hipStream_t st;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
};

static std::mutex g_pmu;
static std::map<hipStream_t, Prof*> g_prof;
static thread_local Prof* t_cur = nullptr;

static hipEvent_t take_event(Prof* p) {
  if (p->used < p->pool.size()) return p->pool[p->used++];
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  p->pool.push_back(e);
  p->used++;
  return e;
}

void prof_attach(hipStream_t st) {
  std::lock_guard<std::mutex> lock(g_pmu);
  auto it = g_prof.find(st);
  t_cur = it == g_prof.end() ? nullptr : it->second;
}

void prof_detach() { t_cur = nullptr; }

void prof_begin(int kind, int tag, double bytes, double flops) {
  Prof* p = t_cur;
  if (!p) return;
  ProfRec r{kind, tag, take_event(p), take_event(p), bytes, flops, nullptr};
  if (r.a) (void)hipEventRecord(r.a, p->st);
  p->recs.push_back(r);
}

void prof_model(double bytes, double flops) {
  Prof* p = t_cur;
  if (p && !p->recs.empty()) {
    p->recs.back().bytes = bytes;
    p->recs.back().flops = flops;
  }
}

void prof_retag(int tag) {
  Prof* p = t_cur;
  if (p && !p->recs.empty()) p->recs.back().tag = tag;
}

// names live for the whole process, so records keep plain pointers
static std::mutex g_nmu;
static std::set<std::string> g_names;

void prof_name(const char* fmt, ...) {
  Prof* p = t_cur;
  if (!p || p->recs.empty()) return;
  char buf[256];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  std::lock_guard<std::mutex> lock(g_nmu);
  p->recs.back().name = g_names.insert(buf).first->c_str();
}

void prof_end() {
  Prof* p = t_cur;
  if (!p || p->recs.empty()) return;
  ProfRec& r = p->recs.back();
  if (r.b) (void)hipEventRecord(r.b, p->st);
}

}  // namespace bcgs

using namespace bcgs;

extern "C" {

bcgs_status bcgs_profile_start(hipStream_t stream) {
  std::lock_guard<std::mutex> lock(g_pmu);
  Prof*& p = g_prof[stream];
  if (!p) p = new Prof();
  p->st = stream;
  p->recs.clear();
  p->used = 0;
  return BCGS_OK;
}

int32_t bcgs_profile_stop(hipStream_t stream, bcgs_launch_record* out,
                          int32_t capacity) {
  Prof* p = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_pmu);
    auto it = g_prof.find(stream);
    if (it == g_prof.end()) return -1;
    p = it->second;
    g_prof.erase(it);
  }
  if (hipStreamSynchronize(stream) != hipSuccess) return -1;
  int32_t n = 0;
  for (const ProfRec& r : p->recs) {
    if (out && n < capacity) {
      float ms = -1.0f;
      if (r.a && r.b && hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
        ms = -1.0f;
      out[n].kind = r.kind;
      out[n].tag = r.tag;
      out[n].ms = ms;
      out[n].bytes = r.bytes;
      out[n].flops = r.flops;
      memset(out[n].name, 0, sizeof out[n].name);
      if (r.name) strncpy(out[n].name, r.name, sizeof out[n].name - 1);
    }
    ++n;
  }
  for (hipEvent_t e : p->pool) (void)hipEventDestroy(e);
  delete p;
  return n;
}

}  // extern "C"
