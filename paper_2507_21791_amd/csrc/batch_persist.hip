// Batched factorizations in one persistent launch.
//
// Each problem's schedule (the launches its variant makes alone: info
// reset, fill, TSQR leaf / node / down / apply, streaming passes,
// reductions, epilogues) is recorded on the host as a list of steps; a
// step is a set of work items, one per workgroup the lone launch would
// have had.  One kernel with two resident workgroups per CU then runs all
// problems: a workgroup claims the next free item of some problem's
// current step (a per-problem 64-bit word: step << 32 | next item), runs
// the same device body the lone kernel runs, with the item as its
// workgroup index, and counts the item done; the workgroup that completes
// a step's last item opens the problem's next step.  That counter is the
// per-problem device-side barrier between dependent steps, while items of
// different problems (iterations, row chunks) run side by side.
//
// Bits: an item computes exactly what workgroup `item` of the lone launch
// computes (same bodies, same row split, same fixed-order sums), so a
// batched result equals the lone one bitwise.  Streaming passes run their
// register-staged form (the LDS tile is identical to the direct-copy one)
// with four waves, whatever shape of four waves the lone run chose.
//
// Visibility: items of one step run on any XCD, and XCDs have separate L2
// caches, so every item ends with an agent-scope release fence before it
// is counted, and every item starts with an agent-scope acquire fence.
//
// Termination: items never wait for one another, so some workgroup always
// makes progress; a workgroup that finds no free item sleeps briefly and
// looks again.  A workgroup that has found nothing to do for about ten
// seconds (the device's 100 MHz clock) gives up, marks the unfinished
// problems' info records BCGS_ERR_HIP and exits, so the launch always
// ends.
#include <string.h>

#include <map>
#include <mutex>
#include <vector>

#include "common.h"
#include "epilogue_impl.h"
#include "pass16_impl.h"
#include "small_impl.h"
#include "tsqr_wave_impl.h"

namespace bcgs {

enum StepKind : int32_t {
  SK_INIT = 0, SK_FILL, SK_LEAF, SK_NODE, SK_DOWN, SK_APPLY, SK_PASS,
  SK_REDUCE, SK_EPI
};

struct LeafA { const double* v; int64_t ldv, m, nchunks; double* rleaf; };
struct NodeA {
  const double* rprev; int64_t nprev; int fan; int64_t nnodes;
  double* rcur; double* qcur; int is_root; double* r_out;
  int64_t r_rs, r_cs; int32_t* syncs;
};
struct DownA {
  const double* qpar; const double* cpar; int64_t nchild; int fan, s;
  double* cchild; int parent_is_root;
};
struct ApplyA {
  const double* v; int64_t ldv, m, nchunks; const double* cleaf;
  double* dst; int64_t ldd;
};
struct RedA {
  const double* partial; int G; int64_t elems; double* out; int32_t* syncs;
};
struct FillA { double* p; int64_t rows, cols, ld; double v; };
struct InitA { bcgs_info* info; };

// One step: `items` work items of one kind; sel is the body (pass: tile
// rows code * 3 + Gram B blocks; TSQR and epilogue: s).
struct BatchStep {
  int32_t kind, items, sel, pad;
  union {
    p16::ArgsT<double> pass;
    EpiArgs epi;
    LeafA leaf;
    NodeA node;
    DownA down;
    ApplyA apply;
    RedA red;
    FillA fill;
    InitA init;
  } u;
};

// per problem: step << 32 | next item to claim; items of the step done
struct ProbCtl {
  unsigned long long w;
  unsigned done;
  unsigned pad;
};

// ------------------------------------------------------------ record ---
namespace {
struct Recorder {
  std::vector<BatchStep> steps;
  bool unsupported = false;
};
thread_local Recorder* t_rec = nullptr;

BatchStep& add(int kind, int64_t items, int sel) {
  BatchStep st;
  memset(&st, 0, sizeof st);
  st.kind = kind;
  st.items = (int32_t)items;
  st.sel = sel;
  if (items < 1 || items > (int64_t(1) << 30)) t_rec->unsupported = true;
  t_rec->steps.push_back(st);
  return t_rec->steps.back();
}
}  // namespace

bool rec_active() { return t_rec != nullptr; }
void rec_unsupported() {
  if (t_rec) t_rec->unsupported = true;
}

void p16::rec_pass16(const p16::ArgsT<double>& a, int tr, int nw,
                     int gram_ntb, int G) {
  const int code = tr == 16 ? 0 : tr == 32 ? 1 : tr == 64 ? 2 : -1;
  // the bodies hold up to 272 (16 rows), 128 (32) or 64 (64) columns
  const int cap = tr == 16 ? 272 : tr == 32 ? 128 : 64;
  if (code < 0 || nw != 4 || gram_ntb > 2 || a.ncols_p > cap) {
    t_rec->unsupported = true;
    return;
  }
  add(SK_PASS, G, code * 3 + gram_ntb).u.pass = a;
}

void rec_reduce(const double* partial, int G, int64_t elems, double* out,
                int32_t* syncs, int64_t blocks) {
  add(SK_REDUCE, blocks, 0).u.red = RedA{partial, G, elems, out, syncs};
}

void rec_fill(double* p, int64_t rows, int64_t cols, int64_t ld, double v,
              int64_t blocks) {
  add(SK_FILL, blocks, 0).u.fill = FillA{p, rows, cols, ld, v};
}

void rec_init(bcgs_info* info) { add(SK_INIT, 1, 0).u.init = InitA{info}; }

void rec_epi(const EpiArgs& a) { add(SK_EPI, 1, a.s).u.epi = a; }

void rec_tsqr_leaf(int S, const double* v, int64_t ldv, int64_t m,
                   int64_t nchunks, double* rleaf, int64_t blocks) {
  add(SK_LEAF, blocks, S).u.leaf = LeafA{v, ldv, m, nchunks, rleaf};
}

void rec_tsqr_node(int S, const double* rprev, int64_t nprev, int fan,
                   int64_t nnodes, double* rcur, double* qcur, int is_root,
                   double* r_out, int64_t r_rs, int64_t r_cs, int32_t* syncs,
                   int64_t blocks) {
  add(SK_NODE, blocks, S).u.node = NodeA{rprev, nprev, fan, nnodes, rcur, qcur,
                                         is_root, r_out, r_rs, r_cs, syncs};
}

void rec_tsqr_down(const double* qpar, const double* cpar, int64_t nchild,
                   int fan, int s, double* cchild, int parent_is_root) {
  add(SK_DOWN, nchild, s).u.down =
      DownA{qpar, cpar, nchild, fan, s, cchild, parent_is_root};
}

void rec_tsqr_apply(int S, const double* v, int64_t ldv, int64_t m,
                    int64_t nchunks, const double* cleaf, double* dst,
                    int64_t ldd, int64_t blocks) {
  add(SK_APPLY, blocks, S).u.apply =
      ApplyA{v, ldv, m, nchunks, cleaf, dst, ldd};
}

// ------------------------------------------------------------ device ---
// LDS of the persistent kernel: two tile buffers and a partial-sum area,
// distinct objects (so the passes' copies into one buffer never make the
// compiler wait before reads of the other); the other bodies use them as
// scratch.  Sized for the largest pass body (272 columns x 16 rows).
constexpr int kPoolTile = 4352;
constexpr int kPoolScr = 1024;
__shared__ double g_pool_b0[kPoolTile];
__shared__ double g_pool_b1[kPoolTile];
__shared__ double g_pool_scr[kPoolScr];

// Every body is its own (not inlined) function, so that each gets the
// register allocation it would have as a kernel instead of sharing one
// allocation with all the others.

// pass bodies: four waves, two register-staged buffers, Gram pair slots for
// the most pairs a wave can get
template <int TR, int CAP, int NTB, bool GRAM>
__device__ __noinline__ void pass_item(const p16::ArgsT<double>* a,
                                       int64_t g, int64_t G) {
  constexpr int kTop = ((CAP / 16) * NTB + 3) / 4;
  constexpr int MAXP = kTop < 1 ? 1 : kTop;
  using K = p16::Kernel<double, TR, 2, CAP, 2, 4, false, MAXP, GRAM, NTB,
                        true, 0>;
  static_assert(TR * CAP <= kPoolTile, "tile fits the pool");
  static_assert(K::kScrElems <= kPoolScr, "partial sums fit the pool");
  K::run_with(*a, g_pool_b0, g_pool_b1, nullptr, nullptr, g_pool_scr, g, G);
}

template <int TR, int CAP>
__device__ __forceinline__ void pass_tr(const p16::ArgsT<double>* a, int ntb,
                                        int64_t g, int64_t G) {
  if (ntb == 0) pass_item<TR, CAP, 1, false>(a, g, G);
  else if (ntb == 1) pass_item<TR, CAP, 1, true>(a, g, G);
  else pass_item<TR, CAP, 2, true>(a, g, G);
}

template <int S>
__device__ __noinline__ void epi_item(const EpiArgs* a) {
  double* p = g_pool_b0;
  const EpiView sm{p, g_pool_b1, p + 256, p + 512, p + 768, p + 1024,
                   p + 1280, p + 1536, p + 1792, p + 2048, p + 2560,
                   reinterpret_cast<int*>(p + 2564)};
  epilogue_all<S>(*a, sm);
}

template <int S>
__device__ __noinline__ void leaf_item(const LeafA* l, int64_t item) {
  tw::leaf_body<double, S>(l->v, l->ldv, l->m, l->nchunks, l->rleaf, item);
}

template <int S>
__device__ __noinline__ void node_item(const NodeA* n, int64_t item) {
  tw::node_body<S>(n->rprev, n->nprev, n->fan, n->nnodes, n->rcur, n->qcur,
                   n->is_root, n->r_out, n->r_rs, n->r_cs, n->syncs,
                   g_pool_b0, item);
}

template <int S>
__device__ __noinline__ void apply_item(const ApplyA* p, int64_t item) {
  tw::apply_body<double, S>(p->v, p->ldv, p->m, p->nchunks, p->cleaf, p->dst,
                            p->ldd, g_pool_b0, item);
}

__device__ __noinline__ void small_item(const BatchStep* st, int64_t item) {
  switch (st->kind) {
    case SK_INIT:
      info_init_body(st->u.init.info);
      break;
    case SK_FILL: {
      const FillA& f = st->u.fill;
      fill_body(f.p, f.rows, f.cols, f.ld, f.v, item);
      break;
    }
    case SK_REDUCE: {
      const RedA& r = st->u.red;
      reduce_body(r.partial, r.G, r.elems, r.out, r.syncs, g_pool_b0, item);
      break;
    }
    default: {
      const DownA& d = st->u.down;
      tsqr_down_body(d.qpar, d.cpar, d.nchild, d.fan, d.s, d.cchild,
                     d.parent_is_root, item);
    }
  }
}

template <int S>
__device__ __forceinline__ void tsqr_item(const BatchStep* st, int64_t item) {
  if (st->kind == SK_LEAF) leaf_item<S>(&st->u.leaf, item);
  else if (st->kind == SK_NODE) node_item<S>(&st->u.node, item);
  else apply_item<S>(&st->u.apply, item);
}

__device__ __forceinline__ void run_item(const BatchStep* st, int64_t item) {
  switch (st->kind) {
    case SK_PASS: {
      const int code = st->sel / 3, ntb = st->sel % 3;
      if (code == 0) pass_tr<16, 272>(&st->u.pass, ntb, item, st->items);
      else if (code == 1) pass_tr<32, 128>(&st->u.pass, ntb, item, st->items);
      else pass_tr<64, 64>(&st->u.pass, ntb, item, st->items);
      break;
    }
    case SK_EPI:
      if (st->sel == 4) epi_item<4>(&st->u.epi);
      else if (st->sel == 8) epi_item<8>(&st->u.epi);
      else epi_item<16>(&st->u.epi);
      break;
    case SK_LEAF:
    case SK_NODE:
    case SK_APPLY:
      if (st->sel == 4) tsqr_item<4>(st, item);
      else if (st->sel == 8) tsqr_item<8>(st, item);
      else tsqr_item<16>(st, item);
      break;
    default:
      small_item(st, item);
  }
}

__global__ void persist_reset(ProbCtl* ctl, int nprob, unsigned* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nprob) {
    ctl[i].w = 0;
    ctl[i].done = 0;
  }
  if (i == 0) {
    flags[0] = 0;   // problems finished
    flags[1] = 0;   // gave up
  }
}

constexpr uint64_t kIdleTicks = 1000000000ull;   // 10 s at 100 MHz

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void persist_kernel(const BatchStep* __restrict__ steps,
                    const int* __restrict__ first,
                    const int* __restrict__ nsteps,
                    bcgs_info* const* __restrict__ infos, int nprob,
                    ProbCtl* ctl, unsigned* flags) {
  __shared__ int sh[4];
  const int tid = threadIdx.x, lane = tid & 63;
  int start = blockIdx.x % nprob;
  uint64_t idle_since = wall_clock64();
  for (;;) {
    // ---- wave 0 looks for a free item, 64 problems at a time ----
    if (tid < 64) {
      int fp = -1, fs = 0, fi = 0, ex = 0;
      if (__hip_atomic_load(&flags[0], __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT) >= (unsigned)nprob ||
          __hip_atomic_load(&flags[1], __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT) != 0)
        ex = 1;
      for (int base = 0; !ex && fp < 0 && base < nprob; base += 64) {
        int p = start + base + lane;
        p = p >= nprob ? p - nprob : p;
        bool open = false;
        if (base + lane < nprob) {
          const unsigned long long w = __hip_atomic_load(
              &ctl[p].w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          const int s = (int)(w >> 32);
          open = s < nsteps[p] &&
                 (unsigned)w < (unsigned)steps[first[p] + s].items;
        }
        unsigned long long cand = __ballot(open);
        // claim from the candidates in order, one at a time
        while (cand && fp < 0) {
          const int k = __ffsll((long long)cand) - 1;
          cand &= cand - 1;
          int got = 0, gs = 0, gi = 0;
          if (lane == k) {
            const unsigned long long w2 = __hip_atomic_fetch_add(
                &ctl[p].w, 1ull, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            gs = (int)(w2 >> 32);
            gi = (int)(unsigned)w2;
            got = gs < nsteps[p] &&
                  (unsigned)gi < (unsigned)steps[first[p] + gs].items;
          }
          got = __shfl(got, k);
          if (got) {
            fp = __shfl(p, k);
            fs = __shfl(gs, k);
            fi = __shfl(gi, k);
          }
        }
      }
      if (lane == 0) {
        sh[0] = fp;
        sh[1] = fs;
        sh[2] = fi;
        sh[3] = ex;
      }
    }
    __syncthreads();
    const int p = sh[0], s = sh[1], it = sh[2], ex = sh[3];
    __syncthreads();
    if (ex) break;
    if (p < 0) {
      if (wall_clock64() - idle_since > kIdleTicks) {
        // nothing became free for a long time: stop, and say so
        if (tid == 0) {
          __hip_atomic_store(&flags[1], 1u, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
          for (int q = 0; q < nprob; ++q) {
            const unsigned long long w = __hip_atomic_load(
                &ctl[q].w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((int)(w >> 32) < nsteps[q]) infos[q]->status = BCGS_ERR_HIP;
          }
        }
        break;
      }
      __builtin_amdgcn_s_sleep(16);
      continue;
    }
    idle_since = wall_clock64();
    // ---- the item, after everything the earlier steps wrote ----
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const BatchStep& st = steps[first[p] + s];
    run_item(&st, it);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0) {
      const unsigned d = __hip_atomic_fetch_add(
          &ctl[p].done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (d + 1 == (unsigned)st.items) {
        // the step is complete: open the next one
        __hip_atomic_store(&ctl[p].done, 0u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctl[p].w, (unsigned long long)(s + 1) << 32,
                           __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (s + 1 == nsteps[p])
          __hip_atomic_fetch_add(&flags[0], 1u, __ATOMIC_RELEASE,
                                 __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    start = p;
  }
}

// -------------------------------------------------------------- host ---
namespace {
struct PersistState {
  std::vector<char> key;
  BatchStep* d_steps = nullptr;
  int* d_first = nullptr;
  int* d_nsteps = nullptr;
  bcgs_info** d_infos = nullptr;
  ProbCtl* d_ctl = nullptr;
  unsigned* d_flags = nullptr;
  int nprob = 0;
  size_t nstep_total = 0;
  hipGraphExec_t exec = nullptr;
  hipStream_t graph_stream = nullptr;
};
std::mutex g_pmu;
std::map<hipStream_t, PersistState> g_persist;

void free_state(PersistState& s) {
  if (s.exec) (void)hipGraphExecDestroy(s.exec);
  (void)hipFree(s.d_steps);
  (void)hipFree(s.d_first);
  (void)hipFree(s.d_nsteps);
  (void)hipFree(s.d_infos);
  (void)hipFree(s.d_ctl);
  (void)hipFree(s.d_flags);
  const hipStream_t gs = s.graph_stream;   // kept for the next batch
  s = PersistState{};
  s.graph_stream = gs;
}

// Record every problem's schedule; false when some step has no persistent
// body (the caller then uses the graph of lone launches).
bool persist_record(const std::vector<Plan>& plans, const bcgs_problem* probs,
                    const std::vector<size_t>& offs, char* arena,
                    std::vector<BatchStep>* steps, std::vector<int>* first,
                    std::vector<int>* nsteps) {
  Recorder rec;
  for (size_t i = 0; i < plans.size(); ++i) {
    const bcgs_problem& p = probs[i];
    if (p.precision != BCGS_FP64) return false;
    first->push_back((int)rec.steps.size());
    t_rec = &rec;
    const bcgs_status r = run_problem(plans[i], p.X, p.ldx, p.Q, p.ldq, p.R,
                                      p.ldr, arena + offs[i], p.d_info,
                                      nullptr);
    t_rec = nullptr;
    if (r != BCGS_OK || rec.unsupported) return false;
    nsteps->push_back((int)rec.steps.size() - first->back());
  }
  *steps = std::move(rec.steps);
  return true;
}

// Launch the recorded batch on `stream` as one graph of two nodes (reset of
// the control words, the persistent kernel); the step tables are uploaded
// once per distinct batch (`key`).
bcgs_status persist_launch(const std::vector<char>& key,
                           const std::vector<BatchStep>& steps,
                           const std::vector<int>& first,
                           const std::vector<int>& nsteps,
                           const bcgs_problem* probs, int count,
                           hipStream_t stream) {
  std::lock_guard<std::mutex> lock(g_pmu);
  PersistState& s = g_persist[stream];
  if (s.key != key || !s.exec) {
    if (s.d_steps && hipStreamSynchronize(stream) != hipSuccess)
      return BCGS_ERR_HIP;
    free_state(s);
    std::vector<bcgs_info*> infos(count);
    for (int i = 0; i < count; ++i) infos[i] = probs[i].d_info;
    if (hipMalloc(&s.d_steps, steps.size() * sizeof(BatchStep)) !=
            hipSuccess ||
        hipMalloc(&s.d_first, count * sizeof(int)) != hipSuccess ||
        hipMalloc(&s.d_nsteps, count * sizeof(int)) != hipSuccess ||
        hipMalloc(&s.d_infos, count * sizeof(bcgs_info*)) != hipSuccess ||
        hipMalloc(&s.d_ctl, count * sizeof(ProbCtl)) != hipSuccess ||
        hipMalloc(&s.d_flags, 2 * sizeof(unsigned)) != hipSuccess) {
      free_state(s);
      return BCGS_ERR_NOMEM;
    }
    if (hipMemcpy(s.d_steps, steps.data(), steps.size() * sizeof(BatchStep),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s.d_first, first.data(), count * sizeof(int),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s.d_nsteps, nsteps.data(), count * sizeof(int),
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s.d_infos, infos.data(), count * sizeof(bcgs_info*),
                  hipMemcpyHostToDevice) != hipSuccess) {
      free_state(s);
      return BCGS_ERR_HIP;
    }
    s.nprob = count;
    s.nstep_total = steps.size();
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                              dev) != hipSuccess)
      return BCGS_ERR_HIP;
    // capture reset + persistent kernel once; replays are one launch
    if (!s.graph_stream &&
        hipStreamCreateWithFlags(&s.graph_stream, hipStreamNonBlocking) !=
            hipSuccess)
      return BCGS_ERR_HIP;
    if (hipStreamBeginCapture(s.graph_stream, hipStreamCaptureModeRelaxed) !=
        hipSuccess)
      return BCGS_ERR_HIP;
    hipLaunchKernelGGL(persist_reset, dim3((unsigned)cdiv(count, 256)),
                       dim3(256), 0, s.graph_stream, s.d_ctl, count,
                       s.d_flags);
    hipLaunchKernelGGL(persist_kernel, dim3((unsigned)(2 * cus)), dim3(256),
                       0, s.graph_stream, s.d_steps, s.d_first, s.d_nsteps,
                       s.d_infos, count, s.d_ctl, s.d_flags);
    hipGraph_t graph = nullptr;
    if (hipStreamEndCapture(s.graph_stream, &graph) != hipSuccess || !graph)
      return BCGS_ERR_HIP;
    const hipError_t ei =
        hipGraphInstantiate(&s.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      s.exec = nullptr;
      return BCGS_ERR_HIP;
    }
    s.key = key;
  }
  return hipGraphLaunch(s.exec, stream) == hipSuccess ? BCGS_OK
                                                      : BCGS_ERR_HIP;
}

}  // namespace

// The batch as one persistent launch on `stream` (see the top of this
// file).  *used = false, nothing enqueued, when some problem has a step the
// persistent kernel cannot run.
bcgs_status persist_run(const std::vector<Plan>& plans,
                        const bcgs_problem* probs,
                        const std::vector<size_t>& offs, void* arena,
                        const std::vector<char>& key, hipStream_t stream,
                        bool* used) {
  *used = false;
  const int count = (int)plans.size();
  {
    std::lock_guard<std::mutex> lock(g_pmu);
    auto it = g_persist.find(stream);
    if (it != g_persist.end() && it->second.exec && it->second.key == key) {
      *used = true;
      return hipGraphLaunch(it->second.exec, stream) == hipSuccess
                 ? BCGS_OK : BCGS_ERR_HIP;
    }
  }
  std::vector<BatchStep> steps;
  std::vector<int> first, nsteps;
  if (!persist_record(plans, probs, offs, static_cast<char*>(arena), &steps,
                      &first, &nsteps))
    return BCGS_OK;
  *used = true;
  return persist_launch(key, steps, first, nsteps, probs, count, stream);
}

void persist_release() {
  std::lock_guard<std::mutex> lock(g_pmu);
  for (auto& kv : g_persist) {
    (void)hipStreamSynchronize(kv.first);
    if (kv.second.graph_stream) (void)hipStreamDestroy(kv.second.graph_stream);
    free_state(kv.second);
  }
  g_persist.clear();
}

}  // namespace bcgs
