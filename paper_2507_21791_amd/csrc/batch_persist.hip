// Batched factorizations in one persistent launch.
//
// Each problem's schedule (the launches its variant makes alone: info
// reset, fill, TSQR leaf / node / down / apply, streaming passes,
// reductions, epilogues) is recorded on the host as a list of steps; a
// step is a set of work items, one per workgroup the lone launch would
// have had, grouped into units of up to 8 consecutive items.  One kernel
// with two resident workgroups per CU then runs all problems: a workgroup
// claims the next free unit of some problem's current step (a per-problem
// 64-bit word: owner << 56 | step << 32 | next unit), runs the same device
// bodies the lone kernels run, with each item as its workgroup index, and
// counts the unit done; the workgroup that completes a step's last unit
// opens the problem's next step.  That counter is the per-problem
// device-side barrier between dependent steps, while units of different
// problems run side by side.
//
// Bits: an item computes exactly what workgroup `item` of the lone launch
// computes (same bodies, same row split, same fixed-order sums, the same
// tile layout whether tiles are copied directly or through registers), so
// a batched result equals the lone one bitwise.
//
// Placement: each XCD has its own L2, so a problem is adopted by one XCD
// (the hardware XCC_ID of the first workgroup that claims it) and all its
// units run there.  Units then communicate through that L2: a unit's
// stores are complete in the L2 before it is counted, without a write-back
// of the L2 to memory, and a workgroup starting a unit of a new step
// invalidates its caches at agent scope.  An XCD adopts the largest
// problem nobody owns yet whenever it runs fewer than six problems, so the
// XCDs share the work as they free up and finish together.
//
// Code generation: every body is its own function; the step record it
// receives is read as wave-uniform constant data (scalar loads), and all
// its global accesses use global instructions (flat ones would be counted
// with the LDS operations, coupling every LDS wait to the loads in
// flight).
//
// Termination: units never wait for one another, so some workgroup always
// makes progress; a workgroup that finds no free unit sleeps briefly and
// looks again.  A workgroup that has found nothing to do for about ten
// seconds (the device's 100 MHz clock) gives up, marks the unfinished
// problems' info records BCGS_ERR_HIP and exits, so the launch always
// ends.
#include <string.h>

#include <algorithm>
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
  int32_t kind, items, sel;
  int32_t chunk;     // items run back to back per claim (a unit)
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

// Per problem: w = owner << 56 | step << 32 | next unit to claim (owner
// 0xFF: not adopted yet); units of the step done.
struct ProbCtl {
  unsigned long long w;
  unsigned done;
  unsigned pad;
};
constexpr unsigned long long kNoOwner = 0xFFull << 56;

// ------------------------------------------------------------ record ---
namespace {
struct Recorder {
  std::vector<BatchStep> steps;
  bool unsupported = false;
};
thread_local Recorder* t_rec = nullptr;

// Items per unit: lone launches with many workgroups become fewer, longer
// units (up to 8 items), so that per-claim costs are spread; at least 32
// units remain for the XCD's workgroups to share.
int chunk_for(int64_t items) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(8, items / 32));
}

BatchStep& add(int kind, int64_t items, int sel) {
  BatchStep st;
  memset(&st, 0, sizeof st);
  st.kind = kind;
  st.items = (int32_t)items;
  st.sel = sel;
  st.chunk = chunk_for(items);
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
                     int gram_ntb, int G, bool reg) {
  const int code = tr == 16 ? 0 : tr == 32 ? 1 : tr == 64 ? 2 : -1;
  // the bodies hold up to 272 (16 rows), 128 (32) or 64 (64) columns
  const int cap = tr == 16 ? 272 : tr == 32 ? 128 : 64;
  if (code < 0 || nw != 4 || gram_ntb > 2 || a.ncols_p > cap) {
    t_rec->unsupported = true;
    return;
  }
  add(SK_PASS, G, code * 3 + gram_ntb + (reg ? 9 : 0)).u.pass = a;
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
//
// A body receives its step record as a function argument, which the
// compiler must assume divergent and generic.  uniform_const makes the
// record's address wave-uniform and constant-address-space (the records do
// not change while the kernel runs), so its fields come from scalar loads
// into scalar registers and the body's loop control stays scalar, as in
// the lone kernels; the pointers in the record are generic, so the bodies
// access global memory through gload / gstore (global instructions, which
// the hardware does not count with the LDS operations).
template <typename P>
__device__ __forceinline__ const P* uniform_const(const P* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  typedef const __attribute__((address_space(4))) P CP;
  return (const P*)(CP*)(((uint64_t)hi << 32) | lo);
}

// pass bodies: four waves, two tile buffers filled by direct copies or,
// where the lone launch staged through registers (columns not 16-byte
// aligned), through registers (the same tile layout either way), Gram pair
// slots for the most pairs a wave can get
template <int TR, int CAP, int NTB, bool GRAM, bool REG>
__device__ __noinline__ void pass_item(const p16::ArgsT<double>* a,
                                       int64_t g0, int64_t g1, int64_t G) {
  constexpr int kTop = ((CAP / 16) * NTB + 3) / 4;
  constexpr int MAXP = kTop < 1 ? 1 : kTop;
  using K = p16::Kernel<double, TR, 2, CAP, 2, 4, false, MAXP, GRAM, NTB,
                        REG, 0>;
  static_assert(TR * CAP <= kPoolTile, "tile fits the pool");
  static_assert(K::kScrElems <= kPoolScr, "partial sums fit the pool");
  const p16::ArgsT<double>& b = *uniform_const(a);
  for (int64_t g = g0; g < g1; ++g) {
    if (g > g0) __syncthreads();     // the previous item's LDS reads are done
    K::run_with(b, g_pool_b0, g_pool_b1, nullptr, nullptr, g_pool_scr, g, G);
  }
}

template <int TR, int CAP, bool REG>
__device__ __forceinline__ void pass_tr(const p16::ArgsT<double>* a, int ntb,
                                        int64_t g0, int64_t g1, int64_t G) {
  if (ntb == 0) pass_item<TR, CAP, 1, false, REG>(a, g0, g1, G);
  else if (ntb == 1) pass_item<TR, CAP, 1, true, REG>(a, g0, g1, G);
  else pass_item<TR, CAP, 2, true, REG>(a, g0, g1, G);
}

template <bool REG>
__device__ __forceinline__ void pass_unit(const BatchStep* st, int sel,
                                          int64_t g0, int64_t g1) {
  const int code = sel / 3, ntb = sel % 3;
  if (code == 0) pass_tr<16, 272, REG>(&st->u.pass, ntb, g0, g1, st->items);
  else if (code == 1)
    pass_tr<32, 128, REG>(&st->u.pass, ntb, g0, g1, st->items);
  else pass_tr<64, 64, REG>(&st->u.pass, ntb, g0, g1, st->items);
}

template <int S>
__device__ __noinline__ void epi_item(const EpiArgs* a) {
  double* p = g_pool_b0;
  const EpiView sm{p, g_pool_b1, p + 256, p + 512, p + 768, p + 1024,
                   p + 1280, p + 1536, p + 1792, p + 2048, p + 2560,
                   reinterpret_cast<int*>(p + 2564)};
  epilogue_all<S>(*uniform_const(a), sm);
}

template <int S>
__device__ __noinline__ void leaf_item(const LeafA* l, int64_t item) {
  l = uniform_const(l);
  tw::leaf_body<double, S>(l->v, l->ldv, l->m, l->nchunks, l->rleaf, item);
}

template <int S>
__device__ __noinline__ void node_item(const NodeA* n, int64_t item) {
  n = uniform_const(n);
  tw::node_body<S>(n->rprev, n->nprev, n->fan, n->nnodes, n->rcur, n->qcur,
                   n->is_root, n->r_out, n->r_rs, n->r_cs, n->syncs,
                   g_pool_b0, item);
}

template <int S>
__device__ __noinline__ void apply_item(const ApplyA* p, int64_t item) {
  p = uniform_const(p);
  tw::apply_body<double, S>(p->v, p->ldv, p->m, p->nchunks, p->cleaf, p->dst,
                            p->ldd, g_pool_b0, item);
}

__device__ __noinline__ void small_item(const BatchStep* st, int64_t item) {
  st = uniform_const(st);
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

__device__ __forceinline__ void run_one(const BatchStep* st, int64_t item) {
  switch (st->kind) {
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

// Unit `unit` of a step: its items [unit chunk, (unit + 1) chunk), one
// after another (the same bodies with the same item indices as alone).
__device__ __forceinline__ void run_unit(const BatchStep* st, int unit) {
  const int64_t g0 = (int64_t)unit * st->chunk;
  const int64_t g1 = min((int64_t)st->items, g0 + st->chunk);
  if (st->kind == SK_PASS) {
    if (st->sel >= 9) pass_unit<true>(st, st->sel - 9, g0, g1);
    else pass_unit<false>(st, st->sel, g0, g1);
    return;
  }
  for (int64_t g = g0; g < g1; ++g) {
    if (g > g0) __syncthreads();
    run_one(st, g);
  }
}

__device__ __forceinline__ int units_of(const BatchStep* st) {
  return (st->items + st->chunk - 1) / st->chunk;
}

// Identifier of the accelerator complex die (XCD) this wave runs on: its
// L2 cache domain (hardware register XCC_ID, bits 3:0).
__device__ __forceinline__ int xcc_id() {
  return __builtin_amdgcn_s_getreg((3 << 11) | 20) & 15;
}

// flags: [0] problems finished, [1] gave up, [2 + x] problems adopted and
// not finished by XCD x (x < 16)
constexpr int kFlags = 18;

__global__ void persist_reset(ProbCtl* ctl, int nprob, unsigned* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nprob) {
    ctl[i].w = kNoOwner;
    ctl[i].done = 0;
  }
  if (i < kFlags) flags[i] = 0;
}

constexpr uint64_t kIdleTicks = 1000000000ull;   // 10 s at 100 MHz

// Ordering between the units of a problem.  All of a problem's units run on
// the XCD that adopted it, so they share that XCD's L2: a unit's stores
// need only be complete in the L2 (s_waitcnt vmcnt(0)) before the unit is
// counted done, with no write-back of the L2 to memory, which with
// thousands of units per millisecond would keep every L2 writing.  A unit
// that starts a new step invalidates its caches at agent scope (the L1 and
// the non-coherent L2 lines; dirty lines stay): measured on MI355X,
// invalidating the L1 alone left units reading stale data.
__device__ __forceinline__ void unit_acquire() {
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}
__device__ __forceinline__ void unit_release() {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

template <typename W>
__device__ __forceinline__ W ld_agent(W* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void persist_kernel(const BatchStep* __restrict__ steps,
                    const int* __restrict__ first,
                    const int* __restrict__ nsteps,
                    const int* __restrict__ order,
                    bcgs_info* const* __restrict__ infos, int nprob,
                    ProbCtl* ctl, unsigned* flags, int max_live) {
  __shared__ int sh[4];
  const int tid = threadIdx.x, lane = tid & 63;
  const unsigned long long mine = (unsigned long long)xcc_id();
  int start = blockIdx.x % nprob;
  int last_p = -1, last_s = -1;     // step of this workgroup's last unit
  uint64_t idle_since = wall_clock64();
  for (;;) {
    // ---- wave 0 looks for a free unit, 64 problems at a time ----
    if (tid < 64) {
      int fp = -1, fs = 0, fi = 0, ex = 0;
      if (ld_agent(&flags[0]) >= (unsigned)nprob || ld_agent(&flags[1]) != 0)
        ex = 1;
      // 1. a unit of the current step of a problem this XCD owns
      for (int base = 0; !ex && fp < 0 && base < nprob; base += 64) {
        int p = start + base + lane;
        p = p >= nprob ? p - nprob : p;
        bool open = false;
        if (base + lane < nprob) {
          const unsigned long long w = ld_agent(&ctl[p].w);
          const int st = (int)((w >> 32) & 0xFFFFFF);
          open = (w >> 56) == mine && st < nsteps[p] &&
                 (unsigned)w < (unsigned)units_of(&steps[first[p] + st]);
        }
        unsigned long long cand = __ballot(open);
        // claim from the candidates in order, one at a time
        while (cand && fp < 0) {
          const int k = __ffsll((long long)cand) - 1;
          cand &= cand - 1;
          int got = 0, gs = 0, gi = 0;
          if (lane == k) {
            const unsigned long long w2 = __hip_atomic_fetch_add(
                &ctl[p].w, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            gs = (int)((w2 >> 32) & 0xFFFFFF);
            gi = (int)(unsigned)w2;
            got = gs < nsteps[p] &&
                  gi < units_of(&steps[first[p] + gs]);
          }
          got = __shfl(got, k);
          if (got) {
            fp = __shfl(p, k);
            fs = __shfl(gs, k);
            fi = __shfl(gi, k);
          }
        }
      }
      // 2. adopt the largest problem nobody owns yet (claiming
      //    unit 0 of its first step with the same exchange), if this XCD
      //    runs fewer than max_live problems: a slot is reserved first
      //    (and returned when nothing is adopted), so the limit is exact
      //    and problems are handed out as XCDs make room, largest first
      bool slot = false;
      if (!ex && fp < 0 && lane == 0 &&
          ld_agent(&flags[2 + mine]) < (unsigned)max_live) {
        const unsigned had = __hip_atomic_fetch_add(
            &flags[2 + mine], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        slot = had < (unsigned)max_live;
        if (!slot)
          __hip_atomic_fetch_sub(&flags[2 + mine], 1u, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
      }
      slot = __shfl((int)slot, 0) != 0;
      if (slot) {
        for (int base = 0; fp < 0 && base < nprob; base += 64) {
          const int j = base + lane;
          const int p = j < nprob ? order[j] : 0;
          const bool free_p = j < nprob && ld_agent(&ctl[p].w) == kNoOwner;
          unsigned long long cand = __ballot(free_p);
          while (cand && fp < 0) {
            const int k = __ffsll((long long)cand) - 1;
            cand &= cand - 1;
            int got = 0;
            if (lane == k) {
              unsigned long long expect = kNoOwner;
              got = __hip_atomic_compare_exchange_strong(
                  &ctl[p].w, &expect, (mine << 56) | 1ull, __ATOMIC_RELAXED,
                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            got = __shfl(got, k);
            if (got) {
              fp = __shfl(p, k);
              fs = 0;
              fi = 0;
            }
          }
        }
        if (fp < 0 && lane == 0)       // nothing left to adopt
          __hip_atomic_fetch_sub(&flags[2 + mine], 1u, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
      }
      if (lane == 0) {
        sh[0] = fp;
        sh[1] = fs;
        sh[2] = fi;
        sh[3] = ex;
      }
    }
    __syncthreads();
    const int p = __builtin_amdgcn_readfirstlane(sh[0]);
    const int s = __builtin_amdgcn_readfirstlane(sh[1]);
    const int it = __builtin_amdgcn_readfirstlane(sh[2]);
    const int ex = __builtin_amdgcn_readfirstlane(sh[3]);
    __syncthreads();
    if (ex) break;
    if (p < 0) {
      if (wall_clock64() - idle_since > kIdleTicks) {
        // nothing became free for a long time: stop, and say so
        if (tid == 0) {
          __hip_atomic_store(&flags[1], 1u, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
          for (int q = 0; q < nprob; ++q) {
            const unsigned long long w = ld_agent(&ctl[q].w);
            if ((int)((w >> 32) & 0xFFFFFF) < nsteps[q])
              infos[q]->status = BCGS_ERR_HIP;
          }
        }
        break;
      }
      __builtin_amdgcn_s_sleep(16);
      continue;
    }
    idle_since = wall_clock64();
    // ---- the unit, after everything the earlier steps wrote (already
    //      acquired when this workgroup's last unit was of the same step) ----
    if (p != last_p || s != last_s) unit_acquire();
    last_p = p;
    last_s = s;
    const BatchStep* st = &steps[first[p] + s];
    run_unit(st, it);
    unit_release();
    __syncthreads();
    if (tid == 0) {
      const unsigned d = __hip_atomic_fetch_add(
          &ctl[p].done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (d + 1 == (unsigned)units_of(st)) {
        // the step is complete: open the next one
        __hip_atomic_store(&ctl[p].done, 0u, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        unit_release();         // the reset lands before the step opens
        __hip_atomic_store(&ctl[p].w,
                           (mine << 56) | ((unsigned long long)(s + 1) << 32),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (s + 1 == nsteps[p]) {
          __hip_atomic_fetch_add(&flags[0], 1u, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_fetch_sub(&flags[2 + mine], 1u, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
        }
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
  int* d_order = nullptr;
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
  (void)hipFree(s.d_order);
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
                           const std::vector<int>& order,
                           const bcgs_problem* probs, int count,
                           hipStream_t stream) {
  // problems an XCD runs at a time: measured 4 to 6 best on the batched
  // workload (more and the XCDs finish unevenly, fewer and they idle)
  constexpr int max_live = 6;
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
        hipMalloc(&s.d_order, count * sizeof(int)) != hipSuccess ||
        hipMalloc(&s.d_flags, kFlags * sizeof(unsigned)) != hipSuccess) {
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
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s.d_order, order.data(), count * sizeof(int),
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
    hipLaunchKernelGGL(persist_reset,
                       dim3((unsigned)cdiv(std::max(count, kFlags), 256)),
                       dim3(256), 0, s.graph_stream, s.d_ctl, count,
                       s.d_flags);
    hipLaunchKernelGGL(persist_kernel, dim3((unsigned)(2 * cus)), dim3(256),
                       0, s.graph_stream, s.d_steps, s.d_first, s.d_nsteps,
                       s.d_order, s.d_infos, count, s.d_ctl, s.d_flags,
                       max_live);
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
  // adoption order: largest modelled work first (streamed m x n x q)
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  auto work = [&](int i) {
    return (double)probs[i].m * (double)probs[i].n *
           (double)(probs[i].n / probs[i].s);
  };
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return work(a) > work(b); });
  return persist_launch(key, steps, first, nsteps, order, probs, count,
                        stream);
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
