// Device code of the s <= 16 TSQR (one wave per row chunk): included by
// tsqr_wave.hip (its three kernels: leaves, the upward tree, the explicit
// Q) and by the batched persistent kernel, which runs the leaf,
// node, downward and apply bodies as steps of work items (the same
// arithmetic in the same order, so the same bits).
#pragma once

#include "common.h"

namespace bcgs {
namespace tw {

// Store of an R factor that a workgroup on another XCD may read in the
// same launch (the one-launch tree): written through to the device level
// (agent scope), so the writer need not write its whole L2 back.
__device__ __forceinline__ void st_r(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int S>
struct Geo {
  static constexpr int R = 64 / S;       // rows per lane
  static constexpr int L = 64 * R;       // rows per chunk
  static constexpr int P =               // reduction slots (power of two)
      S <= 1 ? 1 : S <= 2 ? 2 : S <= 4 ? 4 : S <= 8 ? 8 : 16;
  static constexpr int SH =              // slot c ends in lane c << SH
      P == 1 ? 6 : P == 2 ? 5 : P == 4 ? 4 : P == 8 ? 3 : 2;
};

constexpr int kRowMirror = 0x140;
constexpr int kRowHalfMirror = 0x141;
constexpr int kQuadXor1 = 0xB1;          // quad_perm [1, 0, 3, 2]
constexpr int kQuadXor2 = 0x4E;          // quad_perm [2, 3, 0, 1]

template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xf,
                                             0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xf,
                                             0xf, false);
  return __hiloint2double(hi, lo);
}

// a + b after exchanging lanes 32..63 of a with lanes 0..31 of b: lanes
// 0..31 get a(l) + a(l + 32), lanes 32..63 get b(l - 32) + b(l).
__device__ __forceinline__ double swap32_sum(double a, double b) {
  const auto l = __builtin_amdgcn_permlane32_swap(
      (unsigned)__double2loint(a), (unsigned)__double2loint(b), false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(
      (unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false, false);
  return __hiloint2double((int)h[0], (int)l[0]) +
         __hiloint2double((int)h[1], (int)l[1]);
}

// the same within each half wave, for lanes 16 apart
__device__ __forceinline__ double swap16_sum(double a, double b) {
  const auto l = __builtin_amdgcn_permlane16_swap(
      (unsigned)__double2loint(a), (unsigned)__double2loint(b), false, false);
  const auto h = __builtin_amdgcn_permlane16_swap(
      (unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false, false);
  return __hiloint2double((int)h[0], (int)l[0]) +
         __hiloint2double((int)h[1], (int)l[1]);
}

__device__ __forceinline__ double bcast(double y, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(y), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(y), lane);
  return __hiloint2double(hi, lo);
}

// Wave sums of the P slots v[0..P-1].  On return slot c's total is held by
// lane c << SH (and the other lanes of its group); read it with bcast().
// Lane bits 5, 4, 3, 2 split the slots (the partner lane keeps the other
// half of the slots); the remaining bits are summed over directly.  With
// HALVED the caller has already done the first split (v[i] = swap32_sum(
// v[i], v[i + P/2]) for i < P/2), so fewer slots are live at once.
template <int P, bool HALVED = false>
__device__ __forceinline__ double wave_sums(double (&v)[P]) {
  const int lane = threadIdx.x & 63;
  if constexpr (P >= 2 && !HALVED) {
#pragma unroll
    for (int i = 0; i < P / 2; ++i) v[i] = swap32_sum(v[i], v[i + P / 2]);
  }
  if constexpr (P >= 4) {
#pragma unroll
    for (int i = 0; i < P / 4; ++i) v[i] = swap16_sum(v[i], v[i + P / 4]);
  }
  if constexpr (P >= 8) {
    const bool hi = (lane >> 3) & 1;
#pragma unroll
    for (int i = 0; i < P / 8; ++i) {
      const double send = hi ? v[i] : v[i + P / 8];
      const double keep = hi ? v[i + P / 8] : v[i];
      v[i] = keep + dpp<kRowMirror>(send);
    }
  }
  if constexpr (P >= 16) {
    const bool hi = (lane >> 2) & 1;
#pragma unroll
    for (int i = 0; i < P / 16; ++i) {
      const double send = hi ? v[i] : v[i + P / 16];
      const double keep = hi ? v[i + P / 16] : v[i];
      v[i] = keep + dpp<kRowHalfMirror>(send);
    }
  }
  double y = v[0];
  y += dpp<kQuadXor1>(y);
  y += dpp<kQuadXor2>(y);
  if constexpr (P < 16) y += dpp<kRowHalfMirror>(y);
  if constexpr (P < 8) y += dpp<kRowMirror>(y);
  if constexpr (P < 4) y = swap16_sum(y, y);
  if constexpr (P < 2) y = swap32_sum(y, y);
  return y;
}

// LDS ordering between the lanes of one wave (no workgroup barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Householder QR of the chunk in a[][] (LAPACK convention: H_j = I - tau_j
// v_j v_j^T, v_j(j) = 1, beta_j = -sign(alpha_j) ||x_j||).  Afterwards the
// rows < S of a[0][] hold R (lane l: row l) and the entries below the
// diagonal hold the reflectors.  With z != nullptr (lane 0 writes) the
// products v_i^T v_j (i < j) go to z[i * S + j].
template <int S>
__device__ __forceinline__ void factor(double (&a)[Geo<S>::R][S],
                                       double (&tau)[S], double* z) {
  using Gm = Geo<S>;
  constexpr int R = Gm::R, P = Gm::P, SH = Gm::SH;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < S; ++j) {
    double pn[1] = {0.0};
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const double x = a[k][j];
      pn[0] += (k > 0 || lane > j) ? x * x : 0.0;
    }
    const double sigma2 = bcast(wave_sums<1>(pn), 0);
    const double alpha = bcast(a[0][j], j);
    double t = 0.0, scal = 0.0, beta = alpha;
    if (sigma2 != 0.0) {
      const double nrm = sqrt(alpha * alpha + sigma2);
      beta = alpha >= 0.0 ? -nrm : nrm;
      t = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    tau[j] = t;
    if (z != nullptr && lane == 0) z[j * S + j] = t;
    double v[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      if (k == 0) {
        v[0] = lane > j ? a[0][j] * scal : (lane == j ? 1.0 : 0.0);
        a[0][j] = lane > j ? v[0] : (lane == j ? beta : a[0][j]);
      } else {
        v[k] = a[k][j] * scal;
        a[k][j] = v[k];
      }
    }
    if constexpr (S > 1) {
      // v^T a[:, c] for the slots c, each pair (c, c + P/2) combined by the
      // first split of wave_sums as soon as both are formed
      double d[P];
#pragma unroll
      for (int c = 0; c < P / 2; ++c) {
        double lo = 0.0, hi = 0.0;
        const int c2 = c + P / 2;
        if (c < S && c != j && (c > j || z != nullptr)) {
#pragma unroll
          for (int k = 0; k < R; ++k) lo += v[k] * a[k][c];
        }
        if (c2 < S && c2 != j && (c2 > j || z != nullptr)) {
#pragma unroll
          for (int k = 0; k < R; ++k) hi += v[k] * a[k][c2];
        }
        d[c] = swap32_sum(lo, hi);
      }
      const double y = wave_sums<P, true>(d);
#pragma unroll
      for (int c = j + 1; c < S; ++c) {
        const double tw = t * bcast(y, c << SH);
#pragma unroll
        for (int k = 0; k < R; ++k) a[k][c] -= tw * v[k];
      }
      if (z != nullptr) {
#pragma unroll
        for (int c = 0; c < j; ++c) {
          const double zc = bcast(y, c << SH);
          if (lane == 0) z[c * S + j] = zc;
        }
      }
    }
  }
}

template <typename T, int S>
__device__ __forceinline__ void load_chunk(const T* __restrict__ v,
                                           int64_t ldv, int64_t m,
                                           int64_t row0,
                                           double (&a)[Geo<S>::R][S]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < Geo<S>::R; ++k) {
    const int64_t row = row0 + lane + 64 * k;
#pragma unroll
    for (int c = 0; c < S; ++c)
      a[k][c] = row < m ? static_cast<double>(v[(int64_t)c * ldv + row]) : 0.0;
  }
}

// Explicit rows of H_1 ... H_s [C; 0], handed row block by row block to
// store(k, c, value) (rows lane + 64 k, column c).  a[][] holds the factored
// chunk and is left unchanged; C (s x s) is read from cc (column-major) or
// is the identity when cc == nullptr.  lds: this wave's own 4 S^2 doubles,
// z and tau already filled by factor().  The s x s work runs on lanes < S
// with its operands in LDS; only the final product E - V W touches the
// register-resident rows.
template <int S, typename Store>
__device__ __forceinline__ void form_q(const double (&a)[Geo<S>::R][S],
                                       const double* __restrict__ cc,
                                       double* lds, Store store) {
  constexpr int R = Geo<S>::R;
  const int lane = threadIdx.x & 63;
  double* z = lds;                   // z[i * S + k] = v_i^T v_k, i < k
  double* vt = lds + S * S;          // vt[r * S + i] = v_i(r), r < S
  double* wl = lds + 2 * S * S;      // W, row-major
  double* cl = lds + 3 * S * S;      // C, row-major; tau in z's diagonal
  if (lane < S) {
#pragma unroll
    for (int i = 0; i < S; ++i) {
      vt[lane * S + i] = i < lane ? a[0][i] : (i == lane ? 1.0 : 0.0);
      cl[lane * S + i] = cc ? cc[i * S + lane] : (i == lane ? 1.0 : 0.0);
    }
  }
  wave_sync();
  if (lane < S) {
    const int c = lane;
#pragma unroll 1
    for (int i = S - 1; i >= 0; --i) {
      double u = cl[i * S + c];
      for (int r = i + 1; r < S; ++r) u += vt[r * S + i] * cl[r * S + c];
      for (int k = i + 1; k < S; ++k) u -= z[i * S + k] * wl[k * S + c];
      wl[i * S + c] = z[i * S + i] * u;
    }
  }
  wave_sync();
#pragma unroll 1
  for (int c = 0; c < S; ++c) {
    double wc[S];
#pragma unroll
    for (int i = 0; i < S; ++i) wc[i] = wl[i * S + c];
    const double e0 = lane < S ? cl[lane * S + c] : 0.0;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      double q = k == 0 ? e0 : 0.0;
#pragma unroll
      for (int i = 0; i < S; ++i) {
        const double vi =
            k > 0 ? a[k][i] : (i < lane ? a[0][i] : (i == lane ? 1.0 : 0.0));
        q -= vi * wc[i];
      }
      store(k, c, q);
    }
  }
}

// leaf pass: R factor of every chunk (column-major s x s); workgroup
// `block` of 256 threads, one chunk per wave
template <typename T, int S>
__device__ __forceinline__ void leaf_body(
    const T* __restrict__ v, int64_t ldv, int64_t m, int64_t nchunks,
    double* __restrict__ rleaf, int64_t block) {
  const int64_t chunk = block * 4 + (threadIdx.x >> 6);
  if (chunk >= nchunks) return;
  const int lane = threadIdx.x & 63;
  double a[Geo<S>::R][S], tau[S];
  load_chunk<T, S>(v, ldv, m, chunk * Geo<S>::L, a);
  factor<S>(a, tau, nullptr);
  if (lane < S) {
    double* out = rleaf + (size_t)chunk * S * S;
#pragma unroll
    for (int c = 0; c < S; ++c)
      st_r(out + c * S + lane, c >= lane ? a[0][c] : 0.0);
  }
}

// one upward level: node stacks children [node*fan, ...) of nprev; stores
// its R and its explicit Q (fan*s x s, column-major); the root normalizes
// signs (R <- D R, Q <- Q D) and also writes R to r_out.  lds: 4 * 4 S^2
// doubles of workgroup memory (one slice per wave).
template <int S>
__device__ __forceinline__ void node_wave(
    const double* __restrict__ rprev, int64_t nprev, int fan, int64_t node,
    double* __restrict__ rcur, double* __restrict__ qcur, int is_root,
    double* r_out, int64_t r_rs, int64_t r_cs, int32_t* syncs, double* my) {
  const int lane = threadIdx.x & 63;
  // the root completes the synchronization point of this TSQR
  if (is_root && syncs != nullptr && lane == 0) *syncs += 1;
  constexpr int R = Geo<S>::R;
  const int64_t c0 = node * fan;
  const int nch = (int)min((int64_t)fan, nprev - c0);
  const int rows = fan * S;
  double a[R][S], tau[S];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    // row i of the stack: row rr of child ch (column c at c * S)
    const int i = lane + 64 * k;
    const int ch = i / S, rr = i % S;
    const bool live = i < rows && ch < nch;
    const double* src = rprev + (size_t)(c0 + (live ? ch : 0)) * S * S + rr;
#pragma unroll
    for (int c = 0; c < S; ++c) a[k][c] = live ? src[c * S] : 0.0;
  }
  factor<S>(a, tau, my);
  // columns whose sign the root flips (bit c), the same on every lane
  unsigned neg = 0;
  if (is_root) {
#pragma unroll
    for (int c = 0; c < S; ++c)
      if (bcast(a[0][c], c) < 0.0) neg |= 1u << c;
  }
  if (lane < S) {
    double* rn = rcur + (size_t)node * S * S;
    const double mine = (neg >> lane) & 1 ? -1.0 : 1.0;   // this lane's row
#pragma unroll
    for (int c = 0; c < S; ++c) {
      const double val = (c >= lane ? a[0][c] : 0.0) * mine;
      st_r(rn + c * S + lane, val);
      if (is_root) r_out[lane * r_rs + c * r_cs] = val;
    }
  }
  double* qn = qcur + (size_t)node * rows * S;
  form_q<S>(a, nullptr, my, [&](int k, int c, double q) {
    const int i = lane + 64 * k;
    const double d = (neg >> c) & 1 ? -1.0 : 1.0;
    if (i < rows) qn[(size_t)c * rows + i] = q * d;
  });
}

// one node per wave: workgroup `block` of 256 threads takes nodes
// 4 block .. 4 block + 3
template <int S>
__device__ __forceinline__ void node_body(
    const double* __restrict__ rprev, int64_t nprev, int fan, int64_t nnodes,
    double* __restrict__ rcur, double* __restrict__ qcur, int is_root,
    double* r_out, int64_t r_rs, int64_t r_cs, int32_t* syncs, double* lds,
    int64_t block) {
  const int wv = threadIdx.x >> 6;
  const int64_t node = block * 4 + wv;
  if (node >= nnodes) return;
  node_wave<S>(rprev, nprev, fan, node, rcur, qcur, is_root, r_out, r_rs,
               r_cs, syncs, lds + wv * 4 * S * S);
}

// apply pass: explicit Q rows of every chunk, optionally in place (lds as
// for node_body)
template <typename T, int S>
__device__ __forceinline__ void apply_wave(
    const T* v, int64_t ldv, int64_t m, int64_t chunk,
    const double* __restrict__ cchunk, T* dst, int64_t ldd, double* my) {
  const int lane = threadIdx.x & 63;
  constexpr int R = Geo<S>::R;
  const int64_t row0 = chunk * Geo<S>::L;
  double a[R][S], tau[S];
  load_chunk<T, S>(v, ldv, m, row0, a);
  factor<S>(a, tau, my);
  form_q<S>(a, cchunk, my,
            [&](int k, int c, double q) {
              const int64_t row = row0 + lane + 64 * k;
              if (row < m) dst[(int64_t)c * ldd + row] = static_cast<T>(q);
            });
}

template <typename T, int S>
__device__ __forceinline__ void apply_body(
    const T* v, int64_t ldv, int64_t m, int64_t nchunks,
    const double* __restrict__ cleaf, T* dst, int64_t ldd, double* lds,
    int64_t block) {
  const int wv = threadIdx.x >> 6;
  const int64_t chunk = block * 4 + wv;
  if (chunk >= nchunks) return;
  apply_wave<T, S>(v, ldv, m, chunk, cleaf + (size_t)chunk * S * S, dst, ldd,
                   lds + wv * 4 * S * S);
}

// Coefficient block of leaf chunk `chunk` (S x S, column-major, into the
// wave's LDS slice out): the downward pass restricted to the chunk's path
// from the root, the same products in the same order as the per-level
// down kernels (C_child = Q_parent[child block] C_parent, the root's
// children taking their Q block).
template <int S>
__device__ __forceinline__ void path_coef(const TsqrPlan& tp,
                                          const double* ws, int64_t chunk,
                                          double* out) {
  const int lane = threadIdx.x & 63;
  const int L = tp.levels, fan = tp.fan, rows = fan * S;
  // ancestor of the chunk at level l: chunk / fan^l (wave-uniform)
  int64_t span = 1;                         // fan^(L - 1)
  for (int l = 1; l < L; ++l) span *= fan;
  constexpr int kPer = (S * S + 63) / 64;
  {
    const double* qb = ws + tp.q_off[L] + (size_t)((chunk / span) % fan) * S;
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const int e = lane + 64 * t;
      if (e < S * S) out[e] = qb[(size_t)(e / S) * rows + e % S];
    }
  }
  for (int l = L - 1; l >= 1; --l) {
    const int64_t below = span / fan;       // fan^(l - 1)
    const double* qb = ws + tp.q_off[l] + (size_t)(chunk / span) * rows * S +
                       (size_t)((chunk / below) % fan) * S;
    span = below;
    double v[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const int e = lane + 64 * t;
      double acc = 0.0;
      if (e < S * S) {
        const int c = e / S, r = e % S;
        for (int k = 0; k < S; ++k)
          acc += qb[(size_t)k * rows + r] * out[c * S + k];
      }
      v[t] = acc;
    }
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const int e = lane + 64 * t;
      if (e < S * S) out[e] = v[t];
    }
  }
}

template <typename T, int S>
__global__ __launch_bounds__(256) void leaf_kernel(
    const T* __restrict__ v, int64_t ldv, int64_t m, int64_t nchunks,
    double* __restrict__ rleaf) {
  leaf_body<T, S>(v, ldv, m, nchunks, rleaf, blockIdx.x);
}

// The whole upward tree in one launch (after the leaves): each wave
// factors one node of the first level, then counts itself in at the parent
// node; the wave that completes a node's children invalidates its caches
// at agent scope and factors that node, and goes on up, so the root is
// done by the last wave to arrive.  Node R factors are written through to
// the device level (st_r), so a wave's release is only the wait for its
// stores.  The counters (ints at tp.cnt_off) start at zero and are put
// back to zero by the wave that completes each node.
template <int S>
__global__ __launch_bounds__(256) void tree_kernel(
    TsqrPlan tp, double* ws, double* r_out, int64_t r_rs, int64_t r_cs,
    int32_t* syncs) {
  __shared__ double lds[4 * 4 * S * S];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t node = (int64_t)blockIdx.x * 4 + wv;
  if (node >= tp.nodes[1]) return;
  double* my = lds + wv * 4 * S * S;
  node_wave<S>(ws + tp.r_off[0], tp.nodes[0], tp.fan, node,
               ws + tp.r_off[1], ws + tp.q_off[1], tp.levels == 1 ? 1 : 0,
               r_out, r_rs, r_cs, syncs, my);
  int* cnt = reinterpret_cast<int*>(ws + tp.cnt_off);
  int64_t child = node, base = tp.nodes[1];
  for (int l = 2; l <= tp.levels; ++l) {
    const int64_t p = child / tp.fan;
    const int nch = (int)min((int64_t)tp.fan, tp.nodes[l - 1] - p * tp.fan);
    // this wave's node factor (written through) is complete
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    int old = 0;
    if (lane == 0) old = atomicAdd(&cnt[base + p], 1);
    old = __shfl(old, 0);
    if (old + 1 != nch) return;             // a sibling completes p
    if (lane == 0) cnt[base + p] = 0;
    // the siblings' factors: drop any stale cached copies
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    node_wave<S>(ws + tp.r_off[l - 1], tp.nodes[l - 1], tp.fan, p,
                 ws + tp.r_off[l], ws + tp.q_off[l], l == tp.levels ? 1 : 0,
                 r_out, r_rs, r_cs, syncs, my);
    base += tp.nodes[l];
    child = p;
  }
}

// Explicit Q of every chunk, each wave forming its chunk's coefficient
// block from the tree's Q factors along its path (no downward launches).
template <typename T, int S>
__global__ __launch_bounds__(256) void apply_path_kernel(
    const T* v, int64_t ldv, int64_t m, TsqrPlan tp, const double* ws,
    T* dst, int64_t ldd) {
  __shared__ double lds[4 * 4 * S * S + 4 * S * S];
  const int wv = threadIdx.x >> 6;
  const int64_t chunk = (int64_t)blockIdx.x * 4 + wv;
  if (chunk >= tp.nchunks) return;
  double* c = lds + 4 * 4 * S * S + wv * S * S;
  path_coef<S>(tp, ws, chunk, c);
  apply_wave<T, S>(v, ldv, m, chunk, c, dst, ldd, lds + wv * 4 * S * S);
}

}  // namespace tw

// downward pass of either TSQR form: C_child = Qnode_parent[child block] *
// C_parent (s x s, column-major); the root's C is the identity.  One child
// per workgroup (`block`); any number of threads.
__device__ __forceinline__ void tsqr_down_body(
    const double* __restrict__ qpar, const double* __restrict__ cpar,
    int64_t nchild, int fan, int s, double* __restrict__ cchild,
    int parent_is_root, int64_t block) {
  const int64_t child = block;
  const int64_t p = child / fan;
  const int idx_in = (int)(child % fan);
  const int rows = fan * s;
  const double* qb = qpar + (size_t)p * rows * s + (size_t)idx_in * s;
  const double* cp = cpar + (size_t)p * s * s;
  double* out = cchild + (size_t)child * s * s;
  for (int e = threadIdx.x; e < s * s; e += blockDim.x) {
    const int c = e / s, r = e % s;
    double acc;
    if (parent_is_root) {
      acc = qb[(size_t)c * rows + r];
    } else {
      acc = 0.0;
      for (int k = 0; k < s; ++k)
        acc += qb[(size_t)k * rows + r] * cp[c * s + k];
    }
    out[e] = acc;
  }
}

}  // namespace bcgs
