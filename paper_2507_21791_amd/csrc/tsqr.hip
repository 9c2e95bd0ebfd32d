// TSQR: the unconditionally stable intra-orthogonalization of the paper
// (section 1; used for X_1 by every variant, for both intra-
// orthogonalizations of BCGSI+ and for the first one of BCGSI+P-2S,
// section 2.3).
//
// The m x s block is cut into row chunks of `cr` rows.
//   leaf pass   each workgroup computes the Householder QR of its chunk and
//               stores the s x s factor R_c;
//   tree        levels of workgroups stack `fan` child R factors
//               (fan * s <= cr rows), factor them, and keep the node's
//               explicit Q (fan*s x s) and R; the root's R is sign-normalized
//               (positive diagonal, the unique factorization) and the signs
//               are folded into the root's Q;
//   downward    each node's coefficient C = (parent Q block) * C_parent;
//   apply pass  each workgroup recomputes its chunk's Householder QR
//               (bitwise the same reflectors) and forms the explicit rows
//               Q_chunk = H_1 ... H_s [C_c; 0].
// The single device-wide reduction of TSQR is its tree.
//
// Register-resident Householder: thread (c, g) of the workgroup owns column
// c of the chunk at the interleaved rows g, g + nseg, g + 2 nseg, ...
// (kRows values; nseg = 256 / s row segments, cr = kRows * nseg).  One
// Householder step publishes the pivot column to LDS, then every thread
// forms its partial dot product with the reflector over its rows; the
// partials of all columns are reduced in one LDS exchange.  Two barriers
// per step; every reduction is summed in a fixed order, so results are
// identical run to run.
#include "common.h"
#include "tsqr_wave_impl.h"

namespace bcgs {

namespace tq {

constexpr int kRows = 32;          // rows per thread
constexpr int kT = kThreads;       // 256

// S > 0: block width known at compile time (row offsets become immediates);
// S == 0: runtime block width.
template <int S>
struct Geo {
  int s, nseg, cr;
  int c, g;          // this thread's column and row segment (c < s valid)
  bool active;
  __device__ Geo(int s_) {
    s = S ? S : s_;
    nseg = S ? kT / S : kT / s_;
    cr = kRows * nseg;
    c = threadIdx.x / nseg;
    g = threadIdx.x % nseg;
    active = c < s;
  }
  __device__ int row(int k) const {
    return g + (S ? (kT / S) : nseg) * k;
  }
};

struct Smem {
  double* vbuf;    // [2][cr]  published pivot column / reflector
  double* red;     // [2][nseg] partial norms
  double* dots;    // [2][s * nseg] partial dot products
  double* tau;     // [kMaxS]
};

__host__ __device__ inline int lds_doubles(int s) {
  const int nseg = kT / s;
  const int cr = kRows * nseg;
  return 2 * cr + 2 * nseg + 2 * s * nseg + kMaxS;
}

__device__ inline Smem carve(double* lds, int s) {
  const int nseg = kT / s, cr = kRows * nseg;
  Smem m;
  m.vbuf = lds;
  m.red = m.vbuf + 2 * cr;
  m.dots = m.red + 2 * nseg;
  m.tau = m.dots + 2 * s * nseg;
  return m;
}

// Householder QR of the chunk held in a[] (column geo.c, rows geo.row(k)).
// Afterwards a[] holds R (rows < s on and above the diagonal) and the
// reflectors (below the diagonal, v_j(j) = 1 implicit); sm.tau the taus.
// LAPACK convention: H_j = I - tau_j v_j v_j^T, beta = -sign(alpha) norm.
template <int S>
__device__ void factor(double (&a)[kRows], const Geo<S>& geo, const Smem& sm) {
  const int s = geo.s, nseg = geo.nseg, cr = geo.cr;
  int par = 0;
  // publish column 0 and its partial norm (rows > 0)
  if (geo.c == 0) {
    double p = 0.0;
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const int i = geo.row(k);
      sm.vbuf[i] = a[k];
      if (i > 0) p += a[k] * a[k];
    }
    sm.red[geo.g] = p;
  }
  __syncthreads();
  for (int j = 0; j < s; ++j) {
    const double* vb = sm.vbuf + par * cr;
    const double* rd = sm.red + par * nseg;
    double* dt = sm.dots + par * s * nseg;
    double sigma2 = 0.0;
    for (int q = 0; q < nseg; ++q) sigma2 += rd[q];
    const double alpha = vb[j];
    double tau = 0.0, scal = 0.0, beta = alpha;
    if (sigma2 != 0.0) {
      const double nrm = sqrt(alpha * alpha + sigma2);
      beta = alpha >= 0.0 ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    if (threadIdx.x == 0) sm.tau[j] = tau;
    if (geo.active && geo.c > j) {
      // partial of w_c = sum_{i >= j} v_i a(i, c), v_j = 1
      double p = 0.0;
#pragma unroll
      for (int k = 0; k < kRows; ++k) {
        const int i = geo.row(k);
        if (i > j) p += vb[i] * scal * a[k];
        else if (i == j) p += a[k];
      }
      dt[geo.c * nseg + geo.g] = p;
    } else if (geo.c == j) {
#pragma unroll
      for (int k = 0; k < kRows; ++k) {
        const int i = geo.row(k);
        if (i > j && tau != 0.0) a[k] *= scal;
        else if (i == j) a[k] = beta;
      }
    }
    __syncthreads();
    if (geo.active && geo.c > j && tau != 0.0) {
      double w = 0.0;
      for (int q = 0; q < nseg; ++q) w += dt[geo.c * nseg + q];
      const double tw = tau * w;
#pragma unroll
      for (int k = 0; k < kRows; ++k) {
        const int i = geo.row(k);
        if (i > j) a[k] -= tw * (vb[i] * scal);
        else if (i == j) a[k] -= tw;
      }
    }
    if (geo.c == j + 1) {
      double* vn = sm.vbuf + (par ^ 1) * cr;
      double p = 0.0;
#pragma unroll
      for (int k = 0; k < kRows; ++k) {
        const int i = geo.row(k);
        vn[i] = a[k];
        if (i > j + 1) p += a[k] * a[k];
      }
      sm.red[(par ^ 1) * nseg + geo.g] = p;
    }
    __syncthreads();
    par ^= 1;
  }
}

// M <- H_0 ... H_{s-1} M for M held like a[] (column geo.c).  The reflectors
// are in v[] (the output of factor()).
template <int S>
__device__ void apply(const double (&v)[kRows], double (&M)[kRows],
                      const Geo<S>& geo, const Smem& sm) {
  const int s = geo.s, nseg = geo.nseg, cr = geo.cr;
  int par = 0;
  // publish reflector s-1
  if (geo.c == s - 1) {
#pragma unroll
    for (int k = 0; k < kRows; ++k) sm.vbuf[geo.row(k)] = v[k];
  }
  __syncthreads();
  for (int j = s - 1; j >= 0; --j) {
    const double* vb = sm.vbuf + par * cr;
    double* dt = sm.dots + par * s * nseg;
    const double tau = sm.tau[j];
    if (geo.active) {
      double p = 0.0;
#pragma unroll
      for (int k = 0; k < kRows; ++k) {
        const int i = geo.row(k);
        if (i > j) p += vb[i] * M[k];
        else if (i == j) p += M[k];
      }
      dt[geo.c * nseg + geo.g] = p;
    }
    __syncthreads();
    if (geo.active && tau != 0.0) {
      double w = 0.0;
      for (int q = 0; q < nseg; ++q) w += dt[geo.c * nseg + q];
      const double tw = tau * w;
#pragma unroll
      for (int k = 0; k < kRows; ++k) {
        const int i = geo.row(k);
        if (i > j) M[k] -= tw * vb[i];
        else if (i == j) M[k] -= tw;
      }
    }
    if (j > 0 && geo.c == j - 1) {
      double* vn = sm.vbuf + (par ^ 1) * cr;
#pragma unroll
      for (int k = 0; k < kRows; ++k) vn[geo.row(k)] = v[k];
    }
    __syncthreads();
    par ^= 1;
  }
}

template <typename T, int S>
__device__ void load_chunk(const T* __restrict__ v, int64_t ldv, int64_t m,
                           int64_t row0, const Geo<S>& geo,
                           double (&a)[kRows]) {
#pragma unroll
  for (int k = 0; k < kRows; ++k) {
    const int64_t row = row0 + geo.row(k);
    a[k] = (geo.active && row < m)
               ? static_cast<double>(v[(int64_t)geo.c * ldv + row])
               : 0.0;
  }
}

// leaf pass: R factor of every chunk (column-major s x s)
template <typename T, int S>
__global__ __launch_bounds__(kT) void leaf_kernel(
    const T* __restrict__ v, int64_t ldv, int64_t m, int s,
    double* __restrict__ rleaf) {
  extern __shared__ double lds[];
  const Geo<S> geo(s);
  const Smem sm = carve(lds, s);
  const int64_t chunk = blockIdx.x;
  double a[kRows];
  load_chunk(v, ldv, m, chunk * geo.cr, geo, a);
  factor(a, geo, sm);
  double* out = rleaf + (size_t)chunk * s * s;
  if (geo.active) {
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const int i = geo.row(k);
      if (i < s) out[geo.c * s + i] = i <= geo.c ? a[k] : 0.0;
    }
  }
}

// one upward tree level: node stacks children [node*fan, ...) of nprev
template <int S>
__global__ __launch_bounds__(kT) void node_kernel(
    const double* __restrict__ rprev, int64_t nprev, int fan, int s,
    double* __restrict__ rcur, double* __restrict__ qcur, int is_root,
    double* r_out, int64_t r_rs, int64_t r_cs, int32_t* syncs) {
  extern __shared__ double lds[];
  const Geo<S> geo(s);
  const Smem sm = carve(lds, s);
  const int64_t node = blockIdx.x;
  const int64_t c0 = node * fan;
  const int nch = (int)min((int64_t)fan, nprev - c0);
  const int rows = fan * s;
  double a[kRows], M[kRows];
#pragma unroll
  for (int k = 0; k < kRows; ++k) {
    const int i = geo.row(k);
    const int ch = i / s, rr = i % s;
    a[k] = (geo.active && i < rows && ch < nch)
               ? rprev[(size_t)(c0 + ch) * s * s + (size_t)geo.c * s + rr]
               : 0.0;
    M[k] = (geo.active && i == geo.c) ? 1.0 : 0.0;
  }
  factor(a, geo, sm);
  apply(a, M, geo, sm);
  // sign normalization at the root: R <- D R, Q <- Q D
  double* sgn = sm.vbuf;          // free again after apply()
  if (is_root && geo.active) {
#pragma unroll
    for (int k = 0; k < kRows; ++k)
      if (geo.row(k) == geo.c) sgn[geo.c] = a[k] < 0.0 ? -1.0 : 1.0;
  }
  __syncthreads();
  // the root completes the synchronization point of this TSQR
  if (is_root && syncs != nullptr && threadIdx.x == 0) *syncs += 1;
  if (!geo.active) return;
  double* rn = rcur + (size_t)node * s * s;
  double* qn = qcur + (size_t)node * rows * s;
  const double dc = is_root ? sgn[geo.c] : 1.0;
#pragma unroll
  for (int k = 0; k < kRows; ++k) {
    const int i = geo.row(k);
    if (i < s) {
      double val = i <= geo.c ? a[k] : 0.0;
      if (is_root) val *= sgn[i];
      rn[geo.c * s + i] = val;
      if (is_root) r_out[i * r_rs + geo.c * r_cs] = val;
    }
    if (i < rows) qn[(size_t)geo.c * rows + i] = M[k] * dc;
  }
}

// downward pass (the body is shared with the s <= 16 TSQR)
__global__ __launch_bounds__(kT) void down_kernel(
    const double* __restrict__ qpar, const double* __restrict__ cpar,
    int64_t nchild, int fan, int s, double* __restrict__ cchild,
    int parent_is_root) {
  tsqr_down_body(qpar, cpar, nchild, fan, s, cchild, parent_is_root,
                 blockIdx.x);
}

// apply pass: explicit Q rows of every chunk, optionally in place
template <typename T, int S>
__global__ __launch_bounds__(kT) void apply_kernel(
    const T* v, int64_t ldv, int64_t m, int s,
    const double* __restrict__ cleaf, T* dst, int64_t ldd) {
  extern __shared__ double lds[];
  const Geo<S> geo(s);
  const Smem sm = carve(lds, s);
  const int64_t chunk = blockIdx.x;
  const int64_t row0 = chunk * geo.cr;
  double a[kRows], M[kRows];
  load_chunk(v, ldv, m, row0, geo, a);
  const double* cc = cleaf + (size_t)chunk * s * s;
#pragma unroll
  for (int k = 0; k < kRows; ++k) {
    const int i = geo.row(k);
    M[k] = (geo.active && i < s) ? cc[geo.c * s + i] : 0.0;
  }
  factor(a, geo, sm);
  apply(a, M, geo, sm);
  if (!geo.active) return;
#pragma unroll
  for (int k = 0; k < kRows; ++k) {
    const int64_t row = row0 + geo.row(k);
    if (row < m) dst[(int64_t)geo.c * ldd + row] = static_cast<T>(M[k]);
  }
}

}  // namespace tq

int wave_tsqr_rows(int s);

template <typename T>
hipError_t launch_wave_tsqr(const TsqrPlan& tp, const T* v, int64_t ldv,
                            T* dst, int64_t ldd, int64_t m, double* ws,
                            double* r_out, int64_t r_rs, int64_t r_cs,
                            int32_t* syncs, hipStream_t st);

// s <= 16: one wave per chunk (tsqr_wave.hip); wider blocks: one workgroup
// per chunk (this file)
TsqrPlan make_tsqr_plan(int64_t m, int s) {
  TsqrPlan p{};
  p.s = s;
  const int nseg = kThreads / s;
  p.wave = s <= 16;
  p.cr = p.wave ? wave_tsqr_rows(s) : tq::kRows * nseg;
  p.fan = p.cr / s;
  if (p.fan < 2) p.fan = 2;
  p.nchunks = cdiv(m, p.cr);
  p.nodes[0] = p.nchunks;
  int l = 0;
  do {
    p.nodes[l + 1] = cdiv(p.nodes[l], p.fan);
    ++l;
  } while (p.nodes[l] > 1);
  p.levels = l;
  int64_t off = 0;
  const int64_t ss = (int64_t)s * s;
  for (int i = 0; i <= p.levels; ++i) {
    p.r_off[i] = off; off += p.nodes[i] * ss;
    p.c_off[i] = off; off += p.nodes[i] * ss;
    if (i >= 1) { p.q_off[i] = off; off += p.nodes[i] * (int64_t)p.fan * s * s; }
    else p.q_off[i] = -1;
  }
  int64_t ncnt = 0;
  for (int i = 1; i <= p.levels; ++i) ncnt += p.nodes[i];
  p.cnt_off = off;
  p.cnt_doubles = (ncnt + 1) / 2;
  off += p.cnt_doubles;
  p.total = off;
  return p;
}

// downward pass of the tree: coefficient blocks from the root to the leaves
void tsqr_down(const TsqrPlan& tp, double* ws, hipStream_t st) {
  const int s = tp.s, fan = tp.fan;
  const double ss = (double)s * s;
  for (int l = tp.levels; l >= 1; --l) {
    const double n = (double)tp.nodes[l - 1];
    if (rec_active()) {
      rec_tsqr_down(ws + tp.q_off[l], ws + tp.c_off[l], tp.nodes[l - 1], fan,
                    s, ws + tp.c_off[l - 1], l == tp.levels ? 1 : 0);
      continue;
    }
    prof_begin(BCGS_KERNEL_TSQR_DOWN, l, 8.0 * n * ss * 2, 2.0 * n * ss * s);
    hipLaunchKernelGGL(tq::down_kernel, dim3((unsigned)tp.nodes[l - 1]),
                       dim3(kThreads), 0, st, ws + tp.q_off[l],
                       ws + tp.c_off[l], tp.nodes[l - 1], fan, s,
                       ws + tp.c_off[l - 1], l == tp.levels ? 1 : 0);
    prof_name("tsqr_down_kernel");
    prof_end();
  }
}

template <typename T, int S>
static hipError_t launch_tsqr_s(const TsqrPlan& tp, const T* v, int64_t ldv,
                                T* dst, int64_t ldd, int64_t m, double* ws,
                                double* r_out, int64_t r_rs, int64_t r_cs,
                                int32_t* syncs, hipStream_t st) {
  if (rec_active()) {
    rec_unsupported();
    return hipSuccess;
  }
  const int s = tp.s, fan = tp.fan;
  const size_t lds = (size_t)tq::lds_doubles(s) * sizeof(double);
  const double ss = (double)s * s, esz = sizeof(T);
  // algorithmic work: Householder QR of the m x s block (2 m s^2) and the
  // formation of its explicit Q (2 m s^2); the tree is O(nchunks s^3)
  prof_begin(BCGS_KERNEL_TSQR_LEAF, 0, esz * m * s, 2.0 * m * ss);
  hipLaunchKernelGGL((tq::leaf_kernel<T, S>), dim3((unsigned)tp.nchunks),
                     dim3(kThreads), lds, st, v, ldv, m, s, ws + tp.r_off[0]);
  prof_name("tsqr_leaf_kernel<%s, %d>", type_name<T>(), S);
  prof_end();
  for (int l = 1; l <= tp.levels; ++l) {
    const double rows = (double)tp.nodes[l - 1] * s;
    prof_begin(BCGS_KERNEL_TSQR_NODE, l, 8.0 * rows * s * 2,
               4.0 * rows * ss);
    hipLaunchKernelGGL(tq::node_kernel<S>, dim3((unsigned)tp.nodes[l]),
                       dim3(kThreads), lds, st, ws + tp.r_off[l - 1],
                       tp.nodes[l - 1], fan, s, ws + tp.r_off[l],
                       ws + tp.q_off[l], l == tp.levels ? 1 : 0, r_out, r_rs,
                       r_cs, syncs);
    prof_name("tsqr_node_kernel<%d>", S);
    prof_end();
  }
  tsqr_down(tp, ws, st);
  prof_begin(BCGS_KERNEL_TSQR_APPLY, 0, 2.0 * esz * m * s, 2.0 * m * ss);
  hipLaunchKernelGGL((tq::apply_kernel<T, S>), dim3((unsigned)tp.nchunks),
                     dim3(kThreads), lds, st, v, ldv, m, s,
                     ws + tp.c_off[0], dst, ldd);
  prof_name("tsqr_apply_kernel<%s, %d>", type_name<T>(), S);
  prof_end();
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tsqr(const TsqrPlan& tp, const T* v, int64_t ldv, T* dst,
                       int64_t ldd, int64_t m, double* ws, double* r_out,
                       int64_t r_rs, int64_t r_cs, int32_t* syncs,
                       hipStream_t st) {
  if (tp.wave)
    return launch_wave_tsqr<T>(tp, v, ldv, dst, ldd, m, ws, r_out, r_rs, r_cs,
                               syncs, st);
  switch (tp.s) {
#define TQ(S_) case S_: return launch_tsqr_s<T, S_>(tp, v, ldv, dst, ldd, m, \
                                                    ws, r_out, r_rs, r_cs, \
                                                    syncs, st);
    TQ(1) TQ(2) TQ(4) TQ(8) TQ(16) TQ(32) TQ(64)
#undef TQ
    default:
      return launch_tsqr_s<T, 0>(tp, v, ldv, dst, ldd, m, ws, r_out, r_rs,
                                 r_cs, syncs, st);
  }
}

template hipError_t launch_tsqr<double>(const TsqrPlan&, const double*,
                                        int64_t, double*, int64_t, int64_t,
                                        double*, double*, int64_t, int64_t,
                                        int32_t*, hipStream_t);
template hipError_t launch_tsqr<float>(const TsqrPlan&, const float*,
                                        int64_t, float*, int64_t, int64_t,
                                        double*, double*, int64_t, int64_t,
                                        int32_t*, hipStream_t);

}  // namespace bcgs
