// TSQR: the unconditionally stable intra-orthogonalization of the paper
// (section 1; used for X_1 by every variant, for both intra-
// orthogonalizations of BCGSI+ and for the first one of BCGSI+P-2S,
// section 2.3).
//
// The m x s block is cut into row chunks of `cr` rows.
//   leaf pass   each workgroup computes the Householder QR of its chunk in
//               LDS and stores the s x s factor R_c;
//   tree        levels of workgroups stack `fan` child R factors
//               (fan * s rows), factor them, and keep the node's explicit
//               Q (fan*s x s) and R; the root's R is sign-normalized
//               (positive diagonal, the unique factorization) and the signs
//               are folded into the root's Q;
//   downward    each node's coefficient C = (parent Q block) * C_parent;
//   apply pass  each workgroup recomputes its chunk's Householder QR
//               (bitwise the same reflectors) and forms the explicit rows
//               Q_chunk = H_1 ... H_s [C_c; 0].
// The single device-wide reduction of TSQR is its tree.
#include "common.h"

namespace bcgs {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum one value over the workgroup (fixed order); result in every thread.
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = red[0];
#pragma unroll
  for (int w = 1; w < kWaves; ++w) t += red[w];
  return t;
}

// Householder QR (LAPACK convention: H_j = I - tau_j v_j v_j^T, v_j(j) = 1)
// of the rows x s matrix A (column-major in LDS, leading dimension lda).
// On return the upper triangle holds R, the strict lower part the v_j.
// `red` is LDS scratch of kWaves * (kMaxS + 1) doubles, `tau` s doubles.
__device__ void householder_lds(double* A, int lda, int rows, int s,
                                double* tau, double* red, double* bcast) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j = 0; j < s; ++j) {
    double* aj = A + (size_t)j * lda;
    double p = 0.0;
    for (int i = j + 1 + tid; i < rows; i += kThreads) p += aj[i] * aj[i];
    const double sigma2 = block_sum(p, red);
    if (tid == 0) {
      const double alpha = aj[j];
      double t = 0.0, scal = 0.0, beta = alpha;
      if (sigma2 != 0.0) {
        const double nrm = sqrt(alpha * alpha + sigma2);
        beta = alpha >= 0.0 ? -nrm : nrm;
        t = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
      tau[j] = t;
      bcast[0] = scal;
      bcast[1] = beta;
    }
    __syncthreads();
    const double scal = bcast[0], tj = tau[j];
    if (tj != 0.0)
      for (int i = j + 1 + tid; i < rows; i += kThreads) aj[i] *= scal;
    __syncthreads();
    if (tid == 0) aj[j] = bcast[1];
    if (tj == 0.0) { __syncthreads(); continue; }
    // w_c = A(j,c) + sum_{i>j} v_i A(i,c) for c > j, then rank-1 update
    const int nc = s - j - 1;
    for (int c = 0; c < nc; ++c) {
      const double* ac = A + (size_t)(j + 1 + c) * lda;
      double q = 0.0;
      for (int i = j + 1 + tid; i < rows; i += kThreads) q += aj[i] * ac[i];
      q = wave_sum(q);
      if (lane == 0) red[wave * (kMaxS + 1) + c] = q;
    }
    __syncthreads();
    if (tid < nc) {
      double t = A[(size_t)(j + 1 + tid) * lda + j];   // v_j(j) = 1 term
      for (int w = 0; w < kWaves; ++w) t += red[w * (kMaxS + 1) + tid];
      bcast[2 + tid] = tj * t;
    }
    __syncthreads();
    for (int c = 0; c < nc; ++c) {
      double* ac = A + (size_t)(j + 1 + c) * lda;
      const double tw = bcast[2 + c];
      if (tid == 0) ac[j] -= tw;
      for (int i = j + 1 + tid; i < rows; i += kThreads) ac[i] -= tw * aj[i];
    }
    __syncthreads();
  }
}

// M (rows x s, LDS, leading dimension ldm) <- H_0 ... H_{s-1} M, with the
// reflectors stored below the diagonal of A.
__device__ void apply_q_lds(const double* A, int lda, int rows, int s,
                            const double* tau, double* M, int ldm,
                            double* red, double* bcast) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j = s - 1; j >= 0; --j) {
    const double tj = tau[j];
    if (tj == 0.0) continue;
    const double* v = A + (size_t)j * lda;
    for (int c = 0; c < s; ++c) {
      const double* mc = M + (size_t)c * ldm;
      double q = 0.0;
      for (int i = j + 1 + tid; i < rows; i += kThreads) q += v[i] * mc[i];
      q = wave_sum(q);
      if (lane == 0) red[wave * (kMaxS + 1) + c] = q;
    }
    __syncthreads();
    if (tid < s) {
      double t = M[(size_t)tid * ldm + j];
      for (int w = 0; w < kWaves; ++w) t += red[w * (kMaxS + 1) + tid];
      bcast[2 + tid] = tj * t;
    }
    __syncthreads();
    for (int c = 0; c < s; ++c) {
      double* mc = M + (size_t)c * ldm;
      const double tw = bcast[2 + c];
      if (tid == 0) mc[j] -= tw;
      for (int i = j + 1 + tid; i < rows; i += kThreads) mc[i] -= tw * v[i];
    }
    __syncthreads();
  }
}

struct TsqrSmem {
  double* A; double* M; double* tau; double* red; double* bcast;
};

__device__ TsqrSmem carve(double* lds, int rows, int s, bool with_m) {
  TsqrSmem t;
  t.A = lds;
  t.M = t.A + (size_t)rows * s;
  t.tau = t.M + (with_m ? (size_t)rows * s : 0);
  t.red = t.tau + kMaxS;
  t.bcast = t.red + kWaves * (kMaxS + 1);
  return t;
}

static size_t tsqr_lds_bytes(int rows, int s, bool with_m) {
  return ((size_t)rows * s * (with_m ? 2 : 1) + kMaxS +
          kWaves * (kMaxS + 1) + kMaxS + 2) * sizeof(double);
}

template <typename T>
__device__ void load_chunk(const T* __restrict__ v, int64_t ldv, int64_t m,
                           int64_t row0, int cr, int s, double* A) {
  for (int idx = threadIdx.x; idx < cr * s; idx += kThreads) {
    const int c = idx / cr, r = idx % cr;
    const int64_t row = row0 + r;
    A[(size_t)c * cr + r] =
        row < m ? static_cast<double>(v[(int64_t)c * ldv + row]) : 0.0;
  }
  __syncthreads();
}

// leaf pass: R factor of every chunk
template <typename T>
__global__ __launch_bounds__(kThreads) void tsqr_leaf_kernel(
    const T* __restrict__ v, int64_t ldv, int64_t m, int cr, int s,
    double* __restrict__ rleaf) {
  extern __shared__ double lds[];
  TsqrSmem sm = carve(lds, cr, s, false);
  const int64_t chunk = blockIdx.x;
  load_chunk(v, ldv, m, chunk * cr, cr, s, sm.A);
  householder_lds(sm.A, cr, cr, s, sm.tau, sm.red, sm.bcast);
  double* out = rleaf + (size_t)chunk * s * s;   // column-major s x s
  for (int idx = threadIdx.x; idx < s * s; idx += kThreads) {
    const int c = idx / s, r = idx % s;
    out[idx] = r <= c ? sm.A[(size_t)c * cr + r] : 0.0;
  }
}

// one upward tree level: node i stacks children [i*fan, min((i+1)*fan, nprev))
__global__ __launch_bounds__(kThreads) void tsqr_node_kernel(
    const double* __restrict__ rprev, int64_t nprev, int fan, int s,
    double* __restrict__ rcur, double* __restrict__ qcur, int is_root,
    double* r_out, int64_t r_rs, int64_t r_cs) {
  extern __shared__ double lds[];
  const int rows = fan * s;
  TsqrSmem sm = carve(lds, rows, s, true);
  const int64_t node = blockIdx.x;
  const int64_t c0 = node * fan;
  const int nch = (int)min((int64_t)fan, nprev - c0);
  const int nrows = nch * s;
  for (int idx = threadIdx.x; idx < rows * s; idx += kThreads) {
    const int c = idx / rows, r = idx % rows;
    const int ch = r / s, rr = r % s;
    sm.A[(size_t)c * rows + r] =
        ch < nch ? rprev[(size_t)(c0 + ch) * s * s + (size_t)c * s + rr] : 0.0;
    sm.M[(size_t)c * rows + r] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  householder_lds(sm.A, rows, nrows, s, sm.tau, sm.red, sm.bcast);
  apply_q_lds(sm.A, rows, nrows, s, sm.tau, sm.M, rows, sm.red, sm.bcast);
  // sign normalization at the root: R <- D R, Q <- Q D
  if (is_root && threadIdx.x < s) {
    const int j = threadIdx.x;
    sm.bcast[2 + j] = sm.A[(size_t)j * rows + j] < 0.0 ? -1.0 : 1.0;
  }
  __syncthreads();
  double* rn = rcur + (size_t)node * s * s;
  for (int idx = threadIdx.x; idx < s * s; idx += kThreads) {
    const int c = idx / s, r = idx % s;
    double val = r <= c ? sm.A[(size_t)c * rows + r] : 0.0;
    if (is_root) val *= sm.bcast[2 + r];
    rn[idx] = val;
    if (is_root) r_out[r * r_rs + c * r_cs] = val;
  }
  double* qn = qcur + (size_t)node * rows * s;
  for (int idx = threadIdx.x; idx < rows * s; idx += kThreads) {
    const int c = idx / rows;
    double val = sm.M[idx];
    if (is_root) val *= sm.bcast[2 + c];
    qn[idx] = val;
  }
}

// downward: C_child = Qnode_parent[child block] * C_parent (all s x s,
// column-major); the root's C is the identity.
__global__ __launch_bounds__(kThreads) void tsqr_down_kernel(
    const double* __restrict__ qpar, const double* __restrict__ cpar,
    int64_t nchild, int fan, int s, double* __restrict__ cchild,
    int parent_is_root) {
  const int64_t child = blockIdx.x;
  const int64_t p = child / fan;
  const int idx_in = (int)(child % fan);
  const int rows = fan * s;
  const double* qb = qpar + (size_t)p * rows * s + (size_t)idx_in * s;
  const double* cp = cpar + (size_t)p * s * s;
  double* out = cchild + (size_t)child * s * s;
  for (int e = threadIdx.x; e < s * s; e += kThreads) {
    const int c = e / s, r = e % s;
    double acc;
    if (parent_is_root) {
      acc = qb[(size_t)c * rows + r];
    } else {
      acc = 0.0;
      for (int k = 0; k < s; ++k) acc += qb[(size_t)k * rows + r] * cp[c * s + k];
    }
    out[e] = acc;
  }
}

// apply pass: explicit Q rows of every chunk, optionally in place
template <typename T>
__global__ __launch_bounds__(kThreads) void tsqr_apply_kernel(
    const T* v, int64_t ldv, int64_t m, int cr, int s,
    const double* __restrict__ cleaf, T* dst, int64_t ldd) {
  extern __shared__ double lds[];
  TsqrSmem sm = carve(lds, cr, s, true);
  const int64_t chunk = blockIdx.x;
  const int64_t row0 = chunk * cr;
  load_chunk(v, ldv, m, row0, cr, s, sm.A);
  householder_lds(sm.A, cr, cr, s, sm.tau, sm.red, sm.bcast);
  const double* cc = cleaf + (size_t)chunk * s * s;
  for (int idx = threadIdx.x; idx < cr * s; idx += kThreads) {
    const int c = idx / cr, r = idx % cr;
    sm.M[idx] = r < s ? cc[c * s + r] : 0.0;
  }
  __syncthreads();
  apply_q_lds(sm.A, cr, cr, s, sm.tau, sm.M, cr, sm.red, sm.bcast);
  for (int idx = threadIdx.x; idx < cr * s; idx += kThreads) {
    const int c = idx / cr, r = idx % cr;
    const int64_t row = row0 + r;
    if (row < m) dst[(int64_t)c * ldd + row] = static_cast<T>(sm.M[idx]);
  }
}

TsqrPlan make_tsqr_plan(int64_t m, int s) {
  TsqrPlan p{};
  p.s = s;
  int cr = 64;
  while (cr * 2 * s <= 8192 && cr < 2048) cr *= 2;
  while (cr < 2 * s) cr *= 2;
  p.cr = cr;
  p.fan = cr / s;
  p.nchunks = cdiv(m, cr);
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
  p.total = off;
  return p;
}

template <typename K>
static void allow_big_lds(K kern) {
  (void)hipFuncSetAttribute((const void*)kern,
                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

template <typename T>
hipError_t launch_tsqr(const TsqrPlan& tp, const T* v, int64_t ldv, T* dst,
                       int64_t ldd, int64_t m, double* ws, double* r_out,
                       int64_t r_rs, int64_t r_cs, hipStream_t st) {
  static bool once = false;
  if (!once) {
    allow_big_lds(tsqr_leaf_kernel<T>);
    allow_big_lds(tsqr_apply_kernel<T>);
    allow_big_lds(tsqr_node_kernel);
    once = true;
  }
  const int s = tp.s, cr = tp.cr, fan = tp.fan;
  const double ss = (double)s * s, esz = sizeof(T);
  // algorithmic work: Householder QR of the m x s block (2 m s^2) and the
  // formation of its explicit Q (2 m s^2); the tree is O(nchunks s^3)
  prof_begin(BCGS_KERNEL_TSQR_LEAF, 0, esz * m * s, 2.0 * m * ss);
  hipLaunchKernelGGL(tsqr_leaf_kernel<T>, dim3((unsigned)tp.nchunks),
                     dim3(kThreads), tsqr_lds_bytes(cr, s, false), st, v, ldv,
                     m, cr, s, ws + tp.r_off[0]);
  prof_end();
  for (int l = 1; l <= tp.levels; ++l) {
    const double rows = (double)tp.nodes[l - 1] * s;
    prof_begin(BCGS_KERNEL_TSQR_NODE, l, 8.0 * rows * s * 2,
               4.0 * rows * ss);
    hipLaunchKernelGGL(tsqr_node_kernel, dim3((unsigned)tp.nodes[l]),
                       dim3(kThreads), tsqr_lds_bytes(fan * s, s, true), st,
                       ws + tp.r_off[l - 1], tp.nodes[l - 1], fan, s,
                       ws + tp.r_off[l], ws + tp.q_off[l],
                       l == tp.levels ? 1 : 0, r_out, r_rs, r_cs);
    prof_end();
  }
  for (int l = tp.levels; l >= 1; --l) {
    const double n = (double)tp.nodes[l - 1];
    prof_begin(BCGS_KERNEL_TSQR_DOWN, l, 8.0 * n * ss * 2, 2.0 * n * ss * s);
    hipLaunchKernelGGL(tsqr_down_kernel, dim3((unsigned)tp.nodes[l - 1]),
                       dim3(kThreads), 0, st, ws + tp.q_off[l],
                       ws + tp.c_off[l], tp.nodes[l - 1], fan, s,
                       ws + tp.c_off[l - 1], l == tp.levels ? 1 : 0);
    prof_end();
  }
  prof_begin(BCGS_KERNEL_TSQR_APPLY, 0, 2.0 * esz * m * s, 2.0 * m * ss);
  hipLaunchKernelGGL(tsqr_apply_kernel<T>, dim3((unsigned)tp.nchunks),
                     dim3(kThreads), tsqr_lds_bytes(cr, s, true), st, v, ldv,
                     m, cr, s, ws + tp.c_off[0], dst, ldd);
  prof_end();
  return hipGetLastError();
}

template hipError_t launch_tsqr<double>(const TsqrPlan&, const double*,
                                        int64_t, double*, int64_t, int64_t,
                                        double*, double*, int64_t, int64_t,
                                        hipStream_t);

}  // namespace bcgs
