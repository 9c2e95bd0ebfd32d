// Small-matrix work between two device-wide reductions (one workgroup).
//
// Reads the reduced Gram matrix of the last synchronization and produces the
// coefficients the next streaming pass needs, plus one block column of R:
//   - Pythagorean Cholesky  Y_kk = chol(Omega - Y^T Y),
//                           S_kk = chol(T - S^T S)           (Alg. 1, Alg. 2)
//   - delayed normalization S_{1:k,k+1} = [Z; Y_kk^{-T}(P - Y^T Z)]  (eq. (1))
//   - R assembly            R_{1:k,k+1} = S + Y S_kk, R_kk = Y_kk S_kk
// A Cholesky pivot that is not strictly positive and finite is a breakdown:
// the first one is recorded in bcgs_info and the factor is filled with NaN,
// which then propagates; nothing waits on the host.
//
// Coefficient matrices (C1, C2: K x s; T1, T2: s x s upper) are row-major
// with row stride sp; the Gram matrix is column-major with leading
// dimension gld; R is column-major with leading dimension ldr.
#include <math.h>

#include "common.h"

namespace bcgs {

struct EpiSmem {
  double A[kMaxS * kMaxS];     // matrix being factored (row-major s x s)
  double B[kMaxS * kMaxS];     // scratch s x s
  double bc[4];
  int flag;
};

// Upper Cholesky of the s x s matrix in sm.A (row-major, symmetric); the
// factor overwrites sm.A's upper triangle and the lower part is zeroed.
// Returns through sm.flag: 0 ok, 1 breakdown (then sm.A is all NaN).
__device__ void chol_lds(EpiSmem& sm, int s, bcgs_info* info, int block,
                         int stage) {
  const int tid = threadIdx.x;
  if (tid == 0) sm.flag = 0;
  __syncthreads();
  for (int j = 0; j < s; ++j) {
    if (tid == 0) {
      const double d = sm.A[j * s + j];
      if (!(isfinite(d) && d > 0.0)) {
        if (sm.flag == 0 && info->status == BCGS_OK) {
          info->status = BCGS_ERR_BREAKDOWN;
          info->block = block;
          info->pivot = j;
          info->stage = stage;
          info->value = d;
        }
        sm.flag = 1;
      }
      sm.bc[0] = sqrt(d);
    }
    __syncthreads();
    const double r = sm.bc[0];
    for (int l = j + 1 + tid; l < s; l += kThreads) sm.A[j * s + l] /= r;
    __syncthreads();
    // trailing update A(i,l) -= R(j,i) R(j,l), j < i <= l
    const int t = s - j - 1;
    for (int e = tid; e < t * t; e += kThreads) {
      const int i = j + 1 + e / t, l = j + 1 + e % t;
      if (l >= i) sm.A[i * s + l] -= sm.A[j * s + i] * sm.A[j * s + l];
    }
    if (tid == 0) sm.A[j * s + j] = r;
    __syncthreads();
  }
  const bool bad = sm.flag != 0;
  for (int e = tid; e < s * s; e += kThreads) {
    const int i = e / s, l = e % s;
    if (bad) sm.A[e] = NAN;
    else if (l < i) sm.A[e] = 0.0;
  }
  __syncthreads();
}

__device__ __forceinline__ double gram_at(const EpiArgs& a, int r, int c) {
  return a.gram[(size_t)c * a.gld + r];
}

__device__ void store_tri(double* dst, int sp, int s, const double* src) {
  for (int e = threadIdx.x; e < sp * sp; e += kThreads) {
    const int i = e / sp, l = e % sp;
    dst[e] = (i < s && l < s) ? src[i * s + l] : 0.0;
  }
}

// R(0:js, j-block) = C2 + C1 * T2 ;  R(j-block, j-block) = T1 * T2
__device__ void assemble_r(const EpiArgs& a, const double* c1,
                           const double* c2, const double* t1,
                           const double* t2) {
  const int s = a.s, sp = a.sp, js = a.j * s;
  for (int e = threadIdx.x; e < js * s; e += kThreads) {
    const int i = e % js, c = e / js;
    double acc = c2[i * sp + c];
    for (int k = 0; k < s; ++k) acc += c1[i * sp + k] * t2[k * sp + c];
    a.r[(size_t)(js + c) * a.ldr + i] = acc;
  }
  for (int e = threadIdx.x; e < s * s; e += kThreads) {
    const int i = e % s, c = e / s;
    double acc = 0.0;
    if (i <= c)
      for (int k = i; k <= c; ++k) acc += t1[i * sp + k] * t2[k * sp + c];
    a.r[(size_t)(js + c) * a.ldr + js + i] = acc;
  }
}

// F = [-C T^{-1}; T^{-1}] (scaled) or [-C; I] (unscaled), C with K rows.
// T^{-1} by back substitution, one column per thread, in FP64.
__device__ void make_coef(EpiSmem& sm, double* F, const double* C, int K,
                          const double* T, int scaled, int s, int sp) {
  const int tid = threadIdx.x;
  double* Ti = sm.B;                  // s x s row-major
  if (scaled) {
    if (tid < s) {
      const int j = tid;
      for (int i = s - 1; i >= 0; --i) {
        double x = 0.0;
        if (i <= j) {
          x = (i == j) ? 1.0 : 0.0;
          for (int k = i + 1; k <= j; ++k) x -= T[i * sp + k] * Ti[k * s + j];
          x /= T[i * sp + i];
        }
        Ti[i * s + j] = x;
      }
    }
  } else {
    for (int e = tid; e < s * s; e += kThreads)
      Ti[e] = (e / s == e % s) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < K * sp; e += kThreads) {
    const int i = e / sp, c = e % sp;
    double v = 0.0;
    if (c < s) {
      if (scaled) {
        for (int k = 0; k <= c; ++k) v -= C[i * sp + k] * Ti[k * s + c];
      } else {
        v = -C[i * sp + c];
      }
    }
    F[e] = v;
  }
  for (int e = tid; e < s * sp; e += kThreads) {
    const int i = e / sp, c = e % sp;
    F[(size_t)(K + i) * sp + c] = c < s ? Ti[i * s + c] : 0.0;
  }
  __syncthreads();
}

__device__ void make_coefs(EpiSmem& sm, const EpiArgs& a) {
  __syncthreads();
  if (a.f1_mode != COEF_NONE)
    make_coef(sm, a.f1, a.c1, a.f1_rows, a.t1, a.f1_mode == COEF_SCALED,
              a.s, a.sp);
  if (a.f2_mode != COEF_NONE)
    make_coef(sm, a.f2, a.c2, a.f2_rows, a.t2, a.f2_mode == COEF_SCALED,
              a.s, a.sp);
}

__device__ void epilogue_body(EpiArgs a, EpiSmem& sm);

__global__ __launch_bounds__(kThreads) void epilogue_kernel(EpiArgs a) {
  __shared__ EpiSmem sm;
  epilogue_body(a, sm);
  make_coefs(sm, a);
}

__device__ void epilogue_body(EpiArgs a, EpiSmem& sm) {
  const int tid = threadIdx.x;
  const int s = a.s, sp = a.sp, js = a.j * s;

  if (a.mode == EPI_S_ONLY || a.mode == EPI_Y_ONLY) {
    double* dst = a.mode == EPI_S_ONLY ? a.c2 : a.c1;
    for (int e = tid; e < js * sp; e += kThreads) {
      const int i = e / sp, c = e % sp;
      dst[e] = c < s ? gram_at(a, i, c) : 0.0;
    }
    return;
  }

  if (a.mode == EPI_R_ASSEMBLE) {
    assemble_r(a, a.c1, a.c2, a.t1, a.t2);
    return;
  }

  if (a.mode == EPI_P1S_INIT) {
    // gram rows [0,s) = S_12, rows [s,2s) = T_2 (columns [0,s))
    for (int e = tid; e < s * sp; e += kThreads) {
      const int i = e / sp, c = e % sp;
      a.c2[e] = c < s ? gram_at(a, i, c) : 0.0;
    }
    for (int e = tid; e < s * s; e += kThreads) {
      const int x = e / s, y = e % s;
      double acc = gram_at(a, s + x, y);
      for (int k = 0; k < s; ++k) acc -= gram_at(a, k, x) * gram_at(a, k, y);
      sm.A[e] = acc;
    }
    __syncthreads();
    chol_lds(sm, s, a.info, 1, 0);
    store_tri(a.t2, sp, s, sm.A);
    return;
  }

  // EPI_ONE_SYNC, after [Q_{0:j-1} U_j (E)]^T [U_j (E)]:
  //   Y = G(0:js, 0:s)     Omega = G(js:js+s, 0:s)
  //   Z = G(0:js, s:2s)    P = G(js:js+s, s:2s)    T = G(js+s:js+2s, s:2s)
  // 1. Y_jj = chol(Omega - Y^T Y)
  for (int e = tid; e < s * s; e += kThreads) {
    const int x = e / s, y = e % s;
    double acc = gram_at(a, js + x, y);
    for (int k = 0; k < js; ++k) acc -= gram_at(a, k, x) * gram_at(a, k, y);
    sm.A[e] = acc;
  }
  __syncthreads();
  chol_lds(sm, s, a.info, a.j, 1);
  // 2. R block column j with the current S (C2, T2) and the new Y, Y_jj
  //    (C1/T1 are overwritten below, so write the new Y into C1 first)
  for (int e = tid; e < js * sp; e += kThreads) {
    const int i = e / sp, c = e % sp;
    a.c1[e] = c < s ? gram_at(a, i, c) : 0.0;
  }
  store_tri(a.t1, sp, s, sm.A);
  __syncthreads();
  assemble_r(a, a.c1, a.c2, a.t1, a.t2);
  __syncthreads();
  if (!a.has_e) return;
  // 3. eq. (1): lower block L = Y_jj^{-T} (P - Y^T Z), forward substitution
  //    with Y_jj^T (lower triangular), one column per thread
  for (int e = tid; e < s * s; e += kThreads) {
    const int x = e / s, y = e % s;
    double acc = gram_at(a, js + x, s + y);
    for (int k = 0; k < js; ++k) acc -= gram_at(a, k, x) * gram_at(a, k, s + y);
    sm.B[e] = acc;                    // M = P - Y^T Z (row-major)
  }
  __syncthreads();
  if (tid < s) {
    const int c = tid;
    for (int i = 0; i < s; ++i) {
      double acc = sm.B[i * s + c];
      for (int k = 0; k < i; ++k) acc -= sm.A[k * s + i] * sm.B[k * s + c];
      sm.B[i * s + c] = acc / sm.A[i * s + i];
    }
  }
  __syncthreads();
  // C2 <- [Z; L]
  for (int e = tid; e < (js + s) * sp; e += kThreads) {
    const int i = e / sp, c = e % sp;
    double v = 0.0;
    if (c < s) v = i < js ? gram_at(a, i, s + c) : sm.B[(i - js) * s + c];
    a.c2[e] = v;
  }
  if (!a.chol_s) return;
  __syncthreads();
  // 4. S_{j+1,j+1} = chol(T - S^T S) with S = [Z; L]
  double tmp[kMaxS * kMaxS / kThreads];
  int nt = 0;
  for (int e = tid; e < s * s; e += kThreads) {
    const int x = e / s, y = e % s;
    double acc = gram_at(a, js + s + x, s + y);
    for (int k = 0; k < js; ++k)
      acc -= gram_at(a, k, s + x) * gram_at(a, k, s + y);
    for (int k = 0; k < s; ++k) acc -= sm.B[k * s + x] * sm.B[k * s + y];
    tmp[nt++] = acc;
  }
  __syncthreads();
  nt = 0;
  for (int e = tid; e < s * s; e += kThreads) sm.A[e] = tmp[nt++];
  __syncthreads();
  chol_lds(sm, s, a.info, a.j + 1, 0);
  store_tri(a.t2, sp, s, sm.A);
}

hipError_t launch_epilogue(const EpiArgs& a, hipStream_t st) {
  prof_begin(BCGS_KERNEL_EPILOGUE, a.mode, 0.0, 0.0);
  hipLaunchKernelGGL(epilogue_kernel, dim3(1), dim3(kThreads), 0, st, a);
  prof_end();
  return hipGetLastError();
}

// p(i, j) = value for i < rows, j < cols of a column-major matrix with
// leading dimension ld (a kernel rather than a memset, so that the sequence
// can be captured in a HIP graph).
__global__ void fill_kernel(double* p, int64_t rows, int64_t cols, int64_t ld,
                            double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < rows * cols) p[(i / rows) * ld + i % rows] = v;
}

hipError_t launch_fill(double* p, int64_t rows, int64_t cols, int64_t ld,
                       double value, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  prof_begin(BCGS_KERNEL_OTHER, 0, 8.0 * rows * cols, 0.0);
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)cdiv(rows * cols, 256)),
                     dim3(256), 0, st, p, rows, cols, ld, value);
  prof_end();
  return hipGetLastError();
}

}  // namespace bcgs
