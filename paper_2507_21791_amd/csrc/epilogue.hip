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
#include "epilogue_impl.h"
#include "small_impl.h"

namespace bcgs {

hipError_t launch_epilogue(const EpiArgs& a, hipStream_t st) {
  if (rec_active()) {
    if (a.s == 4 || a.s == 8 || a.s == 16)
      rec_epi(a);
    else
      rec_unsupported();
    return hipSuccess;
  }
  prof_begin(BCGS_KERNEL_EPILOGUE, a.mode * 1000 + a.j, 0.0, 0.0);
  switch (a.s) {
#define EPI(S_) case S_: hipLaunchKernelGGL(epilogue_kernel<S_>, dim3(1), \
                                            dim3(kThreads), 0, st, a); \
                         prof_name("epilogue_kernel<%d>", S_); break;
    EPI(4) EPI(8) EPI(16) EPI(32)
#undef EPI
    default:
      hipLaunchKernelGGL(epilogue_kernel<0>, dim3(1), dim3(kThreads), 0, st,
                         a);
      prof_name("epilogue_kernel<0>");
  }
  prof_end();
  return hipGetLastError();
}

// p(i, j) = value for i < rows, j < cols of a column-major matrix with
// leading dimension ld (a kernel rather than a memset, so that the sequence
// can be captured in a HIP graph).
__global__ void fill_kernel(double* p, int64_t rows, int64_t cols, int64_t ld,
                            double v) {
  fill_body(p, rows, cols, ld, v, blockIdx.x);
}

hipError_t launch_fill(double* p, int64_t rows, int64_t cols, int64_t ld,
                       double value, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  if (rec_active()) {
    rec_fill(p, rows, cols, ld, value, cdiv(rows * cols, 256));
    return hipSuccess;
  }
  prof_begin(BCGS_KERNEL_OTHER, 0, 8.0 * rows * cols, 0.0);
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)cdiv(rows * cols, 256)),
                     dim3(256), 0, st, p, rows, cols, ld, value);
  prof_name("fill_kernel");
  prof_end();
  return hipGetLastError();
}

__global__ void split_coef_kernel(const double* __restrict__ F, int64_t K,
                                  int sp, int c0, double* __restrict__ fa,
                                  double* __restrict__ fb) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= K * 16) return;
  const int64_t k = e >> 4;
  const int c = (int)(e & 15);
  fa[e] = F[k * sp + c0 + c];
  fb[e] = F[k * sp + c0 + 16 + c];
}

hipError_t launch_split_coef(const double* F, int64_t K, int sp, int c0,
                             double* fa, double* fb, hipStream_t st) {
  if (K <= 0) return hipSuccess;
  prof_begin(BCGS_KERNEL_OTHER, 1, 8.0 * K * 32 * 2, 0.0);
  hipLaunchKernelGGL(split_coef_kernel, dim3((unsigned)cdiv(K * 16, 256)),
                     dim3(256), 0, st, F, K, sp, c0, fa, fb);
  prof_name("split_coef_kernel");
  prof_end();
  return hipGetLastError();
}

}  // namespace bcgs
