// Accuracy checker of a computed factorization X = Q R (the loss of
// orthogonality ||Q^T Q - I|| and the residual ||X - Q R|| / ||X|| of
// section 1 need three n x n Gram matrices; their 2-norms are the largest
// absolute eigenvalues, which the caller takes on the host).
//
//   E = X - Q R            residual_kernel: 64-row x 64-column tiles of E,
//                          FP64 16x16x4 MFMA over the upper triangle of R
//   G = M^T M              gram_check_kernel: workgroup (row range, 64 x 64
//                          output block of the upper triangle); each chunk
//                          of at most 4096 rows is one MFMA product, added
//                          to the running block with a compensated
//                          (two-sum) addition, so the sum over chunks loses
//                          O(u) whatever the row count
//                          gram_check_reduce: the row-range partials summed
//                          in fixed order, again compensated, and mirrored
//                          into the lower triangle
// The element type of X and Q is FP64 or binary32 (FP32-bulk results,
// widened to FP64 as they are read); everything else is FP64.
#include "common.h"

namespace bcgs {
namespace ck {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kChunk = 4096;       // rows per chunk product
constexpr int kBlk = 64;           // output block edge

__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Running sum s with accumulated rounding error c (Knuth's two-sum gives
// the exact error of each addition); the value is s + c.
__device__ __forceinline__ void two_sum_add(double& s, double& c, double t) {
  const double u = s + t;
  const double bp = u - s;
  c += (s - (u - bp)) + (t - bp);
  s = u;
}

template <typename T>
__device__ __forceinline__ double ld(const T* p, int64_t i) {
  return static_cast<double>(p[i]);
}

// E(:, c) = X(:, c) - Q(:, 0:c+1) R(0:c+1, c) for a 64 x 64 tile of E;
// grid (row tiles, column tiles).  Tiles through LDS in steps of 16 of K.
template <typename T>
__global__ __launch_bounds__(256) void residual_kernel(
    const T* __restrict__ X, int64_t ldx, const T* __restrict__ Q,
    int64_t ldq, const double* __restrict__ R, int64_t ldr, int64_t m,
    int64_t n, double* __restrict__ E, int64_t lde) {
  __shared__ double qs[16][kBlk + 1];    // K x rows
  __shared__ double rs[16][kBlk + 1];    // K x columns
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * kBlk;
  const int64_t c0 = (int64_t)blockIdx.y * kBlk;
  // wave w: rows r0 + 16 w .. +16, all 64 columns (four 16 x 16 tiles)
  v4d acc[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
  const int64_t kend = min(n, c0 + kBlk);     // R upper triangular
  for (int64_t k0 = 0; k0 < kend; k0 += 16) {
    for (int e = tid; e < 16 * kBlk; e += 256) {
      const int kk = e / kBlk, rr = e % kBlk;
      const int64_t row = r0 + rr, k = k0 + kk, col = c0 + rr;
      qs[kk][rr] = (row < m && k < n) ? ld(Q, k * ldq + row) : 0.0;
      rs[kk][rr] = (k < n && col < n && k <= col) ? R[col * ldr + k] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const double a = qs[4 * ks + lk][16 * w + li];
#pragma unroll
      for (int t = 0; t < 4; ++t)
        acc[t] = mfma(a, rs[4 * ks + lk][16 * t + li], acc[t]);
    }
    __syncthreads();
  }
  // acc[t][v] at lane l: row 16 w + lk + 4 v, column 16 t + li
#pragma unroll
  for (int t = 0; t < 4; ++t) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = r0 + 16 * w + lk + 4 * v, col = c0 + 16 * t + li;
      if (row < m && col < n)
        E[col * lde + row] = ld(X, col * ldx + row) - acc[t][v];
    }
  }
}

// Partial Gram of rows [g rows_per, (g+1) rows_per) for the 64 x 64 block
// (bi, bj), bi <= bj, of M^T M; grid (row ranges, upper blocks).  Each
// chunk of kChunk rows is accumulated by MFMA, then added to the running
// block with a compensated addition.  part: [range][block][64 x 64].
template <typename T>
__global__ __launch_bounds__(256) void gram_check_kernel(
    const T* __restrict__ M, int64_t ldm, int64_t m, int64_t n,
    int64_t rows_per, int nb, double* __restrict__ part) {
  __shared__ double as[16][kBlk + 1];
  __shared__ double bs[16][kBlk + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  // block index -> (bi, bj) in the upper triangle, row by row
  int blk = blockIdx.y, bi = 0;
  while (blk >= nb - bi) {
    blk -= nb - bi;
    ++bi;
  }
  const int bj = bi + blk;
  const int64_t ca = (int64_t)bi * kBlk, cb = (int64_t)bj * kBlk;
  const int64_t rb = (int64_t)blockIdx.x * rows_per;
  const int64_t re = min(m, rb + rows_per);
  double sum[4][4], cmp[4][4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) sum[t][v] = cmp[t][v] = 0.0;
  for (int64_t c0 = rb; c0 < re; c0 += kChunk) {
    const int64_t c1 = min(re, c0 + kChunk);
    v4d acc[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    for (int64_t k0 = c0; k0 < c1; k0 += 16) {
      for (int e = tid; e < 16 * kBlk; e += 256) {
        const int kk = e % 16, cc = e / 16;
        const int64_t row = k0 + kk;
        const bool in = row < c1;
        as[kk][cc] = (in && ca + cc < n) ? ld(M, (ca + cc) * ldm + row) : 0.0;
        bs[kk][cc] = (in && cb + cc < n) ? ld(M, (cb + cc) * ldm + row) : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const double a = as[4 * ks + lk][16 * w + li];
#pragma unroll
        for (int t = 0; t < 4; ++t)
          acc[t] = mfma(a, bs[4 * ks + lk][16 * t + li], acc[t]);
      }
      __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) two_sum_add(sum[t][v], cmp[t][v], acc[t][v]);
  }
  // sum[t][v] at lane l: row (A column) 16 w + lk + 4 v, column 16 t + li
  double* out = part + ((size_t)blockIdx.x * gridDim.y + blockIdx.y) *
                           (kBlk * kBlk);
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      out[(16 * w + lk + 4 * v) * kBlk + 16 * t + li] = sum[t][v] + cmp[t][v];
}

// G(i, j) = sum over row ranges of the partials (fixed order, compensated);
// both triangles written.  One thread per element of the upper triangle's
// blocks.
__global__ __launch_bounds__(256) void gram_check_reduce(
    const double* __restrict__ part, int nranges, int nblocks, int nb,
    int64_t n, double* __restrict__ G, int64_t ldg) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)nblocks * kBlk * kBlk) return;
  int blk = (int)(e / (kBlk * kBlk));
  const int within = (int)(e % (kBlk * kBlk));
  const int b = blk;
  int bi = 0;
  while (blk >= nb - bi) {
    blk -= nb - bi;
    ++bi;
  }
  const int bj = bi + blk;
  const int64_t i = (int64_t)bi * kBlk + within / kBlk;
  const int64_t j = (int64_t)bj * kBlk + within % kBlk;
  double s = 0.0, c = 0.0;
  for (int r = 0; r < nranges; ++r)
    two_sum_add(s, c, part[((size_t)r * nblocks + b) * (kBlk * kBlk) + within]);
  const double v = s + c;
  if (i < n && j < n) {
    G[j * ldg + i] = v;
    G[i * ldg + j] = v;
  }
}

}  // namespace ck

namespace {

struct CheckPlan {
  int64_t m, n;
  int nb, nblocks, nranges;
  int64_t rows_per;
  size_t off_e, off_part, bytes;
};

CheckPlan check_plan(int64_t m, int64_t n) {
  CheckPlan p{};
  p.m = m;
  p.n = n;
  p.nb = (int)cdiv(n, ck::kBlk);
  p.nblocks = p.nb * (p.nb + 1) / 2;
  // enough row ranges to fill the GPU with (ranges x blocks) workgroups
  const int64_t want = std::max<int64_t>(1, 1024 / p.nblocks);
  p.rows_per = round_up64(cdiv(m, want), ck::kChunk);
  p.nranges = (int)cdiv(m, p.rows_per);
  size_t off = 0;
  p.off_e = off;
  off += (size_t)round_up64(m, 64) * n * sizeof(double);
  off = (off + 255) & ~size_t(255);
  p.off_part = off;
  off += (size_t)p.nranges * p.nblocks * ck::kBlk * ck::kBlk * sizeof(double);
  p.bytes = (off + 255) & ~size_t(255);
  return p;
}

template <typename T>
bcgs_status run_check(const CheckPlan& p, const T* X, int64_t ldx,
                      const T* Q, int64_t ldq, const double* R, int64_t ldr,
                      double* GQ, double* GE, double* GX, int64_t ldg,
                      char* ws, hipStream_t st) {
  double* E = reinterpret_cast<double*>(ws + p.off_e);
  double* part = reinterpret_cast<double*>(ws + p.off_part);
  const int64_t lde = round_up64(p.m, 64);
  hipLaunchKernelGGL(ck::residual_kernel<T>,
                     dim3((unsigned)cdiv(p.m, ck::kBlk), (unsigned)p.nb),
                     dim3(256), 0, st, X, ldx, Q, ldq, R, ldr, p.m, p.n, E,
                     lde);
  const dim3 grid((unsigned)p.nranges, (unsigned)p.nblocks);
  const unsigned rblocks =
      (unsigned)cdiv((int64_t)p.nblocks * ck::kBlk * ck::kBlk, 256);
  auto gram = [&](auto* M, int64_t ldm, double* G) {
    using E_t = std::remove_cv_t<std::remove_pointer_t<decltype(M)>>;
    hipLaunchKernelGGL(ck::gram_check_kernel<E_t>, grid, dim3(256), 0, st, M,
                       ldm, p.m, p.n, p.rows_per, p.nb, part);
    hipLaunchKernelGGL(ck::gram_check_reduce, dim3(rblocks), dim3(256), 0,
                       st, part, p.nranges, p.nblocks, p.nb, p.n, G, ldg);
  };
  gram(Q, ldq, GQ);
  gram(static_cast<const double*>(E), lde, GE);
  gram(X, ldx, GX);
  return hipGetLastError() == hipSuccess ? BCGS_OK : BCGS_ERR_HIP;
}

}  // namespace
}  // namespace bcgs

using namespace bcgs;

extern "C" {

size_t bcgs_check_workspace_size(int64_t m, int64_t n) {
  if (m < 1 || n < 1 || m < n) return 0;
  return check_plan(m, n).bytes;
}

bcgs_status bcgs_check(const void* X, int64_t ldx, const void* Q,
                       int64_t ldq, const double* R, int64_t ldr, int64_t m,
                       int64_t n, bcgs_precision precision, double* GQ,
                       double* GE, double* GX, int64_t ldg, void* workspace,
                       size_t ws_bytes, hipStream_t stream) {
  if (!X || !Q || !R || !GQ || !GE || !GX || !workspace) return BCGS_ERR_ARG;
  if (m < 1 || n < 1 || m < n || ldx < m || ldq < m || ldr < n || ldg < n)
    return BCGS_ERR_ARG;
  if (precision != BCGS_FP64 && precision != BCGS_FP32_BULK)
    return BCGS_ERR_ARG;
  const CheckPlan p = check_plan(m, n);
  if (ws_bytes < p.bytes || reinterpret_cast<uintptr_t>(workspace) % 256)
    return BCGS_ERR_ARG;
  char* ws = static_cast<char*>(workspace);
  if (precision == BCGS_FP64)
    return run_check(p, static_cast<const double*>(X), ldx,
                     static_cast<const double*>(Q), ldq, R, ldr, GQ, GE, GX,
                     ldg, ws, stream);
  return run_check(p, static_cast<const float*>(X), ldx,
                   static_cast<const float*>(Q), ldq, R, ldr, GQ, GE, GX, ldg,
                   ws, stream);
}

}  // extern "C"
