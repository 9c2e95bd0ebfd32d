// Device code of the epilogue (the s x s work between two reductions):
// included by epilogue.hip (its kernel) and by the batched persistent
// kernel, which runs the same body as a work item.
#pragma once

#include <math.h>

#include "common.h"

namespace bcgs {

// LDS of one epilogue (the storage the kernel declares)
struct EpiSmem {
  double A[kMaxS * kMaxS];     // matrix being factored (row-major s x s)
  double B[kMaxS * kMaxS];     // scratch s x s
  double P[256];               // 16 x 16 right operand of mm16
  // s <= 16, one-sync epilogue: the factors stay in LDS for the
  // coefficient matrices (all s x s row-major, stride s)
  double T1[256], T2[256], T1i[256], T2i[256], L[256], N[256];
  double P2[512];              // 32 x 16 right operand of mmk<32>
  double bc[4];
  int flag;
};

// Where the epilogue's LDS arrays are: all inside one EpiSmem for the
// epilogue kernel; spread over the batched persistent kernel's LDS buffers
// there (A, P and the factors in one, B in another).
struct EpiView {
  double *A, *B, *P, *T1, *T2, *T1i, *T2i, *L, *N, *P2, *bc;
  int* flag;
};

__device__ __forceinline__ EpiView view_of(EpiSmem& m) {
  return EpiView{m.A, m.B, m.P, m.T1, m.T2, m.T1i, m.T2i, m.L, m.N, m.P2,
                 m.bc, &m.flag};
}

typedef double v4d __attribute__((ext_vector_type(4)));

// Upper Cholesky of the s x s matrix in sm.A (row-major, symmetric); the
// factor overwrites sm.A's upper triangle and the lower part is zeroed.
// Returns through sm.flag: 0 ok, 1 breakdown (then sm.A is all NaN).
__device__ void chol_lds(const EpiView& sm, int s, bcgs_info* info, int block,
                         int stage) {
  const int tid = threadIdx.x;
  if (tid == 0) *sm.flag = 0;
  __syncthreads();
  for (int j = 0; j < s; ++j) {
    if (tid == 0) {
      const double d = sm.A[j * s + j];
      if (!(isfinite(d) && d > 0.0)) {
        if (*sm.flag == 0 && info->status == BCGS_OK) {
          info->status = BCGS_ERR_BREAKDOWN;
          info->block = block;
          info->pivot = j;
          info->stage = stage;
          info->value = d;
        }
        *sm.flag = 1;
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
  const bool bad = *sm.flag != 0;
  for (int e = tid; e < s * s; e += kThreads) {
    const int i = e / s, l = e % s;
    if (bad) sm.A[e] = NAN;
    else if (l < i) sm.A[e] = 0.0;
  }
  __syncthreads();
}

__device__ __forceinline__ double lane_bcast(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// The same factorization by wave 0 alone for s <= 32 and s = 64: lane
// l holds column l in registers, the pivot and the row of R are broadcast
// with readlane, so no step needs a barrier.  Same breakdown rule, same
// record in bcgs_info, same NaN fill.
template <int S>
__device__ void chol_wave(const EpiView& sm, bcgs_info* info, int block,
                          int stage) {
  if (threadIdx.x < 64) {
    const int l = threadIdx.x;
    double col[S];
#pragma unroll
    for (int i = 0; i < S; ++i) col[i] = l < S ? sm.A[i * S + l] : 0.0;
    bool bad = false;
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const double d = lane_bcast(col[j], j);
      if (!(isfinite(d) && d > 0.0) && !bad) {
        if (l == 0 && info->status == BCGS_OK) {
          info->status = BCGS_ERR_BREAKDOWN;
          info->block = block;
          info->pivot = j;
          info->stage = stage;
          info->value = d;
        }
        bad = true;
      }
      const double r = sqrt(d);
      const double rj = l > j ? col[j] / r : (l == j ? r : col[j]);
      col[j] = rj;                         // R(j, l)
#pragma unroll
      for (int i = j + 1; i < S; ++i) {
        const double rji = lane_bcast(rj, i);   // R(j, i)
        if (l >= i) col[i] -= rji * rj;
      }
    }
    if (l < S) {
#pragma unroll
      for (int i = 0; i < S; ++i)
        sm.A[i * S + l] = bad ? NAN : (i <= l ? col[i] : 0.0);
    }
  }
  __syncthreads();
}

template <int S>
__device__ __forceinline__ void chol(const EpiView& sm, int s, bcgs_info* info,
                                     int block, int stage) {
  if constexpr (S > 0 && S <= 32) {
    chol_wave<S>(sm, info, block, stage);
  } else if constexpr (S == 0) {
    if (s == 64) chol_wave<64>(sm, info, block, stage);
    else chol_lds(sm, s, info, block, stage);
  } else {
    chol_lds(sm, s, info, block, stage);
  }
}

// T^{-1} of the upper triangular s x s matrix T (row-major, LDS) into Ti:
// lane j of wave `w` forms column j by back substitution in registers.
template <int S>
__device__ void tri_inv_wave(const double* T, double* Ti, int w = 0) {
  if ((threadIdx.x >> 6) == w) {
    const int j = threadIdx.x & 63;
    double x[S];
#pragma unroll
    for (int i = S - 1; i >= 0; --i) {
      double v = i == j ? 1.0 : 0.0;
#pragma unroll
      for (int k = i + 1; k < S; ++k) v -= T[i * S + k] * x[k];
      x[i] = i <= j ? v / T[i * S + i] : 0.0;
    }
    if (j < S) {
#pragma unroll
      for (int i = 0; i < S; ++i) Ti[i * S + j] = x[i];
    }
  }
}

__device__ __forceinline__ double gram_at(const EpiArgs& a, int r, int c) {
  return a.gram[(size_t)c * a.gld + r];
}

// out(x, y) = sum_{r < js} G(r, ca + x) G(r, cb + y) for x, y < s (s a
// multiple of 16; out row-major with stride s, in LDS) on the FP64
// 16x16x4 MFMA: the 16 x 16 output tiles go round-robin to the waves, each
// running over all js rows (K = 4 rows per step; the Gram rows are read
// from global memory, where they are L2 resident).
__device__ void gram_mfma(const EpiArgs& a, int js, int ca, int cb, int s,
                          double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nb = s >> 4, ntile = nb * nb;
  constexpr int kT = (kMaxS / 16) * (kMaxS / 16) / kWaves;
  v4d acc[kT];
#pragma unroll
  for (int i = 0; i < kT; ++i) acc[i] = v4d{0.0, 0.0, 0.0, 0.0};
  const int nsteps = (js + 3) >> 2;
  // the operand loads of kG steps are issued before their MFMAs (the
  // accumulation order is that of one step after the other)
  constexpr int kG = 4;
  for (int t0 = 0; t0 < nsteps; t0 += kG) {
    double xs[kG][kT], ys[kG][kT];
#pragma unroll
    for (int u = 0; u < kG; ++u) {
      const int r = 4 * (t0 + u) + lk;
#pragma unroll
      for (int i = 0; i < kT; ++i) {
        const int id = wave + kWaves * i;
        const int bx = id / nb, by = id % nb;
        const bool live = id < ntile && r < js;
        xs[u][i] = live ? gram_at(a, r, ca + 16 * bx + li) : 0.0;
        ys[u][i] = live ? gram_at(a, r, cb + 16 * by + li) : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < kG; ++u) {
      if (t0 + u >= nsteps) break;                    // wave-uniform
#pragma unroll
      for (int i = 0; i < kT; ++i) {
        if (wave + kWaves * i < ntile)
          acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(xs[u][i], ys[u][i],
                                                        acc[i], 0, 0, 0);
      }
    }
  }
  // acc[i][v] at lane l: output row 16 bx + l / 16 + 4 v, column 16 by + l % 16
#pragma unroll
  for (int i = 0; i < kT; ++i) {
    const int id = wave + kWaves * i;
    if (id < ntile) {
      const int bx = id / nb, by = id % nb;
#pragma unroll
      for (int v = 0; v < 4; ++v)
        out[(16 * bx + lk + 4 * v) * s + 16 * by + li] = acc[i][v];
    }
  }
  __syncthreads();
}

// Y^T Y, Y^T Z and Z^T Z over the js Gram rows for s = 32 (Y = Gram columns
// [0, 32), Z = [32, 64); only Y^T Y without Z) in one sweep: each wave owns
// the same 16 x 16 tile (bx, by) of the three products and runs one MFMA
// chain per product over all rows, the tile sequence of gram_mfma (so the
// same sums), with the Gram loads of kG steps issued before their MFMAs.
// out: the three products row-major, 32 x 32 each, one after another.
__device__ __forceinline__ void gram_three32(const EpiArgs& a, int js,
                                             bool has_e, double* out) {
  constexpr int s = 32, kG = 8;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int bx = wave >> 1, by = wave & 1;
  v4d yy = {0.0, 0.0, 0.0, 0.0}, yz = yy, zz = yy;
  const int nsteps = (js + 3) >> 2;
  for (int t0 = 0; t0 < nsteps; t0 += kG) {
    double yb[kG], yc[kG], zb[kG], zc[kG];
#pragma unroll
    for (int u = 0; u < kG; ++u) {
      const int r = 4 * (t0 + u) + lk;
      const bool live = r < js;
      yb[u] = live ? gram_at(a, r, 16 * bx + li) : 0.0;
      yc[u] = live ? gram_at(a, r, 16 * by + li) : 0.0;
      zb[u] = live && has_e ? gram_at(a, r, s + 16 * bx + li) : 0.0;
      zc[u] = live && has_e ? gram_at(a, r, s + 16 * by + li) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kG; ++u) {
      if (t0 + u >= nsteps) break;                    // wave-uniform
      yy = __builtin_amdgcn_mfma_f64_16x16x4f64(yb[u], yc[u], yy, 0, 0, 0);
      if (has_e) {
        yz = __builtin_amdgcn_mfma_f64_16x16x4f64(yb[u], zc[u], yz, 0, 0, 0);
        zz = __builtin_amdgcn_mfma_f64_16x16x4f64(zb[u], zc[u], zz, 0, 0, 0);
      }
    }
  }
  // acc[v] at lane l: row 16 bx + l / 16 + 4 v, column 16 by + l % 16
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int e = (16 * bx + lk + 4 * v) * s + 16 * by + li;
    out[e] = yy[v];
    if (has_e) {
      out[s * s + e] = yz[v];
      out[2 * s * s + e] = zz[v];
    }
  }
  __syncthreads();
}

// Tall-by-small products on the FP64 16x16x4 MFMA, for block widths
// S = 4, 8, 16: out(i, c, v) receives v = sum_{k < S} A(i, k) P(k, c) for
// i < rows and c < 16, with P a 16 x 16 row-major LDS matrix that is zero
// outside its S x S corner (so columns c >= S come out zero).  Row blocks
// of 16 go round-robin to the waves; a_at(i, k) is called only for
// i < rows, k < S.  Operand layout: A[l % 16][l / 16], B[l / 16][l % 16],
// result v at lane l: row l / 16 + 4 v, column l % 16.
template <int S, class FA, class FO>
__device__ __forceinline__ void mm16(int rows, FA a_at, const double* P,
                                     FO out) {
  static_assert(S % 4 == 0 && S <= 32, "whole 16x16x4 K-steps");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  for (int rb = wave; rb * 16 < rows; rb += kWaves) {
    const int i = rb * 16 + li;
    double av[S / 4];
#pragma unroll
    for (int q = 0; q < S / 4; ++q)
      av[q] = i < rows ? a_at(i, 4 * q + lk) : 0.0;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < S / 4; ++q)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], P[(4 * q + lk) * 16 + li],
                                                 acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = rb * 16 + lk + 4 * v;
      if (r < rows) out(r, li, acc[v]);
    }
  }
}

// mm16 with a run-time K (a multiple of 4, at most kMaxS): out(i, c, v)
// receives sum_{k < K} A(i, k) P(k, c) for i < rows and c < 16, P a K x 16
// row-major LDS matrix; the loads of eight K-steps are issued before their
// MFMAs.
template <class FA, class FO>
__device__ __forceinline__ void mm16_rt(int rows, int K, FA a_at,
                                        const double* P, FO out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int nq = K >> 2;
  for (int rb = wave; rb * 16 < rows; rb += kWaves) {
    const int i = rb * 16 + li;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    for (int q0 = 0; q0 < nq; q0 += 8) {
      double av[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        av[u] = (i < rows && q0 + u < nq) ? a_at(i, 4 * (q0 + u) + lk) : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (q0 + u >= nq) break;                      // wave-uniform
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(
            av[u], P[(4 * (q0 + u) + lk) * 16 + li], acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = rb * 16 + lk + 4 * v;
      if (r < rows) out(r, li, acc[v]);
    }
  }
}

// P <- the S x S row-major matrix M (leading dimension ldm), zero-padded
// to 16 x 16
template <int S>
__device__ __forceinline__ void load_p(const EpiView& sm, const double* M,
                                       int ldm) {
  for (int e = threadIdx.x; e < 256; e += kThreads) {
    const int k = e >> 4, c = e & 15;
    sm.P[e] = (k < S && c < S) ? M[k * ldm + c] : 0.0;
  }
}

// W^T W over the js rows of W = Gram columns [0, w) (w = 2S with the E
// block, else S), split into the S x S blocks Y^T Y, Y^T Z, Z^T Z of
// W = [Y Z]: one 16x16x4 MFMA chain per 16 x 16 block, the rows dealt to
// the waves in 4-row steps, the four wave partials summed in a fixed order
// in LDS (scr: 4 x 3 x 256 doubles).  Thread e < S*S receives entry
// (e / S, e % S) of each block.
template <int S>
__device__ __forceinline__ void gram_products(const EpiArgs& a, int js,
                                              bool has_e, double* scr,
                                              double& yy, double& yz,
                                              double& zz) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int w = has_e ? 2 * S : S;
  v4d b00 = {0.0, 0.0, 0.0, 0.0}, b01 = b00, b11 = b00;
  const int nsteps = (js + 3) / 4;
  // column li of the first 16-column block; for S = 16 also of the second.
  // This wave's steps t = wave, wave + kWaves, ...: the Gram loads of kG of
  // them are issued before their MFMAs (the accumulation order is that of
  // one step after the other).
  const int c0 = li, c1 = 16 + li;
  constexpr int kG = 8;
  const bool two = S == 16 && has_e;
  for (int t0 = wave; t0 < nsteps; t0 += kG * kWaves) {
    double x0[kG], x1[kG];
#pragma unroll
    for (int u = 0; u < kG; ++u) {
      const int r = 4 * (t0 + kWaves * u) + lk;
      x0[u] = (r < js && c0 < w) ? gram_at(a, r, c0) : 0.0;
      x1[u] = (two && r < js) ? gram_at(a, r, c1) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kG; ++u) {
      if (t0 + kWaves * u >= nsteps) break;           // wave-uniform
      b00 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0[u], x0[u], b00, 0, 0, 0);
      if (two) {
        b01 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0[u], x1[u], b01, 0, 0,
                                                   0);
        b11 = __builtin_amdgcn_mfma_f64_16x16x4f64(x1[u], x1[u], b11, 0, 0,
                                                   0);
      }
    }
  }
  double* mine = scr + wave * 3 * 256;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int e = (lk + 4 * v) * 16 + li;
    mine[e] = b00[v];
    mine[256 + e] = b01[v];
    mine[512 + e] = b11[v];
  }
  __syncthreads();
  const int e = threadIdx.x;
  if (e < S * S) {
    const int x = e / S, y = e % S;
    // block and offset of (x, y) in Y^T Y, (x, S + y) in Y^T Z and
    // (S + x, S + y) in Z^T Z
    auto sum = [&](int blk, int row, int col) {
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < kWaves; ++q)
        v += scr[q * 3 * 256 + blk * 256 + row * 16 + col];
      return v;
    };
    yy = sum(0, x, y);
    if (has_e) {
      yz = S == 16 ? sum(1, x, y) : sum(0, x, S + y);
      zz = S == 16 ? sum(2, x, y) : sum(0, S + x, S + y);
    }
  }
  __syncthreads();
}

// Coefficient matrices of the one-sync epilogue for s = S <= 16, from
// LDS-resident factors (no round trip through the global copies written
// by the same kernel):
//   F1 = [-Y T1^{-1}; T1^{-1}]   (Y = Gram rows [0, js), columns [0, S))
// and, when the next pass also forms U_{j+1}, F2 with F1 folded in
// (fold_coefs): with M = -L T2^{-1} and N = T1^{-1} M,
//   F2'(0:js)       = Z (-T2^{-1}) + Y (-N)   (one product of K = 2S)
//   F2'(js:js+S)    = N
//   F2'(js+S:js+2S) = T2^{-1}
// where T2 = S_{j+1,j+1} (scaled) or I, Z = Gram columns [S, 2S).
template <int S>
__device__ __forceinline__ void coefs_fused(const EpiView& sm,
                                            const EpiArgs& a, int js) {
  const int tid = threadIdx.x;
  const bool two = a.f2_mode != COEF_NONE;
  const bool scaled2 = a.f2_mode == COEF_SCALED;
  __syncthreads();
  tri_inv_wave<S>(sm.T1, sm.T1i, 0);
  if (two && scaled2) {
    tri_inv_wave<S>(sm.T2, sm.T2i, 1);
  } else if (two) {
    for (int e = tid; e < S * S; e += kThreads)
      sm.T2i[e] = (e / S == e % S) ? 1.0 : 0.0;
  }
  __syncthreads();
  // F1 rows [0, js): -Y T1^{-1}; rows [js, js+S): T1^{-1}
  for (int e = tid; e < 256; e += kThreads) {
    const int k = e >> 4, c = e & 15;
    sm.P[e] = (k < S && c < S) ? -sm.T1i[k * S + c] : 0.0;
  }
  if (two) {
    // M = -L T2^{-1} into sm.N for now (T2^{-1} upper triangular)
    if (tid < S * S) {
      const int x = tid / S, y = tid % S;
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < S; ++k) acc -= sm.L[x * S + k] * sm.T2i[k * S + y];
      sm.A[tid] = acc;
    }
  }
  __syncthreads();
  mm16<S>(
      js, [&](int i, int k) { return gram_at(a, i, k); }, sm.P,
      [&](int i, int c, double v) { a.f1[(size_t)i * 16 + c] = v; });
  for (int e = tid; e < S * 16; e += kThreads) {
    const int i = e / 16, c = e % 16;
    a.f1[(size_t)(js + i) * 16 + c] = c < S ? sm.T1i[i * S + c] : 0.0;
  }
  if (!two) return;
  // N = T1^{-1} M (T1^{-1} upper triangular)
  if (tid < S * S) {
    const int x = tid / S, y = tid % S;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < S; ++k) acc += sm.T1i[x * S + k] * sm.A[k * S + y];
    sm.N[tid] = acc;
  }
  __syncthreads();
  // right operand [-T2^{-1}; -N] (2S x 16, zero beyond S columns)
  for (int e = tid; e < 2 * S * 16; e += kThreads) {
    const int k = e >> 4, c = e & 15;
    double v = 0.0;
    if (c < S) v = k < S ? -sm.T2i[k * S + c] : -sm.N[(k - S) * S + c];
    sm.P2[e] = v;
  }
  __syncthreads();
  mm16<2 * S>(
      js,
      [&](int i, int k) {
        return k < S ? gram_at(a, i, S + k) : gram_at(a, i, k - S);
      },
      sm.P2, [&](int i, int c, double v) { a.f2[(size_t)i * 16 + c] = v; });
  for (int e = tid; e < 2 * S * 16; e += kThreads) {
    const int i = e / 16, c = e % 16;
    double v = 0.0;
    if (c < S) v = i < S ? sm.N[i * S + c] : sm.T2i[(i - S) * S + c];
    a.f2[(size_t)(js + i) * 16 + c] = v;
  }
}

__device__ __forceinline__ void store_identity(double* dst, int sp, int s) {
  for (int e = threadIdx.x; e < sp * sp; e += kThreads) {
    const int i = e / sp, l = e % sp;
    dst[e] = (i == l && i < s) ? 1.0 : 0.0;
  }
}

__device__ __forceinline__ void store_tri(double* dst, int sp, int s,
                                          const double* src) {
  for (int e = threadIdx.x; e < sp * sp; e += kThreads) {
    const int i = e / sp, l = e % sp;
    dst[e] = (i < s && l < s) ? src[i * s + l] : 0.0;
  }
}

// R(0:js, j-block) = C2 + C1 * T2 ;  R(j-block, j-block) = T1 * T2
// T1 (s x s row-major) is already in LDS; T2 is copied to sm.B.  One row of
// C1 / C2 per thread: the row is loaded whole into registers (S > 0: the
// block width is a compile-time constant and the loops unroll).
template <int S>
__device__ __forceinline__ void assemble_r(const EpiView& sm,
                                           const EpiArgs& a, const double* c1,
                                           const double* c2, const double* T1,
                                           const double* t2,
                                           bool c1_is_gram = false) {
  const int s = S ? S : a.s, sp = a.sp, js = a.j * s;
  double* T2 = sm.B;
  __syncthreads();
  for (int e = threadIdx.x; e < s * s; e += kThreads)
    T2[e] = t2[(e / s) * sp + e % s];
  __syncthreads();
  if constexpr (S == 4 || S == 8 || S == 16) {
    load_p<S>(sm, T2, S);
    __syncthreads();
    // R(i, js + c) = C2(i, c) + sum_k C1(i, k) T2(k, c) on the 16x16x4 MFMA
    // (as mm16), row blocks of 16 dealt to the waves; the C1 and C2 loads
    // of kG of a wave's row blocks are issued before their MFMAs
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lk = lane >> 4;
    constexpr int kG = 4;
    for (int rb0 = wave; rb0 * 16 < js; rb0 += kG * kWaves) {
      double av[kG][S / 4], cv[kG][4];
#pragma unroll
      for (int g = 0; g < kG; ++g) {
        const int rb = rb0 + kWaves * g;
        const int i = rb * 16 + li;
#pragma unroll
        for (int q = 0; q < S / 4; ++q)
          av[g][q] = i < js ? (c1_is_gram ? gram_at(a, i, 4 * q + lk)
                                          : c1[(size_t)i * sp + 4 * q + lk])
                            : 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = rb * 16 + lk + 4 * v;
          cv[g][v] = (r < js && li < S) ? c2[(size_t)r * sp + li] : 0.0;
        }
      }
#pragma unroll
      for (int g = 0; g < kG; ++g) {
        const int rb = rb0 + kWaves * g;
        if (rb * 16 >= js) break;                     // wave-uniform
        v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < S / 4; ++q)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(
              av[g][q], sm.P[(4 * q + lk) * 16 + li], acc, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = rb * 16 + lk + 4 * v;
          if (r < js && li < S)
            a.r[(size_t)(js + li) * a.ldr + r] = acc[v] + cv[g][v];
        }
      }
    }
  } else if constexpr (S == 32) {
    // R(i, js + c) = C2(i, c) + sum_k C1(i, k) T2(k, c), one 16-column
    // block of T2 at a time, on the 16x16x4 MFMA
    for (int cb = 0; cb < 2; ++cb) {
      for (int e = threadIdx.x; e < 512; e += kThreads)
        sm.P2[e] = T2[(e >> 4) * 32 + 16 * cb + (e & 15)];
      __syncthreads();
      mm16<32>(
          js, [&](int i, int k) { return c1[(size_t)i * sp + k]; }, sm.P2,
          [&](int i, int c, double v) {
            a.r[(size_t)(js + 16 * cb + c) * a.ldr + i] =
                v + c2[(size_t)i * sp + 16 * cb + c];
          });
      __syncthreads();
    }
  } else if (S == 0 && s % 16 == 0) {
    // run-time s (48, 64): R(i, js + c) = C2(i, c) + sum_k C1(i, k) T2(k, c)
    // on the MFMA, per 16-column block of T2 and K range of 32 rows (the
    // 32 x 16 operand in sm.P2), the later K ranges added to R
    for (int cb = 0; cb < s / 16; ++cb) {
      for (int k0 = 0; k0 < s; k0 += 32) {
        const int kc = min(32, s - k0);
        for (int e = threadIdx.x; e < kc * 16; e += kThreads)
          sm.P2[e] = T2[(k0 + (e >> 4)) * s + 16 * cb + (e & 15)];
        __syncthreads();
        mm16_rt(
            js, kc,
            [&](int i, int k) { return c1[(size_t)i * sp + k0 + k]; }, sm.P2,
            [&](int i, int c, double v) {
              double* o = a.r + (size_t)(js + 16 * cb + c) * a.ldr + i;
              *o = (k0 == 0 ? c2[(size_t)i * sp + 16 * cb + c] : *o) + v;
            });
        __syncthreads();
      }
    }
  } else
  for (int i = threadIdx.x; i < js; i += kThreads) {
    double y[S ? S : kMaxS];
#pragma unroll
    for (int k = 0; k < s; ++k) y[k] = c1[(size_t)i * sp + k];
    // column loop kept rolled: the T2 column is re-read from LDS per
    // column instead of the whole matrix being held in registers
#pragma unroll 1
    for (int c = 0; c < s; ++c) {
      double acc = c2[(size_t)i * sp + c];
      if constexpr (S > 0) {
#pragma unroll
        for (int k = 0; k < S; ++k)
          if (k <= c) acc += y[k] * T2[k * S + c];
      } else {
        for (int k = 0; k <= c; ++k) acc += y[k] * T2[k * s + c];
      }
      a.r[(size_t)(js + c) * a.ldr + i] = acc;
    }
  }
  for (int e = threadIdx.x; e < s * s; e += kThreads) {
    const int i = e % s, c = e / s;
    double acc = 0.0;
    if (i <= c)
      for (int k = i; k <= c; ++k) acc += T1[i * s + k] * T2[k * s + c];
    a.r[(size_t)(js + c) * a.ldr + js + i] = acc;
  }
  __syncthreads();
}

// F = [-C T^{-1}; T^{-1}] (scaled) or [-C; I] (unscaled), C with K rows.
// T^{-1} by back substitution, one column per thread, in FP64.
template <int S>
__device__ __forceinline__ void make_coef(const EpiView& sm, double* F,
                                          const double* C, int K,
                                          const double* T, int scaled, int s_,
                                          int sp) {
  const int tid = threadIdx.x, s = S ? S : s_;
  double* Ti = sm.B;                  // s x s row-major
  double* Tl = sm.A;                  // LDS copy of T (s x s row-major)
  if (scaled) {
    for (int e = tid; e < s * s; e += kThreads)
      Tl[e] = T[(e / s) * sp + e % s];
    __syncthreads();
    if constexpr (S > 0 && S <= 32) {
      tri_inv_wave<S>(Tl, Ti);
    } else if (tid < s) {
      const int j = tid;
      for (int i = s - 1; i >= 0; --i) {
        double x = 0.0;
        if (i <= j) {
          x = (i == j) ? 1.0 : 0.0;
          for (int k = i + 1; k <= j; ++k) x -= Tl[i * s + k] * Ti[k * s + j];
          x /= Tl[i * s + i];
        }
        Ti[i * s + j] = x;
      }
    }
  } else {
    for (int e = tid; e < s * s; e += kThreads)
      Ti[e] = (e / s == e % s) ? 1.0 : 0.0;
  }
  __syncthreads();
  if constexpr (S == 4 || S == 8 || S == 16) {
    // F(0:K, :) = -C T^{-1} (Ti is the identity when unscaled)
    load_p<S>(sm, Ti, S);
    __syncthreads();
    mm16<S>(
        K, [&](int i, int k) { return C[(size_t)i * sp + k]; }, sm.P,
        [&](int i, int c, double v) { F[(size_t)i * sp + c] = -v; });
  } else if constexpr (S == 32) {
    // F(0:K, :) = -C T^{-1}, one 16-column block of T^{-1} at a time
    for (int cb = 0; cb < 2; ++cb) {
      for (int e = tid; e < 512; e += kThreads)
        sm.P2[e] = Ti[(e >> 4) * 32 + 16 * cb + (e & 15)];
      __syncthreads();
      mm16<32>(
          K, [&](int i, int k) { return C[(size_t)i * sp + k]; }, sm.P2,
          [&](int i, int c, double v) {
            F[(size_t)i * sp + 16 * cb + c] = -v;
          });
      __syncthreads();
    }
  } else if (S == 0 && s % 16 == 0) {
    // run-time s (48, 64): F(0:K, :) = -C T^{-1} on the MFMA, one 16-column
    // block of T^{-1} at a time staged in sm.A (free after the inverse)
    for (int cb = 0; cb < s / 16; ++cb) {
      for (int e = tid; e < s * 16; e += kThreads)
        sm.A[e] = Ti[(e >> 4) * s + 16 * cb + (e & 15)];
      __syncthreads();
      mm16_rt(
          K, s, [&](int i, int k) { return C[(size_t)i * sp + k]; }, sm.A,
          [&](int i, int c, double v) {
            F[(size_t)i * sp + 16 * cb + c] = -v;
          });
      __syncthreads();
    }
  } else
  // one row of C per thread: F(i, :) = -C(i, :) T^{-1}  (or -C(i, :))
  for (int i = tid; i < K; i += kThreads) {
    double cr[S ? S : kMaxS];
#pragma unroll
    for (int k = 0; k < s; ++k) cr[k] = C[(size_t)i * sp + k];
    double* fr = F + (size_t)i * sp;
#pragma unroll 1
    for (int c = 0; c < sp; ++c) {
      double v = 0.0;
      if (c < s) {
        if constexpr (S > 0) {
#pragma unroll
          for (int k = 0; k < S; ++k) {
            if (scaled && k <= c) v -= cr[k] * Ti[k * S + c];
            if (!scaled && k == c) v = -cr[k];
          }
        } else if (scaled) {
          for (int k = 0; k <= c; ++k) v -= cr[k] * Ti[k * s + c];
        } else {
          v = -cr[c];
        }
      }
      fr[c] = v;
    }
  }
  for (int e = tid; e < s * sp; e += kThreads) {
    const int i = e / sp, c = e % sp;
    F[(size_t)(K + i) * sp + c] = c < s ? Ti[i * s + c] : 0.0;
  }
  __syncthreads();
}

// The next pass forms B1 = [Q_{0:j-1} U_j] F1 (which replaces U_j) and
// B2 = [Q_{0:j} X] F2 in one sweep over the staged columns [Q_{0:j-1} U_j X],
// so B2 is rewritten on them: the rows of F2 that multiply the new block
// (rows K1 .. K1+s-1, K1 = f1_rows) are replaced by F1 times those rows,
//   F2'(0 : K1+s) = [F2(0 : K1); 0] + F1 F2(K1 : K1+s),
// the same product in exact arithmetic.  One row of F1 per thread.
template <int S>
__device__ __forceinline__ void fold_coefs(const EpiView& sm,
                                           const EpiArgs& a) {
  const int s = S ? S : a.s, sp = a.sp, K1 = a.f1_rows;
  double* M = sm.A;                   // F2(K1 : K1+s), s x s row-major
  if constexpr (S == 4 || S == 8 || S == 16) {
    load_p<S>(sm, a.f2 + (size_t)K1 * sp, sp);
    __syncthreads();
    mm16<S>(
        K1 + s, [&](int i, int k) { return a.f1[(size_t)i * sp + k]; },
        sm.P, [&](int i, int c, double v) {
          double* o = a.f2 + (size_t)i * sp + c;
          *o = (i < K1 ? *o : 0.0) + v;
        });
    __syncthreads();
    return;
  }
  for (int e = threadIdx.x; e < s * s; e += kThreads)
    M[e] = a.f2[(size_t)(K1 + e / s) * sp + e % s];
  __syncthreads();
  if (S == 0 && s % 16 == 0) {
    // run-time s (48, 64): one 16-column block of M at a time, staged in
    // sm.B, on the 16x16x4 MFMA
    for (int cb = 0; cb < s / 16; ++cb) {
      for (int e = threadIdx.x; e < s * 16; e += kThreads)
        sm.B[e] = M[(e >> 4) * s + 16 * cb + (e & 15)];
      __syncthreads();
      mm16_rt(
          K1 + s, s, [&](int i, int k) { return a.f1[(size_t)i * sp + k]; },
          sm.B, [&](int i, int c, double v) {
            double* o = a.f2 + (size_t)i * sp + 16 * cb + c;
            *o = (i < K1 ? *o : 0.0) + v;
          });
      __syncthreads();
    }
    return;
  }
  if constexpr (S == 32) {
    // one 16-column block of M at a time, on the 16x16x4 MFMA
    for (int cb = 0; cb < 2; ++cb) {
      for (int e = threadIdx.x; e < 512; e += kThreads)
        sm.P2[e] = M[(e >> 4) * 32 + 16 * cb + (e & 15)];
      __syncthreads();
      mm16<32>(
          K1 + s, [&](int i, int k) { return a.f1[(size_t)i * sp + k]; },
          sm.P2, [&](int i, int c, double v) {
            double* o = a.f2 + (size_t)i * sp + 16 * cb + c;
            *o = (i < K1 ? *o : 0.0) + v;
          });
      __syncthreads();
    }
    return;
  }
  for (int i = threadIdx.x; i < K1 + s; i += kThreads) {
    double fr[S ? S : kMaxS];
#pragma unroll
    for (int k = 0; k < s; ++k) fr[k] = a.f1[(size_t)i * sp + k];
    double* out = a.f2 + (size_t)i * sp;
#pragma unroll 1
    for (int c = 0; c < s; ++c) {
      double v = i < K1 ? out[c] : 0.0;
      if constexpr (S > 0) {
#pragma unroll
        for (int k = 0; k < S; ++k) v += fr[k] * M[k * S + c];
      } else {
        for (int k = 0; k < s; ++k) v += fr[k] * M[k * s + c];
      }
      out[c] = v;
    }
  }
  __syncthreads();
}

template <int S>
__device__ __forceinline__ void make_coefs(const EpiView& sm,
                                           const EpiArgs& a) {
  __syncthreads();
  if (a.f1_mode != COEF_NONE)
    make_coef<S>(sm, a.f1, a.c1, a.f1_rows, a.t1, a.f1_mode == COEF_SCALED,
              a.s, a.sp);
  if (a.f2_mode != COEF_NONE)
    make_coef<S>(sm, a.f2, a.c2, a.f2_rows, a.t2, a.f2_mode == COEF_SCALED,
              a.s, a.sp);
  if (a.fold12 && a.f1_mode != COEF_NONE && a.f2_mode != COEF_NONE)
    fold_coefs<S>(sm, a);
}

template <int S>
__device__ __forceinline__ bool epilogue_body(EpiArgs a,
                                              const EpiView& sm);

// dst(i, c) = G(i, col0 + c) for c < s, 0 for s <= c < sp (rows i < rows,
// row-major with stride sp): the Gram loads of eight elements per thread
// are issued before their stores.
__device__ __forceinline__ void copy_gram_rows(const EpiArgs& a, double* dst,
                                               int rows, int col0, int s,
                                               int sp) {
  constexpr int kB = 8;
  const int total = rows * sp;
  for (int base = threadIdx.x; base < total; base += kB * kThreads) {
    double v[kB];
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int e = min(base + u * kThreads, total - 1);
      const int i = e / sp, c = e % sp;
      v[u] = c < s ? gram_at(a, i, col0 + c) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kB; ++u) {
      const int e = base + u * kThreads;
      if (e < total) dst[e] = v[u];
    }
  }
}

// The whole epilogue on the LDS arrays of `sm` (one workgroup)
template <int S>
__device__ __forceinline__ void epilogue_all(const EpiArgs& a,
                                             const EpiView& sm) {
  if (!epilogue_body<S>(a, sm)) make_coefs<S>(sm, a);
}

template <int S>
__global__ __launch_bounds__(kThreads) void epilogue_kernel(EpiArgs a) {
  __shared__ EpiSmem sm;
  epilogue_all<S>(a, view_of(sm));
}

// Returns true when it has also written the coefficient matrices.
template <int S>
__device__ __forceinline__ bool epilogue_body(EpiArgs a,
                                              const EpiView& sm) {
  constexpr bool kFast = S == 4 || S == 8 || S == 16;
  const int tid = threadIdx.x;
  const int s = S ? S : a.s, sp = a.sp, js = a.j * s;

  if (a.mode == EPI_S_ONLY || a.mode == EPI_Y_ONLY) {
    double* dst = a.mode == EPI_S_ONLY ? a.c2 : a.c1;
    copy_gram_rows(a, dst, js, 0, s, sp);
    if (a.unit_s) store_identity(a.t2, sp, s);
    return false;
  }

  if (a.mode == EPI_R_ASSEMBLE) {
    for (int e = tid; e < s * s; e += kThreads)
      sm.A[e] = a.t1[(e / s) * sp + e % s];
    assemble_r<S>(sm, a, a.c1, a.c2, sm.A, a.t2);
    return false;
  }

  if (a.mode == EPI_S_CHOL) {
    // gram rows [0, js) = S_{1:j,j+1}, rows [js, js+s) = T_{j+1}
    // (columns [0, s)); S_{j+1,j+1} = chol(T - S^T S)
    copy_gram_rows(a, a.c2, js, 0, s, sp);
    if constexpr (S == 4 || S == 8 || S == 16) {
      double ss = 0.0, unused1 = 0.0, unused2 = 0.0;
      gram_products<S>(a, js, false, sm.B, ss, unused1, unused2);
      if (tid < S * S) sm.A[tid] = gram_at(a, js + tid / S, tid % S) - ss;
    } else if (s % 16 == 0) {
      gram_mfma(a, js, 0, 0, s, sm.B);
      for (int e = tid; e < s * s; e += kThreads)
        sm.A[e] = gram_at(a, js + e / s, e % s) - sm.B[e];
    } else {
      for (int e = tid; e < s * s; e += kThreads) {
        const int x = e / s, y = e % s;
        double acc = gram_at(a, js + x, y);
        for (int k = 0; k < js; ++k)
          acc -= gram_at(a, k, x) * gram_at(a, k, y);
        sm.A[e] = acc;
      }
    }
    __syncthreads();
    chol<S>(sm, s, a.info, a.j, 0);
    store_tri(a.t2, sp, s, sm.A);
    return false;
  }

  // EPI_ONE_SYNC, after [Q_{0:j-1} U_j (E)]^T [U_j (E)]:
  //   Y = G(0:js, 0:s)     Omega = G(js:js+s, 0:s)
  //   Z = G(0:js, s:2s)    P = G(js:js+s, s:2s)    T = G(js+s:js+2s, s:2s)
  // The three products over the js rows of Y and Z (Y^T Y, Y^T Z, Z^T Z)
  // are accumulated together while row chunks of [Y Z] stream through LDS.
  constexpr int kPer =
      S ? (S * S + kThreads - 1) / kThreads : kMaxS * kMaxS / kThreads;
  const int w2 = a.has_e ? 2 * s : s;
  double yy[kPer], yz[kPer], zz[kPer];
#pragma unroll
  for (int t = 0; t < kPer; ++t) yy[t] = yz[t] = zz[t] = 0.0;
  if constexpr (S == 4 || S == 8 || S == 16) {
    gram_products<S>(a, js, a.has_e, sm.B, yy[0], yz[0], zz[0]);
  } else if (S == 32) {
    // the three products in one sweep, through sm.A
    gram_three32(a, js, a.has_e, sm.A);
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const int e = tid + t * kThreads;
      if (e < s * s) {
        yy[t] = sm.A[e];
        if (a.has_e) {
          yz[t] = sm.A[s * s + e];
          zz[t] = sm.A[2 * s * s + e];
        }
      }
    }
    __syncthreads();
  } else if (s % 16 == 0) {
    // the three products one after another through sm.A
    for (int p = 0; p < (a.has_e ? 3 : 1); ++p) {
      gram_mfma(a, js, p == 2 ? s : 0, p == 0 ? 0 : s, s, sm.A);
#pragma unroll
      for (int t = 0; t < kPer; ++t) {
        const int e = tid + t * kThreads;
        if (e < s * s) (p == 0 ? yy : p == 1 ? yz : zz)[t] = sm.A[e];
      }
      __syncthreads();
    }
  } else {
    double* stg = sm.A;               // rows x w2, row-major
    const int crows = (kMaxS * kMaxS) / w2;
    for (int r0 = 0; r0 < js; r0 += crows) {
      const int nr = min(crows, js - r0);
      for (int e = tid; e < nr * w2; e += kThreads) {
        const int c = e / nr, r = e % nr;
        stg[r * w2 + c] = gram_at(a, r0 + r, c);
      }
      __syncthreads();
#pragma unroll
      for (int t = 0; t < kPer; ++t) {
        const int e = tid + t * kThreads;
        if (e < s * s) {
          const int x = e / s, y = e % s;
          double ay = yy[t], az = yz[t], bz = zz[t];
          for (int r = 0; r < nr; ++r) {
            const double* row = stg + r * w2;
            ay += row[x] * row[y];
            if (a.has_e) {
              az += row[x] * row[s + y];
              bz += row[s + x] * row[s + y];
            }
          }
          yy[t] = ay; yz[t] = az; zz[t] = bz;
        }
      }
      __syncthreads();
    }
  }
  // 1. Y_jj = chol(Omega - Y^T Y)
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const int e = tid + t * kThreads;
    if (e < s * s) sm.A[e] = gram_at(a, js + e / s, e % s) - yy[t];
  }
  __syncthreads();
  chol<S>(sm, s, a.info, a.j, 1);
  // 2. R block column j with the current S (C2, T2) and the new Y, Y_jj
  //    (C1/T1 are overwritten below, so write the new Y into C1 first;
  //    the s <= 16 path reads Y from the Gram and keeps Y_jj in LDS)
  if constexpr (kFast) {
    if (tid < S * S) sm.T1[tid] = sm.A[tid];
  } else {
    copy_gram_rows(a, a.c1, js, 0, s, sp);
  }
  store_tri(a.t1, sp, s, sm.A);
  __syncthreads();
  assemble_r<S>(sm, a, a.c1, a.c2, sm.A, a.t2, kFast);
  if (!a.has_e) {
    if constexpr (kFast) {
      coefs_fused<S>(sm, a, js);
      return true;
    }
    return false;
  }
  // 3. eq. (1): lower block L = Y_jj^{-T} (P - Y^T Z), forward substitution
  //    with Y_jj^T (lower triangular), one column per thread
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const int e = tid + t * kThreads;
    if (e < s * s) sm.B[e] = gram_at(a, js + e / s, s + e % s) - yz[t];
  }
  __syncthreads();
  if constexpr (S > 0 && S <= 16) {
    if (tid < S) {
      const int c = tid;
      double x[S];
#pragma unroll
      for (int i = 0; i < S; ++i) {
        double acc = sm.B[i * S + c];
#pragma unroll
        for (int k = 0; k < i; ++k) acc -= sm.A[k * S + i] * x[k];
        x[i] = acc / sm.A[i * S + i];
      }
#pragma unroll
      for (int i = 0; i < S; ++i) sm.B[i * S + c] = x[i];
    }
  } else if (tid < s) {
    const int c = tid;
    for (int i = 0; i < s; ++i) {
      double acc = sm.B[i * s + c];
      for (int k = 0; k < i; ++k) acc -= sm.A[k * s + i] * sm.B[k * s + c];
      sm.B[i * s + c] = acc / sm.A[i * s + i];
    }
  }
  __syncthreads();
  if constexpr (kFast) {
    if (tid < S * S) sm.L[tid] = sm.B[tid];
  }
  // C2 <- [Z; L]
  copy_gram_rows(a, a.c2, js, s, s, sp);
  for (int e = tid; e < s * sp; e += kThreads) {
    const int i = e / sp, c = e % sp;
    a.c2[(size_t)(js + i) * sp + c] = c < s ? sm.B[i * s + c] : 0.0;
  }
  if (a.unit_s) {                     // BCGSI+1s: S_{j+1,j+1} = I
    store_identity(a.t2, sp, s);
  }
  if (a.unit_s || !a.chol_s) {
    if constexpr (kFast) {
      coefs_fused<S>(sm, a, js);
      return true;
    }
    return false;
  }
  // 4. S_{j+1,j+1} = chol(T - S^T S) with S = [Z; L]
  double tmp[kPer];
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const int e = tid + t * kThreads;
    if (e < s * s) {
      const int x = e / s, y = e % s;
      double acc = gram_at(a, js + s + x, s + y) - zz[t];
      for (int k = 0; k < s; ++k) acc -= sm.B[k * s + x] * sm.B[k * s + y];
      tmp[t] = acc;
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const int e = tid + t * kThreads;
    if (e < s * s) sm.A[e] = tmp[t];
  }
  __syncthreads();
  chol<S>(sm, s, a.info, a.j + 1, 0);
  store_tri(a.t2, sp, s, sm.A);
  if constexpr (kFast) {
    if (tid < S * S) sm.T2[tid] = sm.A[tid];
    coefs_fused<S>(sm, a, js);
    return true;
  }
  return false;
}

}  // namespace bcgs
