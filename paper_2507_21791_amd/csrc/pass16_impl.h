// Kernel template of the s <= 16 streaming pass (see pass16.hip for the
// design).  Included by pass16.hip (tiles copied direct to LDS) and
// pass16_reg.hip (tiles staged through registers, for leading dimensions
// or base addresses that are not 16-byte aligned).
#pragma once

#include <stdio.h>
#include <stdlib.h>

#include <algorithm>

#include "common.h"

namespace bcgs {

namespace p16 {

constexpr int kMaxKF = 20;            // C fragments per update per wave

// C fragments per update per wave of a shape with column capacity CAP
__host__ __device__ constexpr int kf_of(int cap) { return cap > 272 ? 20 : 16; }

typedef double v4d __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64: A[l % 16][l / 16], B[l / 16][l % 16],
// D[l / 16 + 4 v][l % 16]
__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// v_mfma_f64_4x4x4f64: four independent 4x4x4 products per wave.  With
// lane l = i + 4 b + 16 k (operand A), l = j + 4 b + 16 k (operand B) and
// l = j + 4 b + 16 i (result), block b computes D_b = A_b B_b + C_b.  On
// gfx950 this form sustains about 1.5x the FP64 rate of the 16x16x4 one.
__device__ __forceinline__ double mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// swizzle key of column c: a permutation of the granule index
template <int TR>
__device__ __forceinline__ int swz(int c) {
  if (TR >= 32) return ((c & 1) << 3) | ((c >> 1) & 7);
  return (c >> 1) & 7;
}

// LDS offset (in doubles) of element (row r, column c) of a tile
template <int TR>
__device__ __forceinline__ int at(int c, int r) {
  return c * TR + (((r >> 1) ^ swz<TR>(c)) << 1) + (r & 1);
}

// s_waitcnt vmcnt(n) (n <= 63), leaving the other counters alone
#define P16_VM(n) (((n) & 15) | (((n) >> 4) << 14) | (7 << 4) | (15 << 8))
__device__ __forceinline__ void wait_vm(int n) {
  switch (n < 63 ? n : 63) {
#define C4(b) case b: __builtin_amdgcn_s_waitcnt(P16_VM(b)); break;   \
              case b + 1: __builtin_amdgcn_s_waitcnt(P16_VM(b + 1)); break; \
              case b + 2: __builtin_amdgcn_s_waitcnt(P16_VM(b + 2)); break; \
              case b + 3: __builtin_amdgcn_s_waitcnt(P16_VM(b + 3)); break;
    C4(0) C4(4) C4(8) C4(12) C4(16) C4(20) C4(24) C4(28)
    C4(32) C4(36) C4(40) C4(44) C4(48) C4(52) C4(56) C4(60)
#undef C4
  }
}

// Workgroup barrier for LDS traffic only.  __syncthreads() also waits for
// every outstanding vector memory operation (vmcnt(0)), which would drain
// the tile copies in flight; LDS visibility needs only lgkmcnt(0), and the
// copies into LDS are waited for explicitly with wait_vm().
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_s_waitcnt((15) | (3 << 14) | (7 << 4) | (0 << 8));
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

struct Args {
  int64_t m;
  int s, ncols, ncols_p;
  int64_t rows_per_wg;
  const double* q; int64_t ldq; int nq;
  const double* f; int64_t ldf; int fcols;
  const double* e; int64_t lde; int ecols;
  int upd1, u1_c0; const double* c1; double* dst1; int64_t ldd1;
  int upd2, u2_c0; const double* c2; double* dst2; int64_t ldd2;
  int gram, ga_p, gb0, gbn_p, skip_a0, skip_b1;
  double* partial;
};

__device__ __forceinline__ const double* col_ptr(const Args& a, int c,
                                                 int64_t* ld) {
  if (c < a.nq) { *ld = a.ldq; return a.q + (int64_t)c * a.ldq; }
  c -= a.nq;
  if (c < a.fcols) { *ld = a.ldf; return a.f + (int64_t)c * a.ldf; }
  c -= a.fcols;
  *ld = a.lde;
  return a.e + (int64_t)c * a.lde;
}

// Synchronous staging of a short last tile: zero past the row count.
template <int TR, int NW>
__device__ void tile_sync(const Args& a, double* buf, int64_t r0, int rows) {
  for (int idx = threadIdx.x; idx < a.ncols * TR; idx += NW * 64) {
    const int c = idx / TR, r = idx % TR;
    double v = 0.0;
    if (r < rows) {
      int64_t ld;
      const double* src = col_ptr(a, c, &ld);
      v = src[r0 + r];
    }
    buf[at<TR>(c, r)] = v;
  }
}

// Sum the K-range partial products of one block update (scr: [KG][TR][17])
// into the tile columns [uc0, uc0 + s) and into dst (rows < rows).
template <int TR, int KG, int NW>
__device__ __forceinline__ void combine(const Args& a, double* tile,
                                        const double* scr, int uc0,
                                        double* dst, int64_t ldd, int64_t r0,
                                        int rows) {
  for (int t = threadIdx.x; t < TR * 16; t += NW * 64) {
    const int r = t % TR, c = t / TR;
    if (c >= a.s) continue;
    double part[KG];
#pragma unroll
    for (int k = 0; k < KG; ++k) part[k] = scr[(k * TR + r) * 17 + c];
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < KG; ++k) sum += part[k];
    tile[at<TR>(uc0 + c, r)] = sum;
    if (r < rows) dst[(int64_t)c * ldd + r0 + r] = sum;
  }
}

// One workgroup per row range.  TR tile rows; NBUF tile buffers of CAP
// columns, each its own LDS object; PC workgroups per CU; NW waves; SCR2:
// LDS room for both updates' partial sums; MAXP Gram pairs per wave; NTB
// B blocks; REG: tiles staged through registers instead of direct copies.
//
// Copy pipeline.  Each wave issues exactly IPW copy instructions per tile
// (waves with fewer instructions repeat their last one, lanes past the last
// column copy a valid column into the zero-weight padding), so the number
// of copies in flight is a compile-time constant: before tile t is read,
// vmcnt((NBUF - 2) IPW) leaves the copies of the next NBUF - 2 tiles in
// flight.  The tile loop is unrolled by NBUF so that every LDS access names
// its buffer statically; the compiler then sees that the copies in flight
// target other buffers and inserts no waits of its own.
//
// Register staging (REG).  The same lanes load the same 16 bytes (as two
// 8-byte loads, which need only the alignment of a double) one tile ahead
// into registers and write them to the LDS position the direct copy would
// use, so the tile layout is identical.  Two buffers: tile t is computed
// while tile t+1 is in registers; then tile t+1 goes to the other buffer
// and the loads of tile t+2 are issued.
template <int TR, int NBUF, int CAP, int PC, int NW, bool SCR2, int MAXP,
          bool GRAM, int NTB, bool REG>
struct Kernel {
  static constexpr int KF = kf_of(CAP);
  static constexpr int MB = TR / 16;          // row blocks per tile
  static constexpr int KG = NW / MB;          // K ranges per update
  static constexpr int kTail = (4 + KG - 1) / KG;
  static constexpr int CPI = 1024 / (TR * 8); // columns per copy instruction
  static constexpr int IPW = ((CAP + CPI - 1) / CPI + NW - 1) / NW;
  static constexpr int TE = CAP * TR;         // doubles per buffer
  static_assert(CAP % CPI == 0, "buffer holds whole copy instructions");

  // register-resident state of one wave
  struct State {
    double c1f[KF], c2f[KF];           // shared K-steps (both updates)
    double c2o[kTail];                 // update 2, steps over its own block
    int kb, ke, nks2, sq;
    int mb, kg;
    double acc[MAXP][4];
    int npairs;
  };

  // direct-to-LDS copy of the full tile at rows r0 .. r0+TR-1
  static __device__ __forceinline__ void dma(const Args& a, double* buf,
                                             int64_t r0) {
    constexpr int kGran = TR / 2;                    // granules per column
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ninst = (a.ncols + CPI - 1) / CPI;
#pragma unroll
    for (int i = 0; i < IPW; ++i) {
      const int ins = min(wave + NW * i, ninst - 1);
      const int c = ins * CPI + lane / kGran;
      const int g = lane % kGran;
      int64_t ld;
      const double* src = col_ptr(a, min(c, a.ncols - 1), &ld);
      const int rr = (g ^ swz<TR>(c)) << 1;
      __builtin_amdgcn_global_load_lds(src + r0 + rr, buf + ins * CPI * TR,
                                       16, 0, 0);
    }
  }

  // register staging: the loads of the tile at rows r0 .. r0+TR-1
  static __device__ __forceinline__ void issue(const Args& a, int64_t r0,
                                               double2 (&pend)[IPW]) {
    constexpr int kGran = TR / 2;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ninst = (a.ncols + CPI - 1) / CPI;
#pragma unroll
    for (int i = 0; i < IPW; ++i) {
      const int ins = min(wave + NW * i, ninst - 1);
      const int c = ins * CPI + lane / kGran;
      const int g = lane % kGran;
      int64_t ld;
      const double* src = col_ptr(a, min(c, a.ncols - 1), &ld);
      const double* p = src + r0 + ((g ^ swz<TR>(c)) << 1);
      pend[i].x = p[0];
      pend[i].y = p[1];
    }
  }

  // ... and their LDS writes, where the direct copy would have put them
  static __device__ __forceinline__ void commit(const Args& a, double* buf,
                                                const double2 (&pend)[IPW]) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ninst = (a.ncols + CPI - 1) / CPI;
#pragma unroll
    for (int i = 0; i < IPW; ++i) {
      const int ins = min(wave + NW * i, ninst - 1);
      *reinterpret_cast<double2*>(buf + ins * CPI * TR + 2 * lane) = pend[i];
    }
  }

  // block updates of one tile (U1: update 1, U2: update 2 present), with
  // the 16x16x4 MFMA: the update reads one tile fragment per K-step and
  // shares it between both updates, which keeps its LDS traffic at a
  // quarter of what the 4x4x4 form would need
  template <bool U1, bool U2>
  static __device__ __forceinline__ void updates(const Args& a, State& S,
                                                 double* tile, double* scr,
                                                 int64_t r0, int rows) {
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    // K-steps in uniform chunks of 4; inside a chunk the four fragment
    // loads are issued first; K-steps past ke read a valid address and
    // meet zero coefficient fragments, so no lane-divergent branches
    v4d acc1 = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};
    v4d acc1b = {0.0, 0.0, 0.0, 0.0}, acc2b = {0.0, 0.0, 0.0, 0.0};
    const int kcl = max(S.kb, S.ke - 1);
    const int row = S.mb * 16 + li;
#pragma unroll
    for (int q = 0; q < KF / 4; ++q) {
      if (4 * q >= S.ke - S.kb) break;
      double av[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = min(S.kb + 4 * q + u, kcl);
        av[u] = tile[at<TR>(4 * k + lk, row)];
      }
#pragma unroll
      for (int u = 0; u < 4; u += 2) {
        if (U1) acc1 = mfma16(av[u], S.c1f[4 * q + u], acc1);
        if (U2) acc2 = mfma16(av[u], S.c2f[4 * q + u], acc2);
        if (U1) acc1b = mfma16(av[u + 1], S.c1f[4 * q + u + 1], acc1b);
        if (U2) acc2b = mfma16(av[u + 1], S.c2f[4 * q + u + 1], acc2b);
      }
    }
    if (U2) {
#pragma unroll
      for (int u = 0; u < kTail; ++u) {
        const int t = S.kg + KG * u;
        if (t < S.sq)
          acc2b = mfma16(tile[at<TR>(4 * (S.nks2 + t) + lk, row)], S.c2o[u],
                         acc2b);
      }
    }
    acc1 += acc1b;
    acc2 += acc2b;
    // partial sums: scr[kg][row][col], row stride 17; result v at lane l is
    // row mb*16 + lk + 4 v, column li
    double* scr1 = scr;
    double* scr2 = SCR2 ? scr + KG * TR * 17 : scr;
    const int wbase = (S.kg * TR + S.mb * 16 + lk) * 17 + li;
    if (U1) {
#pragma unroll
      for (int v = 0; v < 4; ++v) scr1[wbase + 4 * v * 17] = acc1[v];
    }
    if (U2 && (SCR2 || !U1)) {
#pragma unroll
      for (int v = 0; v < 4; ++v) scr2[wbase + 4 * v * 17] = acc2[v];
    }
    lds_barrier();
    if (U1) combine<TR, KG, NW>(a, tile, scr1, a.u1_c0, a.dst1, a.ldd1, r0, rows);
    if (U2 && (SCR2 || !U1))
      combine<TR, KG, NW>(a, tile, scr2, a.u2_c0, a.dst2, a.ldd2, r0, rows);
    lds_barrier();
    if (!SCR2 && U1 && U2) {
      // one partial-sum area: the second update's round
#pragma unroll
      for (int v = 0; v < 4; ++v) scr[wbase + 4 * v * 17] = acc2[v];
      lds_barrier();
      combine<TR, KG, NW>(a, tile, scr, a.u2_c0, a.dst2, a.ldd2, r0, rows);
      lds_barrier();
    }
  }

  static __device__ __forceinline__ void process(const Args& a, State& S,
                                                 double* tile, double* scr,
                                                 int64_t r0, int rows) {
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    // ---- block updates, as out^T = F^T tile^T in 4x4x4 blocks: the A
    //      operand is the F fragment (F[4k + lk][li], kept in registers),
    //      the B operand of instruction q holds rows mb*16 + 4 j + q (j =
    //      lane & 3) of tile column 4k + lk, so a lane's four B values are
    //      four consecutive rows (two 16-byte loads per K-step).  Output
    //      q at lane l: row mb*16 + 4 (l & 3) + q, column 4 ((l >> 2) & 3) +
    //      (l >> 4). ----
    if (a.upd1 && a.upd2) updates<true, true>(a, S, tile, scr, r0, rows);
    else if (a.upd2) updates<false, true>(a, S, tile, scr, r0, rows);
    else if (a.upd1) updates<true, false>(a, S, tile, scr, r0, rows);
    // ---- Gram in 4x4x4 blocks: A operand = the pair's A block fragment
    //      (column pa + li, the 16x16x4 layout), B operand of instruction q
    //      = column gb + 4 (lane & 3) + q; two K-steps per 16-byte load
    //      (lane group lk takes rows kk + 2 lk and kk + 2 lk + 1).  Pair i of
    //      this wave is p = wave + NW i; since NW is a multiple of NTB, all
    //      pairs of a wave share the B block wave % NTB. ----
    if (GRAM) {
      const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
      const int bcol = a.gb0 + (wave % NTB) * 16 + 4 * (lane & 3);
#pragma unroll
      for (int kk = 0; kk < TR; kk += 8) {
        const int r = kk + 2 * lk;
        double2 bq[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          bq[q] = *reinterpret_cast<const double2*>(tile + at<TR>(bcol + q, r));
#pragma unroll
        for (int i = 0; i < MAXP; ++i) {
          const int p = wave + NW * i;
          if (p < S.npairs) {          // wave-uniform
            const double2 af = *reinterpret_cast<const double2*>(
                tile + at<TR>((p / NTB) * 16 + li, r));
#pragma unroll
            for (int q = 0; q < 4; ++q)
              S.acc[i][q] = mfma4(af.x, bq[q].x, S.acc[i][q]);
#pragma unroll
            for (int q = 0; q < 4; ++q)
              S.acc[i][q] = mfma4(af.y, bq[q].y, S.acc[i][q]);
          }
        }
        asm volatile("" ::: "memory");
      }
    }
  }

  // pipelined step on buffer I: tile t is waited for, the copy of tile
  // t + NBUF - 1 goes into the buffer tile t - 1 used, tile t is computed
  template <int I>
  static __device__ __forceinline__ void step(const Args& a, State& S,
                                              double* const (&bufs)[4],
                                              double* scr, int64_t row0,
                                              int64_t t) {
    __builtin_amdgcn_s_waitcnt(P16_VM((NBUF - 2) * IPW));
    lds_barrier();
    dma(a, bufs[(I + NBUF - 1) % NBUF], row0 + (t + NBUF - 1) * TR);
    process(a, S, bufs[I], scr, row0 + t * TR, TR);
  }

  // register-staged step on buffer I: tile t is in buffer I and tile t+1
  // in registers; afterwards tile t+1 is in the other buffer and tile t+2
  // in registers (when it exists)
  template <int I>
  static __device__ __forceinline__ void step_reg(const Args& a, State& S,
                                                  double* const (&bufs)[4],
                                                  double* scr, int64_t row0,
                                                  int64_t t, int64_t nfull,
                                                  double2 (&pend)[IPW]) {
    process(a, S, bufs[I], scr, row0 + t * TR, TR);
    if (t + 1 < nfull) commit(a, bufs[I ^ 1], pend);
    if (t + 2 < nfull) issue(a, row0 + (t + 2) * TR, pend);
    lds_barrier();
  }

  static __device__ __forceinline__ void run(const Args& a) {
    __shared__ double b0[TE];
    __shared__ double b1[TE];
    __shared__ double b2[NBUF > 2 ? TE : 1];
    __shared__ double b3[NBUF > 3 ? TE : 1];
    __shared__ double scr[(SCR2 ? 2 : 1) * KG * TR * 17];
    double* const bufs[4] = {b0, b1, b2, b3};
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform
    const int li = lane & 15, lk = lane >> 4;
    const int64_t g = blockIdx.x;
    const int64_t row_begin = g * a.rows_per_wg;
    const int64_t row_end = min(a.m, row_begin + a.rows_per_wg);

    State S;
    S.mb = wave % MB;
    S.kg = wave / MB;
    // ---- coefficient fragments.  Update 1 runs over the staged columns
    // [0, u1_c0 + s); update 2 over [0, u2_c0) plus its own block F.  With
    // both updates u2_c0 = u1_c0 + s, so the two share all K-steps except
    // update 2's own block. ----
    const int s = a.s;
    S.sq = s / 4;
    const int nks1 = a.upd1 ? (a.u1_c0 + s) / 4 : 0;
    S.nks2 = a.upd2 ? a.u2_c0 / 4 : 0;
    const int shared = max(nks1, S.nks2);
    const int per = (shared + KG - 1) / KG;
    S.kb = S.kg * per;
    S.ke = min(shared, S.kb + per);
#pragma unroll
    for (int i = 0; i < KF; ++i) {
      const int k = S.kb + i;
      const int row = 4 * k + lk;
      S.c1f[i] = (k < S.ke && k < nks1) ? a.c1[row * 16 + li] : 0.0;
      S.c2f[i] = (k < S.ke && k < S.nks2) ? a.c2[row * 16 + li] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kTail; ++u) {
      const int t = S.kg + KG * u;
      S.c2o[u] = (a.upd2 && t < S.sq)
                     ? a.c2[(4 * (S.nks2 + t) + lk) * 16 + li] : 0.0;
    }
    // ---- Gram pairs p = wave + NW i, p = (A block) * NTB + (B block) ----
    const int nta = a.ga_p >> 4;
    S.npairs = GRAM ? nta * NTB : 1;
#pragma unroll
    for (int i = 0; i < MAXP; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) S.acc[i][q] = 0.0;
    // the fragment loads above complete here, so no wait for them is left
    // pending inside the tile loop, where it would drain the copies
    __builtin_amdgcn_s_waitcnt(0);
    // zero the columns past the copied ones (multiplied by zero weights
    // in the updates; their Gram entries are not read)
    for (int idx = a.ncols_p * TR + tid; idx < TE; idx += NW * 64) {
      b0[idx] = 0.0;
      b1[idx] = 0.0;
      if (NBUF > 2) b2[idx] = 0.0;
      if (NBUF > 3) b3[idx] = 0.0;
    }

    // ---- full tiles ----
    const int64_t nfull = row_end > row_begin ? (row_end - row_begin) / TR : 0;
    int64_t t = 0, issued = 0;
    if constexpr (REG) {
      static_assert(NBUF == 2, "register staging uses two buffers");
      double2 pend[IPW];
      if (nfull >= 1) {
        issue(a, row_begin, pend);
        commit(a, b0, pend);
      }
      if (nfull >= 2) issue(a, row_begin + TR, pend);
      lds_barrier();
      for (; t + 1 < nfull; t += 2) {
        step_reg<0>(a, S, bufs, scr, row_begin, t, nfull, pend);
        step_reg<1>(a, S, bufs, scr, row_begin, t + 1, nfull, pend);
      }
      if (t < nfull) {
        step_reg<0>(a, S, bufs, scr, row_begin, t, nfull, pend);
        ++t;
      }
      issued = nfull;
    } else if (nfull >= 2 * NBUF - 1) {
#pragma unroll
      for (int i = 0; i < NBUF - 1; ++i)
        dma(a, bufs[i], row_begin + i * TR);
      for (; t + 2 * NBUF - 2 < nfull; t += NBUF) {
        step<0>(a, S, bufs, scr, row_begin, t);
        step<1>(a, S, bufs, scr, row_begin, t + 1);
        if constexpr (NBUF > 2) step<2>(a, S, bufs, scr, row_begin, t + 2);
        if constexpr (NBUF > 3) step<3>(a, S, bufs, scr, row_begin, t + 3);
      }
      issued = t + NBUF - 1;
    }
    // the last few tiles one at a time, without overlap
    for (; t < nfull; ++t) {
      const int bi = (int)(t % NBUF);
      double* tile = bi == 0 ? b0 : bi == 1 ? b1 : bi == 2 ? b2 : b3;
      if (t >= issued) dma(a, tile, row_begin + t * TR);
      __builtin_amdgcn_s_waitcnt(0);
      lds_barrier();
      process(a, S, tile, scr, row_begin + t * TR, TR);
    }
    // ---- short last tile ----
    const int64_t rt = row_begin + nfull * TR;
    if (rt < row_end) {
      __builtin_amdgcn_s_waitcnt(0);
      lds_barrier();
      tile_sync<TR, NW>(a, b0, rt, (int)(row_end - rt));
      lds_barrier();
      process(a, S, b0, scr, rt, (int)(row_end - rt));
    }

    if (GRAM) {
      double* out = a.partial + (size_t)g * a.ga_p * a.gbn_p;
#pragma unroll
      for (int i = 0; i < MAXP; ++i) {
        const int p = wave + NW * i;
        if (p >= S.npairs) continue;
        const int ta = (p / NTB) * 16, b = p % NTB;
        if (ta >= a.skip_a0 && b * 16 + 16 <= a.skip_b1) continue;
        // acc[i][q] at lane l: A column ta + 4 ((l >> 2) & 3) + lk,
        // B column b * 16 + 4 (l & 3) + q
#pragma unroll
        for (int q = 0; q < 4; ++q)
          out[(size_t)(b * 16 + 4 * (lane & 3) + q) * a.ga_p + ta +
              4 * ((lane >> 2) & 3) + lk] = S.acc[i][q];
      }
    }
  }
};

// two 4-wave workgroups per CU: at most 256 registers per lane
template <int TR, int NBUF, int CAP, int MAXP, bool GRAM, int NTB, bool REG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void pass16_kernel(Args a) {
  Kernel<TR, NBUF, CAP, 2, 4, false, MAXP, GRAM, NTB, REG>::run(a);
}

// one workgroup of NW waves per CU
template <int TR, int NBUF, int CAP, int NW, bool SCR2, int MAXP, bool GRAM,
          int NTB, bool REG>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(NW / 4)))
void pass16_deep_kernel(Args a) {
  Kernel<TR, NBUF, CAP, 1, NW, SCR2, MAXP, GRAM, NTB, REG>::run(a);
}

template <int TR, int NBUF, int CAP, int PC, int NW, bool SCR2, int MAXP,
          bool GRAM, int NTB, bool REG>
static hipError_t go(const Args& a, int G, hipStream_t st, int* tag) {
  // 1 W P B S TT PP N: waves, workgroups per CU, tile buffers (+5 with
  // register staging), both partial-sum areas, tile rows, Gram pairs per
  // wave, B blocks (0: no Gram)
  *tag = 1000000000 + NW * 100000000 + PC * 10000000 +
         (NBUF + (REG ? 5 : 0)) * 1000000 + (SCR2 ? 100000 : 0) + TR * 1000 +
         MAXP * 10 + (GRAM ? NTB : 0);
  if constexpr (PC == 2)
    hipLaunchKernelGGL((pass16_kernel<TR, NBUF, CAP, MAXP, GRAM, NTB, REG>),
                       dim3((unsigned)G), dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(
        (pass16_deep_kernel<TR, NBUF, CAP, NW, SCR2, MAXP, GRAM, NTB, REG>),
        dim3((unsigned)G), dim3(NW * 64), 0, st, a);
  return hipGetLastError();
}

// (tile rows, buffers, column capacity, workgroups per CU, waves, both
// partial-sum areas)
struct Shape { int tr, nbuf, cap, per_cu, nw, scr2; };

// launch_pass16 picks among these (or takes the tuned / BCGS_PASS16_SHAPE
// index); its switch instantiates the same list, entry by entry.
// Taller tiles stream faster (each copy instruction covers fewer columns,
// so fewer pages and longer runs per column: on MI355X about 4.2, 5.7 and
// 6.3 TB/s for 16, 32 and 64 rows), so wide passes take one workgroup of 8
// waves per CU with 32- or 64-row tiles.  The last shape takes up to 544
// columns (n up to 512 at s = 16) in one 8-wave workgroup per CU.
constexpr Shape kShapes[] = {
    {64, 2, 64, 2, 4, 0},  {64, 2, 128, 1, 8, 0}, {32, 2, 272, 1, 8, 0},
    {32, 2, 128, 2, 4, 0}, {16, 2, 272, 2, 4, 0}, {16, 4, 272, 1, 4, 1},
    {16, 2, 544, 1, 8, 0}};
constexpr int kNShapes = sizeof(kShapes) / sizeof(kShapes[0]);

static int shape_maxp(const Shape& sh, int npairs) {
  return (npairs + sh.nw - 1) / sh.nw;
}

static bool shape_fits(const Shape& sh, int ncols_p, int shared_ksteps,
                       int npairs, bool reg) {
  if (reg && sh.nbuf != 2) return false;
  const int kg = sh.nw / (sh.tr / 16);
  if ((shared_ksteps + kg - 1) / kg > kf_of(sh.cap)) return false;
  if (shape_maxp(sh, npairs) > 9) return false;
  return ncols_p <= sh.cap;
}

template <int TR, int NBUF, int CAP, int PC, int NW, bool SCR2, bool REG>
static hipError_t go_shape(const Args& a, int G, bool gram, int ntb,
                           int maxp, hipStream_t st, int* tag) {
#define GO(M_, G_, N_) \
  go<TR, NBUF, CAP, PC, NW, SCR2, M_, G_, N_, REG>(a, G, st, tag)
  // largest pair count per wave this capacity can produce (two B blocks)
  constexpr int kTop = ((CAP / 16) * 2 + NW - 1) / NW;
  if (!gram) return GO(1, false, 1);
  if (ntb == 1) {
    if (kTop <= 2 || maxp <= 2) return GO(2, true, 1);
    if constexpr (kTop > 2) {
      if (kTop <= 5 || maxp <= 5) return GO(5, true, 1);
      if constexpr (kTop > 5) {
        if (kTop <= 7 || maxp <= 7) return GO(7, true, 1);
        if constexpr (kTop > 7) return GO(9, true, 1);
      }
    }
  } else {
    if (kTop <= 2 || maxp <= 2) return GO(2, true, 2);
    if constexpr (kTop > 2) {
      if (kTop <= 5 || maxp <= 5) return GO(5, true, 2);
      if constexpr (kTop > 5) {
        if (kTop <= 7 || maxp <= 7) return GO(7, true, 2);
        if constexpr (kTop > 7) return GO(9, true, 2);
      }
    }
  }
  return hipErrorNotSupported;
#undef GO
}

// Launch shape `pick` of kShapes (REG: register-staged tiles).
// Instantiated in pass16.hip (REG = false) and pass16_reg.hip (REG = true).
#define P16_DISPATCH_BODY(REG_)                                              \
  switch (pick) {                                                            \
    case 0: return go_shape<64, 2, 64, 2, 4, false, REG_>(a, G, gram, ntb,   \
                                                          maxp, st, tag);    \
    case 1: return go_shape<64, 2, 128, 1, 8, false, REG_>(a, G, gram, ntb,  \
                                                           maxp, st, tag);   \
    case 2: return go_shape<32, 2, 272, 1, 8, false, REG_>(a, G, gram, ntb,  \
                                                           maxp, st, tag);   \
    case 3: return go_shape<32, 2, 128, 2, 4, false, REG_>(a, G, gram, ntb,  \
                                                           maxp, st, tag);   \
    case 4: return go_shape<16, 2, 272, 2, 4, false, REG_>(a, G, gram, ntb,  \
                                                           maxp, st, tag);   \
    case 5:                                                                  \
      if constexpr (!REG_)                                                   \
        return go_shape<16, 4, 272, 1, 4, true, REG_>(a, G, gram, ntb, maxp, \
                                                      st, tag);              \
      return hipErrorNotSupported;                                           \
    case 6: return go_shape<16, 2, 544, 1, 8, false, REG_>(a, G, gram, ntb,  \
                                                           maxp, st, tag);   \
  }                                                                          \
  return hipErrorNotSupported;

template <bool REG>
hipError_t dispatch(int pick, const Args& a, int G, bool gram, int ntb,
                    int maxp, hipStream_t st, int* tag) {
  P16_DISPATCH_BODY(REG)
}

extern template hipError_t dispatch<false>(int, const Args&, int, bool, int,
                                           int, hipStream_t, int*);
extern template hipError_t dispatch<true>(int, const Args&, int, bool, int,
                                          int, hipStream_t, int*);

}  // namespace p16
}  // namespace bcgs
