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


// C fragments per update per wave of a shape with column capacity CAP:
// binary64 shapes split K over 4 or 8 waves, binary32 shapes (twice the
// rows per tile for the same bytes) over 2 or 4
template <typename T>
__host__ __device__ constexpr int kf_of(int cap) {
  return sizeof(T) == 8 ? (cap > 272 ? 20 : 16) : (cap > 128 ? 36 : 16);
}

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64: A[l % 16][l / 16], B[l / 16][l % 16],
// D[l / 16 + 4 v][l % 16]
__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// v_mfma_f32_16x16x4f32: same operand layout, D[4 (l / 16) + v][l % 16]
__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// storage-type traits: the 16-byte vector, the MFMA accumulator, the row
// of result value v at lane group lk
template <typename T> struct Elt;
template <> struct Elt<double> {
  typedef double2 V16;
  typedef v4d Acc;
  static __device__ __forceinline__ int drow(int lk, int v) {
    return lk + 4 * v;
  }
};
template <> struct Elt<float> {
  typedef float4 V16;
  typedef v4f Acc;
  static __device__ __forceinline__ int drow(int lk, int v) {
    return 4 * lk + v;
  }
};
template <typename T> constexpr int kEpg = 16 / (int)sizeof(T);

// v_mfma_f64_4x4x4f64: four independent 4x4x4 products per wave.  With
// lane l = i + 4 b + 16 k (operand A), l = j + 4 b + 16 k (operand B) and
// l = j + 4 b + 16 i (result), block b computes D_b = A_b B_b + C_b.  On
// gfx950 this form sustains about 1.5x the FP64 rate of the 16x16x4 one.
__device__ __forceinline__ double mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// swizzle key of column c: a permutation of the granule index (granule =
// 16 bytes: 2 doubles or 4 floats; TR / kEpg granules per column)
template <typename T, int TR>
__device__ __forceinline__ int swz(int c) {
  if constexpr (sizeof(T) == 8) {
    if (TR >= 32) return ((c & 1) << 3) | ((c >> 1) & 7);
    return (c >> 1) & 7;
  } else {
    return c & (TR / 4 - 1);
  }
}

// LDS offset (in elements) of element (row r, column c) of a tile
template <typename T, int TR>
__device__ __forceinline__ int at(int c, int r) {
  constexpr int E = kEpg<T>;
  return c * TR + (((r / E) ^ swz<T, TR>(c)) * E) + (r % E);
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

// T: storage type of the streamed columns; coefficients and Gram partials
// are FP64 either way
template <typename T>
struct ArgsT {
  int64_t m;
  int s, ncols, ncols_p;
  int64_t rows_per_wg;
  int interleave;        // tiles dealt round-robin to the workgroups
  const T* q; int64_t ldq; int nq;
  const T* f; int64_t ldf; int fcols;
  const T* e; int64_t lde; int ecols;
  int upd1, u1_c0; const double* c1; T* dst1; int64_t ldd1;
  int upd2, u2_c0; const double* c2; T* dst2; int64_t ldd2;
  int gram, ga_p, gb0, gbn_p, skip_a0, skip_b1;
  double* partial;
};
typedef ArgsT<double> Args;

template <typename T>
__device__ __forceinline__ const T* col_ptr(const ArgsT<T>& a, int c,
                                            int64_t* ld) {
  if (c < a.nq) { *ld = a.ldq; return a.q + (int64_t)c * a.ldq; }
  c -= a.nq;
  if (c < a.fcols) { *ld = a.ldf; return a.f + (int64_t)c * a.ldf; }
  c -= a.fcols;
  *ld = a.lde;
  return a.e + (int64_t)c * a.lde;
}

// Synchronous staging of a short last tile: zero past the row count.
template <typename T, int TR, int NW>
__device__ void tile_sync(const ArgsT<T>& a, T* buf, int64_t r0, int rows) {
  for (int idx = threadIdx.x; idx < a.ncols * TR; idx += NW * 64) {
    const int c = idx / TR, r = idx % TR;
    T v = 0;
    if (r < rows) {
      int64_t ld;
      const T* src = col_ptr(a, c, &ld);
      v = gload(src + r0 + r);
    }
    buf[at<T, TR>(c, r)] = v;
  }
}

// Partial-sum area of a block update: [KG][TR] rows of 16 columns.  Binary64
// rows hold 16 values with column c of row r at position c ^ (r mod 16);
// binary32 rows are padded to 17.  Either way the MFMA result writes (16
// columns of 4 rows per instruction) and the combine reads (16 or 32 rows of
// one column per half wave) hit distinct banks.
template <typename T>
constexpr int kScrRow = sizeof(T) == 8 ? 16 : 17;
template <typename T>
__device__ __forceinline__ int sidx(int row, int col) {
  if constexpr (sizeof(T) == 8) return row * 16 + (col ^ (row & 15));
  return row * 17 + col;
}

// Sum the K-range partial products of one block update (scr: [KG][TR] rows)
// into the tile columns [uc0, uc0 + s) and into dst (rows < rows).
template <typename T, int TR, int KG, int NW>
__device__ __forceinline__ void combine(const ArgsT<T>& a, T* tile,
                                        const T* scr, int uc0, T* dst,
                                        int64_t ldd, int64_t r0, int rows) {
  for (int t = threadIdx.x; t < TR * 16; t += NW * 64) {
    const int r = t % TR, c = t / TR;
    if (c >= a.s) continue;
    T part[KG];
#pragma unroll
    for (int k = 0; k < KG; ++k) part[k] = scr[sidx<T>(k * TR + r, c)];
    T sum = 0;
#pragma unroll
    for (int k = 0; k < KG; ++k) sum += part[k];
    tile[at<T, TR>(uc0 + c, r)] = sum;
    if (r < rows) gstore(dst + (int64_t)c * ldd + r0 + r, sum);
  }
}

// A workgroup streams its share of the row tiles (round-robin tiles, or a
// contiguous row range).  TR tile rows; NBUF tile buffers of CAP
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
template <typename T, int TR, int NBUF, int CAP, int PC, int NW, bool SCR2,
          int MAXP, bool GRAM, int NTB, bool REG, int KS>
struct Kernel {
  typedef ArgsT<T> Args;
  typedef typename Elt<T>::V16 V16;
  typedef typename Elt<T>::Acc Acc;
  static constexpr int E = kEpg<T>;           // elements per 16 bytes
  static constexpr int KF = kf_of<T>(CAP);
  static constexpr int MB = TR / 16;          // row blocks per tile
  static constexpr int KG = NW / MB;          // K ranges per update
  static constexpr int kTail = (4 + KG - 1) / KG;
  static constexpr int CPI = 1024 / (TR * (int)sizeof(T));  // columns per
                                                            // copy instr.
  static constexpr int IPW = ((CAP + CPI - 1) / CPI + NW - 1) / NW;
  static constexpr int TE = CAP * TR;         // elements per buffer
  static_assert(CAP % CPI == 0, "buffer holds whole copy instructions");
  static_assert(KG >= 1, "at least one wave per row block");
  static_assert(KS % 2 == 0 && KS <= KF, "update steps: even, in registers");

  // register-resident state of one wave
  struct State {
    T c1f[KF], c2f[KF];                // shared K-steps (both updates)
    T c2o[kTail];                      // update 2, steps over its own block
    int kb, ke, nks2, sq;
    int mb, kg;
    T acc[MAXP][4];
    int npairs;
    bool fast;                         // uniform-base tile copies
  };

  // Source of copy instruction i of this wave for the tile at row r0.
  // Fast form (S.fast: every instruction's CPI columns lie in one source
  // block, and the lane offsets fit 32 bits): the block's address at row
  // r0 is wave-uniform (scalar registers) and each lane adds a 32-bit
  // offset (its column times the leading dimension plus its swizzled
  // granule), so a tile costs a few instructions per copy instead of a
  // per-lane search of the three source blocks.
  static __device__ __forceinline__ const T* copy_src(const Args& a,
                                                      const State& S, int i,
                                                      int64_t r0) {
    constexpr int kGran = TR / E;                    // granules per column
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ninst = (a.ncols + CPI - 1) / CPI;
    const int ins = min(wave + NW * i, ninst - 1);
    const int lc = lane / kGran, g = lane % kGran;
    if (S.fast) {
      const int c0 = ins * CPI;
      const T* base;
      int64_t ld;
      int cl;
      if (c0 < a.nq) {
        base = a.q; ld = a.ldq; cl = c0;
      } else if (c0 < a.nq + a.fcols) {
        base = a.f; ld = a.ldf; cl = c0 - a.nq;
      } else {
        base = a.e; ld = a.lde; cl = c0 - a.nq - a.fcols;
      }
      const T* sb = base + (int64_t)cl * ld + r0;
      const uint32_t off = (uint32_t)lc * (uint32_t)ld +
                           (uint32_t)((g ^ swz<T, TR>(c0 + lc)) * E);
      return sb + off;
    }
    const int c = ins * CPI + lc;
    int64_t ld;
    const T* src = col_ptr(a, min(c, a.ncols - 1), &ld);
    return src + r0 + (g ^ swz<T, TR>(c)) * E;
  }

  // LDS offset (elements) of copy instruction i of this wave in a buffer
  static __device__ __forceinline__ int copy_dst(const Args& a, int i) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ninst = (a.ncols + CPI - 1) / CPI;
    return min(wave + NW * i, ninst - 1) * CPI * TR;
  }

  // direct-to-LDS copy of the full tile at rows r0 .. r0+TR-1
  static __device__ __forceinline__ void dma(const Args& a, const State& S,
                                             T* buf, int64_t r0) {
#pragma unroll
    for (int i = 0; i < IPW; ++i)
      __builtin_amdgcn_global_load_lds(copy_src(a, S, i, r0),
                                       buf + copy_dst(a, i), 16, 0, 0);
  }

  // register staging: the loads of the tile at rows r0 .. r0+TR-1
  static __device__ __forceinline__ void issue(const Args& a, const State& S,
                                               int64_t r0,
                                               V16 (&pend)[IPW]) {
#pragma unroll
    for (int i = 0; i < IPW; ++i) {
      const T* p = copy_src(a, S, i, r0);
      if constexpr (E == 2) {
        pend[i].x = gload(p);
        pend[i].y = gload(p + 1);
      } else {
        pend[i].x = gload(p);
        pend[i].y = gload(p + 1);
        pend[i].z = gload(p + 2);
        pend[i].w = gload(p + 3);
      }
    }
  }

  // ... and their LDS writes, where the direct copy would have put them
  static __device__ __forceinline__ void commit(const Args& a, T* buf,
                                                const V16 (&pend)[IPW]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < IPW; ++i)
      *reinterpret_cast<V16*>(buf + copy_dst(a, i) + E * lane) = pend[i];
  }

  // block updates of one tile (U1: update 1, U2: update 2 present), with
  // the 16x16x4 MFMA: the update reads one tile fragment per K-step and
  // shares it between both updates, which keeps its LDS traffic at a
  // quarter of what the 4x4x4 form would need
  template <bool U1, bool U2>
  static __device__ __forceinline__ void updates(const Args& a, State& S,
                                                 T* tile, T* scr,
                                                 int64_t r0, int rows) {
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    // K-steps in chunks of CH, the CH fragment loads of a chunk issued
    // first; a step past ke reads a valid address and meets a zero
    // coefficient fragment, so a wave runs its ke - kb steps rounded up to
    // a multiple of CH with no branch inside a chunk.  Chunks of 2 waste
    // fewer MFMAs; register-staged tiles (more registers live) keep
    // chunks of 4, which the compiler fits with fewer spills.
    constexpr int CH = REG ? 4 : 2;
    Acc acc1 = {0, 0, 0, 0}, acc2 = {0, 0, 0, 0};
    Acc acc1b = {0, 0, 0, 0}, acc2b = {0, 0, 0, 0};
    const int kcl = max(S.kb, S.ke - 1);
    const int row = S.mb * 16 + li;
    if constexpr (KS > 0) {
      // a compile-time step count (the launcher guarantees ke - kb <= KS):
      // no branches, so every fragment load of the tile is issued before
      // the first MFMA waits on one
      T av[KS];
#pragma unroll
      for (int u = 0; u < KS; ++u) {
        const int k = min(S.kb + u, kcl);
        av[u] = tile[at<T, TR>(4 * k + lk, row)];
      }
#pragma unroll
      for (int u = 0; u < KS; u += 2) {
        if (U1) acc1 = mfma16(av[u], S.c1f[u], acc1);
        if (U2) acc2 = mfma16(av[u], S.c2f[u], acc2);
        if (U1) acc1b = mfma16(av[u + 1], S.c1f[u + 1], acc1b);
        if (U2) acc2b = mfma16(av[u + 1], S.c2f[u + 1], acc2b);
      }
    } else {
#pragma unroll
      for (int q = 0; q < KF / CH; ++q) {
        if (CH * q >= S.ke - S.kb) break;           // wave-uniform
        T av[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          const int k = min(S.kb + CH * q + u, kcl);
          av[u] = tile[at<T, TR>(4 * k + lk, row)];
        }
#pragma unroll
        for (int u = 0; u < CH; u += 2) {
          if (U1) acc1 = mfma16(av[u], S.c1f[CH * q + u], acc1);
          if (U2) acc2 = mfma16(av[u], S.c2f[CH * q + u], acc2);
          if (U1) acc1b = mfma16(av[u + 1], S.c1f[CH * q + u + 1], acc1b);
          if (U2) acc2b = mfma16(av[u + 1], S.c2f[CH * q + u + 1], acc2b);
        }
      }
    }
    if (U2) {
#pragma unroll
      for (int u = 0; u < kTail; ++u) {
        const int t = S.kg + KG * u;
        if (t < S.sq)
          acc2b = mfma16(tile[at<T, TR>(4 * (S.nks2 + t) + lk, row)],
                         S.c2o[u], acc2b);
      }
    }
    acc1 += acc1b;
    acc2 += acc2b;
    // partial sums: scr[kg][row][col] (sidx); result v at lane l is row
    // mb*16 + drow(lk, v), column li
    T* scr1 = scr;
    T* scr2 = SCR2 ? scr + KG * TR * kScrRow<T> : scr;
    const int wrow = S.kg * TR + S.mb * 16;
    if (U1) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        scr1[sidx<T>(wrow + Elt<T>::drow(lk, v), li)] = acc1[v];
    }
    if (U2 && (SCR2 || !U1)) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        scr2[sidx<T>(wrow + Elt<T>::drow(lk, v), li)] = acc2[v];
    }
    lds_barrier();
    if (U1)
      combine<T, TR, KG, NW>(a, tile, scr1, a.u1_c0, a.dst1, a.ldd1, r0,
                             rows);
    if (U2 && (SCR2 || !U1))
      combine<T, TR, KG, NW>(a, tile, scr2, a.u2_c0, a.dst2, a.ldd2, r0,
                             rows);
    lds_barrier();
    if (!SCR2 && U1 && U2) {
      // one partial-sum area: the second update's round
#pragma unroll
      for (int v = 0; v < 4; ++v)
        scr[sidx<T>(wrow + Elt<T>::drow(lk, v), li)] = acc2[v];
      lds_barrier();
      combine<T, TR, KG, NW>(a, tile, scr, a.u2_c0, a.dst2, a.ldd2, r0,
                             rows);
      lds_barrier();
    }
  }

  static __device__ __forceinline__ void process(const Args& a, State& S,
                                                 T* tile, T* scr,
                                                 int64_t r0, int rows) {
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lk = lane >> 4;
    // ---- block updates (16x16x4 MFMA, see updates()) ----
    if (a.upd1 && a.upd2) updates<true, true>(a, S, tile, scr, r0, rows);
    else if (a.upd2) updates<false, true>(a, S, tile, scr, r0, rows);
    else if (a.upd1) updates<true, false>(a, S, tile, scr, r0, rows);
    // ---- Gram in 4x4x4 blocks: A operand = the pair's A block fragment
    //      (column pa + li, the 16x16x4 layout), B operand of instruction q
    //      = column gb + 4 (lane & 3) + q; two K-steps per 16-byte load
    //      (lane group lk takes rows kk + 2 lk and kk + 2 lk + 1).  Pair i of
    //      this wave is p = wave + NW i; since NW is a multiple of NTB, all
    //      pairs of a wave share the B block wave % NTB. ----
    if constexpr (GRAM && sizeof(T) == 4) {
      // binary32: 16x16x4 MFMA per pair; the rows of a 16-row chunk are
      // assigned to (K-step q, lane group lk) as row kk + 4 lk + q, the
      // same for both operands, so one 16-byte load per operand feeds four
      // MFMAs.  Result v at lane l: A column 4 lk + v, B column li.
      const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
      const int bcol = a.gb0 + (wave % NTB) * 16 + li;
#pragma unroll
      for (int kk = 0; kk < TR; kk += 16) {
        const int r = kk + 4 * lk;
        const V16 bq = *reinterpret_cast<const V16*>(tile + at<T, TR>(bcol, r));
#pragma unroll
        for (int i = 0; i < MAXP; ++i) {
          const int p = wave + NW * i;
          if (p < S.npairs) {          // wave-uniform
            const V16 af = *reinterpret_cast<const V16*>(
                tile + at<T, TR>((p / NTB) * 16 + li, r));
            Acc acc = {S.acc[i][0], S.acc[i][1], S.acc[i][2], S.acc[i][3]};
            acc = mfma16(af.x, bq.x, acc);
            acc = mfma16(af.y, bq.y, acc);
            acc = mfma16(af.z, bq.z, acc);
            acc = mfma16(af.w, bq.w, acc);
#pragma unroll
            for (int v = 0; v < 4; ++v) S.acc[i][v] = acc[v];
          }
        }
        asm volatile("" ::: "memory");
      }
    } else if constexpr (GRAM) {
      const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
      const int bcol = a.gb0 + (wave % NTB) * 16 + 4 * (lane & 3);
#pragma unroll
      for (int kk = 0; kk < TR; kk += 8) {
        const int r = kk + 2 * lk;
        double2 bq[4];
#pragma unroll
        for (int q = 0; q < 4; ++q)
          bq[q] = *reinterpret_cast<const double2*>(
              tile + at<T, TR>(bcol + q, r));
        // With two B blocks (pairs spread evenly: the waves differ by at
        // most one) and up to 7 pair slots the loop is branch-free: a slot
        // past this wave's pairs works on a valid column (pair npairs - 1)
        // and its sums are never stored, so the compiler batches all
        // operand loads (the launcher picks MAXP = the most pairs any wave
        // has).  Otherwise idle slots are skipped by branches: with more
        // slots the operands would not fit the registers, and with one B
        // block many waves would idle a slot.
        constexpr bool kBranchFree = NTB == 2 && MAXP <= 8;
#pragma unroll
        for (int i = 0; i < MAXP; ++i) {
          const int p0 = wave + NW * i;
          if (!kBranchFree && p0 >= S.npairs) continue;   // wave-uniform
          const int p = min(p0, S.npairs - 1);
          const double2 af = *reinterpret_cast<const double2*>(
              tile + at<T, TR>((p / NTB) * 16 + li, r));
#pragma unroll
          for (int q = 0; q < 4; ++q)
            S.acc[i][q] = mfma4(af.x, bq[q].x, (double)S.acc[i][q]);
#pragma unroll
          for (int q = 0; q < 4; ++q)
            S.acc[i][q] = mfma4(af.y, bq[q].y, (double)S.acc[i][q]);
        }
        asm volatile("" ::: "memory");
      }
    }
  }

  // pipelined step on buffer I: tile t is waited for, the copy of tile
  // t + NBUF - 1 goes into the buffer tile t - 1 used, tile t is computed
  template <int I>
  static __device__ __forceinline__ void step(const Args& a, State& S,
                                              T* const (&bufs)[4],
                                              T* scr, int64_t row0,
                                              int64_t ts, int64_t t) {
    __builtin_amdgcn_s_waitcnt(P16_VM((NBUF - 2) * IPW));
    lds_barrier();
    dma(a, S, bufs[(I + NBUF - 1) % NBUF], row0 + (t + NBUF - 1) * ts);
    process(a, S, bufs[I], scr, row0 + t * ts, TR);
  }

  // register-staged step on buffer I: tile t is in buffer I and tile t+1
  // in registers; afterwards tile t+1 is in the other buffer and tile t+2
  // in registers (when it exists)
  template <int I>
  static __device__ __forceinline__ void step_reg(const Args& a, State& S,
                                                  T* const (&bufs)[4],
                                                  T* scr, int64_t row0,
                                                  int64_t ts, int64_t t,
                                                  int64_t nfull,
                                                  V16 (&pend)[IPW]) {
    process(a, S, bufs[I], scr, row0 + t * ts, TR);
    if (t + 1 < nfull) commit(a, bufs[I ^ 1], pend);
    if (t + 2 < nfull) issue(a, S, row0 + (t + 2) * ts, pend);
    lds_barrier();
  }

  static __device__ __forceinline__ void run(const Args& a) {
    __shared__ T b0[TE];
    __shared__ T b1[TE];
    // the third and fourth buffers exist (take LDS) only with NBUF > 2, 3
    T* b2 = nullptr;
    T* b3 = nullptr;
    if constexpr (NBUF > 2) {
      __shared__ T b2s[TE];
      b2 = b2s;
    }
    if constexpr (NBUF > 3) {
      __shared__ T b3s[TE];
      b3 = b3s;
    }
    __shared__ T scr[(SCR2 ? 2 : 1) * KG * TR * kScrRow<T>];
    run_with(a, b0, b1, b2, b3, scr, blockIdx.x, gridDim.x);
  }

  // Elements of LDS the shape needs: NBUF tile buffers of TE, and the
  // partial-sum area
  static constexpr int kScrElems = (SCR2 ? 2 : 1) * KG * TR * kScrRow<T>;

  // The pass as workgroup g of G on the given LDS buffers (b2, b3 used only
  // with NBUF > 2, 3): the body of the pass kernels, and of the batched
  // persistent kernel, which hands it its work items.
  static __device__ __forceinline__ void run_with(const Args& a, T* b0, T* b1,
                                                  T* b2, T* b3, T* scr,
                                                  int64_t g, int64_t G) {
    T* const bufs[4] = {b0, b1, b2, b3};
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform
    const int li = lane & 15, lk = lane >> 4;
    // Tiles of this workgroup: nfull full tiles at rows row_begin + t ts,
    // then possibly one short tile of rows [rt, rt_end).  Contiguous: a
    // range of rows_per_wg rows per workgroup.  Interleaved: full tile i of
    // the matrix goes to workgroup i mod G (the short last tile too), so
    // the workgroups running together read one narrow band of rows of
    // every column.
    int64_t row_begin, ts, nfull, rt, rt_end;
    if (a.interleave) {
      const int64_t nt = a.m / TR;
      row_begin = g * TR;
      ts = G * TR;
      nfull = nt > g ? (nt - g + G - 1) / G : 0;
      rt = nt * TR;
      rt_end = (nt % G == g) ? a.m : rt;
    } else {
      row_begin = g * a.rows_per_wg;
      const int64_t row_end = min(a.m, row_begin + a.rows_per_wg);
      ts = TR;
      nfull = row_end > row_begin ? (row_end - row_begin) / TR : 0;
      rt = row_begin + nfull * TR;
      rt_end = max(rt, row_end);
    }

    State S;
    {
      // every copy instruction within one source block, 32-bit lane offsets
      const int64_t ldm = max(a.ldq, max(a.fcols ? a.ldf : 0,
                                         a.ecols ? a.lde : 0));
      S.fast = a.nq % CPI == 0 && a.fcols % CPI == 0 && a.ecols % CPI == 0 &&
               ldm * CPI + TR < (int64_t(1) << 31);
    }
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
      S.c1f[i] = (k < S.ke && k < nks1) ? (T)gload(a.c1 + row * 16 + li)
                                        : T(0);
      S.c2f[i] = (k < S.ke && k < S.nks2) ? (T)gload(a.c2 + row * 16 + li)
                                           : T(0);
    }
#pragma unroll
    for (int u = 0; u < kTail; ++u) {
      const int t = S.kg + KG * u;
      S.c2o[u] = (a.upd2 && t < S.sq)
                     ? (T)gload(a.c2 + (4 * (S.nks2 + t) + lk) * 16 + li)
                     : T(0);
    }
    // ---- Gram pairs p = wave + NW i, p = (A block) * NTB + (B block) ----
    const int nta = a.ga_p >> 4;
    S.npairs = GRAM ? nta * NTB : 1;
#pragma unroll
    for (int i = 0; i < MAXP; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) S.acc[i][q] = 0;
    // the fragment loads above complete here, so no wait for them is left
    // pending inside the tile loop, where it would drain the copies
    __builtin_amdgcn_s_waitcnt(0);
    // zero the columns past the copied ones (multiplied by zero weights
    // in the updates; their Gram entries are not read)
    for (int idx = a.ncols_p * TR + tid; idx < TE; idx += NW * 64) {
      b0[idx] = 0;
      b1[idx] = 0;
      if constexpr (NBUF > 2) b2[idx] = 0;
      if constexpr (NBUF > 3) b3[idx] = 0;
    }

    // ---- full tiles ----
    int64_t t = 0, issued = 0;
    if constexpr (REG) {
      static_assert(NBUF == 2, "register staging uses two buffers");
      V16 pend[IPW];
      if (nfull >= 1) {
        issue(a, S, row_begin, pend);
        commit(a, b0, pend);
      }
      if (nfull >= 2) issue(a, S, row_begin + ts, pend);
      lds_barrier();
      for (; t + 1 < nfull; t += 2) {
        step_reg<0>(a, S, bufs, scr, row_begin, ts, t, nfull, pend);
        step_reg<1>(a, S, bufs, scr, row_begin, ts, t + 1, nfull, pend);
      }
      if (t < nfull) {
        step_reg<0>(a, S, bufs, scr, row_begin, ts, t, nfull, pend);
        ++t;
      }
      issued = nfull;
    } else if (nfull >= 2 * NBUF - 1) {
#pragma unroll
      for (int i = 0; i < NBUF - 1; ++i)
        dma(a, S, bufs[i], row_begin + i * ts);
      for (; t + 2 * NBUF - 2 < nfull; t += NBUF) {
        step<0>(a, S, bufs, scr, row_begin, ts, t);
        step<1>(a, S, bufs, scr, row_begin, ts, t + 1);
        if constexpr (NBUF > 2) step<2>(a, S, bufs, scr, row_begin, ts, t + 2);
        if constexpr (NBUF > 3) step<3>(a, S, bufs, scr, row_begin, ts, t + 3);
      }
      issued = t + NBUF - 1;
    }
    // the last few tiles one at a time, without overlap
    for (; t < nfull; ++t) {
      const int bi = (int)(t % NBUF);
      T* tile = bi == 0 ? b0 : bi == 1 ? b1 : bi == 2 ? b2 : b3;
      if (t >= issued) dma(a, S, tile, row_begin + t * ts);
      __builtin_amdgcn_s_waitcnt(0);
      lds_barrier();
      process(a, S, tile, scr, row_begin + t * ts, TR);
    }
    // ---- short last tile ----
    if (rt < rt_end) {
      __builtin_amdgcn_s_waitcnt(0);
      lds_barrier();
      tile_sync<T, TR, NW>(a, b0, rt, (int)(rt_end - rt));
      lds_barrier();
      process(a, S, b0, scr, rt, (int)(rt_end - rt));
    }

    if (GRAM) {
      double* out = a.partial + (size_t)g * a.ga_p * a.gbn_p;
#pragma unroll
      for (int i = 0; i < MAXP; ++i) {
        const int p = wave + NW * i;
        if (p >= S.npairs) continue;
        const int ta = (p / NTB) * 16, b = p % NTB;
        if (ta >= a.skip_a0 && b * 16 + 16 <= a.skip_b1) continue;
        if constexpr (sizeof(T) == 4) {
          // acc[i][v] at lane l: A column ta + 4 lk + v, B column b*16 + li
#pragma unroll
          for (int v = 0; v < 4; ++v)
            gstore(out + (size_t)(b * 16 + li) * a.ga_p + ta + 4 * lk + v,
                   (double)S.acc[i][v]);
        } else {
          // acc[i][q] at lane l: A column ta + 4 ((l >> 2) & 3) + lk,
          // B column b * 16 + 4 (l & 3) + q
#pragma unroll
          for (int q = 0; q < 4; ++q)
            gstore(out + (size_t)(b * 16 + 4 * (lane & 3) + q) * a.ga_p +
                       ta + 4 * ((lane >> 2) & 3) + lk,
                   S.acc[i][q]);
        }
      }
    }
  }
};

// two 4-wave workgroups per CU: at most 256 registers per lane
template <typename T, int TR, int NBUF, int CAP, int MAXP, bool GRAM, int NTB,
          bool REG, int KS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void pass16_kernel(ArgsT<T> a) {
  Kernel<T, TR, NBUF, CAP, 2, 4, false, MAXP, GRAM, NTB, REG, KS>::run(a);
}

// the same with both partial-sum areas (one combine round fewer per tile
// when a pass has both block updates)
template <typename T, int TR, int NBUF, int CAP, int MAXP, bool GRAM, int NTB,
          bool REG, int KS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void pass16_s2_kernel(ArgsT<T> a) {
  Kernel<T, TR, NBUF, CAP, 2, 4, true, MAXP, GRAM, NTB, REG, KS>::run(a);
}

// one workgroup of NW waves per CU
template <typename T, int TR, int NBUF, int CAP, int NW, bool SCR2, int MAXP,
          bool GRAM, int NTB, bool REG>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(NW / 4)))
void pass16_deep_kernel(ArgsT<T> a) {
  Kernel<T, TR, NBUF, CAP, 1, NW, SCR2, MAXP, GRAM, NTB, REG, 0>::run(a);
}

// recording of a pass (batch_persist.hip): tile rows, waves, B blocks of
// the Gram (0: none), workgroups, tiles staged through registers
void rec_pass16(const ArgsT<double>& a, int tr, int nw, int gram_ntb, int G,
                bool reg);

template <typename T, int TR, int NBUF, int CAP, int PC, int NW, bool SCR2,
          int MAXP, bool GRAM, int NTB, bool REG, int KS = 0>
static hipError_t go(const ArgsT<T>& a, int G, hipStream_t st, int* tag) {
  // 1 W P B S TT PP N: waves, workgroups per CU (+4 for binary32), tile
  // buffers (+5 with register staging), both partial-sum areas, tile rows
  // (mod 100), Gram pairs per wave (+50 with a compile-time update step
  // count), B blocks (0: no Gram)
  *tag = 1000000000 + NW * 100000000 +
         (PC + (sizeof(T) == 4 ? 4 : 0)) * 10000000 +
         (NBUF + (REG ? 5 : 0)) * 1000000 + (SCR2 ? 100000 : 0) +
         (TR % 100) * 1000 + (MAXP + (KS ? 50 : 0)) * 10 + (GRAM ? NTB : 0);
  if (rec_active()) {
    // the same pass as a step of G work items: any shape with four waves
    // per workgroup (K split four ways, as here) gives the same bits
    if constexpr (sizeof(T) == 8 && NW == 4)
      rec_pass16(a, TR, NW, GRAM ? NTB : 0, G, REG);
    else
      rec_unsupported();
    return hipSuccess;
  }
  if constexpr (PC == 2) {
    if constexpr (SCR2)
      hipLaunchKernelGGL(
          (pass16_s2_kernel<T, TR, NBUF, CAP, MAXP, GRAM, NTB, REG, KS>),
          dim3((unsigned)G), dim3(256), 0, st, a);
    else
      hipLaunchKernelGGL(
          (pass16_kernel<T, TR, NBUF, CAP, MAXP, GRAM, NTB, REG, KS>),
          dim3((unsigned)G), dim3(256), 0, st, a);
    prof_name("%s<%s, %d, %d, %d, %d, %s, %d, %s, %d>",
              SCR2 ? "pass16_s2_kernel" : "pass16_kernel", type_name<T>(), TR,
              NBUF, CAP, MAXP, bool_name(GRAM), NTB, bool_name(REG), KS);
  } else {
    hipLaunchKernelGGL(
        (pass16_deep_kernel<T, TR, NBUF, CAP, NW, SCR2, MAXP, GRAM, NTB, REG>),
        dim3((unsigned)G), dim3(NW * 64), 0, st, a);
    prof_name("pass16_deep_kernel<%s, %d, %d, %d, %d, %s, %d, %s, %d, %s>",
              type_name<T>(), TR, NBUF, CAP, NW, bool_name(SCR2), MAXP,
              bool_name(GRAM), NTB, bool_name(REG));
  }
  return hipGetLastError();
}

// (tile rows, buffers, column capacity, workgroups per CU, waves, both
// partial-sum areas)
struct Shape { int tr, nbuf, cap, per_cu, nw, scr2; };

// problems of at most this many rows take shapes of four waves when one
// fits (see launch_pass16_t)
constexpr int64_t kSmallRows = int64_t(1) << 18;

// Binary64 shapes.  The launcher picks among these (or takes the tuned /
// BCGS_PASS16_SHAPE index); dispatch() instantiates the same list, entry by
// entry.  Taller tiles stream faster (each copy instruction covers fewer
// columns, so fewer pages and longer runs per column: on MI355X about 4.2,
// 5.7 and 6.3 TB/s for 16, 32 and 64 rows), so wide passes take one
// workgroup of 8 waves per CU with 32- or 64-row tiles.  Shape 6 takes up
// to 544 columns (n up to 512 at s = 16) in one 8-wave workgroup per CU.
// Shape 7 is shape 4 with room for both updates' partial sums (one combine
// round per tile instead of two) at 256 columns, the most that keeps two
// workgroups per CU (2 x 81920 bytes of LDS).
constexpr Shape kShapes[] = {
    {64, 2, 64, 2, 4, 0},  {64, 2, 128, 1, 8, 0}, {32, 2, 272, 1, 8, 0},
    {32, 2, 128, 2, 4, 0}, {16, 2, 272, 2, 4, 0}, {16, 4, 272, 1, 4, 1},
    {16, 2, 544, 1, 8, 0}, {16, 2, 256, 2, 4, 1}};
constexpr int kNShapes = sizeof(kShapes) / sizeof(kShapes[0]);

// Binary32 shapes: the same bytes per column and tile as the 16-row
// binary64 ones (32 rows of 4 bytes), so the same LDS budget.
constexpr Shape kShapesF[] = {
    {32, 2, 128, 2, 4, 0}, {32, 2, 272, 2, 4, 0}, {32, 2, 544, 1, 8, 0}};
constexpr int kNShapesF = sizeof(kShapesF) / sizeof(kShapesF[0]);

template <typename T> struct ShapeList;
template <> struct ShapeList<double> {
  static const Shape* get() { return kShapes; }
  static constexpr int n = kNShapes;
};
template <> struct ShapeList<float> {
  static const Shape* get() { return kShapesF; }
  static constexpr int n = kNShapesF;
};

static inline int shape_maxp(const Shape& sh, int npairs) {
  return (npairs + sh.nw - 1) / sh.nw;
}

template <typename T>
static bool shape_fits(const Shape& sh, int ncols_p, int shared_ksteps,
                       int npairs, bool reg) {
  if (reg && sh.nbuf != 2) return false;
  const int kg = sh.nw / (sh.tr / 16);
  if ((shared_ksteps + kg - 1) / kg > kf_of<T>(sh.cap)) return false;
  if (shape_maxp(sh, npairs) > 9) return false;
  return ncols_p <= sh.cap;
}

// Gram launch with the smallest instantiated pair count per wave M >= maxp:
// every count from 2 up to the most pairs a wave of this shape can get (NTB
// B blocks), at most 9.  With two B blocks on a 16-row 4-wave shape, a pass
// whose block-update K-steps per wave fit 2 M - 2 (the one-sync passes: j
// steps for j + 2 staged blocks) takes the form with that compile-time step
// count (ks).
template <typename T, int TR, int NBUF, int CAP, int PC, int NW, bool SCR2,
          bool REG, int NTB, int M>
static hipError_t go_maxp(const ArgsT<T>& a, int G, int maxp, bool ks,
                          hipStream_t st, int* tag) {
  constexpr int kTop = ((CAP / 16) * NTB + NW - 1) / NW;
  constexpr bool kKs = NTB == 2 && TR == 16 && NW == 4 && sizeof(T) == 8 &&
                       2 * M - 2 >= 2 && 2 * M - 2 <= kf_of<T>(CAP);
  if constexpr (M >= kTop || M >= 9) {
    if constexpr (kKs)
      if (ks)
        return go<T, TR, NBUF, CAP, PC, NW, SCR2, M, true, NTB, REG,
                  2 * M - 2>(a, G, st, tag);
    return go<T, TR, NBUF, CAP, PC, NW, SCR2, M, true, NTB, REG>(a, G, st,
                                                                 tag);
  } else {
    if (maxp <= M) {
      if constexpr (kKs)
        if (ks)
          return go<T, TR, NBUF, CAP, PC, NW, SCR2, M, true, NTB, REG,
                    2 * M - 2>(a, G, st, tag);
      return go<T, TR, NBUF, CAP, PC, NW, SCR2, M, true, NTB, REG>(a, G, st,
                                                                   tag);
    }
    return go_maxp<T, TR, NBUF, CAP, PC, NW, SCR2, REG, NTB, M + 1>(
        a, G, maxp, ks, st, tag);
  }
}

template <typename T, int TR, int NBUF, int CAP, int PC, int NW, bool SCR2,
          bool REG>
static hipError_t go_shape(const ArgsT<T>& a, int G, bool gram, int ntb,
                           int maxp, bool ks, hipStream_t st, int* tag) {
  if (!gram)
    return go<T, TR, NBUF, CAP, PC, NW, SCR2, 1, false, 1, REG>(a, G, st,
                                                                tag);
  if (ntb == 1)
    return go_maxp<T, TR, NBUF, CAP, PC, NW, SCR2, REG, 1, 2>(a, G, maxp,
                                                              false, st, tag);
  return go_maxp<T, TR, NBUF, CAP, PC, NW, SCR2, REG, 2, 2>(a, G, maxp, ks,
                                                            st, tag);
}

// Launch shape `pick` of the storage type's list (REG: register-staged
// tiles).  Instantiated once per (T, REG) in pass16.hip, pass16_reg.hip and
// pass16_f32.hip.
template <typename T, bool REG>
hipError_t dispatch(int pick, const ArgsT<T>& a, int G, bool gram, int ntb,
                    int maxp, bool ks, hipStream_t st, int* tag) {
#define GS(...) \
  go_shape<T, __VA_ARGS__, REG>(a, G, gram, ntb, maxp, ks, st, tag)
  if constexpr (sizeof(T) == 8) {
    switch (pick) {
      case 0: return GS(64, 2, 64, 2, 4, false);
      case 1: return GS(64, 2, 128, 1, 8, false);
      case 2: return GS(32, 2, 272, 1, 8, false);
      case 3: return GS(32, 2, 128, 2, 4, false);
      case 4: return GS(16, 2, 272, 2, 4, false);
      case 5:
        if constexpr (!REG) return GS(16, 4, 272, 1, 4, true);
        return hipErrorNotSupported;
      case 6: return GS(16, 2, 544, 1, 8, false);
      case 7: return GS(16, 2, 256, 2, 4, true);
    }
  } else {
    switch (pick) {
      case 0: return GS(32, 2, 128, 2, 4, false);
      case 1: return GS(32, 2, 272, 2, 4, false);
      case 2: return GS(32, 2, 544, 1, 8, false);
    }
  }
  return hipErrorNotSupported;
#undef GS
}

#define P16_DISPATCH_DECL(T_, R_)                                          \
  hipError_t dispatch<T_, R_>(int, const ArgsT<T_>&, int, bool, int, int, \
                              bool, hipStream_t, int*)
extern template P16_DISPATCH_DECL(double, false);
extern template P16_DISPATCH_DECL(double, true);
extern template P16_DISPATCH_DECL(float, false);
extern template P16_DISPATCH_DECL(float, true);

// Shape choice and launch of one pass (hipErrorNotSupported, nothing
// launched, when no shape of the list takes it).  *G_out receives the
// number of workgroups used.
template <typename T>
hipError_t launch_pass16_t(const PassArgs<T>& pa, int64_t m,
                           const Tuning& tune, hipStream_t st, int* tag,
                           int* G_out) {
  const Shape* shapes = ShapeList<T>::get();
  constexpr int nshapes = ShapeList<T>::n;
  const int s = pa.s;
  if (pa.sp != 16 || s % 4 != 0) return hipErrorNotSupported;
  if (pa.groups != 1) return hipErrorNotSupported;
  if (pa.upd1 && pa.upd2 && pa.u2_c0 != pa.u1_c0 + s)
    return hipErrorNotSupported;
  auto al16 = [](const void* p) {
    return (reinterpret_cast<uintptr_t>(p) & 15) == 0;
  };
  // direct copies need 16-byte aligned columns; otherwise the tiles are
  // staged through registers
  constexpr int E = kEpg<T>;
  const bool dma = (pa.ldq % E == 0) && al16(pa.q) &&
                   (!pa.fcols || (pa.ldf % E == 0 && al16(pa.f))) &&
                   (!pa.ecols || (pa.lde % E == 0 && al16(pa.e)));
  const bool reg = !dma;
  const int nks1 = pa.upd1 ? (pa.u1_c0 + s) / 4 : 0;
  const int nks2 = pa.upd2 ? pa.u2_c0 / 4 : 0;
  const int shared = std::max(nks1, nks2);
  const int ntb = pa.gram ? pa.gbn_p / 16 : 1;
  if (ntb > 2) return hipErrorNotSupported;
  const int npairs = pa.gram ? (pa.ga_p / 16) * ntb : 0;
  int pick = -1;
  int f = tune.shape;
  if (f < 0 && sizeof(T) == 8) {
    if (const char* env = getenv("BCGS_PASS16_SHAPE")) f = atoi(env);
  }
  if (f >= 0 && f < nshapes &&
      shape_fits<T>(shapes[f], pa.ncols_p, shared, npairs, reg))
    pick = f;
  if constexpr (sizeof(T) == 8) {
    // Automatic choice, measured on MI355X: passes with two B blocks of
    // Gram (P-1S, P-2S) are bound by the MFMA work and run best with
    // 16-row tiles, two workgroups per CU; the other wide passes are bound
    // by the stream and take the 32-row, 8-wave shape.
    static const int kHeavy[] = {0, 3, 7, 4, 2, 5, 1, 6};
    static const int kLight[] = {0, 3, 2, 4, 7, 5, 1, 6};
    // small problems (the sizes batches and queues mix) keep to shapes of
    // four waves, which the batched persistent kernel also runs, so a
    // problem gives the same bits alone and in a batch
    static const int kSmall[] = {0, 3, 7, 4, 5, 2, 1, 6};
    static_assert(sizeof(kHeavy) / sizeof(int) == nshapes, "every shape");
    const bool small = m <= kSmallRows;
    const int* order = small ? kSmall
                             : (pa.gram && ntb == 2) ? kHeavy : kLight;
    // Measured per pass (tall PIPI+, P-1S): a pass with one Gram B block and
    // a block update runs faster in shape 7 than in the 8-wave 32-row shape
    // from 129 up to 208 columns (256 with both updates); wider, or with the
    // Gram or an update alone (BCGSI+), the 32-row shape is faster.
    if (pick < 0 && !small && pa.gram && ntb == 1 && (pa.upd1 || pa.upd2) &&
        pa.ncols_p > 128 && pa.ncols_p <= (pa.upd1 && pa.upd2 ? 256 : 208) &&
        shape_fits<T>(shapes[7], pa.ncols_p, shared, npairs, reg))
      pick = 7;
    for (int i = 0; pick < 0 && i < nshapes; ++i)
      if (shape_fits<T>(shapes[order[i]], pa.ncols_p, shared, npairs, reg))
        pick = order[i];
  } else {
    for (int i = 0; pick < 0 && i < nshapes; ++i)
      if (shape_fits<T>(shapes[i], pa.ncols_p, shared, npairs, reg)) pick = i;
  }
  if (pick < 0) return hipErrorNotSupported;
  const Shape sh = shapes[pick];
  const int maxp = shape_maxp(sh, npairs);
  ArgsT<T> a{};
  // G = 256 * per_cu workgroups (256 CUs on MI355X), at most tune.max_wg,
  // each with about m / G rows.  The tiles are dealt round-robin to the
  // workgroups (measured on the tall P-1S, P-2S and BCGSI+ runs: 0.1-2 %
  // faster than contiguous row ranges); BCGS_PASS16_INTERLEAVE=0 selects
  // the contiguous ranges.
  const int64_t rpw =
      std::max(round_up64(cdiv(m, 256 * sh.per_cu), 64),
               round_up64(cdiv(m, std::max(1, tune.max_wg)), 64));
  const int G = (int)cdiv(m, rpw);
  a.m = pa.m; a.s = s; a.ncols = pa.ncols; a.ncols_p = pa.ncols_p;
  a.rows_per_wg = rpw;
  {
    const char* e = getenv("BCGS_PASS16_INTERLEAVE");
    a.interleave = e ? atoi(e) != 0 : 1;
  }
  a.q = pa.q; a.ldq = pa.ldq; a.nq = pa.nq;
  a.f = pa.f; a.ldf = pa.ldf; a.fcols = pa.fcols;
  a.e = pa.e; a.lde = pa.lde; a.ecols = pa.ecols;
  a.upd1 = pa.upd1; a.u1_c0 = pa.u1_c0; a.c1 = pa.c1;
  a.dst1 = pa.dst1; a.ldd1 = pa.ldd1;
  a.upd2 = pa.upd2; a.u2_c0 = pa.u2_c0;
  a.c2 = pa.c2; a.dst2 = pa.dst2; a.ldd2 = pa.ldd2;
  a.gram = pa.gram; a.ga_p = pa.ga_p; a.gb0 = pa.gb0; a.gbn_p = pa.gbn_p;
  a.skip_a0 = pa.skip_a0; a.skip_b1 = pa.skip_b1;
  a.partial = pa.partial;
  *G_out = G;
  const bool gram = pa.gram;
  // compile-time update step count: K-steps per wave within 2 maxp - 2
  const int kg = sh.nw / (sh.tr / 16);
  const int per = (shared + kg - 1) / kg;
  const bool ks = gram && ntb == 2 && (pa.upd1 || pa.upd2) && per >= 1 &&
                  per <= 2 * maxp - 2;
  return reg ? dispatch<T, true>(pick, a, G, gram, ntb, maxp, ks, st, tag)
             : dispatch<T, false>(pick, a, G, gram, ntb, maxp, ks, st, tag);
}

}  // namespace p16
}  // namespace bcgs
