// Streaming pass for block widths s <= 16 (one 16-wide MFMA column block),
// the shape of every large workload.  Same operation as pass.hip (block
// updates of Alg. 1 / Alg. 2 fused with the tall-skinny Gram products),
// organised for gfx950:
//
//  * NW = 4 waves per workgroup and two workgroups per CU when the tiles
//    fit (one workgroup's MFMA work overlaps the other's serial phases),
//    else NW = 8 and one workgroup per CU; the row range is walked in tiles
//    of TR rows (16 or 32).
//  * Two LDS tile buffers.  While tile t is being computed, tile t+1 is
//    copied HBM -> LDS by direct-to-LDS loads (global_load_lds_dwordx4),
//    so HBM streaming overlaps the MFMA work.
//  * LDS tile layout: column c occupies TR consecutive doubles; within a
//    column the 16-byte granules (row pairs) are XOR-swizzled by a
//    per-column key, which keeps both MFMA fragment patterns (16 columns x
//    4 rows for the Gram, 4 columns x 16 rows for the updates) free of bank
//    conflicts.
//  * Block updates B <- [Q B] F (F = [-C T^{-1}; T^{-1}], see common.h):
//    waves = (TR/16 row blocks) x (KG K-ranges); every wave keeps its slice
//    of the coefficient fragments in registers for the whole kernel; both
//    updates of a pass share the Q fragments; the K-range partial products
//    are summed in LDS.
//  * Gram A^T B: the 16x16 output tiles are dealt round-robin to the waves,
//    which accumulate them in registers over the whole row range.
#include "common.h"

namespace bcgs {

namespace p16 {

typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kMaxKF = 16;            // C fragments per update per wave

__device__ __forceinline__ v4d mfma(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
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

struct Args {
  int64_t m;
  int s, ncols, ncols_p;
  int64_t rows_per_wg;
  const double* q; int64_t ldq; int nq;
  const double* f; int64_t ldf; int fcols;
  const double* e; int64_t lde; int ecols;
  int dma;                       // all leading dimensions even: 16B loads
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

// Issue the direct-to-LDS copy of a full tile (rows r0 .. r0+TR-1).
template <int NW, int TR>
__device__ __forceinline__ void tile_dma(const Args& a, double* buf,
                                         int64_t r0) {
  constexpr int kColsPerInst = 1024 / (TR * 8);     // 4 (TR=32) or 8 (16)
  constexpr int kGran = TR / 2;                      // granules per column
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ninst = (a.ncols + kColsPerInst - 1) / kColsPerInst;
  for (int ins = wave; ins < ninst; ins += NW) {
    const int c = ins * kColsPerInst + lane / kGran;
    const int g = lane % kGran;
    double* dst = buf + ins * kColsPerInst * TR;     // wave-uniform
    if (c < a.ncols) {
      int64_t ld;
      const double* src = col_ptr(a, c, &ld);
      const int rr = (g ^ swz<TR>(c)) << 1;
      __builtin_amdgcn_global_load_lds(src + r0 + rr, dst, 16, 0, 0);
    }
  }
}

// Synchronous staging (tail tiles, odd leading dimensions): zero past m.
template <int NW, int TR>
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

// Sum the K-range partial products of one block update into the tile
// columns [uc0, uc0 + s).  scr: [KG][TR][17] doubles.
template <int NW, int TR, int KG>
__device__ __forceinline__ void combine(const Args& a, double* tile,
                                        const double* scr, int uc0) {
  const int s = a.s;
  for (int t = threadIdx.x; t < TR * 16; t += NW * 64) {
    const int r = t >> 4, c = t & 15;
    if (c >= s) continue;
    double part[KG];
#pragma unroll
    for (int k = 0; k < KG; ++k) part[k] = scr[(k * TR + r) * 17 + c];
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < KG; ++k) sum += part[k];
    tile[at<TR>(uc0 + c, r)] = sum;
  }
}

// Copy an updated block (tile columns uc0..uc0+s-1) to HBM, coalesced.
template <int NW, int TR>
__device__ __forceinline__ void store_block(const Args& a, const double* tile,
                                            int uc0, double* dst, int64_t ldd,
                                            int64_t r0, int rows) {
  for (int idx = threadIdx.x; idx < a.s * TR; idx += NW * 64) {
    const int c = idx / TR, r = idx % TR;
    if (r < rows) dst[(int64_t)c * ldd + r0 + r] = tile[at<TR>(uc0 + c, r)];
  }
}

// two waves per SIMD: two 4-wave workgroups, or one 8-wave workgroup, per CU
template <int NW, int TR, int MAXA, bool GRAM, int NTB>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(2)))
void pass16_kernel(Args a) {
  constexpr int kT = NW * 64;
  constexpr int MB = TR / 16;         // row blocks per tile
  constexpr int KG = NW / MB;         // K ranges per update
  extern __shared__ double lds[];
  const int tile_elems = a.ncols_p * TR;
  double* buf0 = lds;
  double* buf1 = lds + tile_elems;
  double* scr = buf1 + tile_elems;                  // KG * TR * 17

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int mb = wave % MB, kg = wave / MB;
  const int64_t g = blockIdx.x;
  const int64_t row_begin = g * a.rows_per_wg;
  const int64_t row_end = min(a.m, row_begin + a.rows_per_wg);

  // ---- prologue: coefficient fragments --------------------------------
  // K-steps (4 columns each) of update 1: [0, nks1) over Q_{1:k-1} (shared
  // with update 2) and [nks1, nks1 + sq) over its own block; of update 2:
  // [0, nks1) shared, [nks1, nks2) over the block update 1 rewrites (after
  // it), and [nks2, nks2 + sq) over its own block F.  Without update 1,
  // update 2's steps [0, nks2) are all "shared".
  const int s = a.s;
  const int sq = s / 4;
  const int nks1 = a.upd1 ? a.u1_c0 / 4 : 0;
  const int nks2 = a.upd2 ? a.u2_c0 / 4 : 0;
  const int shared = a.upd1 ? nks1 : nks2;
  const int per = (shared + KG - 1) / KG;
  const int kb = kg * per, ke = min(shared, kb + per);
  double c1f[kMaxKF], c2f[kMaxKF];
#pragma unroll
  for (int i = 0; i < kMaxKF; ++i) {
    const int k = kb + i;
    c1f[i] = 0.0;
    c2f[i] = 0.0;
    if (k < ke) {
      const int row = 4 * k + lk;
      if (a.upd1) c1f[i] = a.c1[row * 16 + li];
      if (a.upd2) c2f[i] = a.c2[row * 16 + li];
    }
  }
  // per-block steps, step t < sq goes to K range t % KG
  constexpr int kTail = (4 + KG - 1) / KG;
  const int ntail = (a.upd1 && a.upd2) ? sq : 0;   // update 2 over new block
  double c1o[kTail], c2o[kTail], c2t[kTail];
#pragma unroll
  for (int u = 0; u < kTail; ++u) {
    const int t = kg + KG * u;
    c1o[u] = (a.upd1 && t < sq) ? a.c1[(4 * (nks1 + t) + lk) * 16 + li] : 0.0;
    c2o[u] = (a.upd2 && t < sq) ? a.c2[(4 * (nks2 + t) + lk) * 16 + li] : 0.0;
    c2t[u] = t < ntail ? a.c2[(4 * (nks1 + t) + lk) * 16 + li] : 0.0;
  }
  for (int idx = a.ncols * TR + tid; idx < tile_elems; idx += kT) {
    buf0[idx] = 0.0;
    buf1[idx] = 0.0;
  }

  // ---- Gram: this wave owns A blocks ta = wave, wave + NW, ... and all
  //      NTB B blocks, so B fragments are shared across its A blocks ----
  v4d acc[MAXA][NTB];
  const int nta = a.ga_p >> 4;
#pragma unroll
  for (int i = 0; i < MAXA; ++i)
#pragma unroll
    for (int b = 0; b < NTB; ++b) acc[i][b] = v4d{0.0, 0.0, 0.0, 0.0};

  // ---- tile loop ---------------------------------------------------------
  bool prefetched = false;
  int it = 0;
  if (row_begin < row_end && a.dma && row_begin + TR <= row_end) {
    tile_dma<NW, TR>(a, buf0, row_begin);
    prefetched = true;
  }
  for (int64_t r0 = row_begin; r0 < row_end; r0 += TR, ++it) {
    double* tile = (it & 1) ? buf1 : buf0;
    double* next = (it & 1) ? buf0 : buf1;
    const int rows = (int)min((int64_t)TR, row_end - r0);
    if (!prefetched) tile_sync<NW, TR>(a, tile, r0, rows);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    // prefetch the next tile while this one is computed
    const int64_t r1 = r0 + TR;
    prefetched = false;
    if (a.dma && r1 + TR <= row_end) {
      tile_dma<NW, TR>(a, next, r1);
      prefetched = true;
    }

    // ---- block updates ----
    if (a.upd1 || a.upd2) {
      // K-steps in uniform chunks of 4; inside a chunk the four Q fragment
      // loads are issued first, K-steps past ke read a valid address and
      // meet zero coefficient fragments, so no lane-divergent branches
      v4d acc1 = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};
      v4d acc1b = {0.0, 0.0, 0.0, 0.0}, acc2b = {0.0, 0.0, 0.0, 0.0};
      const int kcl = max(kb, min(ke, shared) - 1);
#pragma unroll
      for (int q = 0; q < kMaxKF / 4; ++q) {
        if (4 * q >= ke - kb) break;
        double av[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = min(kb + 4 * q + u, kcl);
          av[u] = tile[at<TR>(4 * k + lk, mb * 16 + li)];
        }
#pragma unroll
        for (int u = 0; u < 4; u += 2) {
          if (a.upd1) acc1 = mfma(av[u], c1f[4 * q + u], acc1);
          if (a.upd2) acc2 = mfma(av[u], c2f[4 * q + u], acc2);
          if (a.upd1) acc1b = mfma(av[u + 1], c1f[4 * q + u + 1], acc1b);
          if (a.upd2) acc2b = mfma(av[u + 1], c2f[4 * q + u + 1], acc2b);
        }
      }
      // own-block steps (independent of update 1's result)
#pragma unroll
      for (int u = 0; u < kTail; ++u) {
        const int t = kg + KG * u;
        if (t < sq) {
          if (a.upd1)
            acc1b = mfma(tile[at<TR>(4 * (nks1 + t) + lk, mb * 16 + li)],
                         c1o[u], acc1b);
          if (a.upd2)
            acc2b = mfma(tile[at<TR>(4 * (nks2 + t) + lk, mb * 16 + li)],
                         c2o[u], acc2b);
        }
      }
      acc1 += acc1b;
      acc2 += acc2b;
      if (a.upd1) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          scr[(kg * TR + mb * 16 + lk + 4 * v) * 17 + li] = acc1[v];
        __syncthreads();
        combine<NW, TR, KG>(a, tile, scr, a.u1_c0);
        __syncthreads();
        store_block<NW, TR>(a, tile, a.u1_c0, a.dst1, a.ldd1, r0, rows);
        // update 2 over the block update 1 just formed
#pragma unroll
        for (int u = 0; u < kTail; ++u) {
          const int t = kg + KG * u;
          if (t < ntail)
            acc2 = mfma(tile[at<TR>(4 * (nks1 + t) + lk, mb * 16 + li)],
                        c2t[u], acc2);
        }
      }
      if (a.upd2) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          scr[(kg * TR + mb * 16 + lk + 4 * v) * 17 + li] = acc2[v];
        __syncthreads();
        combine<NW, TR, KG>(a, tile, scr, a.u2_c0);
        __syncthreads();
        store_block<NW, TR>(a, tile, a.u2_c0, a.dst2, a.ldd2, r0, rows);
      }
    }

    // ---- Gram accumulation: two MFMA K-steps per 16-byte LDS load (lane
    //      group lk takes rows kk + 2 lk and kk + 2 lk + 1) ----
    if (GRAM) {
#pragma unroll
      for (int kk = 0; kk < TR; kk += 8) {
        const int r = kk + 2 * lk;
        double2 bf[NTB], af[MAXA];
#pragma unroll
        for (int b = 0; b < NTB; ++b)
          bf[b] = *reinterpret_cast<const double2*>(
              tile + at<TR>(a.gb0 + b * 16 + li, r));
#pragma unroll
        for (int i = 0; i < MAXA; ++i) {
          // A blocks past the last are computed on a valid block and
          // never stored
          const int ta = min(wave + NW * i, nta - 1);
          af[i] = *reinterpret_cast<const double2*>(
              tile + at<TR>(ta * 16 + li, r));
        }
#pragma unroll
        for (int i = 0; i < MAXA; ++i)
#pragma unroll
          for (int b = 0; b < NTB; ++b)
            acc[i][b] = mfma(af[i].x, bf[b].x, acc[i][b]);
#pragma unroll
        for (int i = 0; i < MAXA; ++i)
#pragma unroll
          for (int b = 0; b < NTB; ++b)
            acc[i][b] = mfma(af[i].y, bf[b].y, acc[i][b]);
      }
    }
  }
  __builtin_amdgcn_s_waitcnt(0);

  if (GRAM) {
    double* out = a.partial + (size_t)g * a.ga_p * a.gbn_p;
#pragma unroll
    for (int i = 0; i < MAXA; ++i) {
      const int ta = wave + NW * i;
      if (ta >= nta) continue;
#pragma unroll
      for (int b = 0; b < NTB; ++b) {
        if (ta * 16 >= a.skip_a0 && b * 16 + 16 <= a.skip_b1) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v)
          out[(size_t)(b * 16 + li) * a.ga_p + ta * 16 + lk + 4 * v] =
              acc[i][b][v];
      }
    }
  }
}

template <int NW, int TR, int MAXA, bool GRAM, int NTB>
static hipError_t go(const Args& a, int G, size_t lds, hipStream_t st,
                     int* tag) {
  auto kern = pass16_kernel<NW, TR, MAXA, GRAM, NTB>;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)kern,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    attr = true;
  }
  // 1NWTTMMG: waves, tile rows, A blocks per wave, B blocks (0: no Gram)
  *tag = 10000000 + NW * 1000000 + TR * 1000 + MAXA * 10 + (GRAM ? NTB : 0);
  hipLaunchKernelGGL(kern, dim3((unsigned)G), dim3(NW * 64), lds, st, a);
  return hipGetLastError();
}

}  // namespace p16

size_t pass16_lds_bytes(int ncols_p, int tr, int nw) {
  const int kg = nw / (tr / 16);
  return ((size_t)2 * ncols_p * tr + (size_t)kg * tr * 17) * sizeof(double);
}

// Returns hipErrorNotSupported (without launching) when this kernel cannot
// take the pass.  *G_out receives the number of workgroups used (the row
// split is a function of m and of the chosen shape only).
hipError_t launch_pass16(const PassArgs<double>& pa, int64_t m, hipStream_t st,
                         int* tag, int* G_out) {
  using namespace p16;
  const int s = pa.s;
  if (pa.sp != 16 || s % 4 != 0) return hipErrorNotSupported;
  if (pa.groups != 1) return hipErrorNotSupported;
  const int K1 = pa.upd1 ? pa.u1_c0 : 0;
  const int K2 = pa.upd2 ? pa.u2_c0 : 0;
  const int shared_cols = pa.upd1 ? K1 : K2;
  // shapes in order of preference: (waves, tile rows, workgroups per CU)
  const int shapes[5][3] = {{4, 64, 2}, {4, 32, 2}, {4, 16, 2},
                            {8, 32, 1}, {8, 16, 1}};
  int nw = 0, tr = 0, per_cu = 1;
  for (const auto& sh : shapes) {
    const int kg = sh[0] / (sh[1] / 16);
    const int per = ((shared_cols / 4) + kg - 1) / kg;
    if (per > kMaxKF) continue;
    if (pa.gram && (pa.ga_p / 16 + sh[0] - 1) / sh[0] > 5) continue;
    if (pass16_lds_bytes(pa.ncols_p, sh[1], sh[0]) * sh[2] > 160 * 1024)
      continue;
    nw = sh[0]; tr = sh[1]; per_cu = sh[2];
    break;
  }
  if (!nw) return hipErrorNotSupported;
  const int ntb = pa.gbn_p / 16;
  const int maxa = pa.gram ? (pa.ga_p / 16 + nw - 1) / nw : 0;
  if (pa.gram && (ntb > 2 || maxa > 5)) return hipErrorNotSupported;
  Args a{};
  // rows split over 256 * per_cu workgroups (256 CUs on MI355X)
  const int64_t rpw = round_up64(cdiv(m, 256 * per_cu), 64);
  const int G = (int)cdiv(m, rpw);
  a.m = pa.m; a.s = s; a.ncols = pa.ncols; a.ncols_p = pa.ncols_p;
  a.rows_per_wg = rpw;
  a.q = pa.q; a.ldq = pa.ldq; a.nq = pa.nq;
  a.f = pa.f; a.ldf = pa.ldf; a.fcols = pa.fcols;
  a.e = pa.e; a.lde = pa.lde; a.ecols = pa.ecols;
  auto al16 = [](const void* p) {
    return (reinterpret_cast<uintptr_t>(p) & 15) == 0;
  };
  a.dma = (pa.ldq % 2 == 0) && al16(pa.q) &&
          (!pa.fcols || (pa.ldf % 2 == 0 && al16(pa.f))) &&
          (!pa.ecols || (pa.lde % 2 == 0 && al16(pa.e)));
  a.upd1 = pa.upd1; a.u1_c0 = pa.u1_c0; a.c1 = pa.c1;
  a.dst1 = pa.dst1; a.ldd1 = pa.ldd1;
  a.upd2 = pa.upd2; a.u2_c0 = pa.u2_c0;
  a.c2 = pa.c2; a.dst2 = pa.dst2; a.ldd2 = pa.ldd2;
  a.gram = pa.gram; a.ga_p = pa.ga_p; a.gb0 = pa.gb0; a.gbn_p = pa.gbn_p;
  a.skip_a0 = pa.skip_a0; a.skip_b1 = pa.skip_b1;
  a.partial = pa.partial;
  *G_out = G;
  const size_t lds = pass16_lds_bytes(pa.ncols_p, tr, nw);
  if (!pa.gram) {
    if (nw == 4 && tr == 64) return go<4, 64, 1, false, 1>(a, G, lds, st, tag);
    if (nw == 4 && tr == 32) return go<4, 32, 1, false, 1>(a, G, lds, st, tag);
    if (nw == 4) return go<4, 16, 1, false, 1>(a, G, lds, st, tag);
    if (tr == 32) return go<8, 32, 1, false, 1>(a, G, lds, st, tag);
    return go<8, 16, 1, false, 1>(a, G, lds, st, tag);
  }
#define P16(NW_, TR_, MA_, NTB_)                                          \
  if (nw == NW_ && tr == TR_ && ntb == NTB_ && maxa <= MA_)               \
    return go<NW_, TR_, MA_, true, NTB_>(a, G, lds, st, tag);
  P16(4, 64, 2, 1) P16(4, 64, 3, 1) P16(4, 64, 5, 1)
  P16(4, 64, 2, 2) P16(4, 64, 3, 2) P16(4, 64, 5, 2)
  P16(4, 32, 2, 1) P16(4, 32, 3, 1) P16(4, 32, 5, 1)
  P16(4, 32, 2, 2) P16(4, 32, 3, 2) P16(4, 32, 5, 2)
  P16(4, 16, 2, 1) P16(4, 16, 3, 1) P16(4, 16, 5, 1)
  P16(4, 16, 2, 2) P16(4, 16, 3, 2) P16(4, 16, 5, 2)
  P16(8, 32, 2, 1) P16(8, 32, 3, 1) P16(8, 32, 5, 1)
  P16(8, 32, 2, 2) P16(8, 32, 3, 2) P16(8, 32, 5, 2)
  P16(8, 16, 2, 1) P16(8, 16, 3, 1) P16(8, 16, 5, 1)
  P16(8, 16, 2, 2) P16(8, 16, 3, 2) P16(8, 16, 5, 2)
#undef P16
  return hipErrorNotSupported;
}

}  // namespace bcgs
