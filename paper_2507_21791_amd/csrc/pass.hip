// Streaming pass over the m rows: block updates and tall-skinny Gram
// products of Alg. 1 / Alg. 2 (and of BCGSI+), fused per row tile.
//
// One workgroup owns a contiguous row range and walks it in tiles of TR
// rows.  Per tile:
//   1. stage the needed column window in LDS (coalesced: consecutive lanes
//      read consecutive rows of one column; rows past m are zero),
//   2. optional block update 1 (Q_k = (U_k - Q_{1:k-1} Y) Y_kk^{-1}),
//   3. optional block update 2 (U_{k+1} = (X_{k+1} - Q_{1:k} S) S^{-1}, or
//      V = X_{k+1} - Q_{1:k} S without the triangular factor),
//      both as FP64 MFMA products followed by a row-wise substitution with
//      the upper-triangular factor, written back to HBM in place,
//   4. optional Gram accumulation A^T B of LDS columns (the tall-skinny
//      products that the paper's synchronizations reduce, section 3) with
//      FP64 MFMA; each wave keeps a fixed set of 16x16 output tiles in
//      registers for the whole row range.
// The partial Gram matrices of all workgroups are then summed in a fixed
// order by gram_reduce_kernel, so results do not depend on timing.
//
// The tile, the products and the per-workgroup partial sums are in the
// storage type T: FP64 for the FP64 form, FP32 for the FP32-bulk form
// (whose partials are widened to FP64 before the cross-workgroup sum).
//
// MFMA 16x16x4 operand layout (lane l of 64), FP64 and FP32 alike:
//   A (16 x 4): A[l % 16][l / 16]     B (4 x 16): B[l / 16][l % 16]
// Result D (16 x 16), 4 values v per lane, column l % 16, row
//   FP64 (v_mfma_f64_16x16x4f64): l / 16 + 4 v
//   FP32 (v_mfma_f32_16x16x4f32): 4 (l / 16) + v
#include "common.h"
#include "small_impl.h"

namespace bcgs {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T> struct Mma;
template <> struct Mma<double> {
  typedef v4d acc;
  static __device__ __forceinline__ v4d mac(double a, double b, v4d c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) {
    return lk + 4 * v;
  }
};
template <> struct Mma<float> {
  typedef v4f acc;
  static __device__ __forceinline__ v4f mac(float a, float b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int v) {
    return 4 * lk + v;
  }
};

template <typename T>
__device__ __forceinline__ const T* col_src(const PassArgs<T>& a, int c,
                                            int64_t* ld) {
  if (c < a.nq) { *ld = a.ldq; return a.q + (int64_t)c * a.ldq; }
  c -= a.nq;
  if (c < a.fcols) { *ld = a.ldf; return a.f + (int64_t)c * a.ldf; }
  c -= a.fcols;
  *ld = a.lde;
  return a.e + (int64_t)c * a.lde;
}

// Block update of the tile columns [uc0, uc0 + s):
//   out = tile[:, 0:uc0+s] * F        (MFMA over K = uc0 + s columns)
// with F = [-C T^{-1}; T^{-1}] or [-C; I] (see common.h); the K range is
// split over the waves.  update_partials() leaves the partial products in
// scr; update_finish() sums them into the tile and into dst.  When a pass
// has two updates, both run on the staged columns before either result is
// written back (the second one's coefficients already account for the
// first, see fold_coefs in epilogue.hip).
__device__ __forceinline__ int update_ksplit(int tr, int sp) {
  const int nt = (tr >> 4) * (sp >> 4);
  return nt >= kWaves ? 1 : kWaves / nt;
}

// MULTI: K-steps four at a time on four accumulators (for the kernels
// without Gram accumulators, whose registers allow it); otherwise one
// accumulator, so the Gram kernels keep their occupancy.
template <typename T, bool MULTI>
__device__ void update_partials(const PassArgs<T>& a, const T* tile,
                                int trp, T* scr, int uc0,
                                const double* __restrict__ F) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tr = a.tr, sp = a.sp, s = a.s;
  const int mb = tr >> 4, nb = sp >> 4, nt = mb * nb;
  const int ksplit = update_ksplit(tr, sp);
  const int K = uc0 + s;
  const int ksteps = (K + 3) >> 2;
  const int kper = (ksteps + ksplit - 1) / ksplit;
  const int srow = sp + 1;     // padded scratch row
  const int li = lane & 15, lk = lane >> 4;
  for (int task = wave; task < nt * ksplit; task += kWaves) {
    const int t = task % nt, ks = task / nt;
    const int rb = t % mb, cb = t / mb;
    typename Mma<T>::acc acc = {0, 0, 0, 0};
    const int kb = ks * kper, ke = min(ksteps, kb + kper);
    auto operands = [&](int kk, T& av, T& bv) {
      const int k = kk * 4 + lk;
      av = 0;
      bv = 0;
      if (kk < ke && k < K) {
        av = tile[k * trp + rb * 16 + li];
        bv = static_cast<T>(F[k * sp + cb * 16 + li]);
      }
    };
    if constexpr (MULTI) {
      // four independent MFMA chains over groups of 16 K-steps: the 16
      // coefficient loads (global) and tile loads of a group are issued
      // before its first MFMA; the chains are summed in a fixed order
      typename Mma<T>::acc acc1 = acc, acc2 = acc, acc3 = acc;
      constexpr int kG = 16;
      for (int kk = kb; kk < ke; kk += kG) {
        T av[kG], bv[kG];
#pragma unroll
        for (int u = 0; u < kG; ++u) operands(kk + u, av[u], bv[u]);
#pragma unroll
        for (int u = 0; u < kG; u += 4) {
          acc = Mma<T>::mac(av[u], bv[u], acc);
          acc1 = Mma<T>::mac(av[u + 1], bv[u + 1], acc1);
          acc2 = Mma<T>::mac(av[u + 2], bv[u + 2], acc2);
          acc3 = Mma<T>::mac(av[u + 3], bv[u + 3], acc3);
        }
      }
      acc += acc1;
      acc2 += acc3;
      acc += acc2;
    } else {
      // one chain (the Gram accumulators hold the registers); the loads of
      // four K-steps are issued before their MFMAs
      for (int kk = kb; kk < ke; kk += 4) {
        T av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) operands(kk + u, av[u], bv[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = Mma<T>::mac(av[u], bv[u], acc);
      }
    }
    T* out = scr + (size_t)ks * tr * srow;
#pragma unroll
    for (int v = 0; v < 4; ++v)
      out[(rb * 16 + Mma<T>::row(lk, v)) * srow + cb * 16 + li] = acc[v];
  }
}

template <typename T>
__device__ void update_finish(const PassArgs<T>& a, T* tile, int trp,
                              const T* scr, int uc0, T* dst,
                              int64_t ldd, int64_t r0, int rows) {
  const int tr = a.tr, s = a.s, srow = a.sp + 1;
  const int ksplit = update_ksplit(tr, a.sp);
  for (int e = threadIdx.x; e < tr * s; e += kThreads) {
    const int r = e % tr, c = e / tr;
    T sum = 0;
    for (int ks = 0; ks < ksplit; ++ks)
      sum += scr[(size_t)ks * tr * srow + r * srow + c];
    tile[(uc0 + c) * trp + r] = sum;
    if (r < rows) dst[(int64_t)c * ldd + r0 + r] = sum;
  }
}

template <typename T, bool GRAM, int NTB, int MAXA>
__global__ __launch_bounds__(kThreads) void pass_kernel(PassArgs<T> a) {
  extern __shared__ double lds[];
  const int tr = a.tr, trp = tr + 1;
  T* tile = reinterpret_cast<T*>(lds);
  T* scr = tile + (size_t)a.ncols_p * trp;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int h = blockIdx.x % a.groups;
  const int64_t g = blockIdx.x / a.groups;
  const int64_t row_begin = g * a.rows_per_wg;
  const int64_t row_end = min(a.m, row_begin + a.rows_per_wg);


  typename Mma<T>::acc acc[MAXA][NTB];
  int ta_of[MAXA];
  const int ta_total = a.ga_p >> 4;
  const int ta_lo = h * a.a_blocks_per_group;
  const int ta_hi = min(ta_total, ta_lo + a.a_blocks_per_group);
#pragma unroll
  for (int i = 0; i < MAXA; ++i) {
    ta_of[i] = ta_lo + wave + kWaves * i;
#pragma unroll
    for (int b = 0; b < NTB; ++b) acc[i][b] = typename Mma<T>::acc{0, 0, 0, 0};
  }
  __syncthreads();

  const int tr_shift = __ffs(tr) - 1;
  const int nstage = a.ncols_p << tr_shift;
  for (int64_t r0 = row_begin; r0 < row_end; r0 += tr) {
    const int rows = (int)min((int64_t)tr, row_end - r0);
    // 1. stage the column window (zero past m and past ncols), eight
    //    elements per thread at a time: all eight loads are issued before
    //    the first is written to LDS
    constexpr int kBatch = 8;
    for (int base = tid; base < nstage; base += kBatch * kThreads) {
      T v[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int idx = base + u * kThreads;
        const int c = idx >> tr_shift, r = idx & (tr - 1);
        v[u] = 0;
        if (idx < nstage && r < rows && c < a.ncols) {
          int64_t ld;
          const T* src = col_src(a, c, &ld);
          v[u] = src[r0 + r];
        }
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int idx = base + u * kThreads;
        if (idx < nstage)
          tile[(idx >> tr_shift) * trp + (idx & (tr - 1))] = v[u];
      }
    }
    __syncthreads();
    // 2-3. block updates, both on the staged columns
    if (a.upd1 || a.upd2) {
      T* scr2 = a.upd1 ? scr + (size_t)update_ksplit(tr, a.sp) * tr *
                                        (a.sp + 1)
                            : scr;
      if (a.upd1) update_partials<T, !GRAM>(a, tile, trp, scr, a.u1_c0, a.c1);
      if (a.upd2)
        update_partials<T, !GRAM>(a, tile, trp, scr2, a.u2_c0, a.c2);
      __syncthreads();
      if (a.upd1)
        update_finish(a, tile, trp, scr, a.u1_c0, a.dst1, a.ldd1, r0, rows);
      if (a.upd2)
        update_finish(a, tile, trp, scr2, a.u2_c0, a.dst2, a.ldd2, r0, rows);
      __syncthreads();
    }
    // 4. Gram accumulation over this tile's rows
    if (GRAM) {
      for (int kk = 0; kk < tr; kk += 4) {
        const int r = kk + lk;
        T bf[NTB];
#pragma unroll
        for (int b = 0; b < NTB; ++b)
          bf[b] = tile[(a.gb0 + b * 16 + li) * trp + r];
#pragma unroll
        for (int i = 0; i < MAXA; ++i) {
          const int ta = ta_of[i];
          if (ta < ta_hi) {
            const T af = tile[(ta * 16 + li) * trp + r];
#pragma unroll
            for (int b = 0; b < NTB; ++b) {
              if (ta * 16 >= a.skip_a0 && b * 16 + 16 <= a.skip_b1) continue;
              acc[i][b] = Mma<T>::mac(af, bf[b], acc[i][b]);
            }
          }
        }
      }
    }
    __syncthreads();
  }

  if (GRAM) {
    double* out = a.partial + (size_t)g * a.ga_p * a.gbn_p;
#pragma unroll
    for (int i = 0; i < MAXA; ++i) {
      const int ta = ta_of[i];
      if (ta >= ta_hi) continue;
#pragma unroll
      for (int b = 0; b < NTB; ++b) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          out[(size_t)(b * 16 + li) * a.ga_p + ta * 16 + Mma<T>::row(lk, v)] =
              static_cast<double>(acc[i][b][v]);
      }
    }
  }
}

__global__ __launch_bounds__(kRedWaves * 64) void gram_reduce_kernel(
    const double* __restrict__ partial, int G, int64_t elems,
    double* __restrict__ out, int32_t* syncs) {
  __shared__ double red[kRedWaves * 64];
  reduce_body(partial, G, elems, out, syncs, red, blockIdx.x);
}

hipError_t launch_gram_reduce(const double* partial, int G, int64_t elems,
                              double* out, int32_t* syncs, hipStream_t st) {
  const int64_t blocks = cdiv(elems, 64);
  if (rec_active()) {
    rec_reduce(partial, G, elems, out, syncs, blocks);
    return hipSuccess;
  }
  prof_begin(BCGS_KERNEL_REDUCE, 0, 8.0 * elems * (G + 1),
             (double)elems * G);
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)blocks),
                     dim3(kRedWaves * 64), 0, st, partial, G, elems, out,
                     syncs);
  prof_name("gram_reduce_kernel");
  prof_end();
  return hipGetLastError();
}

template <typename T>
size_t pass_lds_bytes(const PassArgs<T>& a) {
  const int nt = (a.tr / 16) * (a.sp / 16);
  const int ksplit = nt >= kWaves ? 1 : kWaves / nt;
  const int nupd = (a.upd1 ? 1 : 0) + (a.upd2 ? 1 : 0);
  size_t d = (size_t)a.ncols_p * (a.tr + 1) +
             (size_t)(nupd > 1 ? 2 : 1) * ksplit * a.tr * (a.sp + 1);
  return d * sizeof(T);
}

template <typename T, bool GRAM, int NTB, int MAXA>
static hipError_t launch_one(const PassArgs<T>& a, int G, hipStream_t st,
                             int* tag) {
  *tag = (sizeof(T) == 4 ? 1000 : 0) + (GRAM ? 100 : 0) + 10 * NTB + MAXA;
  if (rec_active()) {
    rec_unsupported();
    return hipSuccess;
  }
  auto kern = pass_kernel<T, GRAM, NTB, MAXA>;
  const size_t lds = pass_lds_bytes(a);
  static bool attr_done = false;
  if (!attr_done) {
    (void)hipFuncSetAttribute((const void*)kern,
                        hipFuncAttributeMaxDynamicSharedMemorySize,
                        160 * 1024);
    attr_done = true;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)(G * a.groups)), dim3(kThreads),
                     lds, st, a);
  prof_name("pass_kernel<%s, %s, %d, %d>", type_name<T>(), bool_name(GRAM),
            NTB, MAXA);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pass(const PassArgs<T>& a, int G, hipStream_t st,
                       int* tag) {
  if (!a.gram) return launch_one<T, false, 1, 1>(a, G, st, tag);
  const int ntb = a.gbn_p / 16;
  const int maxa = (a.a_blocks_per_group + kWaves - 1) / kWaves;
#define BCGS_TRY(NTB_, MAXA_)                                  \
  if (ntb == NTB_ && maxa <= MAXA_)                            \
    return launch_one<T, true, NTB_, MAXA_>(a, G, st, tag);
  BCGS_TRY(1, 1) BCGS_TRY(1, 2) BCGS_TRY(1, 4) BCGS_TRY(1, 8)
  BCGS_TRY(2, 1) BCGS_TRY(2, 2) BCGS_TRY(2, 4) BCGS_TRY(2, 8)
  BCGS_TRY(4, 1) BCGS_TRY(4, 2) BCGS_TRY(4, 4)
  BCGS_TRY(8, 1) BCGS_TRY(8, 2)
#undef BCGS_TRY
  return hipErrorInvalidValue;
}

template hipError_t launch_pass<double>(const PassArgs<double>&, int,
                                        hipStream_t, int*);
template size_t pass_lds_bytes<double>(const PassArgs<double>&);
template hipError_t launch_pass<float>(const PassArgs<float>&, int,
                                       hipStream_t, int*);
template size_t pass_lds_bytes<float>(const PassArgs<float>&);

}  // namespace bcgs
