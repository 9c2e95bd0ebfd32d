// TSQR for block widths s <= 16 with one 64-lane wave per row chunk.
//
// Same tree as the workgroup TSQR (leaf pass, upward node levels with the
// sign normalization at the root, downward coefficients, apply pass that
// recomputes the chunk reflectors and forms the explicit Q rows); see the
// section 1 / section 2.3 description of TSQR as the unconditionally stable
// intra-orthogonalization.  What changes is the granularity: a wave owns a
// chunk of L = 64 R rows (R = 64 / s rows per lane, lane l holding rows
// l, l + 64, ... with all s columns in registers), so a Householder step
// needs no LDS and no barrier:
//   - the column norm and the s dot products with the reflector are wave
//     sums; the s partial sums are transposed across lanes while they are
//     added (permlane32/permlane16 swaps, then DPP row mirrors), so
//     summing s values costs about as much as summing two;
//   - every reduction uses the same fixed pairing, so the leaf pass and
//     the apply pass compute bitwise the same reflectors and results do not
//     depend on timing.
// The explicit Q of a chunk is formed in compact form: with V the unit
// lower-trapezoidal reflectors and E = [C; 0],
//   H_1 ... H_s E = E - V W,   w_i = tau_i (v_i^T E - sum_{k>i} (v_i^T v_k) w_k)
// (rows w_i of W, i = s-1 down to 0), where v_i^T v_k come out of the same
// wave sums as the factorization's dot products.
#include "tsqr_wave_impl.h"

namespace bcgs {


int wave_tsqr_rows(int s) { return s <= 16 ? 64 * (64 / s) : 0; }

void tsqr_down(const TsqrPlan& tp, double* ws, hipStream_t st);

template <typename T, int S>
static hipError_t launch_wave_tsqr_s(const TsqrPlan& tp, const T* v,
                                     int64_t ldv, T* dst, int64_t ldd,
                                     int64_t m, double* ws, double* r_out,
                                     int64_t r_rs, int64_t r_cs,
                                     int32_t* syncs, hipStream_t st) {
  const int fan = tp.fan;
  const double ss = (double)S * S, esz = sizeof(T);
  auto wgs = [](int64_t waves) { return dim3((unsigned)cdiv(waves, 4)); };
  if (rec_active()) {
    // the same kernels as steps of work items (binary64, s = 4, 8, 16)
    if constexpr (sizeof(T) == 8 && (S == 4 || S == 8 || S == 16)) {
      rec_tsqr_leaf(S, v, ldv, m, tp.nchunks, ws + tp.r_off[0],
                    cdiv(tp.nchunks, 4));
      for (int l = 1; l <= tp.levels; ++l)
        rec_tsqr_node(S, ws + tp.r_off[l - 1], tp.nodes[l - 1], fan,
                      tp.nodes[l], ws + tp.r_off[l], ws + tp.q_off[l],
                      l == tp.levels ? 1 : 0, r_out, r_rs, r_cs, syncs,
                      cdiv(tp.nodes[l], 4));
      tsqr_down(tp, ws, st);
      rec_tsqr_apply(S, v, ldv, m, tp.nchunks, ws + tp.c_off[0], dst, ldd,
                     cdiv(tp.nchunks, 4));
    } else {
      rec_unsupported();
    }
    return hipSuccess;
  }
  // three launches: the leaves, the whole upward tree, then the explicit
  // Q with each chunk's coefficients formed along its path
  prof_begin(BCGS_KERNEL_TSQR_LEAF, 0, esz * m * S, 2.0 * m * ss);
  hipLaunchKernelGGL((tw::leaf_kernel<T, S>), wgs(tp.nchunks), dim3(256), 0,
                     st, v, ldv, m, tp.nchunks, ws + tp.r_off[0]);
  prof_name("tsqr_wave_leaf_kernel<%s, %d>", type_name<T>(), S);
  prof_end();
  double tree_rows = 0.0;
  for (int l = 1; l <= tp.levels; ++l) tree_rows += (double)tp.nodes[l - 1] * S;
  prof_begin(BCGS_KERNEL_TSQR_NODE, 0, 16.0 * tree_rows * S,
             4.0 * tree_rows * ss);
  hipLaunchKernelGGL(tw::tree_kernel<S>, wgs(tp.nodes[1]), dim3(256), 0, st,
                     tp, ws, r_out, r_rs, r_cs, syncs);
  prof_name("tsqr_wave_tree_kernel<%d>", S);
  prof_end();
  prof_begin(BCGS_KERNEL_TSQR_APPLY, 0, 2.0 * esz * m * S,
             2.0 * m * ss + 2.0 * (double)tp.nchunks * tp.levels * ss * S);
  hipLaunchKernelGGL((tw::apply_path_kernel<T, S>), wgs(tp.nchunks),
                     dim3(256), 0, st, v, ldv, m, tp, ws, dst, ldd);
  prof_name("tsqr_wave_apply_path_kernel<%s, %d>", type_name<T>(), S);
  prof_end();
  return hipGetLastError();
}

template <typename T>
hipError_t launch_wave_tsqr(const TsqrPlan& tp, const T* v, int64_t ldv,
                            T* dst, int64_t ldd, int64_t m, double* ws,
                            double* r_out, int64_t r_rs, int64_t r_cs,
                            int32_t* syncs, hipStream_t st) {
  switch (tp.s) {
#define TW(S_) case S_: return launch_wave_tsqr_s<T, S_>(tp, v, ldv, dst, ldd, \
                                                         m, ws, r_out, r_rs, \
                                                         r_cs, syncs, st);
    TW(1) TW(2) TW(3) TW(4) TW(5) TW(6) TW(7) TW(8) TW(9) TW(10) TW(11)
    TW(12) TW(13) TW(14) TW(15) TW(16)
#undef TW
    default:
      return hipErrorNotSupported;
  }
}

template hipError_t launch_wave_tsqr<double>(const TsqrPlan&, const double*,
                                             int64_t, double*, int64_t,
                                             int64_t, double*, double*,
                                             int64_t, int64_t, int32_t*,
                                             hipStream_t);
template hipError_t launch_wave_tsqr<float>(const TsqrPlan&, const float*,
                                             int64_t, float*, int64_t,
                                             int64_t, double*, double*,
                                             int64_t, int64_t, int32_t*,
                                             hipStream_t);

}  // namespace bcgs
