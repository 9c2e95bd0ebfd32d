// Host side: argument checks, workspace plan, the per-variant schedule of
// streaming passes / reductions / epilogues, and the C ABI of bcgs.h.
//
// Schedules (0-based block columns j; B = one m x s block):
//   BCGSI+ (section 1, Table 1; four reductions per block column)
//     TSQR(X_0) -> Q_0, R_00
//     for j = 1..q-1:
//       S   = Q_{0:j-1}^T X_j                      pass + reduce
//       V   = X_j - Q S -> slot j; TSQR(V) -> U_j, S_jj
//       Y   = Q^T U_j                              pass + reduce
//       W   = U_j - Q Y -> slot j; TSQR(W) -> Q_j, Y_jj
//       R column block j from S, Y, S_jj, Y_jj
//   BCGSI+P-1S (Alg. 2; one reduction per block column)
//     TSQR(X_0); [S_01; T_1] = [Q_0 X_1]^T X_1; S_11 = chol(T_1 - S^T S)
//     for j = 1..q-1: one pass that forms Q_{j-1} from U_{j-1} (j >= 2),
//       forms U_j from X_j, and accumulates [Q_{0:j-1} U_j]^T [U_j X_{j+1}]
//       and X_{j+1}^T X_{j+1}; then the epilogue (Y_jj, R, eq. (1), S_{j+1})
//     last pass forms Q_{q-1}
//   BCGSI+P-2S (section 2.3; two reductions per block column)
//     as P-1S, but V_j = X_j - Q S is written and factored by TSQR, and
//     the Gram pass runs after it; S_01 = Q_0^T X_1 is its own reduction.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "common.h"
#include "small_impl.h"

namespace bcgs {

template <typename T>
size_t pass_lds_bytes(const PassArgs<T>& a);

static bool valid_args(int64_t m, int64_t n, int64_t s, int variant,
                       int precision) {
  if (s < 1 || s > kMaxS || n < 1 || m < n || n % s != 0) return false;
  if (variant < BCGS_I_PLUS || variant > BCGS_I_PLUS_1S) return false;
  if (precision != BCGS_FP64 && precision != BCGS_FP32_BULK) return false;
  if (m > (int64_t(1) << 40)) return false;
  return true;
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool make_plan(int64_t m, int64_t n, int64_t s, int variant, int precision,
               Plan* p, const Tuning* t) {
  if (!valid_args(m, n, s, variant, precision)) return false;
  Plan P{};
  P.m = m; P.n = n; P.s = (int)s; P.sp = round_up((int)s, 16);
  P.q = (int)(n / s);
  P.variant = variant; P.precision = precision;
  if (t) P.tune = *t;
  if (P.tune.max_wg < 1 || P.tune.max_wg > 512) return false;
  const int64_t target_wg = P.tune.max_wg;
  P.rows_per_wg = round_up64(cdiv(m, target_wg), 64);
  P.G = (int)cdiv(m, P.rows_per_wg);
  P.gram_ld = round_up64(n + s, 16);
  const int64_t gbn = round_up((int)(2 * s), 16);
  P.partial_elems = P.gram_ld * gbn;
  P.tsqr = make_tsqr_plan(m, (int)s);
  size_t off = 0;
  P.off_scratch_info = off; off = align256(off + sizeof(bcgs_info));
  const size_t tri = (size_t)P.sp * P.sp * sizeof(double);
  const size_t col = (size_t)(n + s) * P.sp * sizeof(double);
  P.off_t1 = off; off = align256(off + tri);
  P.off_t2 = off; off = align256(off + tri);
  P.off_c1 = off; off = align256(off + col);
  P.off_c2 = off; off = align256(off + col);
  P.off_f1 = off; off = align256(off + col);
  P.off_f2 = off; off = align256(off + col);
  P.off_gram = off; off = align256(off + P.partial_elems * sizeof(double));
  P.off_partial = off;
  off = align256(off + (size_t)P.G * P.partial_elems * sizeof(double));
  P.off_tsqr = off; off = align256(off + P.tsqr.total * sizeof(double));
  P.off_fsplit = off;
  if (s == 32 || s == 64)
    off = align256(off + 2 * (size_t)(n + s) * 16 * sizeof(double));
  P.bytes = off;
  *p = P;
  return true;
}

static int planned_syncs(int variant, int q) {
  if (q == 1) return 1;
  switch (variant) {
    case BCGS_P_1S: return q + 1;
    case BCGS_I_PLUS_1S: return q + 1;
    case BCGS_P_2S: return 2 * q;
    case BCGS_PIPI_PLUS: return 2 * q - 1;
    default: return 4 * q - 3;
  }
}

void prof_retag(int tag);

// syncs starts at zero; every reduction and every TSQR root adds one as it
// completes, so the record reports the synchronization points that ran
__global__ void info_init_kernel(bcgs_info* info) { info_init_body(info); }

// ------------------------------------------------------------ schedule ---
template <typename T>
struct Run {
  Plan p;
  const T* X; int64_t ldx;
  T* Q; int64_t ldq;
  double* R; int64_t ldr;
  char* ws;
  bcgs_info* info;
  hipStream_t st;
  hipError_t err = hipSuccess;

  double* dws(size_t off) { return reinterpret_cast<double*>(ws + off); }
  const T* xb(int j) const { return X + (int64_t)j * p.s * ldx; }
  T* qb(int j) const { return Q + (int64_t)j * p.s * ldq; }
  void check(hipError_t e) { if (err == hipSuccess && e != hipSuccess) err = e; }

  // Description of one streaming pass.
  struct Pass {
    int nq = 0;                        // Q columns staged
    const T* f = nullptr; int64_t ldf = 0;   // block F (s columns)
    const T* e = nullptr; int64_t lde = 0;   // block E (s columns)
    bool upd1 = false;                 // Q slot (nq/s - 1): U -> Q (F1)
    bool upd2 = false;                 // F block -> dst2 (F2 or c2)
    const double* c2 = nullptr;        // override of F2
    T* dst2 = nullptr;
    bool gram = false; int gb0 = 0; int gbn = 0;
    bool skip_eu = false;              // skip the E^T U tiles
    int64_t needed = 0;                // Gram entries the method needs
    bool scaled2 = true;               // update 2 has a triangular factor
  };

  // The block updates of a pass without a Gram at s = 32 or 64 (g: the
  // pass as the generic kernel would run it) on the s <= 16 pass, whose two
  // updates of 16 columns each become two neighbouring 16-column parts of a
  // block: the second part's K range takes in the first part's staged
  // (old) columns, and the pass forms both products before writing either.
  // A block of 64 columns takes two launches, its last 32 columns first: a
  // launch writes only columns that no later launch reads, so every launch
  // reads old columns, as the folded coefficients assume.  Update 2 runs
  // first (its block is not among update 1's staged columns), then update
  // 1, which rewrites its own block in place.  The caller has put the
  // coefficient parts of the first launch in the split buffer and opened a
  // launch record; each launch gets a record of its own with its own byte
  // and flop model.  Returns hipErrorNotSupported, with nothing launched,
  // where the s <= 16 pass does not take the shape; the generic pass then
  // runs.
  hipError_t split_updates(const Pass& d, const PassArgs<T>& g, int* tag) {
    if constexpr (sizeof(T) != 8) {
      return hipErrorNotSupported;
    } else {
      const int s = p.s;
      double* fa = dws(p.off_fsplit);
      double* fb = fa + (size_t)(p.n + s) * 16;
      const double mr = (double)p.m;
      // columns [c0, c0 + 32) of the block at staged column b0 (into dst),
      // staging the columns up to the part's end: Q columns, then with
      // with_f the first columns of block F (the block is F at b0 = nq)
      auto part = [&](int nq, bool with_f, int b0, int c0,
                      T* dst) -> hipError_t {
        PassArgs<T> h = g;
        h.s = 16; h.sp = 16;
        h.nq = with_f ? nq : b0 + c0 + 32;
        h.fcols = with_f ? c0 + 32 : 0;
        h.e = nullptr; h.ecols = 0;
        h.ncols = h.nq + h.fcols;
        h.ncols_p = round_up(h.ncols, 16);
        h.upd1 = 1; h.u1_c0 = b0 + c0; h.c1 = fa;
        h.dst1 = dst + (int64_t)c0 * ldq; h.ldd1 = ldq;
        h.upd2 = 1; h.u2_c0 = b0 + c0 + 16; h.c2 = fb;
        h.dst2 = dst + (int64_t)(c0 + 16) * ldq; h.ldd2 = ldq;
        h.gram = 0; h.groups = 1;
        prof_model(8.0 * mr * (h.ncols + 32),
                   mr * (2.0 * (b0 + c0) * 32 + 32.0 * 32));
        int g16 = 0;
        return launch_pass16(h, p.m, p.tune, st, tag, &g16);
      };
      struct Job { bool with_f; int b0; const double* F; T* dst; };
      Job jobs[2];
      int nj = 0;
      if (d.upd2) jobs[nj++] = {true, d.nq, g.c2, d.dst2};
      if (d.upd1)
        jobs[nj++] = {false, d.nq - s, g.c1, Q + (int64_t)(d.nq - s) * ldq};
      bool first = true;
      for (int j = 0; j < nj; ++j) {
        const Job& jb = jobs[j];
        for (int c0 = s - 32; c0 >= 0; c0 -= 32) {
          if (!first) {
            // close the last launch's record; this launch's coefficient
            // parts replace the last ones in the split buffer (ordered after
            // that launch on the stream); then a record of its own
            prof_end();
            prof_retag(*tag);
            check(launch_split_coef(jb.F, jb.b0 + c0 + 32, p.sp, c0, fa, fb,
                                    st));
            prof_begin(BCGS_KERNEL_PASS, -1, 0.0, 0.0);
          }
          const hipError_t e = part(d.nq, jb.with_f, jb.b0, c0, jb.dst);
          if (e != hipSuccess) return e;
          first = false;
        }
      }
      return hipSuccess;
    }
  }

  // The Gram of a pass without updates at s = 32 as one launch of the
  // s <= 16 pass per 32 B columns (its two 16-column B blocks), each
  // followed by its reduction into its columns of the reduced Gram (only
  // the last one counts as the synchronization point).  False, with
  // nothing launched, where the s <= 16 pass does not take the shape.
  bool gram_halves(const Pass& d) {
    if constexpr (sizeof(T) != 8) {
      return false;
    } else {
      const int s = p.s;
      PassArgs<T> h{};
      h.m = p.m; h.s = 16; h.sp = 16;
      h.q = Q; h.ldq = ldq; h.nq = d.nq;
      h.f = d.f; h.ldf = d.ldf; h.fcols = d.f ? s : 0;
      h.e = d.e; h.lde = d.lde; h.ecols = d.e ? s : 0;
      h.ncols = h.nq + h.fcols + h.ecols;
      h.ncols_p = round_up(h.ncols, 16);
      h.gram = 1; h.groups = 1;
      h.ga_p = h.ncols_p;
      h.gbn_p = 32;
      h.partial = dws(p.off_partial);
      const int nh = d.gbn > 32 ? 2 : 1;
      const double mr = (double)p.m;
      for (int k = 0; k < nh; ++k) {
        h.gb0 = d.gb0 + 32 * k;
        // the E^T U tiles the method does not need lie in the first half
        h.skip_a0 = d.skip_eu ? d.nq + s : 1 << 30;
        h.skip_b1 = d.skip_eu && k == 0 ? s : 0;
        int tag = 0, g16 = 0;
        prof_begin(BCGS_KERNEL_PASS, -1, 8.0 * mr * h.ncols,
                   2.0 * mr * (double)d.needed / nh);
        const hipError_t e = launch_pass16(h, p.m, p.tune, st, &tag, &g16);
        if (e == hipErrorNotSupported && k == 0) {
          // nothing launched: close the record on an empty launch
          prof_model(0.0, 0.0);
          prof_end();
          return false;
        }
        check(e);
        prof_end();
        prof_retag(tag);
        check(launch_gram_reduce(h.partial, g16, (int64_t)h.ga_p * 32,
                                 dws(p.off_gram) + (size_t)k * h.ga_p * 32,
                                 k == nh - 1 ? &info->syncs : nullptr, st));
      }
      gram_ld_last = h.ga_p;
      return true;
    }
  }

  void pass(const Pass& d) {
    const int s = p.s;
    PassArgs<T> a{};
    a.m = p.m; a.s = s; a.sp = p.sp;
    a.q = Q; a.ldq = ldq; a.nq = d.nq;
    a.f = d.f; a.ldf = d.ldf; a.fcols = d.f ? s : 0;
    a.e = d.e; a.lde = d.lde; a.ecols = d.e ? s : 0;
    a.ncols = a.nq + a.fcols + a.ecols;
    a.upd1 = d.upd1; a.u1_c0 = d.nq - s;
    a.c1 = dws(p.off_f1);
    a.dst1 = Q + (int64_t)(d.nq - s) * ldq; a.ldd1 = ldq;
    a.upd2 = d.upd2; a.u2_c0 = d.nq;
    a.c2 = d.c2 ? d.c2 : dws(p.off_f2);
    a.dst2 = d.dst2; a.ldd2 = ldq;
    a.gram = d.gram;
    a.ga_p = round_up(a.ncols, 16);
    a.gb0 = d.gb0; a.gbn_p = round_up(d.gbn > 0 ? d.gbn : 1, 16);
    a.skip_a0 = d.skip_eu ? d.nq + s : 1 << 30;
    a.skip_b1 = d.skip_eu ? s : 0;
    a.partial = dws(p.off_partial);
    int ncp = round_up(a.ncols, 16);
    if (d.gram) ncp = std::max(ncp, std::max(a.ga_p, round_up(a.gb0 + a.gbn_p, 16)));
    a.ncols_p = ncp;
    // A blocks per wave limited by register budget (16 tiles per wave)
    const int ntb = a.gbn_p / 16;
    const int maxa = ntb >= 8 ? 2 : ntb >= 4 ? 4 : 8;
    const int ta_total = a.ga_p / 16;
    int groups = 1;
    if (d.gram) groups = (int)cdiv(ta_total, kWaves * maxa);
    if (sizeof(T) == 8 && p.sp == 32 && s == 32 && d.gram && !rec_active()) {
      // s = 32: the updates on their own (split_updates), then the Gram in
      // halves of 32 B columns on the s <= 16 pass (gram_halves)
      Pass gdesc = d;
      if (d.upd1 || d.upd2) {
        Pass u = d;
        u.gram = false;
        pass(u);
        gdesc.upd1 = false;
        gdesc.upd2 = false;
        if (d.upd2) { gdesc.f = d.dst2; gdesc.ldf = ldq; }
      }
      if (gram_halves(gdesc)) return;
      if (d.upd1 || d.upd2) { pass(gdesc); return; }
    }
    if (groups > 1 && (d.upd1 || d.upd2)) {
      // the Gram is split over several workgroups per row range: run the
      // updates on their own first, then the Gram reading their results
      Pass u = d;
      u.gram = false;
      pass(u);
      Pass gdesc = d;
      gdesc.upd1 = false;
      gdesc.upd2 = false;
      if (d.upd2) { gdesc.f = d.dst2; gdesc.ldf = ldq; }
      pass(gdesc);
      return;
    }
    a.groups = groups;
    a.a_blocks_per_group = d.gram ? (int)cdiv(ta_total, groups) : 0;
    // tile rows: largest that keeps two workgroups per CU
    int tr = 64;
    while (tr > 16) {
      a.tr = tr;
      if (pass_lds_bytes(a) <= 80 * 1024) break;
      tr /= 2;
    }
    a.tr = tr;
    a.rows_per_wg = p.rows_per_wg;
    int G = p.G;
    // algorithmic work of this pass: the staged columns are read once, the
    // updated blocks written once; 2 K s flops per row and block update
    // plus s^2 for the triangular solve; 2 flops per needed Gram entry
    const double mr = (double)p.m, esz = sizeof(T);
    double flops = 0.0, cols_rw = a.ncols;
    if (d.upd1) { flops += mr * (2.0 * a.u1_c0 * s + (double)s * s); cols_rw += s; }
    if (d.upd2) {
      flops += mr * (2.0 * a.u2_c0 * s + (d.scaled2 ? (double)s * s : 0.0));
      cols_rw += s;
    }
    if (d.gram) flops += 2.0 * mr * (double)d.needed;
    int tag = 0;
    // s = 32, 64 block updates without a Gram on the s <= 16 pass (see
    // split_updates)
    const bool split = sizeof(T) == 8 && (s == 32 || s == 64) && !d.gram &&
                       (d.upd1 || d.upd2) && !rec_active();
    if (split) {
      // the first launch's parts: the last 32 columns of the first update
      double* fa = dws(p.off_fsplit);
      double* fb = fa + (size_t)(p.n + s) * 16;
      const double* F = d.upd2 ? a.c2 : a.c1;
      const int K = d.upd2 ? a.u2_c0 + s : a.u1_c0 + s;
      check(launch_split_coef(F, K, p.sp, s - 32, fa, fb, st));
    }
    prof_begin(BCGS_KERNEL_PASS, -1, esz * mr * cols_rw, flops);
    hipError_t e = hipErrorNotSupported;
    if (split) e = split_updates(d, a, &tag);
    if (p.sp == 16) {
      int g16 = 0;
      if constexpr (sizeof(T) == 8)
        e = launch_pass16(a, p.m, p.tune, st, &tag, &g16);
      else
        e = launch_pass16_f32(a, p.m, p.tune, st, &tag, &g16);
      if (e != hipErrorNotSupported) G = g16;
    }
    if (e == hipErrorNotSupported) e = launch_pass(a, G, st, &tag);
    check(e);
    prof_end();
    prof_retag(tag);
    if (d.gram)
      check(launch_gram_reduce(a.partial, G, (int64_t)a.ga_p * a.gbn_p,
                               dws(p.off_gram), &info->syncs, st));
    gram_ld_last = a.ga_p;
  }
  int64_t gram_ld_last = 0;

  // f1/f2: which coefficient matrices the next pass needs (CoefMode) and
  // the number of rows of C1 / C2 they are built from
  // With both f1 and f2 the next pass runs both block updates on the
  // staged columns, so F1 is folded into F2 (fold_coefs).
  void epi(int mode, int j, bool has_e, bool chol_s, int f1 = COEF_NONE,
           int f1_rows = 0, int f2 = COEF_NONE, int f2_rows = 0,
           bool unit_s = false) {
    EpiArgs e{};
    e.mode = mode; e.s = p.s; e.sp = p.sp; e.j = j;
    e.has_e = has_e; e.chol_s = chol_s;
    e.gram = dws(p.off_gram); e.gld = gram_ld_last;
    e.c1 = dws(p.off_c1); e.c2 = dws(p.off_c2);
    e.t1 = dws(p.off_t1); e.t2 = dws(p.off_t2);
    e.f1 = dws(p.off_f1); e.f2 = dws(p.off_f2);
    e.f1_mode = f1; e.f1_rows = f1_rows;
    e.f2_mode = f2; e.f2_rows = f2_rows;
    e.fold12 = f1 != COEF_NONE && f2 != COEF_NONE;
    e.unit_s = unit_s;
    e.r = R; e.ldr = ldr; e.info = info;
    check(launch_epilogue(e, st));
  }

  void tsqr(const T* v, int64_t ldv, T* dst, double* rout, int64_t rs,
            int64_t cs) {
    check(launch_tsqr(p.tsqr, v, ldv, dst, ldq, p.m, dws(p.off_tsqr), rout,
                      rs, cs, &info->syncs, st));
  }

  void run() {
    prof_attach(st);
    run_steps();
    prof_detach();
  }

  void run_steps() {
    const int s = p.s, q = p.q, sp = p.sp;
    check(launch_fill(R, p.n, p.n, ldr, 0.0, st));
    if (rec_active()) {
      rec_init(info);
    } else {
      hipLaunchKernelGGL(info_init_kernel, dim3(1), dim3(64), 0, st, info);
      check(hipGetLastError());
      // the one-wave TSQR's node counters start at zero (each TSQR leaves
      // them at zero again)
      if (p.tsqr.wave)
        check(launch_fill(dws(p.off_tsqr) + p.tsqr.cnt_off,
                          p.tsqr.cnt_doubles, 1, p.tsqr.cnt_doubles, 0.0,
                          st));
    }
    // [Q_0, R_00] = TSQR(X_0)
    tsqr(xb(0), ldx, qb(0), R, 1, ldr);
    if (q == 1) return;
    if (p.variant == BCGS_I_PLUS) { run_i_plus(); return; }
    if (p.variant == BCGS_PIPI_PLUS) { run_pipi_plus(); return; }
    // BCGSI+1s runs the P-1S schedule with S_{j,j} = I: unscaled U, no T
    const bool unit = p.variant == BCGS_I_PLUS_1S;
    const bool one = p.variant == BCGS_P_1S || unit;
    const bool chol1 = p.variant == BCGS_P_1S;
    {
      Pass d;
      d.nq = s; d.f = xb(1); d.ldf = ldx;
      d.gram = true;
      d.gb0 = s; d.gbn = s;                   // [Q_0 X_1]^T X_1
      d.needed = chol1 ? 2 * s * s : s * s;   // P-2S needs Q_0^T X_1 only
      pass(d);
      // next: U_1 = (X_1 - Q_0 S_01) S_11^{-1} (P-1S) or X_1 - Q_0 S_01
      epi(chol1 ? EPI_S_CHOL : EPI_S_ONLY, 1, false, false, COEF_NONE, 0,
          chol1 ? COEF_SCALED : COEF_UNSCALED, s, unit);
    }
    for (int j = 1; j < q; ++j) {
      const bool has_e = j < q - 1;
      if (one) {
        Pass d;
        d.nq = j * s;
        d.upd1 = j >= 2;
        d.f = xb(j); d.ldf = ldx;
        d.upd2 = true; d.dst2 = qb(j);
        d.scaled2 = chol1;
        if (has_e) { d.e = xb(j + 1); d.lde = ldx; }
        d.gram = true; d.gb0 = j * s; d.gbn = has_e ? 2 * s : s;
        d.skip_eu = has_e;
        d.needed = (int64_t)(j + 1) * s * d.gbn +
                   (has_e && chol1 ? s * s : 0);
        pass(d);
        // next: Q_j from U_j (Y, Y_jj) and U_{j+1} from X_{j+1} (S, S_jj)
        epi(EPI_ONE_SYNC, j, has_e, chol1, COEF_SCALED, j * s,
            has_e ? (chol1 ? COEF_SCALED : COEF_UNSCALED) : COEF_NONE,
            (j + 1) * s, unit);
      } else {
        Pass u;                       // Q_{j-1} and V_j = X_j - Q S
        u.nq = j * s; u.upd1 = j >= 2;
        u.f = xb(j); u.ldf = ldx;
        u.upd2 = true; u.scaled2 = false; u.dst2 = qb(j);
        pass(u);
        tsqr(qb(j), ldq, qb(j), dws(p.off_t2), sp, 1);   // U_j, S_jj
        Pass d;                       // [Q_{0:j-1} U_j]^T [U_j X_{j+1}]
        d.nq = (j + 1) * s;
        if (has_e) { d.e = xb(j + 1); d.lde = ldx; }
        d.gram = true; d.gb0 = j * s; d.gbn = has_e ? 2 * s : s;
        d.skip_eu = has_e;
        d.needed = (int64_t)(j + 1) * s * d.gbn;
        pass(d);
        // next: Q_j from U_j (Y, Y_jj) and V_{j+1} = X_{j+1} - Q S
        epi(EPI_ONE_SYNC, j, has_e, false, COEF_SCALED, j * s,
            has_e ? COEF_UNSCALED : COEF_NONE, (j + 1) * s);
      }
    }
    Pass fin;                         // Q_{q-1} = (U - Q Y) Y_kk^{-1}
    fin.nq = q * s; fin.upd1 = true;
    pass(fin);
  }

  // BCGS-PIPI+ (Alg. 1): two reductions per block column.  Forming Q_{j-1}
  // from U_{j-1} is fused into the first pass of block column j.
  void run_pipi_plus() {
    const int s = p.s, q = p.q;
    for (int j = 1; j < q; ++j) {
      Pass a1;                        // [S; T] = [Q_{0:j-1} X_j]^T X_j
      a1.nq = j * s; a1.upd1 = j >= 2;
      a1.f = xb(j); a1.ldf = ldx;
      a1.gram = true; a1.gb0 = j * s; a1.gbn = s;
      a1.needed = (int64_t)(j + 1) * s * s;
      pass(a1);
      // S_jj = chol(T - S^T S); F2 for U_j = (X_j - Q S) S_jj^{-1}
      epi(EPI_S_CHOL, j, false, false, COEF_NONE, 0, COEF_SCALED, j * s);
      Pass a2;                        // U_j; [Y; Omega] = [Q U_j]^T U_j
      a2.nq = j * s;
      a2.f = xb(j); a2.ldf = ldx;
      a2.upd2 = true; a2.dst2 = qb(j);
      a2.gram = true; a2.gb0 = j * s; a2.gbn = s;
      a2.needed = (int64_t)(j + 1) * s * s;
      pass(a2);
      // Y_jj = chol(Omega - Y^T Y), R block column, F1 for Q_j
      epi(EPI_ONE_SYNC, j, false, false, COEF_SCALED, j * s);
    }
    Pass fin;                         // Q_{q-1} = (U - Q Y) Y_kk^{-1}
    fin.nq = q * s; fin.upd1 = true;
    pass(fin);
  }

  void run_i_plus() {
    const int s = p.s, q = p.q, sp = p.sp;
    for (int j = 1; j < q; ++j) {
      Pass a1;                        // S = Q^T X_j
      a1.nq = j * s; a1.f = xb(j); a1.ldf = ldx;
      a1.gram = true; a1.gb0 = j * s; a1.gbn = s;
      a1.needed = (int64_t)j * s * s;
      pass(a1);
      epi(EPI_S_ONLY, j, false, false, COEF_NONE, 0, COEF_UNSCALED, j * s);
      Pass a2;                        // V = X_j - Q S
      a2.nq = j * s; a2.f = xb(j); a2.ldf = ldx;
      a2.upd2 = true; a2.scaled2 = false; a2.dst2 = qb(j);
      pass(a2);
      tsqr(qb(j), ldq, qb(j), dws(p.off_t2), sp, 1);     // U_j, S_jj
      Pass a3;                        // Y = Q^T U_j
      a3.nq = j * s; a3.f = qb(j); a3.ldf = ldq;
      a3.gram = true; a3.gb0 = j * s; a3.gbn = s;
      a3.needed = (int64_t)j * s * s;
      pass(a3);
      epi(EPI_Y_ONLY, j, false, false, COEF_UNSCALED, j * s);
      Pass a4;                        // W = U_j - Q Y
      a4.nq = j * s; a4.f = qb(j); a4.ldf = ldq;
      a4.upd2 = true; a4.scaled2 = false; a4.dst2 = qb(j);
      a4.c2 = dws(p.off_f1);
      pass(a4);
      tsqr(qb(j), ldq, qb(j), dws(p.off_t1), sp, 1);     // Q_j, Y_jj
      epi(EPI_R_ASSEMBLE, j, false, false);
    }
  }
};

template <typename T>
static bcgs_status run_plan(const Plan& p, const T* X, int64_t ldx, T* Q,
                            int64_t ldq, double* R, int64_t ldr, void* ws,
                            bcgs_info* info, hipStream_t st) {
  Run<T> r;
  r.p = p; r.X = X; r.ldx = ldx; r.Q = Q; r.ldq = ldq; r.R = R; r.ldr = ldr;
  r.ws = static_cast<char*>(ws); r.info = info; r.st = st;
  r.run();
  return r.err == hipSuccess ? BCGS_OK : BCGS_ERR_HIP;
}

bcgs_status run_problem(const Plan& p, const void* X, int64_t ldx, void* Q,
                        int64_t ldq, double* R, int64_t ldr, void* ws,
                        bcgs_info* info, hipStream_t st) {
  if (p.precision == BCGS_FP32_BULK)
    return run_plan<float>(p, static_cast<const float*>(X), ldx,
                           static_cast<float*>(Q), ldq, R, ldr, ws, info, st);
  return run_plan<double>(p, static_cast<const double*>(X), ldx,
                          static_cast<double*>(Q), ldq, R, ldr, ws, info, st);
}

static bool overlaps(const void* a, size_t an, const void* b, size_t bn) {
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + bn && pb < pa + an;
}

bcgs_status check_problem(const void* X, int64_t ldx, int64_t m, int64_t n,
                          int64_t s, int variant, int precision,
                          const void* Q, int64_t ldq, const double* R,
                          int64_t ldr, const bcgs_info* d_info, Plan* p) {
  if (!X || !Q || !R || !d_info) return BCGS_ERR_ARG;
  if (!valid_args(m, n, s, variant, precision)) return BCGS_ERR_ARG;
  if (ldx < m || ldq < m || ldr < n) return BCGS_ERR_ARG;
  Tuning t;
  const bool tuned = tuned_choice(m, n, (int)s, variant, precision, &t);
  if (!make_plan(m, n, s, variant, precision, p, tuned ? &t : nullptr))
    return BCGS_ERR_ARG;
  const size_t esz = precision == BCGS_FP64 ? 8 : 4;
  const size_t xbytes = (size_t)((n - 1) * ldx + m) * esz;
  const size_t qbytes = (size_t)((n - 1) * ldq + m) * esz;
  const size_t rbytes = (size_t)((n - 1) * ldr + n) * 8;
  if (overlaps(X, xbytes, Q, qbytes)) return BCGS_ERR_ARG;
  if (overlaps(R, rbytes, Q, qbytes) || overlaps(R, rbytes, X, xbytes))
    return BCGS_ERR_ARG;
  return BCGS_OK;
}

// --------------------------------------------------- library workspace ---
struct StreamWs {
  void* ptr = nullptr;
  size_t bytes = 0;
  int device = -1;
};
static std::mutex g_mu;
static std::map<hipStream_t, StreamWs> g_ws;

}  // namespace bcgs

using namespace bcgs;

extern "C" {

size_t bcgs_workspace_size(int64_t m, int64_t n, int64_t s,
                           bcgs_variant variant, bcgs_precision precision) {
  Plan p;
  if (!make_plan(m, n, s, variant, precision, &p)) return 0;
  return p.bytes;
}

int32_t bcgs_sync_count(int64_t m, int64_t n, int64_t s,
                        bcgs_variant variant) {
  if (!valid_args(m, n, s, variant, BCGS_FP64)) return -1;
  return planned_syncs(variant, (int)(n / s));
}

bcgs_status bcgs_qr_ex(const void* X, int64_t ldx, int64_t m, int64_t n,
                       int64_t s, bcgs_variant variant,
                       bcgs_precision precision, void* Q, int64_t ldq,
                       double* R, int64_t ldr, void* workspace,
                       size_t ws_bytes, bcgs_info* d_info,
                       hipStream_t stream) {
  Plan p;
  const bcgs_status st = check_problem(X, ldx, m, n, s, variant, precision, Q,
                                       ldq, R, ldr, d_info, &p);
  if (st != BCGS_OK) return st;
  if (!workspace || ws_bytes < p.bytes) return BCGS_ERR_ARG;
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return BCGS_ERR_ARG;
  return run_problem(p, X, ldx, Q, ldq, R, ldr, workspace, d_info, stream);
}

bcgs_status bcgs_qr(const double* X, int64_t m, int64_t n, int64_t s,
                    bcgs_variant variant, double* Q, double* R,
                    hipStream_t stream) {
  Plan p;
  if (!X || !Q || !R) return BCGS_ERR_ARG;
  {
    Tuning t;
    const bool tuned = valid_args(m, n, s, variant, BCGS_FP64) &&
                       tuned_choice(m, n, (int)s, variant, BCGS_FP64, &t);
    if (!make_plan(m, n, s, variant, BCGS_FP64, &p, tuned ? &t : nullptr))
      return BCGS_ERR_ARG;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return BCGS_ERR_HIP;
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    StreamWs& w = g_ws[stream];
    if (w.bytes < p.bytes || w.device != dev) {
      if (w.ptr) {
        if (hipStreamSynchronize(stream) != hipSuccess) return BCGS_ERR_HIP;
        (void)hipFree(w.ptr);
        w.ptr = nullptr;
        w.bytes = 0;
      }
      if (hipMalloc(&w.ptr, p.bytes) != hipSuccess) {
        w.ptr = nullptr;
        return BCGS_ERR_NOMEM;
      }
      w.bytes = p.bytes;
      w.device = dev;
    }
    ws = w.ptr;
  }
  bcgs_info* info = reinterpret_cast<bcgs_info*>(
      static_cast<char*>(ws) + p.off_scratch_info);
  return bcgs_qr_ex(X, m, m, n, s, variant, BCGS_FP64, Q, m, R, n, ws,
                    p.bytes, info, stream);
}

bcgs_status bcgs_get_info(hipStream_t stream, bcgs_info* host_out) {
  if (!host_out) return BCGS_ERR_ARG;
  void* ptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_ws.find(stream);
    if (it == g_ws.end() || !it->second.ptr) return BCGS_ERR_ARG;
    ptr = it->second.ptr;
  }
  if (hipStreamSynchronize(stream) != hipSuccess) return BCGS_ERR_HIP;
  if (hipMemcpy(host_out, ptr, sizeof(bcgs_info), hipMemcpyDeviceToHost) !=
      hipSuccess)
    return BCGS_ERR_HIP;
  return BCGS_OK;
}

void bcgs_release(void) {
  batch_release();
  std::lock_guard<std::mutex> lock(g_mu);
  for (auto& kv : g_ws) {
    if (kv.second.ptr) {
      (void)hipStreamSynchronize(kv.first);
      (void)hipFree(kv.second.ptr);
    }
  }
  g_ws.clear();
}

const char* bcgs_status_string(bcgs_status st) {
  switch (st) {
    case BCGS_OK: return "ok";
    case BCGS_ERR_ARG: return "invalid argument";
    case BCGS_ERR_BREAKDOWN: return "Cholesky breakdown";
    case BCGS_ERR_NOMEM: return "out of device memory";
    case BCGS_ERR_HIP: return "HIP runtime error";
    case BCGS_ERR_QUEUE_FULL: return "queue full";
    case BCGS_PENDING: return "pending";
    case BCGS_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

}  // extern "C"
