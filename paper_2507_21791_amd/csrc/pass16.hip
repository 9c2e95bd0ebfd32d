// Streaming pass for block widths s <= 16 (one 16-wide MFMA column block),
// the shape of every large workload.  Same operation as pass.hip (block
// updates of Alg. 1 / Alg. 2 fused with the tall-skinny Gram products of one
// synchronization point), organised for gfx950:
//
//  * 4 waves per workgroup.  Either two workgroups per CU with two LDS tile
//    buffers each, or one workgroup per CU with three or four buffers (a
//    deeper copy pipeline for the widest passes).  The row range of a
//    workgroup is walked in full tiles of TR rows (16, 32 or 64); a short
//    last tile is staged synchronously after the loop.
//  * Tiles arrive by direct-to-LDS copies (global_load_lds_dwordx4) issued
//    NBUF - 1 tiles ahead.  Waiting for a tile counts only the copies issued
//    after it (vector memory operations complete in issue order), so the
//    copies of later tiles stay in flight.  Columns that are not 16-byte
//    aligned (odd leading dimensions) take the register-staged form of the
//    same kernel (pass16_reg.hip), which builds the identical LDS tile.
//  * LDS tile layout: column c occupies TR consecutive doubles; within a
//    column the 16-byte granules (row pairs) are XOR-swizzled by a
//    per-column key, which keeps both MFMA fragment patterns (16 columns x
//    4 rows for the Gram, 4 columns x 16 rows for the updates) free of bank
//    conflicts.
//  * The Gram uses the FP64 4x4x4 MFMA (four 4x4 blocks per instruction),
//    which gfx950 runs at about 1.5x the rate of the 16x16x4 form (a 16x16
//    output tile is four such instructions); the block updates use the
//    16x16x4 form, whose operands cost a quarter of the LDS reads.
//  * Block updates B <- [Q B] F (F = [-C T^{-1}; T^{-1}], see common.h):
//    waves = (TR/16 row blocks) x (KG K-ranges); every wave keeps its slice
//    of the coefficient fragments in registers for the whole kernel.  When
//    a pass has two updates, both read the staged (old) columns (the second
//    one's coefficients have the first one's folded in by the epilogue), so
//    they share the fragment loads and their K-range partial sums are
//    combined in one LDS round; the combine writes the results both to HBM
//    (coalesced) and into the tile for the Gram.
//  * Gram A^T B: the (A block, B block) pairs of 16x16 outputs are dealt
//    round-robin to the waves (equal MFMA counts), which accumulate them in
//    registers over the whole row range.
#include "pass16_impl.h"

namespace bcgs {
namespace p16 {

template hipError_t dispatch<false>(int, const Args&, int, bool, int, int,
                                   hipStream_t, int*);

}  // namespace p16

size_t pass16_lds_bytes(int ncols_p, int tr, int nw) {
  (void)nw;
  return ((size_t)2 * ncols_p * tr + 64 * 17) * sizeof(double);
}

// Returns hipErrorNotSupported (without launching) when this kernel cannot
// take the pass.  *G_out receives the number of workgroups used (the row
// split is a function of m and of the chosen shape only).
int pass16_shape_count() { return p16::kNShapes; }

hipError_t launch_pass16(const PassArgs<double>& pa, int64_t m,
                         const Tuning& tune, hipStream_t st, int* tag,
                         int* G_out) {
  using namespace p16;
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
  const bool dma = (pa.ldq % 2 == 0) && al16(pa.q) &&
                   (!pa.fcols || (pa.ldf % 2 == 0 && al16(pa.f))) &&
                   (!pa.ecols || (pa.lde % 2 == 0 && al16(pa.e)));
  const bool reg = !dma;
  const int nks1 = pa.upd1 ? (pa.u1_c0 + s) / 4 : 0;
  const int nks2 = pa.upd2 ? pa.u2_c0 / 4 : 0;
  const int shared = std::max(nks1, nks2);
  const int ntb = pa.gram ? pa.gbn_p / 16 : 1;
  if (ntb > 2) return hipErrorNotSupported;
  const int npairs = pa.gram ? (pa.ga_p / 16) * ntb : 0;
  int pick = -1;
  int f = tune.shape;
  if (f < 0) {
    if (const char* env = getenv("BCGS_PASS16_SHAPE")) f = atoi(env);
  }
  if (f >= 0 && f < kNShapes &&
      shape_fits(kShapes[f], pa.ncols_p, shared, npairs, reg))
    pick = f;
  // Automatic choice, measured on MI355X: passes with two B blocks of
  // Gram (P-1S, P-2S) are bound by the MFMA work and run best with 16-row
  // tiles, two workgroups per CU; the other wide passes are bound by the
  // stream and take the 32-row, 8-wave shape.
  static const int kHeavy[] = {0, 3, 4, 2, 5, 1, 6};
  static const int kLight[] = {0, 3, 2, 4, 5, 1, 6};
  static_assert(sizeof(kHeavy) / sizeof(int) == kNShapes, "every shape");
  const int* order = (pa.gram && ntb == 2) ? kHeavy : kLight;
  for (int i = 0; pick < 0 && i < kNShapes; ++i)
    if (shape_fits(kShapes[order[i]], pa.ncols_p, shared, npairs, reg))
      pick = order[i];
  if (pick < 0) return hipErrorNotSupported;
  const Shape sh = kShapes[pick];
  const int maxp = shape_maxp(sh, npairs);
  Args a{};
  // rows split over 256 * per_cu workgroups (256 CUs on MI355X), at most
  // tune.max_wg of them
  const int64_t rpw =
      std::max(round_up64(cdiv(m, 256 * sh.per_cu), 64),
               round_up64(cdiv(m, std::max(1, tune.max_wg)), 64));
  const int G = (int)cdiv(m, rpw);
  a.m = pa.m; a.s = s; a.ncols = pa.ncols; a.ncols_p = pa.ncols_p;
  a.rows_per_wg = rpw;
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
  return reg ? dispatch<true>(pick, a, G, gram, ntb, maxp, st, tag)
             : dispatch<false>(pick, a, G, gram, ntb, maxp, st, tag);
}

}  // namespace bcgs
