// Streaming pass for block widths s <= 16 (one 16-wide MFMA column block),
// the shape of every large workload.  Same operation as pass.hip (block
// updates of Alg. 1 / Alg. 2 fused with the tall-skinny Gram products of one
// synchronization point), organised for gfx950:
//
//  * Either two 4-wave workgroups per CU with two LDS tile buffers each, or
//    one workgroup per CU with 8 waves or with four buffers.  Full tiles of
//    TR rows (16, 32 or 64) are dealt round-robin to the workgroups, so the
//    workgroups running together read one narrow band of rows of every
//    column; the short last tile is staged synchronously after the loop.
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
//    they share the fragment loads.  Their K-range partial sums are combined
//    through LDS, one round per update, or one round for both where the
//    shape has room for both partial-sum areas (three barriers per tile
//    instead of five); the combine writes the results both to HBM
//    (coalesced) and into the tile for the Gram.
//  * Gram A^T B: the (A block, B block) pairs of 16x16 outputs are dealt
//    round-robin to the waves (equal MFMA counts), which accumulate them in
//    registers over the whole row range.
#include "pass16_impl.h"

namespace bcgs {
namespace p16 {

template P16_DISPATCH_DECL(double, false);

}  // namespace p16

size_t pass16_lds_bytes(int ncols_p, int tr, int nw) {
  (void)nw;
  return ((size_t)2 * ncols_p * tr + 64 * 17) * sizeof(double);
}

int pass16_shape_count() { return p16::kNShapes; }

bool pass16_shape_four_waves(int shape) {
  return shape >= 0 && shape < p16::kNShapes && p16::kShapes[shape].nw == 4;
}

int64_t pass16_small_rows() { return p16::kSmallRows; }

// Returns hipErrorNotSupported (without launching) when this kernel cannot
// take the pass.  *G_out receives the number of workgroups used (the row
// split is a function of m and of the chosen shape only).
hipError_t launch_pass16(const PassArgs<double>& pa, int64_t m,
                         const Tuning& tune, hipStream_t st, int* tag,
                         int* G_out) {
  return p16::launch_pass16_t<double>(pa, m, tune, st, tag, G_out);
}

}  // namespace bcgs
