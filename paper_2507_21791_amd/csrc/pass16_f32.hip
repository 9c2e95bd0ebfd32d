// Binary32 instantiations of the s <= 16 streaming pass, for the FP32-bulk
// form: tiles of 32 rows x 4 bytes (the bytes per column of the 16-row
// binary64 tiles), block updates and Gram products on the FP32 16x16x4
// MFMA with FP32 accumulation, per-workgroup Gram partials widened to FP64
// for the cross-workgroup sum.  Both copy forms: direct to LDS for 16-byte
// aligned columns, register-staged otherwise.
#include "pass16_impl.h"

namespace bcgs {
namespace p16 {

template P16_DISPATCH_DECL(float, false);
template P16_DISPATCH_DECL(float, true);

}  // namespace p16

hipError_t launch_pass16_f32(const PassArgs<float>& pa, int64_t m,
                             const Tuning& tune, hipStream_t st, int* tag,
                             int* G_out) {
  return p16::launch_pass16_t<float>(pa, m, tune, st, tag, G_out);
}

}  // namespace bcgs
