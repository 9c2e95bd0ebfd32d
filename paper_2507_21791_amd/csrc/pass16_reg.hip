// Register-staged instantiations of the s <= 16 streaming pass: the same
// kernels as pass16.hip for columns whose addresses are not 16-byte aligned
// (odd leading dimensions, e.g. an odd row count with ld = m).  Tiles are
// loaded one ahead into registers and written to LDS in the layout the
// direct copies produce.
#include "pass16_impl.h"

namespace bcgs {
namespace p16 {

template P16_DISPATCH_DECL(double, true);

}  // namespace p16
}  // namespace bcgs
