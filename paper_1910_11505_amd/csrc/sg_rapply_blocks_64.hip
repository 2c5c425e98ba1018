// Compile-time field-split block kernels of the register apply for (M, p) =
// (6, 4), in a translation unit of their own so that they compile
// beside the rest of the library (the kernels and tables come from
// sg_rapply.hip, read here for its device templates only).
#define SG_RAPPLY_BLOCK_TU
#include "sg_rapply.hip"

namespace sg {
SG_RBLOCK_DECL(6, 4)
}  // namespace sg
