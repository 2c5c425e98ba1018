// Compile-time field-split block kernels of the register apply for the chaos
// spaces of at most 35 modes, in a translation unit of their own so that they
// compile beside the rest of the library (the kernels and tables come from
// sg_rapply.hip, read here for its device templates only).
#define SG_RAPPLY_BLOCK_TU
#include "sg_rapply.hip"

namespace sg {
SG_RAPPLY_LIST(SG_RBLOCK_DECL)
}  // namespace sg
