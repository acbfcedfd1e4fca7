// Blocked int8 form: kernels of product depth(s) K_pad / 32 = 8, 9.
#include "gemm_blk.h"

namespace hpmap {

HP_BLK_DEPTH(8)
HP_BLK_DEPTH(9)

}  // namespace hpmap
