// Blocked int8 form: kernels of product depth(s) K_pad / 32 = 1, 2, 3.
#include "gemm_blk.h"

namespace hpmap {

HP_BLK_DEPTH(1)
HP_BLK_DEPTH(2)
HP_BLK_DEPTH(3)

}  // namespace hpmap
