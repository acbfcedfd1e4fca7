// Blocked int8 form: kernels of product depth(s) K_pad / 32 = 6, 7.
#include "gemm_blk.h"

namespace hpmap {

HP_BLK_DEPTH(6)
HP_BLK_DEPTH(7)

}  // namespace hpmap
