// Blocked int8 form: kernels of product depth(s) K_pad / 32 = 11, 12.
#include "gemm_blk.h"

namespace hpmap {

HP_BLK_DEPTH(11)
HP_BLK_DEPTH(12)

}  // namespace hpmap
