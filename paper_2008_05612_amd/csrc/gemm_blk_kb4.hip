// Blocked int8 form: kernels of product depth(s) K_pad / 32 = 4.
#include "gemm_blk.h"

namespace hpmap {

HP_BLK_DEPTH(4)

}  // namespace hpmap
