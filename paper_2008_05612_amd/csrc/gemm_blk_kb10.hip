// Blocked int8 form: kernels of product depth(s) K_pad / 32 = 10.
#include "gemm_blk.h"

namespace hpmap {

HP_BLK_DEPTH(10)

}  // namespace hpmap
