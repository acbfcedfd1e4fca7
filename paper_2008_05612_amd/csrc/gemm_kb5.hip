// int8-MFMA ground-state kernels for product depth K_pad = 160 (5x5 and the
// 3x3x3 cube).  The first entry is the default shape; the autotuner may pick
// any other.
#include "gemm_body.h"

namespace hpmap {

static const GemmVariant kVariants[] = {
    HP_GEMM_VARIANT(5, 2, 8, kLds),
    HP_GEMM_VARIANT(5, 2, 4, kLds),
    HP_GEMM_VARIANT(5, 2, 4, kDirect),
    HP_GEMM_VARIANT(5, 4, 4, kLds),
    HP_GEMM_VARIANT(5, 4, 4, kDirect),
    HP_GEMM_VARIANT(5, 3, 4, kLds),
    HP_GEMM_VARIANT(5, 3, 4, kDirect),
    HP_GEMM_VARIANT(5, 1, 8, kDirect),
    HP_GEMM_VARIANT(5, 2, 8, kPipe),
    HP_GEMM_VARIANT(5, 2, 4, kPipe),
    HP_GEMM_VARIANT(5, 4, 4, kPipe),
    HP_GEMM_VARIANT(5, 3, 4, kPipe),
};

int gemm_variants_kb5(const GemmVariant **out)
{
    *out = kVariants;
    return int(sizeof(kVariants) / sizeof(kVariants[0]));
}

}  // namespace hpmap
