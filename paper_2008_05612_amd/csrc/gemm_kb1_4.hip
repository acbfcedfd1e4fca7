// int8-MFMA ground-state kernels for product depths K_pad = 32 .. 128
// (boxes up to N = 24, e.g. 4x4 and 2x3x4).  The first entry per depth is the
// default shape; the autotuner may pick any other.
#include "gemm_body.h"

namespace hpmap {

static const GemmVariant kVariants[] = {
    HP_GEMM_VARIANT(1, 2, 4, kLds),
    HP_GEMM_VARIANT(2, 2, 4, kLds),
    HP_GEMM_VARIANT(2, 4, 4, kLds),
    HP_GEMM_VARIANT(2, 2, 4, kDirect),
    HP_GEMM_VARIANT(3, 2, 4, kLds),
    HP_GEMM_VARIANT(4, 4, 4, kLds),
    HP_GEMM_VARIANT(4, 2, 4, kLds),
    HP_GEMM_VARIANT(4, 2, 4, kDirect),
    HP_GEMM_VARIANT(4, 2, 8, kPipe),
    HP_GEMM_VARIANT(4, 4, 4, kPipe),
    HP_GEMM_VARIANT(2, 2, 4, kPipe),
};

int gemm_variants_kb1_4(const GemmVariant **out)
{
    *out = kVariants;
    return int(sizeof(kVariants) / sizeof(kVariants[0]));
}

}  // namespace hpmap
