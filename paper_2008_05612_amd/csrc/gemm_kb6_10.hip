// int8-MFMA ground-state kernels for product depths K_pad = 192 .. 320
// (N = 28 .. 36, e.g. the 6x6 square; the 3x3x3 cube with a two-letter
// contact table).  The first entry per depth is the
// default shape; the autotuner may pick any other.
#include "gemm_body.h"

namespace hpmap {

static const GemmVariant kVariants[] = {
    HP_GEMM_VARIANT(6, 2, 8, kLds),
    HP_GEMM_VARIANT(6, 2, 4, kLds),
    HP_GEMM_VARIANT(6, 2, 8, kPipe),
    HP_GEMM_VARIANT(6, 2, 4, kPipe),
    HP_GEMM_VARIANT(7, 2, 4, kLds),
    HP_GEMM_VARIANT(8, 2, 4, kLds),
    HP_GEMM_VARIANT(9, 2, 4, kLds),
    HP_GEMM_VARIANT(10, 2, 4, kLds),
    HP_GEMM_VARIANT(10, 2, 4, kDirect),
    HP_GEMM_VARIANT(10, 1, 4, kLds),
    HP_GEMM_VARIANT(10, 1, 8, kDirect),
    HP_GEMM_VARIANT(10, 2, 8, kLds),
    HP_GEMM_VARIANT(10, 3, 4, kLds),
    HP_GEMM_VARIANT(10, 2, 4, kPipe),
    HP_GEMM_VARIANT(10, 2, 8, kPipe),
    HP_GEMM_VARIANT(10, 1, 8, kPipe),
};

int gemm_variants_kb6_10(const GemmVariant **out)
{
    *out = kVariants;
    return int(sizeof(kVariants) / sizeof(kVariants[0]));
}

}  // namespace hpmap
