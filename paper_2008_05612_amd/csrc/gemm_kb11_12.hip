// int8-MFMA ground-state kernels for product depths K_pad = 352 .. 384 (N up
// to 36 with a two-letter contact table, e.g. the 6x6 square).  The first
// entry per depth is the default shape; the autotuner may pick any other.
#include "gemm_body.h"

namespace hpmap {

static const GemmVariant kVariants[] = {
    HP_GEMM_VARIANT(11, 2, 4, kLds),
    HP_GEMM_VARIANT(11, 2, 4, kPipe),
    HP_GEMM_VARIANT(11, 1, 8, kPipe),
    HP_GEMM_VARIANT(12, 2, 4, kLds),
    HP_GEMM_VARIANT(12, 2, 4, kPipe),
};

int gemm_variants_kb11_12(const GemmVariant **out)
{
    *out = kVariants;
    return int(sizeof(kVariants) / sizeof(kVariants[0]));
}

}  // namespace hpmap
