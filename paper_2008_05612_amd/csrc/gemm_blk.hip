// Dispatch of the block-factorised int8 form by product depth.  The kernels
// themselves (gemm_blk.h) are instantiated per depth in gemm_blk_kb*.hip.
#include "hp_internal.h"
#include "kernels.h"

namespace hpmap {

#define HP_BLK_DECLARE(KB)                                                                    \
    hipError_t launch_gemm_blocked_kb##KB(const EnumJob &j, int nw, int mode, hipStream_t st); \
    hipError_t launch_gemm_blk_batch_kb##KB(BatchHeader *hdr, int item_lo, unsigned grid,     \
                                            bool unary, int wide, hipStream_t st);            \
    hipError_t launch_gemm_wide_kb##KB(const EnumJob &j, hipStream_t st);
HP_BLK_DECLARE(1)
HP_BLK_DECLARE(2)
HP_BLK_DECLARE(3)
HP_BLK_DECLARE(4)
HP_BLK_DECLARE(5)
HP_BLK_DECLARE(6)
HP_BLK_DECLARE(7)
HP_BLK_DECLARE(8)
HP_BLK_DECLARE(9)
HP_BLK_DECLARE(10)
HP_BLK_DECLARE(11)
HP_BLK_DECLARE(12)
#undef HP_BLK_DECLARE

namespace {

using BlockedLaunch = hipError_t (*)(const EnumJob &, int, int, hipStream_t);
using BlockedBatchLaunch = hipError_t (*)(BatchHeader *, int, unsigned, bool, int, hipStream_t);

// Index = product depth / 32 (1 .. kMaxKB).
const BlockedLaunch kBlocked[] = {
    nullptr,
    launch_gemm_blocked_kb1, launch_gemm_blocked_kb2, launch_gemm_blocked_kb3,
    launch_gemm_blocked_kb4, launch_gemm_blocked_kb5, launch_gemm_blocked_kb6,
    launch_gemm_blocked_kb7, launch_gemm_blocked_kb8, launch_gemm_blocked_kb9,
    launch_gemm_blocked_kb10, launch_gemm_blocked_kb11, launch_gemm_blocked_kb12,
};
const BlockedBatchLaunch kBlockedBatch[] = {
    nullptr,
    launch_gemm_blk_batch_kb1, launch_gemm_blk_batch_kb2, launch_gemm_blk_batch_kb3,
    launch_gemm_blk_batch_kb4, launch_gemm_blk_batch_kb5, launch_gemm_blk_batch_kb6,
    launch_gemm_blk_batch_kb7, launch_gemm_blk_batch_kb8, launch_gemm_blk_batch_kb9,
    launch_gemm_blk_batch_kb10, launch_gemm_blk_batch_kb11, launch_gemm_blk_batch_kb12,
};
using WideLaunch = hipError_t (*)(const EnumJob &, hipStream_t);
const WideLaunch kWide[] = {
    nullptr,
    launch_gemm_wide_kb1, launch_gemm_wide_kb2, launch_gemm_wide_kb3, launch_gemm_wide_kb4,
    launch_gemm_wide_kb5, launch_gemm_wide_kb6, launch_gemm_wide_kb7, launch_gemm_wide_kb8,
    launch_gemm_wide_kb9, launch_gemm_wide_kb10, launch_gemm_wide_kb11, launch_gemm_wide_kb12,
};
constexpr int kDepths = int(sizeof(kBlocked) / sizeof(kBlocked[0])) - 1;

}  // namespace

uint64_t blk_batch_seqs_per_item() { return uint64_t(1) << kWideBits; }

bool blk_batch_wide(const hp_structs *s)
{
    const int mode = blocked_selected_mode();
    return s->wide_ok && (mode < 0 || mode == kBlkStageWide);
}

bool blk_batch_wide8(const hp_structs *s, uint64_t lo, uint64_t hi)
{
    const uint64_t m = (uint64_t(1) << kWide11ChunkBits) - 1;
    const int mode = blocked_selected_mode();
    return blk_batch_wide(s) && (mode < 0 || blocked_selected_nw() == 8) &&
           s->N >= kWide11ChunkBits && hi > lo && (lo & m) == 0 && (hi & m) == 0;
}

hipError_t launch_gemm_blk_batch(void *d_batch_ws, int kb, bool unary, int wide, int item_lo,
                                 int item_hi, hipStream_t st)
{
    if (kb < 1 || kb > kDepths)
        return hipErrorInvalidValue;
    return kBlockedBatch[kb](static_cast<BatchHeader *>(d_batch_ws), item_lo,
                             unsigned(item_hi - item_lo), unary, wide, st);
}

hipError_t launch_gemm_blocked(const EnumJob &j, int nw, int mode, hipStream_t st)
{
    // automatic staging: shallow products keep the second operand in LDS,
    // which frees registers for a fourth wave per SIMD (measured faster for
    // K_pad <= 160, slower for 320)
    // wide blocks cover plain ranges with pure pair energies only; elsewhere
    // the staging falls back to the automatic choice, which takes wide blocks
    // where they apply (measured faster at every depth) and otherwise keeps
    // the second operand in LDS for shallow products
    const bool wide_ok = j.wide_s2 && j.mode == kSeqPlain && j.blk_ngroups == 0 &&
                         j.blk_coefB == 0;
    // wide blocks: 8 waves (blocks of 2048 where the range allows) by default
    // or when 8 waves are selected; 4 waves (blocks of 1024) when 4 are
    const bool wide8 = mode < 0 || nw == 8;
    if (mode == kBlkStageWide && !wide_ok)
        mode = -1;
    if (mode < 0)
        mode = wide_ok ? kBlkStageWide : (j.blk_KB <= 6 ? kBlkStageS2Lds : kBlkStageLds);
    if (mode == kBlkStageWide)
        nw = wide8 ? 8 : 4;
    if (j.blk_KB < 1 || j.blk_KB > kDepths)
        return hipErrorInvalidValue;
    return kBlocked[j.blk_KB](j, nw, mode, st);
}

}  // namespace hpmap

namespace hpmap {

hipError_t launch_gemm_wide_canonical(const EnumJob &j, hipStream_t st)
{
    if (j.blk_KB < 1 || j.blk_KB > kDepths || !j.wide_s2 || j.mode != kSeqCanonical)
        return hipErrorInvalidValue;
    return kWide[j.blk_KB](j, st);
}

}  // namespace hpmap
