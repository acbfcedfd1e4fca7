// Batched launch of the dense int8-MFMA form: the jobs of a batch (different
// lattices, uneven sizes) are grouped by product depth, and one launch of the
// kernel compiled for that depth covers each group's items, one workgroup per
// item.
#include "gemm_body.h"

namespace hpmap {

// Batched form for jobs of one product depth KB: workgroup b scores item
// item_lo + b, a fixed-size sequence tile of the job whose item range holds
// it.  (A persistent loop over items would keep values live across items and
// cost about 90 registers here.)
template <int KB, int T, int NW, int MODE>
__global__ __launch_bounds__(NW * 64) void k_gemm_batch(BatchHeader *hdr, int item_lo)
{
    __shared__ v4i lds[2 * KB * 64];
    const EnumJob *jobs = reinterpret_cast<const EnumJob *>(hdr + 1);
    const int njobs = hdr->njobs;
    const int64_t *start = reinterpret_cast<const int64_t *>(jobs + njobs);
    {
        // uniform indices let the job be read with scalar loads instead of
        // occupying vector registers
        const int it = item_lo + int(blockIdx.x);
        int lo = 0, hi = njobs - 1;   // job with start[job] <= it < start[job+1]
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (start[mid] <= it)
                lo = mid;
            else
                hi = mid - 1;
        }
        lo = __builtin_amdgcn_readfirstlane(lo);
        const EnumJob &j = jobs[lo];
        const uint64_t seq0 = j.lo + uint64_t(it - start[lo]) * (NW * T * 32);
        gemm_body<KB, T, NW, MODE>(j, seq0, lds);
    }
}

namespace {

template <int KB>
hipError_t launch_batch_kb(BatchHeader *hdr, int item_lo, unsigned grid, hipStream_t st)
{
    hipLaunchKernelGGL((k_gemm_batch<KB, 2, 4, kLds>), dim3(grid), dim3(256), 0, st, hdr, item_lo);
    return hipGetLastError();
}

}  // namespace

uint64_t gemm_batch_seqs_per_item()
{
    return 2 * 4 * 32;   // T = 2 sequence tiles x 4 waves x 32 sequences
}

hipError_t launch_gemm_batch(void *d_batch_ws, int kb, int item_lo, int item_hi, hipStream_t st)
{
    BatchHeader *hdr = static_cast<BatchHeader *>(d_batch_ws);
    const unsigned grid = unsigned(item_hi - item_lo);
    switch (kb) {
    case 1: return launch_batch_kb<1>(hdr, item_lo, grid, st);
    case 2: return launch_batch_kb<2>(hdr, item_lo, grid, st);
    case 3: return launch_batch_kb<3>(hdr, item_lo, grid, st);
    case 4: return launch_batch_kb<4>(hdr, item_lo, grid, st);
    case 5: return launch_batch_kb<5>(hdr, item_lo, grid, st);
    case 6: return launch_batch_kb<6>(hdr, item_lo, grid, st);
    case 7: return launch_batch_kb<7>(hdr, item_lo, grid, st);
    case 8: return launch_batch_kb<8>(hdr, item_lo, grid, st);
    case 9: return launch_batch_kb<9>(hdr, item_lo, grid, st);
    case 10: return launch_batch_kb<10>(hdr, item_lo, grid, st);
    case 11: return launch_batch_kb<11>(hdr, item_lo, grid, st);
    case 12: return launch_batch_kb<12>(hdr, item_lo, grid, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hpmap
