// Persistent batched launch of the int8-MFMA form: one kernel processes a
// list of enumeration jobs of different lattices and uneven sizes.
#include "gemm_body.h"

namespace hpmap {

// Persistent batched form: workgroups take fixed-size sequence tiles of any
// job from a shared counter until the list is exhausted, dispatching to the
// body compiled for that job's K_pad.  Every workgroup exits once the counter
// passes the last item.
template <int KBMAX, int T, int NW, int MODE>
__global__ __launch_bounds__(NW * 64) void k_gemm_batch(BatchHeader *hdr)
{
    __shared__ v4i lds[2 * KBMAX * 64];
    __shared__ int item_sh;
    const EnumJob *jobs = reinterpret_cast<const EnumJob *>(hdr + 1);
    const int njobs = hdr->njobs;
    const int64_t *start = reinterpret_cast<const int64_t *>(jobs + njobs);
    const int n_items = hdr->n_items;
    for (;;) {
        if (threadIdx.x == 0)
            item_sh = int(atomicAdd(&hdr->counter, 1u));
        __syncthreads();
        const int it = item_sh;
        __syncthreads();
        if (it >= n_items)
            break;
        int lo = 0, hi = njobs - 1;   // job with start[job] <= it < start[job+1]
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (start[mid] <= it)
                lo = mid;
            else
                hi = mid - 1;
        }
        const EnumJob j = jobs[lo];
        const uint64_t seq0 = j.lo + uint64_t(it - start[lo]) * (NW * T * 32);
        switch (j.KB) {
#define HP_CASE(kb)                                     \
    case kb:                                            \
        if constexpr (kb <= KBMAX)                      \
            gemm_body<kb, T, NW, MODE>(j, seq0, lds);         \
        break;
            HP_CASE(1) HP_CASE(2) HP_CASE(3) HP_CASE(4) HP_CASE(5)
            HP_CASE(6) HP_CASE(7) HP_CASE(8) HP_CASE(9) HP_CASE(10) HP_CASE(11) HP_CASE(12)
#undef HP_CASE
        default:
            break;
        }
    }
}

uint64_t gemm_batch_seqs_per_item(int kb_max)
{
    (void)kb_max;
    return 2 * 4 * 32;   // T = 2 sequence tiles x 4 waves x 32 sequences
}

hipError_t launch_gemm_batch(void *d_batch_ws, int kb_max, int n_items, hipStream_t st)
{
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess)
        return e;
    BatchHeader *hdr = static_cast<BatchHeader *>(d_batch_ws);
    e = launch_fill_u32(&hdr->counter, 0u, 1, st);
    if (e != hipSuccess)
        return e;
    const unsigned grid = unsigned(std::max(1, std::min(n_items, cus * 2)));  // two resident workgroups per CU
    if (kb_max <= 5)
        hipLaunchKernelGGL((k_gemm_batch<5, 2, 4, kLds>), dim3(grid), dim3(256), 0, st, hdr);
    else
        hipLaunchKernelGGL((k_gemm_batch<12, 2, 4, kLds>), dim3(grid), dim3(256), 0, st, hdr);
    return hipGetLastError();
}

}  // namespace hpmap
