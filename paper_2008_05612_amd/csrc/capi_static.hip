// hp_enumerate_batch_static: the batched enumeration of hp_enumerate_batch
// for callers that cannot allocate device memory.  The work list lives in a
// file-scope device array instead of a caller workspace, and reaches it
// through small install kernels whose arguments carry the bytes, so the call
// needs no allocation, no host buffer that outlives it and no host wait.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "hp_internal.h"
#include "kernels.h"

namespace hpmap {
namespace {

constexpr int kStaticJobs = HP_STATIC_BATCH_MAX_JOBS;
constexpr size_t kStaticBytes =
    (sizeof(BatchHeader) + sizeof(EnumJob) * kStaticJobs + sizeof(int64_t) * (kStaticJobs + 1) +
     255) & ~size_t(255);
static_assert(kStaticBytes % 4 == 0, "work list is copied in 32-bit words");

// Work-list bytes carried by one install launch (kernel arguments stay well
// below the 4 KiB argument limit).
constexpr uint32_t kChunkWords = 896;
struct PlanChunk {
    uint32_t off_words, n_words;
    uint32_t words[kChunkWords];
};

__global__ __launch_bounds__(256) void k_install(uint32_t *dst, PlanChunk c)
{
    for (uint32_t i = threadIdx.x; i < c.n_words; i += blockDim.x)
        dst[c.off_words + i] = c.words[i];
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

}  // namespace
}  // namespace hpmap

// The work list of hp_enumerate_batch_static on each GPU (one copy per
// device, held until the process ends).  Host code never passes this name to
// a kernel: it uses the device address that hipGetSymbolAddress returns.
static __device__ __align__(256) unsigned char scratch[hpmap::kStaticBytes];

namespace hpmap {
namespace {

// Device address of `scratch` on the current device, looked up once per
// device and kept.
hp_status static_scratch(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail(HP_EDEVICE, std::string("hp_enumerate_batch_static: hipGetDevice: ") +
                                    hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(HP_EUNSUPPORTED, "hp_enumerate_batch_static: device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(HP_EDEVICE,
                        std::string("hp_enumerate_batch_static: hipGetSymbolAddress: ") +
                            hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HP_OK;
}

}  // namespace
}  // namespace hpmap

using namespace hpmap;

extern "C" hp_status hp_enumerate_batch_static(const hp_job *jobs, int njobs, int form,
                                               void *stream)
{
    if (!jobs || njobs < 1)
        return fail(HP_EINVAL, "batch needs at least one job");
    if (njobs > kStaticJobs)
        return fail(HP_ERANGE, "hp_enumerate_batch_static takes at most " +
                                   std::to_string(kStaticJobs) + " jobs");
    if (form == HP_FORM_POPCOUNT) {
        for (int i = 0; i < njobs; ++i) {
            hp_status st = hp_enumerate(jobs[i].structs, jobs[i].d_ws, form, jobs[i].seq_lo,
                                        jobs[i].seq_hi, jobs[i].d_out, jobs[i].d_emin,
                                        jobs[i].d_designability, jobs[i].d_nondesign, stream);
            if (st != HP_OK)
                return st;
        }
        return HP_OK;
    }
    if (form != HP_FORM_GEMM_I8 && form != HP_FORM_BLOCKED_I8)
        return fail(HP_EINVAL, "unknown kernel form");
    alignas(16) char host[kStaticBytes];
    int order[kStaticJobs];
    int64_t start[kStaticJobs + 1];
    BatchGroup groups[kStaticJobs];
    int ngroups = 0;
    hp_status st = plan_batch(jobs, njobs, form, kStaticBytes, host, order, start, groups,
                              &ngroups);
    if (st != HP_OK)
        return st;
    void *d_list = nullptr;
    if ((st = static_scratch(&d_list)) != HP_OK)
        return st;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const uint32_t words = uint32_t(hp_batch_workspace_bytes(njobs) / 4);
    PlanChunk c;
    for (uint32_t off = 0; off < words; off += kChunkWords) {
        c.off_words = off;
        c.n_words = std::min(kChunkWords, words - off);
        std::memcpy(c.words, host + size_t(off) * 4, size_t(c.n_words) * 4);
        hipLaunchKernelGGL(k_install, dim3(1), dim3(256), 0, hs, static_cast<uint32_t *>(d_list),
                           c);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return fail(HP_EDEVICE, std::string("hp_enumerate_batch_static install: ") +
                                        hipGetErrorString(e));
    }
    hipError_t e = launch_plan(groups, ngroups, form, d_list, hs);
    if (e != hipSuccess)
        return fail(HP_EDEVICE,
                    std::string("hp_enumerate_batch_static launch: ") + hipGetErrorString(e));
    return HP_OK;
}
