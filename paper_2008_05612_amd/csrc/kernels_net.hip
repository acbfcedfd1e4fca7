// Genotype-network kernels of libhpmap: single-point-mutation counts (the
// numerators of phi_pq, robustness and phi_del of Eq. 2) and neutral-network
// components by union-find on the N-cube of sequences.
//
// Both kernels stream the uint16 phenotype map; they are bound by HBM
// bandwidth, not arithmetic.
#include <hip/hip_runtime.h>

#include "hp_internal.h"
#include "kernels.h"

namespace hpmap {

namespace {

unsigned grid_for(uint64_t n, unsigned block)
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;   // a grid-size hint only
    const uint64_t want = (n + block - 1) / block;
    const uint64_t cap = uint64_t(cus) * 16;
    return unsigned(std::max<uint64_t>(1, std::min(want, cap)));
}

}  // namespace

// For each designing genotype g (phenotype q) and each one-bit mutant p:
// neutral / deleterious / other counts of q, and the phi row of phi_q.
__global__ __launch_bounds__(256) void k_neighbors(const uint16_t *__restrict__ map, int N,
                                                   uint64_t total, int n_class,
                                                   unsigned long long *neutral,
                                                   unsigned long long *deleterious,
                                                   unsigned long long *other, int phi_q,
                                                   unsigned long long *phi_row)
{
    for (uint64_t g = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += uint64_t(gridDim.x) * blockDim.x) {
        const uint16_t q = map[g];
        if (q == HP_NONE || int(q) >= n_class)   // ids beyond n_class are not phenotypes
            continue;
        unsigned a = 0, d = 0, o = 0;
        for (int i = 0; i < N; ++i) {
            const uint16_t p = map[g ^ (uint64_t(1) << i)];
            a += p == q;
            d += p == HP_NONE;
            o += (p != q) & (p != HP_NONE);
            if (phi_row && int(q) == phi_q)
                atomicAdd(&phi_row[(p == HP_NONE || int(p) >= n_class) ? n_class : int(p)], 1ull);
        }
        if (neutral && a)
            atomicAdd(&neutral[q], (unsigned long long)a);
        if (deleterious && d)
            atomicAdd(&deleterious[q], (unsigned long long)d);
        if (other && o)
            atomicAdd(&other[q], (unsigned long long)o);
    }
}

hipError_t launch_neighbors(const uint16_t *map, int N, int n_class, unsigned long long *neutral,
                            unsigned long long *deleterious, unsigned long long *other, int phi_q,
                            unsigned long long *phi_row, hipStream_t st)
{
    const uint64_t total = uint64_t(1) << N;
    hipLaunchKernelGGL(k_neighbors, dim3(grid_for(total, 256)), dim3(256), 0, st, map, N, total,
                       n_class, neutral, deleterious, other, phi_q, phi_row);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Union-find.  parent[x] <= x always holds and roots satisfy parent[x] == x;
// two roots are joined by pointing the larger at the smaller with a CAS, so
// the root of every tree is its smallest member and the final labels do not
// depend on the schedule.  Path halving writes only ancestors, so concurrent
// readers always see a valid (older or newer) ancestor.
// ---------------------------------------------------------------------------

constexpr uint32_t kNoLabel = 0xFFFFFFFFu;

__device__ __forceinline__ uint32_t uf_root(uint32_t *parent, uint32_t x)
{
    uint32_t p = parent[x];
    while (p != x) {
        const uint32_t gp = parent[p];
        if (gp != p)
            parent[x] = gp;
        x = p;
        p = gp;
    }
    return x;
}

__device__ __forceinline__ void uf_unite(uint32_t *parent, uint32_t a, uint32_t b)
{
    uint32_t ra = uf_root(parent, a), rb = uf_root(parent, b);
    while (ra != rb) {
        const uint32_t hi = max(ra, rb), lo = min(ra, rb);
        const uint32_t old = atomicCAS(&parent[hi], hi, lo);
        if (old == hi)
            break;
        ra = uf_root(parent, old);
        rb = uf_root(parent, lo);
    }
}

__global__ __launch_bounds__(256) void k_uf_init(const uint16_t *__restrict__ map, uint32_t *parent,
                                                 uint32_t *compsize, uint64_t total)
{
    for (uint64_t g = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += uint64_t(gridDim.x) * blockDim.x) {
        parent[g] = map[g] == HP_NONE ? kNoLabel : uint32_t(g);
        compsize[g] = 0;
    }
}

// Edge g -- g|bit for every clear bit of g between equal designing phenotypes.
__global__ __launch_bounds__(256) void k_uf_hook(const uint16_t *__restrict__ map, int N,
                                                 uint32_t *parent, uint64_t total)
{
    for (uint64_t g = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += uint64_t(gridDim.x) * blockDim.x) {
        const uint16_t q = map[g];
        if (q == HP_NONE)
            continue;
        for (int i = 0; i < N; ++i) {
            const uint64_t u = g | (uint64_t(1) << i);
            if (u != g && map[u] == q)
                uf_unite(parent, uint32_t(g), uint32_t(u));
        }
    }
}

__global__ __launch_bounds__(256) void k_uf_compress(const uint16_t *__restrict__ map,
                                                     uint32_t *parent, uint32_t *compsize,
                                                     uint64_t total)
{
    for (uint64_t g = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += uint64_t(gridDim.x) * blockDim.x) {
        if (map[g] == HP_NONE)
            continue;
        uint32_t r = uint32_t(g);
        while (parent[r] != r)
            r = parent[r];
        parent[g] = r;
        atomicAdd(&compsize[r], 1u);
    }
}

__global__ __launch_bounds__(256) void k_uf_count(const uint16_t *__restrict__ map,
                                                  const uint32_t *__restrict__ labels,
                                                  const uint32_t *__restrict__ compsize,
                                                  uint32_t *ncomp, uint32_t *largest,
                                                  int n_class, uint64_t total)
{
    for (uint64_t g = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += uint64_t(gridDim.x) * blockDim.x) {
        const uint16_t q = map[g];
        if (q == HP_NONE || int(q) >= n_class || labels[g] != uint32_t(g))
            continue;
        if (ncomp)
            atomicAdd(&ncomp[q], 1u);
        if (largest)
            atomicMax(&largest[q], compsize[g]);
    }
}

hipError_t launch_components(const uint16_t *map, int N, uint32_t *labels, uint32_t *compsize,
                             uint32_t *ncomp, uint32_t *largest, int n_class, hipStream_t st)
{
    const uint64_t total = uint64_t(1) << N;
    const dim3 grid(grid_for(total, 256)), block(256);
    hipError_t e;
    if (ncomp && (e = launch_fill_u32(ncomp, 0u, uint64_t(n_class), st)) != hipSuccess)
        return e;
    if (largest && (e = launch_fill_u32(largest, 0u, uint64_t(n_class), st)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_uf_init, grid, block, 0, st, map, labels, compsize, total);
    hipLaunchKernelGGL(k_uf_hook, grid, block, 0, st, map, N, labels, total);
    hipLaunchKernelGGL(k_uf_compress, grid, block, 0, st, map, labels, compsize, total);
    hipLaunchKernelGGL(k_uf_count, grid, block, 0, st, map, labels, compsize, ncomp, largest,
                       n_class, total);
    return hipGetLastError();
}

}  // namespace hpmap
