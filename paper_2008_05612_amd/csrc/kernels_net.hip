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

// ---------------------------------------------------------------------------
// Eight genotypes per lane.  The map is read as 16-byte vectors holding the
// genotypes 8k .. 8k+7: the mutants of bits 0..2 lie in the same vector, and
// the mutants of bit i >= 3 of all eight are the eight entries of vector
// k ^ 2^(i-3).  One 16-byte load then replaces eight 2-byte loads, so a wave
// issues an eighth of the load instructions.  These kernels serve 16-byte
// aligned maps with N >= 3; the one-genotype kernels cover the rest.
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t geno8(const uint4 &v, int r)
{
    const uint32_t w = r < 2 ? v.x : (r < 4 ? v.y : (r < 6 ? v.z : v.w));
    return (w >> (16 * (r & 1))) & 0xffffu;
}

__device__ __forceinline__ void unpack8(const uint4 &v, uint32_t q[8])
{
#pragma unroll
    for (int r = 0; r < 8; ++r)
        q[r] = geno8(v, r);
}

static bool use_geno8(const uint16_t *map, int N)
{
    return N >= 3 && (reinterpret_cast<uintptr_t>(map) & 15u) == 0;
}

__global__ __launch_bounds__(256) void k_neighbors8(const uint4 *__restrict__ m4, int N, uint64_t n8,
                                                    int n_class, unsigned long long *neutral,
                                                    unsigned long long *deleterious,
                                                    unsigned long long *other, int phi_q,
                                                    unsigned long long *phi_row)
{
    const uint16_t *__restrict__ map = reinterpret_cast<const uint16_t *>(m4);
    for (uint64_t k = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n8;
         k += uint64_t(gridDim.x) * blockDim.x) {
        uint32_t q[8];
        unpack8(m4[k], q);
        bool any = false;
#pragma unroll
        for (int r = 0; r < 8; ++r)
            any |= int(q[r]) < n_class;   // 0xFFFF and ids beyond n_class are not phenotypes
        if (!any)
            continue;
        // a: neutral mutants, d: deleterious ones; the other N - a - d change the phenotype
        uint32_t a[8], d[8];
#pragma unroll
        for (int r = 0; r < 8; ++r)
            a[r] = d[r] = 0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const uint32_t p = q[r ^ (1 << i)];
                a[r] += p == q[r] ? 1u : 0u;
                d[r] += p == HP_NONE ? 1u : 0u;
            }
        for (int i = 3; i < N; ++i) {
            const uint4 nv = m4[k ^ (uint64_t(1) << (i - 3))];
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const uint32_t p = geno8(nv, r);
                a[r] += p == q[r] ? 1u : 0u;
                d[r] += p == HP_NONE ? 1u : 0u;
            }
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            if (int(q[r]) >= n_class)
                continue;
            const uint32_t o = uint32_t(N) - a[r] - d[r];
            if (neutral && a[r])
                atomicAdd(&neutral[q[r]], (unsigned long long)a[r]);
            if (deleterious && d[r])
                atomicAdd(&deleterious[q[r]], (unsigned long long)d[r]);
            if (other && o)
                atomicAdd(&other[q[r]], (unsigned long long)o);
            if (phi_row && int(q[r]) == phi_q) {
                const uint64_t g = 8 * k + uint64_t(r);
                for (int i = 0; i < N; ++i) {
                    const uint16_t p = map[g ^ (uint64_t(1) << i)];
                    atomicAdd(&phi_row[(p == HP_NONE || int(p) >= n_class) ? n_class : int(p)],
                              1ull);
                }
            }
        }
    }
}

hipError_t launch_neighbors(const uint16_t *map, int N, int n_class, unsigned long long *neutral,
                            unsigned long long *deleterious, unsigned long long *other, int phi_q,
                            unsigned long long *phi_row, hipStream_t st)
{
    const uint64_t total = uint64_t(1) << N;
    if (use_geno8(map, N)) {
        const uint64_t n8 = total / 8;
        hipLaunchKernelGGL(k_neighbors8, dim3(grid_for(n8, 256)), dim3(256), 0, st,
                           reinterpret_cast<const uint4 *>(map), N, n8, n_class, neutral,
                           deleterious, other, phi_q, phi_row);
    } else {
        hipLaunchKernelGGL(k_neighbors, dim3(grid_for(total, 256)), dim3(256), 0, st, map, N,
                           total, n_class, neutral, deleterious, other, phi_q, phi_row);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The whole phi_pq matrix (Eq. 2) as dense counts: row q (phenotype of the
// genotype, q < n_class), column p (phenotype of its single-point mutant,
// column n_class for deleterious ids).  Neutral and deleterious mutants of
// a genotype are summed in registers and added once; each mutant into
// another phenotype adds one at (q, p).
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_phi_counts(const uint16_t *__restrict__ map, int N,
                                                    uint64_t total, int n_class,
                                                    unsigned long long *counts)
{
    const uint64_t ld = uint64_t(n_class) + 1;
    for (uint64_t g = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < total;
         g += uint64_t(gridDim.x) * blockDim.x) {
        const int q = map[g];
        if (q >= n_class)   // 0xFFFF and ids beyond n_class have no row
            continue;
        unsigned long long *row = counts + uint64_t(q) * ld;
        unsigned neutral = 0, del = 0;
        for (int i = 0; i < N; ++i) {
            const int p = map[g ^ (uint64_t(1) << i)];
            if (p == q)
                ++neutral;
            else if (p >= n_class)
                ++del;
            else
                atomicAdd(&row[p], 1ull);
        }
        if (neutral)
            atomicAdd(&row[q], (unsigned long long)neutral);
        if (del)
            atomicAdd(&row[n_class], (unsigned long long)del);
    }
}

// Eight genotypes per lane (the vector layout of k_neighbors8).
__global__ __launch_bounds__(256) void k_phi_counts8(const uint4 *__restrict__ m4, int N,
                                                     uint64_t n8, int n_class,
                                                     unsigned long long *counts)
{
    const uint64_t ld = uint64_t(n_class) + 1;
    for (uint64_t k = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n8;
         k += uint64_t(gridDim.x) * blockDim.x) {
        uint32_t q[8];
        unpack8(m4[k], q);
        bool any = false;
#pragma unroll
        for (int r = 0; r < 8; ++r)
            any |= int(q[r]) < n_class;
        if (!any)
            continue;
        uint32_t neutral[8], del[8];
#pragma unroll
        for (int r = 0; r < 8; ++r)
            neutral[r] = del[r] = 0;
        // one mutant p of genotype r: neutral and deleterious ones are
        // counted in registers, one into another phenotype adds at (q, p)
        auto take = [&](int r, uint32_t p) {
            if (int(q[r]) >= n_class)
                return;
            if (p == q[r])
                ++neutral[r];
            else if (int(p) >= n_class)
                ++del[r];
            else
                atomicAdd(&counts[uint64_t(q[r]) * ld + p], 1ull);
        };
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int r = 0; r < 8; ++r)
                take(r, q[r ^ (1 << i)]);
        for (int i = 3; i < N; ++i) {
            const uint4 nv = m4[k ^ (uint64_t(1) << (i - 3))];
#pragma unroll
            for (int r = 0; r < 8; ++r)
                take(r, geno8(nv, r));
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            if (int(q[r]) >= n_class)
                continue;
            unsigned long long *row = counts + uint64_t(q[r]) * ld;
            if (neutral[r])
                atomicAdd(&row[q[r]], (unsigned long long)neutral[r]);
            if (del[r])
                atomicAdd(&row[n_class], (unsigned long long)del[r]);
        }
    }
}

// Sparse rows (CSR, columns ascending).  Both passes stream the dense
// matrix once (HBM-bound); each thread keeps kPhiUnroll loads in flight, a
// workgroup covers kPhiChunk consecutive columns per iteration.
constexpr int kPhiUnroll = 4;
constexpr int kPhiChunk = 256 * kPhiUnroll;

// k_phi_row_nnz: one workgroup per row writes its number of non-zero
// entries to row_ptr[q].
__global__ __launch_bounds__(256) void k_phi_row_nnz(const unsigned long long *__restrict__ counts,
                                                     int n_class, uint64_t *row_ptr)
{
    __shared__ unsigned part[4];
    const uint64_t ld = uint64_t(n_class) + 1;
    const unsigned long long *row = counts + uint64_t(blockIdx.x) * ld;
    unsigned c = 0;
    for (uint64_t base = 0; base < ld; base += kPhiChunk) {
        unsigned long long v[kPhiUnroll];
#pragma unroll
        for (int k = 0; k < kPhiUnroll; ++k) {
            const uint64_t p = base + k * 256 + threadIdx.x;
            v[k] = p < ld ? row[p] : 0;
        }
#pragma unroll
        for (int k = 0; k < kPhiUnroll; ++k)
            c += v[k] != 0;
    }
    for (int o = 32; o; o >>= 1)
        c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0)
        row_ptr[blockIdx.x] = uint64_t(part[0]) + part[1] + part[2] + part[3];
}

// In-place exclusive scan of row_ptr[0 .. n) with the total written to
// row_ptr[n]: one workgroup, thread t owns a contiguous chunk.
__global__ __launch_bounds__(1024) void k_phi_scan(uint64_t *row_ptr, int n)
{
    __shared__ uint64_t sums[1024];
    const int t = threadIdx.x;
    const int per = (n + 1023) / 1024;
    const int lo = min(n, t * per), hi = min(n, lo + per);
    uint64_t s = 0;
    for (int i = lo; i < hi; ++i)
        s += row_ptr[i];
    sums[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {   // inclusive scan of the chunk sums
        const uint64_t v = t >= off ? sums[t - off] : 0;
        __syncthreads();
        sums[t] += v;
        __syncthreads();
    }
    uint64_t run = t ? sums[t - 1] : 0;
    for (int i = lo; i < hi; ++i) {
        const uint64_t c = row_ptr[i];
        row_ptr[i] = run;
        run += c;
    }
    if (t == 1023)
        row_ptr[n] = sums[1023];
}

// One workgroup per row: the non-zero entries in column order, from
// row_ptr[q] onwards.  Sub-chunk k of a chunk holds columns base + 256 k ..
// base + 256 k + 255 (thread t reads column base + 256 k + t); an entry's
// slot is the count of non-zeros in earlier sub-chunks, earlier waves of its
// sub-chunk (per-wave counts in LDS) and earlier lanes of its wave (ballot).
__global__ __launch_bounds__(256) void k_phi_compact(const unsigned long long *__restrict__ counts,
                                                     int n_class, const uint64_t *__restrict__ row_ptr,
                                                     uint32_t *cols, uint64_t *vals)
{
    __shared__ unsigned wave_n[kPhiUnroll][4];
    const uint64_t ld = uint64_t(n_class) + 1;
    const unsigned long long *row = counts + uint64_t(blockIdx.x) * ld;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const unsigned long long below = (1ull << lane) - 1;
    uint64_t at = row_ptr[blockIdx.x];
    for (uint64_t base = 0; base < ld; base += kPhiChunk) {
        unsigned long long v[kPhiUnroll];
        unsigned before[kPhiUnroll];
#pragma unroll
        for (int k = 0; k < kPhiUnroll; ++k) {
            const uint64_t p = base + k * 256 + threadIdx.x;
            v[k] = p < ld ? row[p] : 0;
        }
#pragma unroll
        for (int k = 0; k < kPhiUnroll; ++k) {
            const unsigned long long m = __ballot(v[k] != 0);
            before[k] = __popcll(m & below);
            if (lane == 0)
                wave_n[k][wave] = __popcll(m);
        }
        __syncthreads();
        unsigned run = 0;
#pragma unroll
        for (int k = 0; k < kPhiUnroll; ++k) {
            unsigned off = 0;
            for (int w = 0; w < 4; ++w) {
                off += w < wave ? wave_n[k][w] : 0;
            }
            if (v[k]) {
                const uint64_t slot = at + run + off + before[k];
                cols[slot] = uint32_t(base + k * 256 + threadIdx.x);
                vals[slot] = v[k];
            }
            run += wave_n[k][0] + wave_n[k][1] + wave_n[k][2] + wave_n[k][3];
        }
        at += run;
        __syncthreads();   // wave_n is rewritten by the next chunk
    }
}

hipError_t launch_phi_counts(const uint16_t *map, int N, int n_class, unsigned long long *counts,
                             hipStream_t st)
{
    const uint64_t total = uint64_t(1) << N;
    if (use_geno8(map, N)) {
        const uint64_t n8 = total / 8;
        hipLaunchKernelGGL(k_phi_counts8, dim3(grid_for(n8, 256)), dim3(256), 0, st,
                           reinterpret_cast<const uint4 *>(map), N, n8, n_class, counts);
    } else {
        hipLaunchKernelGGL(k_phi_counts, dim3(grid_for(total, 256)), dim3(256), 0, st, map, N,
                           total, n_class, counts);
    }
    return hipGetLastError();
}

hipError_t launch_phi_row_ptr(const unsigned long long *counts, int n_class, uint64_t *row_ptr,
                              hipStream_t st)
{
    hipLaunchKernelGGL(k_phi_row_nnz, dim3(n_class), dim3(256), 0, st, counts, n_class, row_ptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_phi_scan, dim3(1), dim3(1024), 0, st, row_ptr, n_class);
    return hipGetLastError();
}

hipError_t launch_phi_compact(const unsigned long long *counts, int n_class,
                              const uint64_t *row_ptr, uint32_t *cols, uint64_t *vals,
                              hipStream_t st)
{
    hipLaunchKernelGGL(k_phi_compact, dim3(n_class), dim3(256), 0, st, counts, n_class, row_ptr,
                       cols, vals);
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

// Eight genotypes per lane (the vector layout of k_neighbors8): the edges
// g -- g|bit of the genotypes 8k .. 8k+7.
__global__ __launch_bounds__(256) void k_uf_hook8(const uint4 *__restrict__ m4, int N,
                                                  uint32_t *parent, uint64_t n8)
{
    for (uint64_t k = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n8;
         k += uint64_t(gridDim.x) * blockDim.x) {
        uint32_t q[8];
        unpack8(m4[k], q);
        bool any = false;
#pragma unroll
        for (int r = 0; r < 8; ++r)
            any |= q[r] != HP_NONE;
        if (!any)
            continue;
        const uint32_t g0 = uint32_t(8 * k);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int r = 0; r < 8; ++r)
                if (!(r & (1 << i)) && q[r] != HP_NONE && q[r | (1 << i)] == q[r])
                    uf_unite(parent, g0 + r, g0 + (r | (1 << i)));
        for (int i = 3; i < N; ++i) {
            const uint64_t u = k | (uint64_t(1) << (i - 3));
            if (u == k)
                continue;
            const uint4 nv = m4[u];
            const uint32_t u0 = uint32_t(8 * u);
#pragma unroll
            for (int r = 0; r < 8; ++r)
                if (q[r] != HP_NONE && geno8(nv, r) == q[r])
                    uf_unite(parent, g0 + r, u0 + r);
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

// Eight genotypes per lane (map and labels read as vectors).
__global__ __launch_bounds__(256) void k_uf_count8(const uint4 *__restrict__ m4,
                                                   const uint4 *__restrict__ labels4,
                                                   const uint32_t *__restrict__ compsize,
                                                   uint32_t *ncomp, uint32_t *largest,
                                                   int n_class, uint64_t n8)
{
    for (uint64_t k = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n8;
         k += uint64_t(gridDim.x) * blockDim.x) {
        uint32_t q[8];
        unpack8(m4[k], q);
        bool any = false;
#pragma unroll
        for (int r = 0; r < 8; ++r)
            any |= int(q[r]) < n_class;
        if (!any)
            continue;
        const uint4 la = labels4[2 * k], lb = labels4[2 * k + 1];
        const uint32_t lab[8] = {la.x, la.y, la.z, la.w, lb.x, lb.y, lb.z, lb.w};
        const uint32_t g0 = uint32_t(8 * k);
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            if (int(q[r]) >= n_class || lab[r] != g0 + uint32_t(r))
                continue;
            if (ncomp)
                atomicAdd(&ncomp[q[r]], 1u);
            if (largest)
                atomicMax(&largest[q[r]], compsize[g0 + r]);
        }
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
    // eight genotypes per lane where the map (and, for the count, the labels)
    // are 16-byte vectors; one genotype per lane otherwise.  The init pass
    // stays one genotype per lane: its 4-byte stores are contiguous per wave
    // (measured 0.30 ms against 0.36 ms for 8 per lane on the 3x3x3 map).
    const bool v8 = use_geno8(map, N) && (reinterpret_cast<uintptr_t>(labels) & 15u) == 0;
    const uint64_t n8 = total / 8;
    const dim3 grid8(grid_for(n8, 256));
    const uint4 *m4 = reinterpret_cast<const uint4 *>(map);
    hipLaunchKernelGGL(k_uf_init, grid, block, 0, st, map, labels, compsize, total);
    if (use_geno8(map, N))
        hipLaunchKernelGGL(k_uf_hook8, grid8, block, 0, st, m4, N, labels, n8);
    else
        hipLaunchKernelGGL(k_uf_hook, grid, block, 0, st, map, N, labels, total);
    hipLaunchKernelGGL(k_uf_compress, grid, block, 0, st, map, labels, compsize, total);
    if (v8)
        hipLaunchKernelGGL(k_uf_count8, grid8, block, 0, st, m4,
                           reinterpret_cast<const uint4 *>(labels), compsize, ncomp, largest,
                           n_class, n8);
    else
        hipLaunchKernelGGL(k_uf_count, grid, block, 0, st, map, labels, compsize, ncomp, largest,
                           n_class, total);
    return hipGetLastError();
}

}  // namespace hpmap
