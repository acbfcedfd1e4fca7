// Ground-state kernels of libhpmap for gfx950: the plain popcount form and the
// int8-MFMA form, plus the persistent batched launch.
//
// Both forms evaluate, for every (sequence s, conformation c) pair, the number
// of H-H contacts n(s,c) (the energy of Eq. 1 with E_HH = -1 is -n), keep the
// running best and second-best, and finally test uniqueness of the minimum
// energy (Methods, end of "HP and MJ lattice models").
//
// Running state is a pair of 32-bit keys per sequence.  A key orders first by
// n and then by conformation, so the largest key is a minimum-energy
// conformation and the second-largest key has the same n exactly when the
// minimum is shared.  The global key is (n << 17) | c.
//
// Pair products.  Contacts on the bipartite lattice join monomers whose
// separation j - i is odd and >= 3; index these K pairs as k.  For sequence s,
// P_k(s) = h_i h_j, so n(s,c) = sum_k P_k(s) C_k(c) where C_k(c) = 1 iff pair k
// is a contact of c.
//   popcount form:  P and C as K-bit masks, n = popcount(P & C);
//   int8 form:      n as an int8 x int8 -> int32 matrix product on MFMA.
//
// int8 form in detail.  A = C^T in 32-conformation x 32-pair blocks (MFMA
// operand A, one 16-byte slice per lane), B = P for 32 sequences, generated in
// registers once per sequence tile.  Entries are scaled to -128 on both sides,
// so each H-H contact adds 16384.  Two extra rows carry the conformation's
// position idx in its window of 16384 conformations: row K has P = 1 and
// C = idx & 127, row K+1 has P = -128 and C = -(idx >> 7).  The MFMA output is
// therefore directly the window key 16384 n + idx, and the epilogue is two
// VALU ops per pair (max3 and med3 over two keys, then one max).  Padding
// columns carry C = -1 in row K, i.e. key -1, which never wins.  At every
// window boundary the window's top-2 keys are converted to global keys.
#include <hip/hip_runtime.h>

#include <climits>

#include "hp_internal.h"
#include "kernels.h"

namespace hpmap {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kWinShift = 14;   // window key = (n << 14) | idx

__device__ __forceinline__ int med3_i32(int a, int b, int c)
{
    int r;
    asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// (b, s) is the running top-2, b >= s.  Absorb keys k1 and k2.
__device__ __forceinline__ void top2_add2(int &b, int &s, int k1, int k2)
{
    int m = med3_i32(b, k1, k2);     // second largest of {b, k1, k2}
    b = max(max(b, k1), k2);
    s = max(s, m);
}

__device__ __forceinline__ void top2_add1(int &b, int &s, int k)
{
    s = max(s, min(b, k));
    b = max(b, k);
}

__device__ __forceinline__ void top2_merge(int &b, int &s, int b2, int s2)
{
    s = max(min(b, b2), max(s, s2));
    b = max(b, b2);
}

// Window key -> global key; negative keys (padding, empty) stay negative.
__device__ __forceinline__ int window_to_global(int k, int conf_base)
{
    int g = ((k >> kWinShift) << kKeyConfBits) | (conf_base + (k & (kWindowConf - 1)));
    return k < 0 ? -1 : g;
}

// Final decision for one sequence and the per-sequence outputs.
__device__ __forceinline__ void finish_sequence(const EnumJob &j, uint64_t s, bool valid, int gb,
                                                int gs, bool count_lane)
{
    const int nb = gb >> kKeyConfBits;
    const int ns = gs >> kKeyConfBits;   // arithmetic shift keeps "none" negative
    const bool uniq = nb != ns;
    uint16_t q = HP_NONE;
    if (valid && uniq)   // the clamp keeps the table read in bounds for any key
        q = j.c2q[min(gb & int(kMaxConf - 1), j.n_conf - 1)];
    if (valid) {
        if (j.out)
            j.out[s - j.lo] = q;
        if (j.emin)
            j.emin[s - j.lo] = -nb;
        if (uniq && j.desig)
            atomicAdd(&j.desig[q], 1ull);
    }
    const unsigned long long del = __ballot(valid && !uniq);
    if (count_lane && j.nondesign && del)
        atomicAdd(j.nondesign, (unsigned long long)__popcll(del));
}

// ---------------------------------------------------------------------------
// Popcount form: one sequence per lane, contact masks read as wave-uniform
// (scalar) loads, running keys in VGPRs.
// ---------------------------------------------------------------------------

template <int W>
__global__ __launch_bounds__(256) void k_popcount(EnumJob j, const uint32_t *__restrict__ masks,
                                                  const uint8_t *__restrict__ pairs)
{
    const uint64_t s = j.lo + uint64_t(blockIdx.x) * 256 + threadIdx.x;
    const bool valid = s < j.hi;
    uint32_t P[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        uint32_t v = 0;
        for (int b = 0; b < 32; ++b) {
            const int k = w * 32 + b;
            if (k < j.K) {
                const uint32_t hi = pairs[2 * k], hj = pairs[2 * k + 1];
                v |= uint32_t((s >> hi) & (s >> hj) & 1u) << b;
            }
        }
        P[w] = v;
    }
    int best = INT_MIN, second = INT_MIN;
    const int n_conf = j.n_conf;
    int c = 0;
    for (; c + 2 <= n_conf; c += 2) {
        const uint32_t *m = masks + size_t(c) * W;
        int n0 = 0, n1 = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            n0 += __popc(P[w] & m[w]);
            n1 += __popc(P[w] & m[W + w]);
        }
        top2_add2(best, second, (n0 << kKeyConfBits) | c, (n1 << kKeyConfBits) | (c + 1));
    }
    if (c < n_conf) {
        const uint32_t *m = masks + size_t(c) * W;
        int n0 = 0;
#pragma unroll
        for (int w = 0; w < W; ++w)
            n0 += __popc(P[w] & m[w]);
        top2_add1(best, second, (n0 << kKeyConfBits) | c);
    }
    finish_sequence(j, s, valid, best, second, (threadIdx.x & 63) == 0);
}

// ---------------------------------------------------------------------------
// int8 MFMA form.
// ---------------------------------------------------------------------------

// 16 bytes of B for one lane: P values of sequence s for pair rows
// kbase .. kbase+15 (byte q of the fragment is row kbase+q).
__device__ __forceinline__ v4i p_fragment(uint64_t s, int kbase, int K, const uint8_t *pairs)
{
    v4i r;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        uint32_t word = 0;
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) {
            const int k = kbase + 4 * q + bb;
            uint32_t byte = 0;
            if (k < K) {
                const uint32_t hi = pairs[2 * k], hj = pairs[2 * k + 1];
                byte = ((s >> hi) & (s >> hj) & 1u) ? 0x80u : 0u;
            } else if (k == K) {
                byte = 0x01u;
            } else if (k == K + 1) {
                byte = 0x80u;
            }
            word |= byte << (8 * bb);
        }
        r[q] = int(word);
    }
    return r;
}

template <int KB, int NW>
struct TileStage {
    static constexpr int kVecs = KB * 64;                       // 16-byte vectors per tile
    static constexpr int kPer = (kVecs + NW * 64 - 1) / (NW * 64);
    v4i v[kPer];

    __device__ __forceinline__ void load(const v4i *__restrict__ A, int tile)
    {
        const v4i *src = A + size_t(tile) * kVecs;
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int i = threadIdx.x + r * NW * 64;
            if (kVecs % (NW * 64) == 0 || i < kVecs)
                v[r] = src[i];
        }
    }
    __device__ __forceinline__ void store(v4i *dst) const
    {
#pragma unroll
        for (int r = 0; r < kPer; ++r) {
            const int i = threadIdx.x + r * NW * 64;
            if (kVecs % (NW * 64) == 0 || i < kVecs)
                dst[i] = v[r];
        }
    }
};

// One workgroup scores NW*T*32 consecutive sequences starting at seq0 against
// every conformation tile.  lds must hold 2 * KB * 64 vectors.
template <int KB, int T, int NW>
__device__ __forceinline__ void gemm_body(const EnumJob &j, uint64_t seq0_wg, v4i *lds)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 31;
    const int half = lane >> 5;
    const uint64_t seq0 = seq0_wg + uint64_t(wave) * (T * 32);
    const v4i *__restrict__ A = reinterpret_cast<const v4i *>(j.gemm_a);

    v4i pf[T][KB];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const uint64_t s = seq0 + t * 32 + col;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
            pf[t][kb] = p_fragment(s, kb * 32 + half * 16, j.K, j.pairs);
    }

    int b[T], sc[T], gb[T], gs[T];
#pragma unroll
    for (int t = 0; t < T; ++t)
        b[t] = sc[t] = gb[t] = gs[t] = INT_MIN;

    const int n_tiles = j.n_tiles;
    TileStage<KB, NW> stg;
    stg.load(A, 0);
    stg.store(lds);
    __syncthreads();

    int wend = min(kWindowTiles, n_tiles);
    int conf_base = 0;
    for (int tile = 0; tile < n_tiles; ++tile) {
        const bool more = tile + 1 < n_tiles;
        if (more)
            stg.load(A, tile + 1);
        const v4i *cur = lds + (tile & 1) * (KB * 64);
        v16i acc[T];
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            const v4i a = cur[kb * 64 + lane];
#pragma unroll
            for (int t = 0; t < T; ++t) {
                const v16i zero = {};
                acc[t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, pf[t][kb], kb == 0 ? zero : acc[t],
                                                                0, 0, 0);
            }
        }
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int r = 0; r < 16; r += 2)
                top2_add2(b[t], sc[t], acc[t][r], acc[t][r + 1]);
        if (tile + 1 == wend) {
#pragma unroll
            for (int t = 0; t < T; ++t) {
                top2_merge(gb[t], gs[t], window_to_global(b[t], conf_base),
                           window_to_global(sc[t], conf_base));
                b[t] = sc[t] = INT_MIN;
            }
            conf_base += kWindowConf;
            wend = min(wend + kWindowTiles, n_tiles);
        }
        if (more)
            stg.store(lds + ((tile + 1) & 1) * (KB * 64));
        __syncthreads();
    }

#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int ob = __shfl_xor(gb[t], 32);
        const int os = __shfl_xor(gs[t], 32);
        top2_merge(gb[t], gs[t], ob, os);
        const uint64_t s = seq0 + t * 32 + col;
        finish_sequence(j, s, half == 0 && s < j.hi, gb[t], gs[t], lane == 0);
    }
}

template <int KB, int T, int NW>
__global__ __launch_bounds__(NW * 64) void k_gemm(EnumJob j)
{
    __shared__ v4i lds[2 * KB * 64];
    const uint64_t seq0 = j.lo + uint64_t(blockIdx.x) * (NW * T * 32);
    gemm_body<KB, T, NW>(j, seq0, lds);
}

// Persistent batched form: workgroups take fixed-size sequence tiles of any
// job from a shared counter until the list is exhausted, dispatching to the
// body compiled for that job's K_pad.  Every workgroup exits once the counter
// passes the last item.
template <int KBMAX, int T, int NW>
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
            gemm_body<kb, T, NW>(j, seq0, lds);         \
        break;
            HP_CASE(1) HP_CASE(2) HP_CASE(3) HP_CASE(4) HP_CASE(5)
            HP_CASE(6) HP_CASE(7) HP_CASE(8) HP_CASE(9) HP_CASE(10)
#undef HP_CASE
        default:
            break;
        }
    }
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, uint64_t n)
{
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += uint64_t(gridDim.x) * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u64(unsigned long long *p, unsigned long long v, uint64_t n)
{
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += uint64_t(gridDim.x) * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, uint64_t n, hipStream_t st)
{
    if (n == 0)
        return hipSuccess;
    const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_fill_u32, dim3(unsigned(blocks)), dim3(256), 0, st, p, value, n);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long *p, unsigned long long value, uint64_t n,
                           hipStream_t st)
{
    if (n == 0)
        return hipSuccess;
    const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 65536);
    hipLaunchKernelGGL(k_fill_u64, dim3(unsigned(blocks)), dim3(256), 0, st, p, value, n);
    return hipGetLastError();
}

hipError_t launch_popcount(const EnumJob &j, hipStream_t st)
{
    const uint64_t n = j.hi - j.lo;
    const dim3 grid(unsigned((n + 255) / 256));
    switch (j.W) {
#define HP_W(w)                                                                                \
    case w:                                                                                    \
        hipLaunchKernelGGL(k_popcount<w>, grid, dim3(256), 0, st, j, j.masks, j.pairs); \
        break;
        HP_W(1) HP_W(2) HP_W(3) HP_W(4) HP_W(5) HP_W(6) HP_W(7) HP_W(8) HP_W(9) HP_W(10)
#undef HP_W
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

GemmShape default_gemm_shape(int KB)
{
    if (KB <= 5)
        return GemmShape{4, 4};
    return GemmShape{2, 4};
}

uint64_t gemm_seqs_per_item(GemmShape shape) { return uint64_t(shape.T) * shape.NW * 32; }

template <int KB>
static hipError_t launch_gemm_kb(const EnumJob &j, GemmShape sh, hipStream_t st)
{
    const uint64_t n = j.hi - j.lo;
    const uint64_t per = gemm_seqs_per_item(sh);
    const dim3 grid(unsigned((n + per - 1) / per));
    if (sh.T == 4 && sh.NW == 4)
        hipLaunchKernelGGL((k_gemm<KB, 4, 4>), grid, dim3(256), 0, st, j);
    else if (sh.T == 2 && sh.NW == 4)
        hipLaunchKernelGGL((k_gemm<KB, 2, 4>), grid, dim3(256), 0, st, j);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_gemm(const EnumJob &j, GemmShape shape, hipStream_t st)
{
    switch (j.KB) {
#define HP_KB(kb)                                  \
    case kb:                                       \
        return launch_gemm_kb<kb>(j, shape, st);
        HP_KB(1) HP_KB(2) HP_KB(3) HP_KB(4) HP_KB(5) HP_KB(6) HP_KB(7) HP_KB(8) HP_KB(9) HP_KB(10)
#undef HP_KB
    default:
        return hipErrorInvalidValue;
    }
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
    const unsigned grid = unsigned(std::max(1, std::min(n_items, cus * 2)));
    if (kb_max <= 5)
        hipLaunchKernelGGL((k_gemm_batch<5, 4, 4>), dim3(grid), dim3(256), 0, st, hdr);
    else
        hipLaunchKernelGGL((k_gemm_batch<10, 2, 4>), dim3(grid), dim3(256), 0, st, hdr);
    return hipGetLastError();
}

}  // namespace hpmap
