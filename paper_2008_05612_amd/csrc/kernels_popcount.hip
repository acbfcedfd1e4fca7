// Popcount form of the ground-state search (the plain form) and small fill
// kernels of libhpmap for gfx950.
//
// Contacts on the bipartite lattice join monomers whose separation j - i is
// odd and >= 3; index these K pairs as k.  For sequence s, P_k(s) = h_i h_j is
// a K-bit mask built once per sequence, and each conformation's contacts are
// a K-bit mask C, so n(s,c) = popcount(P & C) H-H contacts and E = -n (Eq. 1
// with E_HH = -1).  A general two-letter table adds B sum_i h_i c_i, taken
// from bit planes of the per-monomer contact counts c_i.  One sequence per
// lane; the conformation loop is wave-uniform, so the masks arrive through
// scalar loads and the pure-HP cost per pair is W ANDs + W bit counts + the
// key update.
#include "device_common.h"

namespace hpmap {

// ---------------------------------------------------------------------------
// Popcount form: one sequence per lane, contact masks read as wave-uniform
// (scalar) loads, running keys in VGPRs.
// ---------------------------------------------------------------------------

// Unary part of F for one conformation: sum_i h_i c_i from the bit planes
// of the contact counts c_i (plane b holds bit b of every c_i).
__device__ __forceinline__ int unary_sum(const uint32_t *m, int planes, int uw, uint32_t s_lo,
                                         uint32_t s_hi)
{
    int u = 0;
    for (int b = 0; b < planes; ++b) {
        int cnt = __popc(s_lo & m[b * uw]);
        if (uw > 1)
            cnt += __popc(s_hi & m[b * uw + 1]);
        u += cnt << b;
    }
    return u;
}

// UN = false: pure pair energies (B = 0); the key carries n and F = A n is
// formed only for the energy output.  UN = true: F = A n + B u per pair.
template <int W, bool UN>
__global__ __launch_bounds__(256) void k_popcount(EnumJob j, const uint32_t *__restrict__ masks,
                                                  const uint8_t *__restrict__ pairs)
{
    const uchar4 *rows = reinterpret_cast<const uchar4 *>(pairs);
    const uint64_t idx = j.lo + uint64_t(blockIdx.x) * 256 + threadIdx.x;
    const bool valid = idx < j.hi;
    uint64_t rs;
    const uint64_t s = sequence_at(j, idx, &rs);
    uint32_t P[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        uint32_t v = 0;
        for (int b = 0; b < 32; ++b) {
            const int k = w * 32 + b;
            if (k < j.K) {
                const uchar4 row = rows[k];
                v |= uint32_t((s >> row.x) & (s >> row.y) & 1u) << b;
            }
        }
        P[w] = v;
    }
    const uint32_t s_lo = uint32_t(s), s_hi = uint32_t(s >> 32);
    const int MW = UN ? j.MW : W;
    int best = 0, second = 0;
    const int n_conf = j.n_conf;
    int c = 0;
    for (; c + 2 <= n_conf; c += 2) {
        const uint32_t *m = masks + size_t(c) * MW;
        int n0 = 0, n1 = 0;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            n0 += __popc(P[w] & m[w]);
            n1 += __popc(P[w] & m[MW + w]);
        }
        if (UN) {
            n0 = j.A * n0 + j.B * unary_sum(m + W, j.planes, j.uw, s_lo, s_hi);
            n1 = j.A * n1 + j.B * unary_sum(m + MW + W, j.planes, j.uw, s_lo, s_hi);
        }
        top2_add2(best, second, (n0 << kKeyConfBits) | (c + 1), (n1 << kKeyConfBits) | (c + 2));
    }
    if (c < n_conf) {
        const uint32_t *m = masks + size_t(c) * MW;
        int n0 = 0;
#pragma unroll
        for (int w = 0; w < W; ++w)
            n0 += __popc(P[w] & m[w]);
        if (UN)
            n0 = j.A * n0 + j.B * unary_sum(m + W, j.planes, j.uw, s_lo, s_hi);
        top2_add1(best, second, (n0 << kKeyConfBits) | (c + 1));
    }
    finish_sequence(j, idx, s, rs, valid, best, second, (threadIdx.x & 63) == 0, UN ? 1 : j.A);
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
#define HP_W(w)                                                                           \
    case w:                                                                               \
        if (j.U)                                                                          \
            hipLaunchKernelGGL((k_popcount<w, true>), grid, dim3(256), 0, st, j, j.masks,  \
                               j.pairs);                                                  \
        else                                                                              \
            hipLaunchKernelGGL((k_popcount<w, false>), grid, dim3(256), 0, st, j, j.masks, \
                               j.pairs);                                                  \
        break;
        HP_W(1) HP_W(2) HP_W(3) HP_W(4) HP_W(5) HP_W(6) HP_W(7) HP_W(8) HP_W(9) HP_W(10)
#undef HP_W
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace hpmap
