// int8-MFMA form of the ground-state search (internal templates; instantiated
// per product depth in gemm_kb*.hip).
//
// Contacts on the bipartite lattice join monomers whose separation j - i is
// odd and >= 3; index these K pairs as k.  For sequence s, P_k(s) = h_i h_j
// and C_k(c) = 1 iff pair k is a contact of conformation c, so the number of
// H-H contacts is n(s,c) = sum_k P_k(s) C_k(c): a K-deep integer matrix
// product (the energy of Eq. 1 with E_HH = -1 is -n).
//
// Operands of v_mfma_i32_32x32x32_i8: A = C^T, 32 conformations x 32 rows per
// block, stored pre-swizzled so that lane l's 16 bytes are one load; B = P for
// 32 sequences, generated in registers once per sequence tile and held for
// the whole sweep over conformations.  For pure HP the entries are -128 on
// both sides, so each H-H contact adds S = 16384.  A general two-letter table
// maximises F = A n + B sum_i h_i c_i: pair rows carry C = -A m, N more
// "unary" rows carry P = -128 h_i and C = -B c_i m, so the product is S F with
// S = 128 m.  The two rows after them carry u = 1 + the conformation's
// position within its key window (P = 1, C = u & 127 and P = -128,
// C = -(u >> 7)), so the accumulator IS the window key S F + u and the
// epilogue needs no index arithmetic: per two values one med3, one max3 and
// half of a max3.  Padding columns hold key 0.
//
// Three staging modes for A:
//   kLds    : the workgroup copies each conformation tile global -> LDS
//             (double-buffered, one barrier per tile) and every wave reads its
//             fragments from LDS;
//   kDirect : every wave loads its fragments straight from global memory
//             (L1/L2-resident, all waves sweep the same tiles) into registers,
//             one tile ahead; no LDS, no barriers;
//   kPipe   : as kLds, but software-pipelined: the MFMAs of tile t+1 are
//             issued before the epilogue of tile t, into a second set of
//             accumulators, so one wave's matrix and vector work overlap.
#pragma once

#include "device_common.h"

namespace hpmap {

enum { kLds = 0, kDirect = 1, kPipe = 2 };

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

template <int KB, int T>
__device__ __forceinline__ void mma_tile(const v4i (&a)[KB], const v4i (&pf)[T][KB], v16i (&acc)[T])
{
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const v16i zero = {};
            acc[t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[kb], pf[t][kb], kb == 0 ? zero : acc[t],
                                                            0, 0, 0);
        }
}

template <int T>
__device__ __forceinline__ void epilogue_tile(const v16i (&acc)[T], int (&b)[T], int (&sc)[T])
{
#pragma unroll
    for (int t = 0; t < T; ++t)
#pragma unroll
        for (int r = 0; r < 16; r += 2)
            top2_add2(b[t], sc[t], acc[t][r], acc[t][r + 1]);
}

template <int T>
__device__ __forceinline__ void fold_window(int (&b)[T], int (&sc)[T], int (&gb)[T], int (&gs)[T],
                                            int conf_base, int win_shift)
{
#pragma unroll
    for (int t = 0; t < T; ++t) {
        top2_merge(gb[t], gs[t], window_to_global(b[t], conf_base, win_shift),
                   window_to_global(sc[t], conf_base, win_shift));
        b[t] = sc[t] = 0;
    }
}

// One workgroup scores NW*T*32 consecutive sequences starting at seq0_wg
// against every conformation tile.  lds holds 2*KB*64 vectors (kLds only).
template <int KB, int T, int NW, int MODE>
__device__ __forceinline__ void gemm_body(const EnumJob &j, uint64_t seq0_wg, v4i *lds)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 31;
    const int half = lane >> 5;
    const uint64_t seq0 = seq0_wg + uint64_t(wave) * (T * 32);
    const v4i *__restrict__ A = reinterpret_cast<const v4i *>(j.gemm_a);

    v4i pf[T][KB];
    {
        uint64_t seqs[T], revs[T];
#pragma unroll
        for (int t = 0; t < T; ++t)
            seqs[t] = sequence_at(j, seq0 + t * 32 + col, &revs[t]);
        p_fragments<KB, T>(seqs, half, j.N, j.K, j.U, pf);
    }

    int b[T], sc[T], gb[T], gs[T];
#pragma unroll
    for (int t = 0; t < T; ++t)
        b[t] = sc[t] = gb[t] = gs[t] = 0;

    const int n_tiles = j.n_tiles;
    const int win_tiles = j.win_tiles;
    const int win_shift = j.win_shift;
    int wend = min(win_tiles, n_tiles);
    int conf_base = 0;

    if constexpr (MODE == kLds) {
        TileStage<KB, NW> stg;
        stg.load(A, 0);
        stg.store(lds);
        __syncthreads();
        for (int tile = 0; tile < n_tiles; ++tile) {
            const bool more = tile + 1 < n_tiles;
            if (more)
                stg.load(A, tile + 1);
            const v4i *cur = lds + (tile & 1) * (KB * 64);
            v4i a[KB];
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
                a[kb] = cur[kb * 64 + lane];
            v16i acc[T];
            mma_tile<KB, T>(a, pf, acc);
            epilogue_tile<T>(acc, b, sc);
            if (tile + 1 == wend) {
                fold_window<T>(b, sc, gb, gs, conf_base, win_shift);
                conf_base += win_tiles * kTileConf;
                wend = min(wend + win_tiles, n_tiles);
            }
            if (more)
                stg.store(lds + ((tile + 1) & 1) * (KB * 64));
            __syncthreads();
        }
    } else if constexpr (MODE == kPipe) {
        // Double-buffered LDS; half-step t: prefetch tile t+2 from global,
        // MFMAs of tile t+1 (buffer (t+1)&1), epilogue of tile t, store tile
        // t+2 into buffer t&1 (last read by the MFMAs of tile t, before the
        // previous barrier), barrier.  Unrolled by two so the accumulator
        // sets alternate without copies.
        constexpr int TV = KB * 64;
        TileStage<KB, NW> stg;
        stg.load(A, 0);
        stg.store(lds);
        if (n_tiles > 1) {
            stg.load(A, 1);
            stg.store(lds + TV);
        }
        __syncthreads();
        v16i acc0[T], acc1[T];
        {
            v4i a[KB];
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
                a[kb] = lds[kb * 64 + lane];
            mma_tile<KB, T>(a, pf, acc0);
        }
        // Every wave has read tile 0 before any wave overwrites buffer 0
        // with tile 2 in the first half-step.
        __syncthreads();
        for (int tile = 0; tile < n_tiles; tile += 2) {
            const bool has1 = tile + 1 < n_tiles;
            const bool has2 = tile + 2 < n_tiles;
            const bool has3 = tile + 3 < n_tiles;
            const v4i *buf0 = lds + (tile & 1) * TV;         // holds tile (then tile+2)
            const v4i *buf1 = lds + ((tile + 1) & 1) * TV;   // holds tile+1 (then tile+3)
            if (has2)
                stg.load(A, tile + 2);
            if (has1) {
                v4i a[KB];
#pragma unroll
                for (int kb = 0; kb < KB; ++kb)
                    a[kb] = buf1[kb * 64 + lane];
                mma_tile<KB, T>(a, pf, acc1);
            }
            epilogue_tile<T>(acc0, b, sc);
            if (tile + 1 == wend) {
                fold_window<T>(b, sc, gb, gs, conf_base, win_shift);
                conf_base += win_tiles * kTileConf;
                wend = min(wend + win_tiles, n_tiles);
            }
            if (has2)
                stg.store(lds + (tile & 1) * TV);
            __syncthreads();
            if (!has1)
                break;
            if (has3)
                stg.load(A, tile + 3);
            if (has2) {
                v4i a[KB];
#pragma unroll
                for (int kb = 0; kb < KB; ++kb)
                    a[kb] = buf0[kb * 64 + lane];
                mma_tile<KB, T>(a, pf, acc0);
            }
            epilogue_tile<T>(acc1, b, sc);
            if (tile + 2 == wend) {
                fold_window<T>(b, sc, gb, gs, conf_base, win_shift);
                conf_base += win_tiles * kTileConf;
                wend = min(wend + win_tiles, n_tiles);
            }
            if (has3)
                stg.store(lds + ((tile + 1) & 1) * TV);
            __syncthreads();
        }
    } else {
        v4i a[KB], an[KB];
        const v4i *src = A + lane;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
            a[kb] = src[kb * 64];
        for (int tile = 0; tile < n_tiles; ++tile) {
            const int nt = min(tile + 1, n_tiles - 1);   // re-reads the last tile: in bounds
            const v4i *nsrc = A + size_t(nt) * (KB * 64) + lane;
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
                an[kb] = nsrc[kb * 64];
            v16i acc[T];
            mma_tile<KB, T>(a, pf, acc);
            epilogue_tile<T>(acc, b, sc);
            if (tile + 1 == wend) {
                fold_window<T>(b, sc, gb, gs, conf_base, win_shift);
                conf_base += win_tiles * kTileConf;
                wend = min(wend + win_tiles, n_tiles);
            }
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
                a[kb] = an[kb];
        }
    }

#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int ob = __shfl_xor(gb[t], 32);
        const int os = __shfl_xor(gs[t], 32);
        top2_merge(gb[t], gs[t], ob, os);
        const uint64_t idx = seq0 + t * 32 + col;
        uint64_t rs;
        const uint64_t sq = sequence_at(j, idx, &rs);
        finish_sequence(j, idx, sq, rs, half == 0 && idx < j.hi, gb[t], gs[t], lane == 0, 1);
    }
}

template <int KB, int T, int NW, int MODE>
__global__ __launch_bounds__(NW * 64) void k_gemm(EnumJob j)
{
    __shared__ v4i lds[MODE == kDirect ? 1 : 2 * KB * 64];
    const uint64_t seq0 = j.lo + uint64_t(blockIdx.x) * (NW * T * 32);
    gemm_body<KB, T, NW, MODE>(j, seq0, lds);
}

template <int KB, int T, int NW, int MODE>
hipError_t launch_gemm_variant(const EnumJob &j, hipStream_t st)
{
    const uint64_t n = j.hi - j.lo;
    const uint64_t per = uint64_t(T) * NW * 32;
    const dim3 grid(unsigned((n + per - 1) / per));
    hipLaunchKernelGGL((k_gemm<KB, T, NW, MODE>), grid, dim3(NW * 64), 0, st, j);
    return hipGetLastError();
}

#define HP_GEMM_VARIANT(KB, T, NW, MODE) \
    GemmVariant{KB, T, NW, MODE, &launch_gemm_variant<KB, T, NW, MODE>}

}  // namespace hpmap
