// Block-factorised int8-MFMA form of the ground-state search (pure pair
// energies, plain sequence ranges).
//
// A block is 2^8 consecutive sequences: they share every monomer above the
// low 8 bits.  Splitting each pair (i, j) by whether i and j are low (< 8)
// or high, the quantity maximised, F = A sum_k C_k(c) h_i h_j (the negated
// energy of Eq. 1 up to a constant), becomes
//   F(s, c) = base(c) + sum_{v < 8} h_v w_v(c) + sum_{low pairs} A C_vv'(c) h_v h_v'
// with base(c) = A sum over high-high contacts of h_i h_j and
// w_v(c) = A sum over contacts (v, j), j high, of h_j: numbers that depend on
// the block and the conformation but not on the low bits.  Two products:
//
//   stage one  D1 = V x C1, per 32-conformation tile: V holds 32 block-
//              dependent "virtual rows" (weights -m2 A on high-high pairs for
//              base, -m2 A h_j on the pairs of v for w_v, unit rows picking
//              the 9 low-low pairs and the 2 window index rows) and C1 is the
//              0/1 contact matrix with the index rows.  D1[m][c] is, for each
//              conformation, the int8 byte of quantity m: -m2 base, -m2 w_v,
//              -m2 A C_vv', u & 127 and -(u >> 7).
//   stage two  key = A2 x S2: A2 = D1 packed to bytes (a lane of the stage-one
//              result holds one conformation and 16 of its virtual rows,
//              exactly the 16 bytes it supplies as the A operand of the next
//              product, so no data moves between lanes), S2 = per-sequence
//              indicators -128 (1, h_v, h_v h_v') and (1, -128) for the index
//              bytes.  The accumulator is the window key 128 m2 F + u.
//
// Per 32 x 32 (conformation x sequence) tile this issues one MFMA of depth
// 32 instead of K_pad/32 of them; stage one adds K_pad/32 MFMAs per
// conformation tile per 256 sequences.  The epilogue is the same top-2 key
// update as the dense form, which now bounds the kernel.
#include "gemm_body.h"

namespace hpmap {

namespace {

constexpr int kBlkTiles = (1 << kBlkBits) / 32;   // sequence tiles per block (8)

// Virtual rows: m = 0 base; 1 .. 8 w_v with v = m - 1; 9 .. 17 the low-low
// pairs below; 18 and 19 the index bytes; 20 .. 31 zero.
constexpr int kRowW = 1, kRowVV = 9, kRowIdx = 18;

// Low-low pairs (a, b) of odd separation >= 3 inside the low 8 monomers.
// Pairs 0 .. 4: (p, p + 3); 5 .. 7: (p - 5, p); 8: (0, 7).
__device__ __forceinline__ int vv_a(int p) { return p < 5 ? p : (p < 8 ? p - 5 : 0); }
__device__ __forceinline__ int vv_b(int p) { return p < 5 ? p + 3 : (p < 8 ? p : 7); }

// Row of the stage-one result held in accumulator register r of a lane in
// half `half` of the wave (32 x 32 MFMA result layout).
__device__ __forceinline__ int d1_row(int r, int half) { return 8 * (r >> 2) + 4 * half + (r & 3); }

// Stage-one A operand: this lane's virtual row m = lane & 31 over product
// rows k = 32 kb + 16 half + q of C1.
template <int KB>
__device__ __forceinline__ void blk_v_fragments(const EnumJob &j, uint64_t outer, int m, int half,
                                                v4i (&vf)[KB])
{
    const uchar4 *rows = reinterpret_cast<const uchar4 *>(j.pairs);
    const int coef = j.blk_coef;
    const int va = m >= kRowVV && m < kRowIdx ? vv_a(m - kRowVV) : -1;
    const int vb = m >= kRowVV && m < kRowIdx ? vv_b(m - kRowVV) : -1;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        uint32_t w[4];
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
            uint32_t word = 0;
#pragma unroll
            for (int bb = 0; bb < 4; ++bb) {
                const int k = kb * 32 + half * 16 + q4 * 4 + bb;
                int v = 0;
                if (k == j.K) {
                    v = m == kRowIdx ? 1 : 0;
                } else if (k == j.K + 1) {
                    v = m == kRowIdx + 1 ? -1 : 0;
                } else if (k < j.K) {
                    const uchar4 r = rows[k];
                    const int i = r.x, jj = r.y;
                    const bool hi_i = i >= kBlkBits, hi_j = jj >= kBlkBits;
                    const int hh = int((outer >> i) & (outer >> jj) & 1u);
                    const int hj = int((outer >> jj) & 1u);
                    if (m == 0)
                        v = hi_i && hi_j && hh ? -coef : 0;
                    else if (m < kRowVV)
                        v = i == m - kRowW && hi_j && hj ? -coef : 0;
                    else if (m < kRowIdx)
                        v = i == va && jj == vb ? -coef : 0;
                }
                word |= (uint32_t(v) & 0xffu) << (8 * bb);
            }
            w[q4] = word;
        }
        vf[kb] = v4i{int(w[0]), int(w[1]), int(w[2]), int(w[3])};
    }
}

// Stage-two B operand for sequence tile t of the block: this lane's sequence
// x = 32 t + (lane & 31) (the low 8 bits), byte q of half `half` carrying the
// indicator of virtual row d1_row(q, half).
__device__ __forceinline__ void blk_s_fragments(int col, int half, v4i (&sf)[kBlkTiles])
{
#pragma unroll
    for (int t = 0; t < kBlkTiles; ++t) {
        const int x = 32 * t + col;
        uint32_t w[4];
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
            uint32_t word = 0;
#pragma unroll
            for (int bb = 0; bb < 4; ++bb) {
                const int m = d1_row(q4 * 4 + bb, half);
                uint32_t byte = 0;
                if (m == 0)
                    byte = 0x80u;
                else if (m < kRowVV)
                    byte = ((x >> (m - kRowW)) & 1) ? 0x80u : 0u;
                else if (m < kRowIdx)
                    byte = ((x >> vv_a(m - kRowVV)) & (x >> vv_b(m - kRowVV)) & 1) ? 0x80u : 0u;
                else if (m == kRowIdx)
                    byte = 0x01u;
                else if (m == kRowIdx + 1)
                    byte = 0x80u;
                word |= byte << (8 * bb);
            }
            w[q4] = word;
        }
        sf[t] = v4i{int(w[0]), int(w[1]), int(w[2]), int(w[3])};
    }
}

// Low bytes of four int32 values (each in [-128, 127]) packed little-endian,
// three byte permutes: v_perm_b32(x, y, sel) picks result byte i as byte
// sel_i of the 8-byte value {x (bytes 4..7), y (bytes 0..3)}; 0x0c gives 0.
__device__ __forceinline__ int pack4(int a, int b, int c, int d)
{
    const uint32_t ab = __builtin_amdgcn_perm(uint32_t(b), uint32_t(a), 0x0c0c0400u);
    const uint32_t cd = __builtin_amdgcn_perm(uint32_t(d), uint32_t(c), 0x0c0c0400u);
    return int(__builtin_amdgcn_perm(cd, ab, 0x05040100u));
}

template <int KB>
__device__ __forceinline__ v16i stage_one(const v4i (&vf)[KB], const v4i *tile, int lane)
{
    v16i d1;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        const v16i zero = {};
        d1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(vf[kb], tile[kb * 64 + lane],
                                                   kb == 0 ? zero : d1, 0, 0, 0);
    }
    return d1;
}

__device__ __forceinline__ v4i pack_d1(const v16i &d1)
{
    return v4i{pack4(d1[0], d1[1], d1[2], d1[3]), pack4(d1[4], d1[5], d1[6], d1[7]),
               pack4(d1[8], d1[9], d1[10], d1[11]), pack4(d1[12], d1[13], d1[14], d1[15])};
}

// Stage two of one conformation tile for the wave's 8 sequence tiles, with
// the top-2 key update of each result.  The product of sequence tile t+1 is
// issued before the key updates of tile t (two accumulators), so the wave
// does not wait on each product's latency.
__device__ __forceinline__ void stage_two(const v4i &a2, const v4i (&sf)[kBlkTiles],
                                          int (&b)[kBlkTiles], int (&sc)[kBlkTiles])
{
    const v16i zero = {};
    v16i acc[2];
    acc[0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a2, sf[0], zero, 0, 0, 0);
#pragma unroll
    for (int t = 0; t < kBlkTiles; ++t) {
        if (t + 1 < kBlkTiles)
            acc[(t + 1) & 1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a2, sf[t + 1], zero, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 16; r += 2)
            top2_add2(b[t], sc[t], acc[t & 1][r], acc[t & 1][r + 1]);
    }
}

// Staging of the C1 tiles:
//   kBlkLds  : double-buffered LDS, one barrier per tile; stage one of a tile
//              runs right before its stage two.
//   kBlkPipe : triple-buffered LDS; the stage-one products of tile t+1 are
//              issued during iteration t, so the matrix pipe works on them
//              while the vector ALU runs tile t's key updates.
enum { kBlkLds = 0, kBlkPipe = 1 };

// One wave scores one block of 256 sequences against every conformation
// tile; the NW waves of a workgroup take consecutive blocks and share the
// C1 tiles through LDS.
template <int KB, int NW, int MODE>
__global__ __launch_bounds__(NW * 64) void k_gemm_blk(EnumJob j)
{
    __shared__ v4i lds[(MODE == kBlkPipe ? 3 : 2) * KB * 64];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 31;
    const int half = lane >> 5;
    const uint64_t blk = (j.lo >> kBlkBits) + uint64_t(blockIdx.x) * NW + wave;
    const uint64_t outer = blk << kBlkBits;
    const v4i *__restrict__ B1 = reinterpret_cast<const v4i *>(j.gemm_b);

    v4i vf[KB];
    blk_v_fragments<KB>(j, outer, col, half, vf);
    v4i sf[kBlkTiles];
    blk_s_fragments(col, half, sf);

    int b[kBlkTiles], sc[kBlkTiles], gb[kBlkTiles], gs[kBlkTiles];
#pragma unroll
    for (int t = 0; t < kBlkTiles; ++t)
        b[t] = sc[t] = gb[t] = gs[t] = 0;

    const int n_tiles = j.n_tiles;
    const int win_tiles = j.blk_win_tiles;
    const int win_shift = j.blk_shift;
    int wend = min(win_tiles, n_tiles);
    int conf_base = 0;

    TileStage<KB, NW> stg;
    constexpr int TV = KB * 64;   // vectors per staged tile
    if constexpr (MODE == kBlkLds) {
        stg.load(B1, 0);
        stg.store(lds);
        __syncthreads();
        for (int tile = 0; tile < n_tiles; ++tile) {
            const bool more = tile + 1 < n_tiles;
            if (more)
                stg.load(B1, tile + 1);
            const v16i d1 = stage_one<KB>(vf, lds + (tile & 1) * TV, lane);
            stage_two(pack_d1(d1), sf, b, sc);
            if (tile + 1 == wend) {
                fold_window<kBlkTiles>(b, sc, gb, gs, conf_base, win_shift);
                conf_base += win_tiles * kTileConf;
                wend = min(wend + win_tiles, n_tiles);
            }
            if (more)
                stg.store(lds + ((tile + 1) & 1) * TV);
            __syncthreads();
        }
    } else {
        // Buffer t % 3 holds tile t.  Iteration t: prefetch tile t+2 from
        // global memory, pack tile t's stage-one result, issue stage one of
        // tile t+1 (buffer (t+1) % 3) and stage two of tile t, store tile t+2
        // into buffer (t+2) % 3 = (t-1) % 3 -- last read by stage one of tile
        // t-1 in iteration t-2, two barriers back -- then one barrier.
        stg.load(B1, 0);
        stg.store(lds);
        if (n_tiles > 1) {
            stg.load(B1, 1);
            stg.store(lds + TV);
        }
        __syncthreads();
        v16i d1 = stage_one<KB>(vf, lds, lane);
        int cur = 0;   // buffer of tile `tile`
        for (int tile = 0; tile < n_tiles; ++tile) {
            const bool has1 = tile + 1 < n_tiles;
            const bool has2 = tile + 2 < n_tiles;
            if (has2)
                stg.load(B1, tile + 2);
            const v4i a2 = pack_d1(d1);
            const int nxt = cur == 2 ? 0 : cur + 1;
            const int nn = nxt == 2 ? 0 : nxt + 1;
            if (has1)
                d1 = stage_one<KB>(vf, lds + nxt * TV, lane);
            stage_two(a2, sf, b, sc);
            if (tile + 1 == wend) {
                fold_window<kBlkTiles>(b, sc, gb, gs, conf_base, win_shift);
                conf_base += win_tiles * kTileConf;
                wend = min(wend + win_tiles, n_tiles);
            }
            if (has2)
                stg.store(lds + nn * TV);
            __syncthreads();
            cur = nxt;
        }
    }

#pragma unroll
    for (int t = 0; t < kBlkTiles; ++t) {
        const int ob = __shfl_xor(gb[t], 32);
        const int os = __shfl_xor(gs[t], 32);
        top2_merge(gb[t], gs[t], ob, os);
        const uint64_t idx = outer + uint64_t(t * 32 + col);
        finish_sequence(j, idx, idx, idx, half == 0 && idx >= j.lo && idx < j.hi, gb[t], gs[t],
                        lane == 0, 1);
    }
}

template <int KB, int NW, int MODE>
hipError_t launch_blk_shape(const EnumJob &j, hipStream_t st)
{
    const uint64_t first = j.lo >> kBlkBits, last = (j.hi - 1) >> kBlkBits;
    const uint64_t n_blocks = last - first + 1;
    const dim3 grid(unsigned((n_blocks + NW - 1) / NW));
    hipLaunchKernelGGL((k_gemm_blk<KB, NW, MODE>), grid, dim3(NW * 64), 0, st, j);
    return hipGetLastError();
}

template <int KB>
hipError_t launch_blk(const EnumJob &j, int nw, int mode, hipStream_t st)
{
    if (mode == kBlkPipe) {
        switch (nw) {
        case 2: return launch_blk_shape<KB, 2, kBlkPipe>(j, st);
        case 8: return launch_blk_shape<KB, 8, kBlkPipe>(j, st);
        default: return launch_blk_shape<KB, 4, kBlkPipe>(j, st);
        }
    }
    switch (nw) {
    case 2: return launch_blk_shape<KB, 2, kBlkLds>(j, st);
    case 8: return launch_blk_shape<KB, 8, kBlkLds>(j, st);
    default: return launch_blk_shape<KB, 4, kBlkLds>(j, st);
    }
}

}  // namespace

hipError_t launch_gemm_blocked(const EnumJob &j, int nw, int mode, hipStream_t st)
{
    switch (j.KB) {
    case 1: return launch_blk<1>(j, nw, mode, st);
    case 2: return launch_blk<2>(j, nw, mode, st);
    case 3: return launch_blk<3>(j, nw, mode, st);
    case 4: return launch_blk<4>(j, nw, mode, st);
    case 5: return launch_blk<5>(j, nw, mode, st);
    case 6: return launch_blk<6>(j, nw, mode, st);
    case 7: return launch_blk<7>(j, nw, mode, st);
    case 8: return launch_blk<8>(j, nw, mode, st);
    case 9: return launch_blk<9>(j, nw, mode, st);
    case 10: return launch_blk<10>(j, nw, mode, st);
    case 11: return launch_blk<11>(j, nw, mode, st);
    case 12: return launch_blk<12>(j, nw, mode, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hpmap
