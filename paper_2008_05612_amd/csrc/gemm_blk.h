// Block-factorised int8-MFMA form of the ground-state search (internal
// templates; instantiated per product depth in gemm_blk_kb*.hip).
//
// A block is 256 sequences that differ only in 8 "varying" monomers: the low
// 8 for plain ranges (256 consecutive sequences), the middle 8 for the
// reversal-canonical blocks (reversal then maps blocks onto blocks).
// Splitting each pair (i, j) by whether i and j vary, the quantity
// maximised, F = A sum_k C_k(c) h_i h_j (the negated energy of Eq. 1 up to a
// constant), becomes
//   F(s, c) = base(c) + sum_{v varying} h_v w_v(c) + sum_{varying pairs} A C_vv'(c) h_v h_v'
// with base(c) = A sum over contacts of two outer monomers of h_i h_j and
// w_v(c) = A sum over contacts of v with an outer monomer j of h_j: numbers
// that depend on the block and the conformation but not on the varying
// monomers.  Two products:
//
//   stage one  D1 = V x C1, per 32-conformation tile: V holds 32 block-
//              dependent "virtual rows" (weights -m2 A on outer-outer pairs
//              for base, -m2 A h_j on the pairs of v for w_v, unit rows
//              picking the varying pairs and the 2 window index rows) and C1
//              is the 0/1 contact matrix with the index rows.  D1[m][c] is,
//              for each conformation, the int8 byte of quantity m: -m2 base,
//              -m2 w_v, -m2 A C_vv', u & 127 and -(u >> 7).
//   stage two  key = A2 x S2: A2 = D1 packed to bytes (a lane of the stage-one
//              result holds one conformation and 16 of its virtual rows,
//              exactly the 16 bytes it supplies as the A operand of the next
//              product, so no data moves between lanes), S2 = per-sequence
//              indicators -128 (1, h_v, h_v h_v') and (1, -128) for the index
//              bytes, precomputed on the host per block geometry.  The
//              accumulator is the window key 128 m2 F + u.
//
// Per 32 x 32 (conformation x sequence) tile this issues one MFMA of depth
// 32 instead of K_pad/32 of them; stage one adds K_pad/32 MFMAs per
// conformation tile per 256 sequences.  The epilogue is the same top-2 key
// update as the dense form, which now bounds the kernel.
#pragma once

#include "gemm_body.h"

namespace hpmap {

namespace {

constexpr int kBlkTiles = (1 << kBlkBits) / 32;   // sequence tiles per block (8)

// The 8 varying monomers of a block sit at positions pos(x) (x = 0 .. 7,
// packed 8 bits each in j.blk_pos); j.blk_vmask has their bits.  Virtual
// rows: m = 0 base; 1 .. 8 w_v for v = pos(m - 1); then one row per pair of
// varying monomers with odd separation >= 3 (j.blk_npp pairs, x-indices a | b << 4
// packed a byte each in j.blk_pp[]); then j.blk_ngroups rows of unary terms
// (two-letter tables: B c_i h_i summed over a group of outer monomers); then
// the two index bytes; zero beyond.
// Plain ranges (CANON false) use the low 8 monomers, a geometry known at
// compile time: pos(x) = x and the pairs kLow8Pairs, the same list the host
// lays the second product's operand out by.
constexpr int kRowW = 1, kRowVV = 9;

template <bool CANON>
__device__ __forceinline__ int blk_pos(const EnumJob &j, int x)
{
    return CANON ? int((j.blk_pos >> (8 * x)) & 0xffu) : x;
}

template <bool CANON>
__device__ __forceinline__ int blk_pair(const EnumJob &j, int p)
{
    if (!CANON)
        return p < 8 ? int((kLow8Pairs >> (8 * p)) & 0xffu) : kLow8Pair8;
    const uint64_t w = p < 8 ? j.blk_pp[0] : (p < 16 ? j.blk_pp[1] : j.blk_pp[2]);
    return int((w >> (8 * (p & 7))) & 0xffu);
}

template <bool CANON>
__device__ __forceinline__ int blk_npp(const EnumJob &j) { return CANON ? j.blk_npp : kLow8NumPairs; }

template <bool CANON>
__device__ __forceinline__ uint64_t blk_vmask(const EnumJob &j) { return CANON ? j.blk_vmask : 0xffull; }

// Unary group of monomer i (15: none).  Selects, not an indexed read: a
// runtime index into the job's array would place the job in scratch memory.
__device__ __forceinline__ int blk_group(const EnumJob &j, int i)
{
    const uint64_t w = i < 16 ? j.blk_grp[0] : (i < 32 ? j.blk_grp[1] : j.blk_grp[2]);
    return int((w >> (4 * (i & 15))) & 15u);
}

// Stage-one A operand: this lane's virtual row m = lane & 31 over product
// rows k = 32 kb + 16 half + q of C1, for the block whose outer monomers are
// the bits of `outer`.
// UNARY: the job has unary-group rows (two-letter tables); compiled apart so
// that the pure-pair instances keep this fully unrolled loop small enough to
// stay in registers at every depth.
template <int KB, bool CANON, bool UNARY>
__device__ __forceinline__ void blk_v_fragments(const EnumJob &j, uint64_t outer, int m, int half,
                                                v4i (&vf)[KB])
{
    const int N = j.N;
    const int coef = j.blk_coef;
    const int coefB = UNARY ? j.blk_coefB : 0;
    const uint64_t vmask = blk_vmask<CANON>(j);
    const int row_un = kRowVV + blk_npp<CANON>(j);
    const int row_idx = row_un + (UNARY ? j.blk_ngroups : 0);
    // unary-group rows (two-letter tables): the outer H monomers of this
    // lane's group, as a bit mask over monomer positions
    uint64_t gmask = 0;
    if (UNARY && m >= row_un && m < row_idx)
        for (int i = 0; i < N; ++i)
            if (blk_group(j, i) == m - row_un && ((outer >> i) & 1u) && !((vmask >> i) & 1u))
                gmask |= uint64_t(1) << i;
    const int wv = m >= kRowW && m < kRowVV ? blk_pos<CANON>(j, m - kRowW) : -1;
    int va = -1, vb = -1;
    if (m >= kRowVV && m < row_un) {
        const int pr = blk_pair<CANON>(j, m - kRowVV);
        va = blk_pos<CANON>(j, pr & 15);
        vb = blk_pos<CANON>(j, pr >> 4);
    }
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        // product row k < K is the pair (i, i + d) of the k-th odd separation
        // d >= 3 in (d, i) order: find the first row's pair by skipping whole
        // runs of length N - d, then advance row by row
        const int kbase = kb * 32 + half * 16;
        int d = 3, i = kbase;
        while (d < N && i >= N - d) {
            i -= N - d;
            d += 2;
        }
        uint32_t w[4];
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
            uint32_t word = 0;
#pragma unroll
            for (int bb = 0; bb < 4; ++bb) {
                const int k = kbase + q4 * 4 + bb;
                int v = 0;
                if (k == j.K) {
                    v = m == row_idx ? 1 : 0;
                } else if (k == j.K + 1) {
                    v = m == row_idx + 1 ? -1 : 0;
                } else if (d < N) {
                    const int jj = i + d;
                    const bool out_i = !((vmask >> i) & 1u), out_j = !((vmask >> jj) & 1u);
                    const bool h_i = (outer >> i) & 1u, h_j = (outer >> jj) & 1u;
                    if (m == 0) {
                        v = out_i && out_j && h_i && h_j ? -coef : 0;
                    } else if (m < kRowVV) {
                        v = (i == wv && out_j && h_j) || (jj == wv && out_i && h_i) ? -coef : 0;
                        v -= i == wv || jj == wv ? coefB : 0;   // B c_v: every contact of v
                    } else if (m < row_un) {
                        v = i == va && jj == vb ? -coef : 0;
                    } else if (UNARY && m < row_idx) {
                        v = -coefB * int(((gmask >> i) & 1u) + ((gmask >> jj) & 1u));
                    }
                }
                word |= (uint32_t(v) & 0xffu) << (8 * bb);
                ++i;   // next row: next i, or the next run
                if (d < N && i + d >= N) {
                    i = 0;
                    d += 2;
                }
            }
            w[q4] = word;
        }
        vf[kb] = v4i{int(w[0]), int(w[1]), int(w[2]), int(w[3])};
    }
}

// Sequence of block sequence x: the outer bits plus x's bits deposited at the
// varying positions.
__device__ __forceinline__ uint64_t blk_sequence(const EnumJob &j, uint64_t outer, int x)
{
    uint64_t s = outer;
#pragma unroll
    for (int b = 0; b < 8; ++b)
        s |= uint64_t((x >> b) & 1) << blk_pos<true>(j, b);
    return s;
}

// Canonical block index t -> outer bits.  With h = j.half_bits outer bits on
// each side (low: b, high: a) and, for odd N, the middle monomer m as an
// outer bit, reversal maps the block (a, m, b) onto (rev b, m, rev a); the
// canonical blocks are a <= b' = rev(b).  The index runs over m, then row
// pairs p < 2^(h-1) of the (a, b') triangle, each holding row b' = p
// (a = 0 .. p) and row b' = 2^h - 1 - p (a = 0 .. 2^h - 1 - p).  *diag is
// set when a == b', i.e. the block is its own reverse.
// (Block counts stay below 2^28 for N <= 36, so 32-bit arithmetic suffices.)
__device__ __forceinline__ uint64_t blk_canonical_outer(const EnumJob &j, uint64_t t64, bool *diag)
{
    const int h = j.half_bits;
    const int odd = j.N & 1;
    const uint32_t t = uint32_t(t64);
    const uint32_t side = 1u << h;
    const uint32_t span = side + 1;
    const uint32_t per_m = h ? (side >> 1) * span : 1;
    const uint32_t m = t / per_m;
    const uint32_t r = t - m * per_m;
    const uint32_t p = h ? r / span : 0;
    const uint32_t o = r - p * span;
    const bool first = o <= p;
    const uint32_t bp = first ? p : side - 1 - p;
    const uint32_t a = first ? o : o - p - 1;
    *diag = a == bp;
    const uint32_t b = h ? (__builtin_bitreverse32(bp) >> (32 - h)) : 0;
    return (uint64_t(a) << (h + 8 + odd)) | (uint64_t(m) << (h + 4)) | b;
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

// Largest of a lane's 16 keys of one product (a v_max3 chain).
__device__ __forceinline__ int max16(const v16i &a)
{
    int m = max(max(a[0], a[1]), a[2]);
#pragma unroll
    for (int r = 3; r < 15; r += 2)
        m = max(max(m, a[r]), a[r + 1]);
    return max(m, a[15]);
}

// Smallest window key S F + u whose F exceeds the F of the global key gs,
// i.e. (F(gs) + 1) S; 0 while gs is "no conformation", so that every real key
// is absorbed until a lane holds two.
__device__ __forceinline__ int absorb_threshold(int gs, int win_shift)
{
    return int((unsigned(gs) + kMaxConf) >> kKeyConfBits) << win_shift;
}

// Stage two of one conformation tile for the wave's 8 sequence tiles.
//
// The running state of a lane (one sequence, half of each tile's 32
// conformations) is the top-2 of global keys (gb, gs) and thr, the window
// key threshold of absorb_threshold(gs).  A product whose 16 keys in every
// lane all have F <= F(gs) is skipped: such a conformation can neither beat
// the lowest energy nor tie it unless the second already does, nor raise the
// second-lowest energy, so the lowest energy, its conformation when unique,
// the uniqueness decision and the gap come out exactly as if every key had
// been absorbed.  Which conformation the second key names may differ; it is
// never reported.  Absorbing is rare once a lane has seen a few windows, so
// the vector ALU spends 9 instructions per product on the test (max3 chain
// and compare) instead of 20 on the key update.  The product of sequence
// tile t+1 is issued before tile t's test (two accumulators), so the wave
// does not wait on each product's latency.
template <bool S2_LDS>
__device__ __forceinline__ void stage_two(const v4i &a2, const v4i (&sf)[S2_LDS ? 1 : kBlkTiles],
                                          const v4i *s2, int lane, int (&gb)[kBlkTiles],
                                          int (&gs)[kBlkTiles], int (&thr)[kBlkTiles],
                                          int conf_base, int win_shift)
{
    const v16i zero = {};
    v16i acc[2];
    acc[0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a2, S2_LDS ? s2[lane] : sf[0], zero, 0, 0, 0);
#pragma unroll
    for (int t = 0; t < kBlkTiles; ++t) {
        if (t + 1 < kBlkTiles)
            acc[(t + 1) & 1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(
                a2, S2_LDS ? s2[(t + 1) * 64 + lane] : sf[S2_LDS ? 0 : t + 1], zero, 0, 0, 0);
        const v16i &a = acc[t & 1];
        if (__builtin_expect(__any(max16(a) >= thr[t]), 0)) {
            // top-2 of the 16 window keys (one window, so their order is the
            // global keys' order), then only those two become global keys
            int b = 0, sc = 0;
#pragma unroll
            for (int r = 0; r < 16; r += 2)
                top2_add2(b, sc, a[r], a[r + 1]);
            top2_merge(gb[t], gs[t], window_to_global(b, conf_base, win_shift),
                       window_to_global(sc, conf_base, win_shift));
            thr[t] = absorb_threshold(gs[t], win_shift);
        }
    }
}

// Stage two of one conformation tile in the wide kernel: as stage_two, with
// two changes that free registers for a third accumulator (four waves per
// SIMD still fit): the running top-2 of each lane lives in LDS (g[t * 64],
// read and written only by the rare key update), and the product of
// sequence tile t + 2 is issued right after tile t's test, so each test reads
// a product issued a full test earlier.  Issuing that product after the test
// rather than before or inside it measured fastest (full 3x3x3 map, 8 waves:
// 310 ms against 314 ms where the compiler placed it and 318 ms before the
// test): a wave that reaches an MFMA while the matrix pipe still runs another
// wave's product waits there, and after its nine test instructions the pipe
// is more often free.
__device__ __forceinline__ void stage_two_wide(const v4i &a2, const v4i (&sf)[kBlkTiles], int2 *g,
                                               int (&thr)[kBlkTiles], int conf_base,
                                               int win_shift)
{
    const v16i zero = {};
    v16i acc[3];
    acc[0] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a2, sf[0], zero, 0, 0, 0);
    acc[1] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a2, sf[1], zero, 0, 0, 0);
#pragma unroll
    for (int t = 0; t < kBlkTiles; ++t) {
        if (t + 2 < kBlkTiles)
            acc[(t + 2) % 3] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a2, sf[t + 2], zero, 0, 0, 0);
        const v16i &a = acc[t % 3];
        const bool hit = __any(max16(a) >= thr[t]);
        if (t + 2 < kBlkTiles) {
            // the test's 9 vector instructions (8 v_max3, 1 compare), then the MFMA
            __builtin_amdgcn_sched_group_barrier(0x002, 9, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        }
        if (__builtin_expect(hit, 0)) {
            int b = 0, sc = 0;
#pragma unroll
            for (int r = 0; r < 16; r += 2)
                top2_add2(b, sc, a[r], a[r + 1]);
            int2 v = g[t * 64];
            top2_merge(v.x, v.y, window_to_global(b, conf_base, win_shift),
                       window_to_global(sc, conf_base, win_shift));
            g[t * 64] = v;
            thr[t] = absorb_threshold(v.y, win_shift);
        }
    }
}

// Staging of the C1 tiles:
//   kBlkLds  : double-buffered LDS, one barrier per tile; stage one of a tile
//              runs right before its stage two.
//   kBlkPipe : triple-buffered LDS; the stage-one products of tile t+1 are
//              issued during iteration t, so the matrix pipe works on them
//              while the vector ALU runs tile t's key updates.
//   kBlkLdsS2: as kBlkLds, with the per-sequence operand of stage two held in
//              LDS (shared by the workgroup) instead of registers.
enum { kBlkLds = kBlkStageLds, kBlkPipe = kBlkStagePipe, kBlkLdsS2 = kBlkStageS2Lds };

// One wave scores one block of 256 sequences against every conformation
// tile; the NW waves of a workgroup take consecutive blocks and share the
// C1 tiles through LDS.
// The work of one workgroup: wave w scores block blk0 + w (plain jobs: the
// 256 sequences sharing the bits above the low 8, block index = sequence >> 8;
// canonical jobs: canonical block index).  lds holds the staged C1 tiles,
// s2lds the stage-two operand (mode kBlkLdsS2).  Starts and ends at a
// workgroup barrier, so consecutive calls may reuse the LDS.
template <int KB, int NW, int MODE, bool CANON, bool UNARY>
__device__ __forceinline__ void blk_body(const EnumJob &j, uint64_t blk0, v4i *lds, v4i *s2lds)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 31;
    const int half = lane >> 5;
    const uint64_t blk = blk0 + wave;
    bool diag = false;
    const uint64_t outer = CANON ? blk_canonical_outer(j, blk, &diag) : blk << kBlkBits;
    const v4i *__restrict__ B1 = reinterpret_cast<const v4i *>(j.gemm_b);

    v4i vf[KB];
    blk_v_fragments<KB, CANON, UNARY>(j, outer, col, half, vf);
    // stage-two B operand: per-sequence indicators, precomputed per geometry
    v4i sf[MODE == kBlkLdsS2 ? 1 : kBlkTiles];
    const v4i *__restrict__ S2 = reinterpret_cast<const v4i *>(j.blk_s2);
    if constexpr (MODE == kBlkLdsS2) {
        for (int i = threadIdx.x; i < kBlkTiles * 64; i += NW * 64)
            s2lds[i] = S2[i];   // made visible by the barrier before the tile loop
    } else {
#pragma unroll
        for (int t = 0; t < kBlkTiles; ++t)
            sf[t] = S2[t * 64 + lane];
    }

    int gb[kBlkTiles], gs[kBlkTiles], thr[kBlkTiles];
#pragma unroll
    for (int t = 0; t < kBlkTiles; ++t)
        gb[t] = gs[t] = thr[t] = 0;

    const int n_tiles = j.n_tiles;
    const int win_tiles = j.blk_win_tiles;
    const int win_shift = j.blk_shift;
    int wend = min(win_tiles, n_tiles);
    int conf_base = 0;

    TileStage<KB, NW> stg;
    constexpr int TV = KB * 64;   // vectors per staged tile
    if constexpr (MODE == kBlkLds || MODE == kBlkLdsS2) {
        stg.load(B1, 0);
        stg.store(lds);
        __syncthreads();
        for (int tile = 0; tile < n_tiles; ++tile) {
            const bool more = tile + 1 < n_tiles;
            if (more)
                stg.load(B1, tile + 1);
            const v16i d1 = stage_one<KB>(vf, lds + (tile & 1) * TV, lane);
            stage_two<MODE == kBlkLdsS2>(pack_d1(d1), sf, s2lds, lane, gb, gs, thr, conf_base,
                                         win_shift);
            if (tile + 1 == wend) {
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
            stage_two<false>(a2, sf, s2lds, lane, gb, gs, thr, conf_base, win_shift);
            if (tile + 1 == wend) {
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
        if constexpr (CANON) {
            // off the diagonal the block's reverse is never scored: write both;
            // a diagonal block holds each sequence and its reverse itself
            const uint64_t sq = blk_sequence(j, outer, t * 32 + col);
            const uint64_t rs = diag ? sq : __builtin_bitreverse64(sq) >> (64 - j.N);
            finish_sequence(j, sq, sq, rs, half == 0 && blk < j.hi, gb[t], gs[t], lane == 0, 1);
        } else {
            const uint64_t idx = outer + uint64_t(t * 32 + col);
            finish_sequence(j, idx, idx, idx, half == 0 && idx >= j.lo && idx < j.hi, gb[t],
                            gs[t], lane == 0, 1);
        }
    }
}

template <int KB, int NW, int MODE, bool CANON, bool UNARY>
__global__ __launch_bounds__(NW * 64) void k_gemm_blk(EnumJob j)
{
    __shared__ v4i lds[(MODE == kBlkPipe ? 3 : 2) * KB * 64];
    __shared__ v4i s2lds[MODE == kBlkLdsS2 ? kBlkTiles * 64 : 1];
    const uint64_t blk0 = (CANON ? j.lo : j.lo >> kBlkBits) + uint64_t(blockIdx.x) * NW;
    blk_body<KB, NW, MODE, CANON, UNARY>(j, blk0, lds, s2lds);
}

// Batched form for jobs of one product depth: workgroup b scores item
// item_lo + b, NW consecutive blocks of the job whose item range holds it.
template <int KB, int NW, int MODE, bool UNARY>
__global__ __launch_bounds__(NW * 64) void k_gemm_blk_batch(BatchHeader *hdr, int item_lo)
{
    __shared__ v4i lds[2 * KB * 64];
    __shared__ v4i s2lds[MODE == kBlkLdsS2 ? kBlkTiles * 64 : 1];
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
        const uint64_t blk0 = (j.lo >> kBlkBits) + uint64_t(it - start[lo]) * NW;
        blk_body<KB, NW, MODE, false, UNARY>(j, blk0, lds, s2lds);
    }
}

// ---------------------------------------------------------------------------
// Wide blocks (pure pair energies): one block of sequences sharing every
// outer monomer per workgroup, wave w scoring the 256 sequences whose
// varying monomers above the low 8 are the bits of w.  The block term, the
// weights w_v of the varying monomers and their 16 pair terms fill all but
// one or three of the 32 virtual rows, so ONE first product per
// conformation tile serves every wave of the workgroup: each wave computes
// it for every NW-th tile (one group of NW tiles ahead) and hands the packed
// result to the others through LDS.  Three geometries (G):
//   0  plain ranges, 1024 sequences (the low 10 monomers), 4 waves;
//   1  reversal-canonical blocks, 1024 sequences (the 10 around the middle),
//      4 waves;
//   2  plain ranges cut at multiples of 2^17, 2048 sequences (monomers 0 .. 4
//      and the even ones 6 .. 16: equal parity never touches, so 11 varying
//      monomers have only 14 pairs), 8 waves, so a first product serves 2048
//      sequences; the default where it applies.
// Per 32 x 32 tile the matrix pipe runs one depth-32 product plus 1/NW of the
// first product's K_pad/32, and the first product is packed once per
// workgroup.
// ---------------------------------------------------------------------------

template <int G>
constexpr int wide_bits() { return G == 2 ? kWide11Bits : kWideBits; }
template <int G>
constexpr int wide_waves() { return G == 2 ? kWide11Waves : 4; }
// virtual rows: 0 block term, 1 .. nb weights, then 16 pairs, then 2 index rows
template <int G>
constexpr int wide_row_vv() { return 1 + wide_bits<G>(); }
template <int G>
constexpr int wide_row_idx() { return wide_row_vv<G>() + 16; }

// Varying monomer x of a wide block: G 0 the low 10; G 1 the 10 around the
// middle, h = j.half_bits outer monomers on each side (and, for odd N, the
// middle monomer h + 5 outer as well); G 2 monomers 0 .. 4, 6, 8, .., 16.
template <int G>
__device__ __forceinline__ int wide_pos(const EnumJob &j, int x)
{
    if constexpr (G == 1)
        return j.half_bits + x + (x >= 5 ? (j.N & 1) : 0);
    else if constexpr (G == 2)
        return x < 5 ? x : 2 * x - 4;
    else
        return x;
}

template <int G>
__device__ __forceinline__ bool wide_varies(const EnumJob &j, int i)
{
    if constexpr (G == 0) {
        return i < kWideBits;
    } else if constexpr (G == 2) {
        return i < 5 || (i >= 6 && i <= 16 && !(i & 1));
    } else {
        const int h = j.half_bits, odd = j.N & 1;
        return i >= h && i < h + kWideBits + odd && !(odd && i == h + 5);
    }
}

// Pair p (0 .. 15) of the block's varying monomers as x-indices a | b << 4.
template <int G>
__device__ __forceinline__ int wide_pair(const EnumJob &j, int p)
{
    const uint64_t w = G == 2                     ? (p < 8 ? kW11Pairs0 : kW11Pairs1)
                       : (G == 1 && (j.N & 1)) ? (p < 8 ? kMid10OddPairs0 : kMid10OddPairs1)
                                                 : (p < 8 ? kLow10Pairs0 : kLow10Pairs1);
    return int((w >> (8 * (p & 7))) & 0xffu);
}

// First-product A operand of a wide block, fragment kb of this lane:
// virtual row m (0 block term, 1 .. nb the weight of varying monomer m - 1,
// then the 16 varying pairs, then the two index rows) over product rows
// k = 32 kb + 16 half + q of C1.
template <int G>
__device__ __forceinline__ v4i wide_v_fragment(const EnumJob &j, uint64_t outer, int m, int half,
                                               int kb)
{
    constexpr int kRowVV = wide_row_vv<G>(), kRowIdx = wide_row_idx<G>();
    const int N = j.N;
    const int coef = j.blk_coef;
    const int wv = m >= 1 && m < kRowVV ? wide_pos<G>(j, m - 1) : -1;
    int va = -1, vb = -1;
    if (m >= kRowVV && m < kRowIdx) {
        const int pr = wide_pair<G>(j, m - kRowVV);
        va = wide_pos<G>(j, pr & 15);
        vb = wide_pos<G>(j, pr >> 4);
    }
    // product row k < K is the pair (i, i + d) of the k-th odd separation
    // d >= 3 in (d, i) order
    const int kbase = kb * 32 + half * 16;
    int d = 3, i = kbase;
    while (d < N && i >= N - d) {
        i -= N - d;
        d += 2;
    }
    uint32_t w[4];
#pragma unroll
    for (int q4 = 0; q4 < 4; ++q4) {
        uint32_t word = 0;
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) {
            const int k = kbase + q4 * 4 + bb;
            int v = 0;
            if (k == j.K) {
                v = m == kRowIdx ? 1 : 0;
            } else if (k == j.K + 1) {
                v = m == kRowIdx + 1 ? -1 : 0;
            } else if (d < N) {
                const int jj = i + d;
                const bool out_i = !wide_varies<G>(j, i), out_j = !wide_varies<G>(j, jj);
                const bool h_i = (outer >> i) & 1u, h_j = (outer >> jj) & 1u;
                if (m == 0)
                    v = out_i && out_j && h_i && h_j ? -coef : 0;
                else if (m < kRowVV)
                    v = (i == wv && out_j && h_j) || (jj == wv && out_i && h_i) ? -coef : 0;
                else if (m < kRowIdx)
                    v = i == va && jj == vb ? -coef : 0;
            }
            word |= (uint32_t(v) & 0xffu) << (8 * bb);
            ++i;   // next row: next i, or the next run
            if (d < N && i + d >= N) {
                i = 0;
                d += 2;
            }
        }
        w[q4] = word;
    }
    return v4i{int(w[0]), int(w[1]), int(w[2]), int(w[3])};
}

// Canonical wide block index t -> outer bits, as blk_canonical_outer with 10
// varying monomers: (a, m, b) = high h, middle (odd N), low h bits; the
// canonical blocks are a <= b' = reverse_h(b), indexed over m, then row pairs
// p < 2^(h-1) holding row b' = p (a = 0 .. p) and row b' = 2^h - 1 - p
// (a = 0 .. 2^h - 1 - p).  *diag: a == b', the block is its own reverse.
__device__ __forceinline__ uint64_t wide_canonical_outer(const EnumJob &j, uint64_t t64, bool *diag)
{
    const int h = j.half_bits;
    const int odd = j.N & 1;
    const uint32_t t = uint32_t(t64);
    const uint32_t side = 1u << h;
    const uint32_t span = side + 1;
    const uint32_t per_m = h ? (side >> 1) * span : 1;
    const uint32_t m = t / per_m;
    const uint32_t r = t - m * per_m;
    const uint32_t p = h ? r / span : 0;
    const uint32_t o = r - p * span;
    const bool first = o <= p;
    const uint32_t bp = first ? p : side - 1 - p;
    const uint32_t a = first ? o : o - p - 1;
    *diag = a == bp;
    const uint32_t b = h ? (__builtin_bitreverse32(bp) >> (32 - h)) : 0;
    return (uint64_t(a) << (h + kWideBits + odd)) | (uint64_t(m) << (h + 5)) | b;
}

// Plain-11 block index t -> outer bits: chunk t >> 6 of 2^17 sequences, and
// within it bits 0 .. 5 of t on the outer monomers 5, 7, .., 15.
__device__ __forceinline__ uint64_t wide11_outer(uint64_t t)
{
    uint64_t o = (t >> 6) << kWide11ChunkBits;
#pragma unroll
    for (int k = 0; k < 6; ++k)
        o |= ((t >> k) & 1u) << (5 + 2 * k);
    return o;
}

// The work of one workgroup: wave w of NW = wide_waves<G>() scores the 256
// sequences x = 256 w + 32 t + col (t = 0 .. 7) of block `blk` (plain 10:
// sequence >> 10; canonical: canonical block index; plain 11: chunk << 6 |
// the outer bits of the chunk).  vlds holds the block's first-product
// fragments, a2s the packed first products of two groups of NW tiles
// ([2][NW][64]), gbs every lane's running top-2 keys ([NW][8][64]).
template <int KB, int G>
__device__ __forceinline__ void wide_body(const EnumJob &j, uint64_t blk, v4i *vlds, v4i *a2s,
                                          int2 *gbs)
{
    constexpr int NW = wide_waves<G>();
    bool diag = false;
    const uint64_t outer = G == 1   ? wide_canonical_outer(j, blk, &diag)
                           : G == 2 ? wide11_outer(blk)
                                    : blk << kWideBits;
    // Contact tiles of the first product are loaded one group ahead into
    // registers for shallow products; deep ones (K_pad > 160) load right
    // before use, which keeps four waves per SIMD.
    constexpr bool kPrefetch = KB <= 5;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = lane & 31;
    const int half = lane >> 5;
    const v4i *__restrict__ B1 = reinterpret_cast<const v4i *>(j.gemm_b);

    // the waves build the block's fragments, one kb at a time
    for (int kb = wave; kb < KB; kb += NW)
        vlds[kb * 64 + lane] = wide_v_fragment<G>(j, outer, col, half, kb);
    v4i sf[kBlkTiles];
    const v4i *__restrict__ S2 = reinterpret_cast<const v4i *>(j.wide_s2) +
                                 ((G == 0 ? 0 : G == 1 ? 4 : 8) + wave) * (kBlkTiles * 64);
#pragma unroll
    for (int t = 0; t < kBlkTiles; ++t)
        sf[t] = S2[t * 64 + lane];
    // Wait for these loads here (s_waitcnt vmcnt(0)): the compiler's wait
    // counts are the same for every pass of the tile loop, so loads of the
    // second operand still counted as in flight there would make each pass
    // also wait for the contact-tile loads issued one group ahead.
    __builtin_amdgcn_s_waitcnt(0x0f70);

    // this lane's running top-2 (global keys) per sequence tile, in LDS
    int2 *const top2 = gbs + wave * (kBlkTiles * 64) + lane;
    int thr[kBlkTiles];
#pragma unroll
    for (int t = 0; t < kBlkTiles; ++t) {
        top2[t * 64] = int2{0, 0};
        thr[t] = 0;
    }

    const int n_tiles = j.n_tiles;
    const int win_tiles = j.blk_win_tiles;
    const int win_shift = j.blk_shift;

    // contact tile `tile` of the first product (this lane's fragments); every
    // wave reads only its own tiles, straight from global memory (L2-resident)
    auto load_c1 = [&](int tile, v4i (&c1)[KB]) {
        const v4i *__restrict__ src = B1 + size_t(tile) * (KB * 64) + lane;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb)
            c1[kb] = src[kb * 64];
    };
    // first product of a tile into this wave's slot of buffer `buf`
    auto first = [&](const v4i (&c1)[KB], int buf) {
        v16i d1;
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
            const v16i zero = {};
            d1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(vlds[kb * 64 + lane], c1[kb],
                                                       kb == 0 ? zero : d1, 0, 0, 0);
        }
        a2s[(buf * NW + wave) * 64 + lane] = pack_d1(d1);
    };

    v4i c1[KB];
    __syncthreads();   // vlds
    if (wave < n_tiles) {
        load_c1(wave, c1);
        first(c1, 0);
    }
    if (kPrefetch && NW + wave < n_tiles)
        load_c1(NW + wave, c1);
    __syncthreads();
    int conf_base = 0;
    int wnext = win_tiles;   // first tile of the next key window
    // The packed first product of the next tile is read from LDS one tile
    // ahead, so no tile starts by waiting for it.  With 8 waves the group's
    // barrier sits before its last tile: by then every wave has read all of
    // this group's buffer and written its first product of the next group,
    // so the next group's first tile can be read ahead as well.  (With 4 waves
    // that needs registers beyond four waves per SIMD where the contact tiles
    // are prefetched, and measured slower where they are not; there the
    // barrier stays at the group's end and each group's first tile is read at
    // its start.)
    constexpr bool kEarlyBarrier = NW == 8;
    v4i a2n = a2s[lane];
    for (int g = 0; g * NW < n_tiles; ++g) {
        const int buf = g & 1;
        const int nt = (g + 1) * NW + wave;   // this wave's tile of the next group
        if constexpr (!kEarlyBarrier)
            a2n = a2s[(buf * NW) * 64 + lane];
#pragma unroll
        for (int tt = 0; tt < NW; ++tt) {
            const int tile = g * NW + tt;
            const v4i a2 = a2n;
            if (tt + 1 < NW) {
                a2n = a2s[(buf * NW + tt + 1) * 64 + lane];
            } else if constexpr (kEarlyBarrier) {
                // the next group's first products are visible, and this
                // group's buffer is free for the group after it
                __syncthreads();
                a2n = a2s[((buf ^ 1) * NW) * 64 + lane];
            }
            if (tile < n_tiles) {
                if (tile == wnext) {
                    conf_base += win_tiles * kTileConf;
                    wnext += win_tiles;
                }
                stage_two_wide(a2, sf, top2, thr, conf_base, win_shift);
            }
            if (tt == 0 && nt < n_tiles) {
                if (!kPrefetch)
                    load_c1(nt, c1);
                first(c1, buf ^ 1);
                if (kPrefetch && nt + NW < n_tiles)
                    load_c1(nt + NW, c1);
            }
        }
        if constexpr (!kEarlyBarrier)
            __syncthreads();   // as above, at the group's end
    }

    int gb[kBlkTiles], gs[kBlkTiles];
#pragma unroll
    for (int t = 0; t < kBlkTiles; ++t) {
        const int2 v = top2[t * 64];
        gb[t] = v.x;
        gs[t] = v.y;
    }
#pragma unroll
    for (int t = 0; t < kBlkTiles; ++t) {
        const int ob = __shfl_xor(gb[t], 32);
        const int os = __shfl_xor(gs[t], 32);
        top2_merge(gb[t], gs[t], ob, os);
        const int x = wave * 256 + t * 32 + col;
        if constexpr (G == 1) {
            // off the diagonal the block's reverse is never scored: write both;
            // a diagonal block holds each sequence and its reverse itself
            uint64_t sq = outer;
#pragma unroll
            for (int b = 0; b < kWideBits; ++b)
                sq |= uint64_t((x >> b) & 1) << wide_pos<1>(j, b);
            const uint64_t rs = diag ? sq : __builtin_bitreverse64(sq) >> (64 - j.N);
            finish_sequence(j, sq, sq, rs, half == 0 && blk < j.hi, gb[t], gs[t], lane == 0, 1);
        } else if constexpr (G == 2) {
            uint64_t sq = outer | uint64_t(x & 31);
#pragma unroll
            for (int b = 5; b < kWide11Bits; ++b)
                sq |= uint64_t((x >> b) & 1) << wide_pos<2>(j, b);
            finish_sequence(j, sq, sq, sq, half == 0 && sq >= j.lo && sq < j.hi, gb[t], gs[t],
                            lane == 0, 1);
        } else {
            const uint64_t idx = outer + uint64_t(x);
            finish_sequence(j, idx, idx, idx, half == 0 && idx >= j.lo && idx < j.hi, gb[t],
                            gs[t], lane == 0, 1);
        }
    }
}

template <int KB, bool CANON>
__global__ __launch_bounds__(256) void k_gemm_wide(EnumJob j)
{
    // first-product A operand of the block (the same for all four waves), the
    // packed first products of the current and the next group of 4 tiles and
    // every lane's running top-2 keys
    __shared__ v4i vlds[KB * 64];
    __shared__ v4i a2s[2 * 4 * 64];
    __shared__ int2 gbs[4 * kBlkTiles * 64];
    wide_body<KB, CANON ? 1 : 0>(j, (CANON ? j.lo : j.lo >> kWideBits) + blockIdx.x, vlds, a2s,
                                 gbs);
}

// Plain ranges cut at multiples of 2^17: blocks of 2048 sequences, 8 waves
// (two workgroups per CU: 53 KB of LDS each at K_pad 160).
template <int KB>
__global__ __launch_bounds__(512) void k_gemm_wide_w8(EnumJob j)
{
    __shared__ v4i vlds[KB * 64];
    __shared__ v4i a2s[2 * kWide11Waves * 64];
    __shared__ int2 gbs[kWide11Waves * kBlkTiles * 64];
    wide_body<KB, 2>(j, ((j.lo >> kWide11ChunkBits) << 6) + blockIdx.x, vlds, a2s, gbs);
}

// Batched wide blocks for jobs of one product depth: workgroup b scores the
// wide block of item item_lo + b, in the job whose item range holds it.
template <int KB>
__global__ __launch_bounds__(256) void k_gemm_wide_batch(BatchHeader *hdr, int item_lo)
{
    __shared__ v4i vlds[KB * 64];
    __shared__ v4i a2s[2 * 4 * 64];
    __shared__ int2 gbs[4 * kBlkTiles * 64];
    const EnumJob *jobs = reinterpret_cast<const EnumJob *>(hdr + 1);
    const int njobs = hdr->njobs;
    const int64_t *start = reinterpret_cast<const int64_t *>(jobs + njobs);
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
    wide_body<KB, 0>(j, (j.lo >> kWideBits) + uint64_t(it - start[lo]), vlds, a2s, gbs);
}

// The same with blocks of 2048 sequences on 8 waves, for jobs whose range
// ends are multiples of 2^17: item b of a job is its block b of the chunked
// 2048-sequence geometry.
template <int KB>
__global__ __launch_bounds__(512) void k_gemm_wide_batch_w8(BatchHeader *hdr, int item_lo)
{
    __shared__ v4i vlds[KB * 64];
    __shared__ v4i a2s[2 * kWide11Waves * 64];
    __shared__ int2 gbs[kWide11Waves * kBlkTiles * 64];
    const EnumJob *jobs = reinterpret_cast<const EnumJob *>(hdr + 1);
    const int njobs = hdr->njobs;
    const int64_t *start = reinterpret_cast<const int64_t *>(jobs + njobs);
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
    wide_body<KB, 2>(j, ((j.lo >> kWide11ChunkBits) << 6) + uint64_t(it - start[lo]), vlds, a2s,
                     gbs);
}

// wide: 1 blocks of 1024 on 4 waves, 2 blocks of 2048 on 8 waves
template <int KB>
hipError_t launch_wide_batch(BatchHeader *hdr, int item_lo, unsigned grid, int wide,
                             hipStream_t st)
{
    if (wide == 2)
        hipLaunchKernelGGL((k_gemm_wide_batch_w8<KB>), dim3(grid), dim3(512), 0, st, hdr,
                           item_lo);
    else
        hipLaunchKernelGGL((k_gemm_wide_batch<KB>), dim3(grid), dim3(256), 0, st, hdr, item_lo);
    return hipGetLastError();
}

// With 8 waves allowed, plain ranges take blocks of 2048 when both ends are
// multiples of 2^17 and monomer 16 exists; otherwise blocks of 1024 (4
// waves).  The 2048 geometry issues half the first products and re-reads the
// contact matrix half as often, and two workgroups per CU keep the SIMDs
// busy while one meets at its group barrier (16 waves in one workgroup per
// CU, tried, left them idle there).
inline bool wide11_applies(const EnumJob &j)
{
    const uint64_t m = (uint64_t(1) << kWide11ChunkBits) - 1;
    return j.N >= kWide11ChunkBits && j.hi > j.lo && (j.lo & m) == 0 && (j.hi & m) == 0;
}

template <int KB>
hipError_t launch_wide(const EnumJob &j, bool waves8, hipStream_t st)
{
    if (j.mode == kSeqCanonical) {
        hipLaunchKernelGGL((k_gemm_wide<KB, true>), dim3(unsigned(j.hi - j.lo)), dim3(256), 0, st,
                           j);
    } else if (waves8 && wide11_applies(j)) {
        const uint64_t n = ((j.hi - j.lo) >> kWide11ChunkBits) << 6;
        hipLaunchKernelGGL((k_gemm_wide_w8<KB>), dim3(unsigned(n)), dim3(512), 0, st, j);
    } else {
        const uint64_t n = ((j.hi - 1) >> kWideBits) - (j.lo >> kWideBits) + 1;
        hipLaunchKernelGGL((k_gemm_wide<KB, false>), dim3(unsigned(n)), dim3(256), 0, st, j);
    }
    return hipGetLastError();
}

template <int KB>
hipError_t launch_blk_batch_kb(BatchHeader *hdr, int item_lo, unsigned grid, bool unary, int wide,
                               hipStream_t st)
{
    if (wide)
        return unary ? hipErrorInvalidValue : launch_wide_batch<KB>(hdr, item_lo, grid, wide, st);
    constexpr int MODE = KB <= 6 ? kBlkLdsS2 : kBlkLds;
    if constexpr (KB <= kBlkUnaryMaxKB) {
        if (unary) {
            hipLaunchKernelGGL((k_gemm_blk_batch<KB, 4, MODE, true>), dim3(grid), dim3(256), 0,
                               st, hdr, item_lo);
            return hipGetLastError();
        }
    }
    if (unary)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_gemm_blk_batch<KB, 4, MODE, false>), dim3(grid), dim3(256), 0, st, hdr,
                       item_lo);
    return hipGetLastError();
}

template <int KB, int NW, int MODE>
hipError_t launch_blk_shape(const EnumJob &j, hipStream_t st)
{
    const bool canon = j.mode == kSeqCanonical;
    const uint64_t n_blocks =
        canon ? j.hi - j.lo : ((j.hi - 1) >> kBlkBits) - (j.lo >> kBlkBits) + 1;
    const dim3 grid(unsigned((n_blocks + NW - 1) / NW));
    if (canon)
        hipLaunchKernelGGL((k_gemm_blk<KB, NW, MODE, true, false>), grid, dim3(NW * 64), 0, st, j);
    else
        hipLaunchKernelGGL((k_gemm_blk<KB, NW, MODE, false, false>), grid, dim3(NW * 64), 0, st, j);
    return hipGetLastError();
}

// Two-letter tables: one launch shape (4 waves, staging by depth).
template <int KB>
hipError_t launch_blk_unary(const EnumJob &j, hipStream_t st)
{
    if constexpr (KB > kBlkUnaryMaxKB) {
        return hipErrorInvalidValue;
    } else {
        constexpr int MODE = KB <= 6 ? kBlkLdsS2 : kBlkLds;
        const bool canon = j.mode == kSeqCanonical;
        const uint64_t n_blocks =
            canon ? j.hi - j.lo : ((j.hi - 1) >> kBlkBits) - (j.lo >> kBlkBits) + 1;
        const dim3 grid(unsigned((n_blocks + 3) / 4));
        if (canon)
            hipLaunchKernelGGL((k_gemm_blk<KB, 4, MODE, true, true>), grid, dim3(256), 0, st, j);
        else
            hipLaunchKernelGGL((k_gemm_blk<KB, 4, MODE, false, true>), grid, dim3(256), 0, st, j);
        return hipGetLastError();
    }
}

template <int KB>
hipError_t launch_blk(const EnumJob &j, int nw, int mode, hipStream_t st)
{
    if (j.blk_ngroups > 0 || j.blk_coefB != 0)
        return launch_blk_unary<KB>(j, st);
    if (mode == kBlkStageWide)
        return launch_wide<KB>(j, nw == 8, st);
    if (mode == kBlkLdsS2) {
        switch (nw) {
        case 2: return launch_blk_shape<KB, 2, kBlkLdsS2>(j, st);
        case 8: return launch_blk_shape<KB, 8, kBlkLdsS2>(j, st);
        default: return launch_blk_shape<KB, 4, kBlkLdsS2>(j, st);
        }
    }
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

// One product depth's launchers, defined by the gemm_blk_kb*.hip units
// (each instantiates the kernels of its depths, so they compile in parallel).
#define HP_BLK_DEPTH(KB)                                                                  \
    hipError_t launch_gemm_blocked_kb##KB(const EnumJob &j, int nw, int mode, hipStream_t st) \
    {                                                                                     \
        return launch_blk<KB>(j, nw, mode, st);                                           \
    }                                                                                     \
    hipError_t launch_gemm_blk_batch_kb##KB(BatchHeader *hdr, int item_lo, unsigned grid,  \
                                            bool unary, int wide, hipStream_t st)         \
    {                                                                                     \
        return launch_blk_batch_kb<KB>(hdr, item_lo, grid, unary, wide, st);              \
    }                                                                                     \
    hipError_t launch_gemm_wide_kb##KB(const EnumJob &j, hipStream_t st)                  \
    {                                                                                     \
        return launch_wide<KB>(j, false, st);                                             \
    }

}  // namespace hpmap
