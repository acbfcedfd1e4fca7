// Device helpers shared by the ground-state kernels of libhpmap (internal).
//
// Running state of a sequence is a pair of 32-bit keys (best, second).  A key
// orders first by the number n of H-H contacts and then by conformation, so
// the largest key is a minimum-energy conformation (E = -n, Eq. 1 with
// E_HH = -1) and the second-largest key has the same n exactly when the
// minimum is shared, i.e. when the sequence does not fold (Methods, end of
// "HP and MJ lattice models").  Keys are non-negative: global keys are
// (n << 17) | (conformation + 1) and 0 stands for "no conformation", so
// signed and unsigned comparisons agree.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>

#include "hp_internal.h"
#include "kernels.h"

namespace hpmap {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// Median of three, written as max(min(a, b), min(max(a, b), c)), which the
// backend selects as one v_med3_i32.  No inline assembly here: the compiler
// must see the instruction to insert the wait states between an MFMA and the
// VALU reads of its result registers.
__device__ __forceinline__ int med3_i32(int a, int b, int c)
{
    return max(min(a, b), min(max(a, b), c));
}

// (b, s) is the running top-2, b >= s >= 0.  Absorb keys k1, k2 >= 0.
// The new best uses unsigned comparisons and the median signed ones (equal
// orders on non-negative keys): being different operations, the compiler
// cannot merge their common max(b, k1), and each selects to a single
// three-operand instruction (v_max3_u32, v_med3_i32); the second then folds
// two medians per v_max3_i32.
__device__ __forceinline__ void top2_add2(int &b, int &s, int k1, int k2)
{
    const int m = med3_i32(b, k1, k2);   // second largest of {b, k1, k2}
    b = int(max(max(unsigned(b), unsigned(k1)), unsigned(k2)));
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

// Window key S F + u (S = 2^win_shift, u = position + 1) -> global key
// (F << 17) | (conformation + 1); 0 stays 0.
__device__ __forceinline__ int window_to_global(int k, int conf_base, int win_shift)
{
    const int g = ((k >> win_shift) << kKeyConfBits) | (conf_base + (k & ((1 << win_shift) - 1)));
    return k == 0 ? 0 : g;
}

// Bits 0 .. n-1 of x reversed (n <= 32).
__device__ __forceinline__ uint32_t reverse_bits(uint32_t x, int n)
{
    return n ? __builtin_bitreverse32(x) >> (32 - n) : 0u;
}

// Draw t of the splitmix64 stream seeded with `seed` (Steele, Lea and Flood,
// OOPSLA 2014), evaluated directly from the counter: the generator's state
// after t + 1 steps is seed + (t + 1) * golden-ratio increment, followed by
// the variant-13 64-bit finaliser.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t t)
{
    uint64_t z = seed + (t + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Sequence at index t of the enumeration.  Plain jobs: s = t.  Sampled jobs:
// the low N bits of draw t (N independent fair H/P choices).  Symmetric jobs
// enumerate only canonical sequences s <= reverse(s): with h = floor(N/2),
// s = (a, m, b) = high h bits, middle bit (odd N), low h bits, and
// reverse(s) = (rev b, m, rev a), so s is canonical iff a <= b' = rev b.  Row
// b' holds the b' + 1 values a = 0 .. b'; rows p and 2^h - 1 - p together
// hold 2^h + 1, so the index runs over m, then the row pair p < 2^(h-1), then
// its 2^h + 1 entries (first row p, then row 2^h - 1 - p).  (For h = 0 there
// is one row holding a = 0.)  *rs receives reverse(s).
__device__ __forceinline__ uint64_t sequence_at(const EnumJob &j, uint64_t t, uint64_t *rs)
{
    if (j.mode == kSeqPlain) {
        *rs = t;
        return t;
    }
    if (j.mode == kSeqSampled) {
        const uint64_t s = splitmix64_at(j.seed, t) & ((uint64_t(1) << j.N) - 1);
        *rs = s;
        return s;
    }
    const int h = j.half_bits;
    const int mid = j.N & 1;
    const uint64_t side = uint64_t(1) << h;
    const uint64_t span = side + 1;                         // entries per row pair
    const uint64_t per_m = h ? (side >> 1) * span : 1;      // canonical count per middle bit
    const uint64_t m = t / per_m;
    const uint64_t r = t - m * per_m;
    const uint64_t p = h ? r / span : 0;
    const uint64_t o = r - p * span;
    const bool first = o <= p;
    const uint64_t bp = first ? p : side - 1 - p;
    const uint64_t a = first ? o : o - p - 1;
    const int hi_shift = h + mid;
    *rs = (bp << hi_shift) | (m << h) | reverse_bits(uint32_t(a), h);
    return (a << hi_shift) | (m << h) | reverse_bits(uint32_t(bp), h);
}

// Final decision for sequence s at index t and the per-sequence outputs.
// The keys' high part times fmul is F, the minimum energy is e0 - F, and the
// energy gap to the best other conformation is fmul times the difference of
// the two keys' high parts (0 when the minimum is shared).  The sequence
// folds iff that gap reaches the threshold, or it has no other conformation.
// Plain and sampled jobs write at t - lo; symmetric jobs write the full-size
// maps at s and reverse(s) and count a non-palindromic sequence twice.
__device__ __forceinline__ void finish_sequence(const EnumJob &j, uint64_t t, uint64_t s,
                                                uint64_t rs, bool valid, int gb, int gs,
                                                bool count_lane, int fmul)
{
    const int nb = gb >> kKeyConfBits;
    const int ns = gs >> kKeyConfBits;
    const int diff = fmul * (nb - ns);
    const bool uniq = gs == 0 || diff >= j.threshold;   // no second conformation, or far enough
    uint16_t q = HP_NONE;
    if (valid && uniq)   // the clamp keeps the table read in bounds for any key
        q = j.c2q[min(max((gb & int(kMaxConf)) - 1, 0), j.n_conf - 1)];
    const bool twin = j.mode == kSeqCanonical && rs != s;
    if (valid) {
        const uint64_t at = j.mode == kSeqCanonical ? s : t - j.lo;
        const int e = j.e0 - fmul * nb;
        if (j.out) {
            j.out[at] = q;
            if (twin)
                j.out[rs] = q;
        }
        if (j.emin) {
            j.emin[at] = e;
            if (twin)
                j.emin[rs] = e;
        }
        if (j.gap) {
            const uint8_t g = uint8_t(gs == 0 ? 255 : min(diff, 255));
            j.gap[at] = g;
            if (twin)
                j.gap[rs] = g;
        }
        if (j.seqs)
            j.seqs[at] = s;
        if (uniq && j.desig)
            atomicAdd(&j.desig[q], twin ? 2ull : 1ull);
    }
    const unsigned long long del = __ballot(valid && !uniq);
    const unsigned long long del2 = __ballot(valid && !uniq && twin);
    if (count_lane && j.nondesign && del)
        atomicAdd(j.nondesign, (unsigned long long)(__popcll(del) + __popcll(del2)));
}

// B-operand fragments of one lane for T sequences: bytes of product rows
// kbase .. kbase+15 with kbase = 32 kb + 16 half (byte q of a fragment is row
// kbase + q).  Row k < K is the pair (i, i + d) of the k-th odd separation
// d >= 3 in (d, i) order, and its byte is 0x80 * h_i h_{i+d}; rows K .. K+U-1
// are the unary rows 0x80 * h_{k-K}; row K+U is the constant 0x01 and row
// K+U+1 the constant 0x80 (the index rows); rows beyond are 0.  The row walk
// needs no table: the pair of the first row is found by skipping whole runs
// of length N - d, consecutive rows advance (d, i), and after the last run
// the walk continues with d = 0, where h_i h_{i+d} = h_i is the unary row.
template <int KB, int T>
__device__ __forceinline__ void p_fragments(const uint64_t (&s)[T], int half, int N, int K, int U,
                                            v4i (&pf)[T][KB])
{
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        const int kbase = kb * 32 + half * 16;
        int d = 3, i = kbase;
        while (d < N && i >= N - d) {   // skip whole runs of separation d
            i -= N - d;
            d += 2;
        }
        if (d >= N)                     // past the pairs: unary row i = kbase - K
            d = 0;
        uint32_t w[T][4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
            for (int t = 0; t < T; ++t)
                w[t][q] = 0;
#pragma unroll
            for (int bb = 0; bb < 4; ++bb) {
                const int k = kbase + 4 * q + bb;
                const int ki = K + U;
                const uint32_t c = k == ki ? 0x01u : (k == ki + 1 ? 0x80u : 0u);
                const bool real = k < ki;
#pragma unroll
                for (int t = 0; t < T; ++t) {
                    const uint32_t bit = real ? uint32_t((s[t] >> i) & (s[t] >> (i + d)) & 1u) : 0u;
                    w[t][q] |= ((bit << 7) | c) << (8 * bb);
                }
                ++i;                       // next row: next i, or the next run
                if (d > 0 && i + d >= N) {
                    i = 0;
                    d += 2;
                    if (d >= N)
                        d = 0;
                }
            }
        }
#pragma unroll
        for (int t = 0; t < T; ++t)
            pf[t][kb] = v4i{int(w[t][0]), int(w[t][1]), int(w[t][2]), int(w[t][3])};
    }
}

}  // namespace hpmap
