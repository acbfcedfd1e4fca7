// Device-side job descriptors and kernel launchers of libhpmap (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

struct hp_structs;

namespace hpmap {

// One enumeration job as the kernels see it.  Plain data, copied into kernel
// arguments (single launches) or into the batch work list (device memory).
struct EnumJob {
    const uint16_t *c2q;            // conformation -> class
    const uint8_t *pairs;           // K_pad x 4 row table (i, j, constant, 0)
    const uint32_t *masks;          // n_conf x W contact bitmasks
    const int8_t *gemm_a;           // int8 contact matrix, MFMA A-operand order
    const int8_t *gemm_b;           // blocked form: 0/1 contacts + window index rows
    uint16_t *out;                  // phenotype per sequence, or null
    int32_t *emin;                  // ground-state energy per sequence, or null
    unsigned long long *desig;      // designability, += (or null)
    unsigned long long *nondesign;  // deleterious count, += (or null)
    uint64_t lo, hi;                // sequence range [lo, hi)
    int32_t N, K, W, KB;            // chain length, pairs, pair-mask words, K_pad/32
    int32_t n_conf, n_tiles;        // conformations, 32-conformation tiles
    int32_t U;                      // unary product rows (0 for pure HP)
    int32_t win_tiles, win_shift;   // int8-form key windows
    int32_t A, B, e0;               // F = A n + B u, E = e0 - F
    int32_t planes, uw, MW;         // popcount form: unary bit planes, words, mask stride
    int32_t mode;                   // how [lo, hi) maps to sequences (SeqMode)
    int32_t half_bits;              // floor(N / 2)
    int32_t threshold;              // folds iff second-lowest - lowest energy >= threshold
    uint8_t *gap;                   // energy gap per sequence (saturated at 255), or null
    uint64_t *seqs;                 // sampled mode: the sequence drawn at each index, or null
    uint64_t seed;                  // sampled mode: generator seed
    int32_t blk_shift, blk_win_tiles, blk_coef;   // blocked form: key scale, windows, m2 A
    // blocked form block geometry: varying monomers (mask; positions packed a
    // byte each), their odd-separation pairs (x-indices a | b << 4, a byte
    // each) and how many
    uint64_t blk_vmask, blk_pos, blk_pp[3];
    int32_t blk_npp;
    int32_t blk_KB, blk_coefB, blk_ngroups;   // first-product depth / 32, m2 B, unary rows
    uint64_t blk_grp[3];                      // unary group of each outer monomer (4 bits)
    const int8_t *blk_s2;           // second-product operand of this geometry (8 x 64 x 16 B)
    const int8_t *wide_s2;          // wide blocks: second-product operand ((4 + 4 + 8) waves
                                    // x 8 x 64 x 16 B: plain 10, canonical 10 and plain 11
                                    // geometries), or null where wide blocks do not apply
};

// Index -> sequence maps of a job.  kSeqPlain: index t is sequence t.
// kSeqCanonical: t ranks the canonical sequences s <= reverse(s) (results are
// written at s and reverse(s)).  kSeqSampled: t is a draw of the random
// generator (results are written at t - lo).
enum SeqMode { kSeqPlain = 0, kSeqCanonical = 1, kSeqSampled = 2 };

// Work list of a batched launch, laid out in the batch workspace: this
// header, EnumJob[njobs] ordered by product depth, int64 item_start[njobs+1].
// One launch per product depth covers the items of its jobs, one workgroup
// per item.
struct BatchHeader {
    uint32_t reserved;
    int32_t njobs;
    int32_t n_items;
    int32_t kb_max;
};

// One compiled tile shape of the int8 form: KB = K_pad/32 product depth, T
// sequence tiles of 32 per wave, NW waves per workgroup, A staged through
// LDS (mode 0) or loaded per wave from global memory (mode 1).
struct GemmVariant {
    int KB, T, NW, mode;
    hipError_t (*launch)(const EnumJob &j, hipStream_t st);
};

// Compiled variants, grouped by the translation unit that instantiates them.
int gemm_variants_kb1_4(const GemmVariant **out);
int gemm_variants_kb5(const GemmVariant **out);
int gemm_variants_kb6_10(const GemmVariant **out);
int gemm_variants_kb11_12(const GemmVariant **out);

// Shape used for product depth KB (process-wide choice; default: first listed).
const GemmVariant *gemm_selected_variant(int KB);

hipError_t launch_popcount(const EnumJob &j, hipStream_t st);
// Block-factorised int8 form over a plain range (pure pair energies); nw
// waves per workgroup (2, 4 or 8), one 256-sequence block per wave; mode 0
// stages contact tiles through double-buffered LDS, mode 1 through triple-
// buffered LDS with the next tile's first product overlapping this tile's
// key updates.
hipError_t launch_gemm_blocked(const EnumJob &j, int nw, int mode, hipStream_t st);
// Reversal-canonical wide blocks [j.lo, j.hi) (j.mode kSeqCanonical,
// j.half_bits the outer monomers on each side).
hipError_t launch_gemm_wide_canonical(const EnumJob &j, hipStream_t st);
// Staging modes of the blocked form's contact tiles (gemm_blk.h); mode < 0
// picks by product depth.
// kBlkStageWide: wide blocks of 1024 sequences per workgroup of 4 waves,
// the first product shared by the waves (pure pair energies, plain ranges).
enum BlkStage { kBlkStageLds = 0, kBlkStagePipe = 1, kBlkStageS2Lds = 2, kBlkStageWide = 3 };
// Batched launch of the blocked form (plain jobs), same work-list layout:
// items of blk_batch_seqs_per_item() sequences, one wide block of 1024 (wide
// jobs: blk_batch_wide) or 4 blocks of 256, or one wide block of 2048 (jobs
// whose range ends are multiples of 2^17: blk_batch_wide8), one workgroup per
// item; wide = 0, 1 (blocks of 1024) or 2 (blocks of 2048).
uint64_t blk_batch_seqs_per_item();
bool blk_batch_wide(const hp_structs *s);
bool blk_batch_wide8(const hp_structs *s, uint64_t lo, uint64_t hi);
hipError_t launch_gemm_blk_batch(void *d_batch_ws, int kb, bool unary, int wide, int item_lo,
                                 int item_hi, hipStream_t st);
// Process-wide launch shape of the blocked form (runtime.cpp).
int blocked_selected_nw();
int blocked_selected_mode();
// Sequences per work item of the dense persistent batched kernel.
uint64_t gemm_batch_seqs_per_item();
// Persistent launch over items [item_lo, item_hi) of the work list at
// d_batch_ws, all of product depth kb.
hipError_t launch_gemm_batch(void *d_batch_ws, int kb, int item_lo, int item_hi, hipStream_t st);
// One launch per group of a batch plan (hp_internal.h), in order on `st`,
// over the work list at d_batch_ws (capi.cpp).
struct BatchGroup;
hipError_t launch_plan(const BatchGroup *groups, int ngroups, int form, void *d_batch_ws,
                       hipStream_t st);
hipError_t launch_fill_u32(uint32_t *p, uint32_t value, uint64_t n, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long value, uint64_t n,
                           hipStream_t st);

hipError_t launch_neighbors(const uint16_t *map, int N, int n_class, unsigned long long *neutral,
                            unsigned long long *deleterious, unsigned long long *other, int phi_q,
                            unsigned long long *phi_row, hipStream_t st);
hipError_t launch_phi_counts(const uint16_t *map, int N, int n_class, unsigned long long *counts,
                             hipStream_t st);
hipError_t launch_phi_row_ptr(const unsigned long long *counts, int n_class, uint64_t *row_ptr,
                              hipStream_t st);
hipError_t launch_phi_compact(const unsigned long long *counts, int n_class,
                              const uint64_t *row_ptr, uint32_t *cols, uint64_t *vals,
                              hipStream_t st);
hipError_t launch_components(const uint16_t *map, int N, uint32_t *labels, uint32_t *compsize,
                             uint32_t *ncomp, uint32_t *largest, int n_class, hipStream_t st);

}  // namespace hpmap
