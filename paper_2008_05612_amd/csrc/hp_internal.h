// Internal definitions shared by the host structure code, the C ABI and the
// kernel launchers of libhpmap.  Not installed; the public surface is hp.h.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "hp.h"

namespace hpmap {

constexpr int kMaxN = 36;            // sequences are 64-bit, ids 16-bit
constexpr int kTileConf = 32;        // conformations per MFMA tile (rows of A)
// Keys of the running minimum search are non-negative; 0 means "no
// conformation".  F is the quantity maximised (F = A n_HH + B sum_i h_i c_i,
// the negated energy up to a constant; F = n_HH for pure HP).  Global key =
// (F << 17) | (conformation + 1); window key of the int8 form =
// S F + (position in window + 1) with S = 2^win_shift, windows being the
// largest whole number of 32-conformation tiles below S.
constexpr int kKeyConfBits = 17;
constexpr uint32_t kMaxConf = (1u << kKeyConfBits) - 1;
constexpr int kMaxKB = 12;              // product depth K_pad <= 384
constexpr int kBlkUnaryMaxKB = 8;       // blocked form with unary rows: first-product depth <= 256
// Block-factorised int8 form: blocks of 2^kBlkBits consecutive sequences
// share every monomer above the low kBlkBits.
constexpr int kBlkBits = 8;

// Byte offsets of the packed tables inside the device workspace.
struct WsLayout {
    size_t c2q = 0;      // uint16_t[n_conf]
    size_t pairs = 0;    // uint8_t[K_pad][4] row table (i, j, constant, 0)
    size_t masks = 0;    // uint32_t[n_conf][MW]: W pair words, then unary bit planes
    size_t gemm_a = 0;   // int8_t[n_tiles][K_pad/32][64 lanes][16]
    size_t gemm_b = 0;   // blocked form: int8_t[n_tiles][K_pad/32][64 lanes][16], or none
    size_t blk_s2 = 0;   // blocked form: int8_t[2 geometries][8 tiles][64 lanes][16], or none
    size_t wide_s2 = 0;  // wide blocks: int8_t[4 + 4 + 8 waves][8 tiles][64 lanes][16] (geometries:
                         // plain 10, canonical 10, plain 11), or none
    size_t total = 0;
};

}  // namespace hpmap

struct hp_structs {
    int X = 0, Y = 0, Z = 0, N = 0;
    uint32_t G = 0;
    uint64_t n_walks = 0;
    uint32_t n_conf = 0, n_class = 0, n_selfrev = 0, nbp = 0, K = 0, W = 0, K_pad = 0;
    // energy model: table {E_PP, E_PH, E_HP, E_HH}; maximised F = A n + B u
    int32_t table[4] = {0, 0, 0, -1};
    int32_t A = 1, B = 0, e0 = 0;     // E = e0 - F, e0 = E_PP * nbp
    uint32_t U = 0;                   // unary rows (N when B != 0)
    uint32_t cmax = 0;                // largest contact count of one monomer
    uint32_t planes = 0, uw = 0;      // bit planes of c_i and 32-bit words per plane
    uint32_t MW = 0;                  // mask words per conformation: W + planes * uw
    uint32_t win_shift = 14, win_tiles = 511;
    // blocked int8 form (pure pair energies, N >= kBlkBits): key scale
    // 2^blk_shift, windows of blk_win_tiles tiles, stage-one weight blk_coef
    bool blk_ok = false;
    uint32_t blk_shift = 0, blk_win_tiles = 0;
    int32_t blk_coef = 0, blk_coefB = 0;   // m2 A, m2 B
    uint32_t blk_KB = 0;                   // depth of the first product / 32
    int32_t blk_ngroups[2] = {0, 0};       // unary-term rows per geometry (plain, canonical)
    uint64_t blk_grp[2][3] = {};           // group id of each outer monomer, 4 bits, 15 = none
    std::vector<uint8_t> walks;       // n_conf * N canonical site sequences, ascending
    std::vector<uint16_t> c2q;        // conformation -> class
    std::vector<uint32_t> rev_conf;   // conformation of the reversed chain
    std::vector<uint8_t> self_rev;    // per class
    std::vector<uint8_t> pairs;       // K * 2: (i, j) of bit / row k
    std::vector<uint8_t> contacts;    // n_conf * nbp * 2, (i, j) ascending
    std::vector<uint32_t> masks;      // n_conf * W contact bitmasks
    std::vector<int8_t> gemm_a;       // int8 contact matrix in MFMA A-operand order
    std::vector<int8_t> gemm_b;       // blocked form: 0/1 contact matrix + window index rows
    std::vector<int8_t> blk_s2;       // blocked form: per-sequence operand of the second product
    bool wide_ok = false;             // wide blocks apply (pure pair energies, N >= 10)
    std::vector<int8_t> wide_s2;      // wide blocks: per-sequence operand of the second product
    std::vector<uint8_t> pair_rows;   // K_pad * 4: (i, j, constant, 0) per product row
    hpmap::WsLayout ws;
};

namespace hpmap {

// Block geometry of the blocked form: the 8 varying monomers pos[0..7]
// (ascending) -- the low 8 for plain ranges, the middle 8 (around the middle
// monomer for odd N) for reversal-canonical blocks -- and the pairs among
// them with odd separation >= 3 as x-indices (a, b), a < b (at most 16).
// Pairs of the low 8 monomers with odd separation >= 3, as x-indices
// a | b << 4 a byte each (pairs 0 .. 7) plus the ninth pair: the plain
// geometry, shared by the host tables and the kernel's compile-time copy.
constexpr uint64_t kLow8Pairs = 0x6372526141705030ull;   // (0,3) (0,5) (0,7) (1,4) (1,6) (2,5) (2,7) (3,6)
constexpr int kLow8Pair8 = 0x74;                          // (4,7)
constexpr int kLow8NumPairs = 9;

// Wide blocks of the blocked form: 2^kWideBits = 1024 sequences sharing
// every monomer above the low 10, scored by the 4 waves of one workgroup.
// Pairs of the low 10 monomers with odd separation >= 3, as x-indices
// a | b << 4 a byte each: pairs 0 .. 7 in kLow10Pairs0, 8 .. 15 in
// kLow10Pairs1 (shared by the host tables and the kernel).
constexpr int kWideBits = 10;
constexpr uint64_t kLow10Pairs0 = 0x5096857463524130ull;   // (0,3) (1,4) (2,5) (3,6) (4,7) (5,8) (6,9) (0,5)
constexpr uint64_t kLow10Pairs1 = 0x9092817094837261ull;   // (1,6) (2,7) (3,8) (4,9) (0,7) (1,8) (2,9) (0,9)
constexpr int kLow10NumPairs = 16;
// Reversal-canonical wide blocks vary the 10 monomers around the middle:
// pos(x) = h + x for even N; for odd N the middle monomer h + 5 stays outer,
// pos(x) = h + x + (x >= 5).  With even N the pairs are those of the low 10;
// with odd N (x-indices, same byte layout):
constexpr uint64_t kMid10OddPairs0 = 0x7151806096854130ull;  // (0,3) (1,4) (5,8) (6,9) (0,6) (0,8) (1,5) (1,7)
constexpr uint64_t kMid10OddPairs1 = 0x8464937353826291ull;  // (1,9) (2,6) (2,8) (3,5) (3,7) (3,9) (4,6) (4,8)
// Wide blocks of 2048 sequences for plain ranges, scored by the 8 waves of
// one workgroup: the 11 varying monomers are 0 .. 4 and the even monomers
// 6, 8, .., 16 (pos(x) = x for x < 5, 2 x - 4 after).  Monomers of equal
// parity are never in contact (odd separation), so the only varying pairs
// are (0,3), (1,4) and those of monomers 1 and 3 with the six even ones: 14
// pairs, padded to 16 with two pairs of equal parity whose rows stay zero;
// base, 11 weights, 16 pair rows and 2 index rows fill 30 of the 32 virtual
// rows.  The outer monomers 5, 7, .., 15 of a 2^17-sequence chunk index its
// 64 blocks.  Pairs as x-indices a | b << 4:
constexpr int kWide11Bits = 11;
constexpr int kWide11Waves = 8;
constexpr int kWide11ChunkBits = 17;
constexpr uint64_t kW11Pairs0 = 0xA191817161514130ull;   // (0,3) (1,4) (1,5) (1,6) (1,7) (1,8) (1,9) (1,10)
constexpr uint64_t kW11Pairs1 = 0x4220A39383736353ull;   // (3,5) (3,6) (3,7) (3,8) (3,9) (3,10) (0,2) (2,4)

struct BlockGeometry {
    int pos[8];
    int npp;
    int pa[16], pb[16];
    int half;   // canonical blocks: outer monomers on each side
};
BlockGeometry block_geometry(int N, bool canonical);

// Host enumeration (structures.cpp).  Returns HP_OK or an error with msg set.
hp_status build_structures(int X, int Y, int Z, const int32_t table[4], hp_structs *s,
                           std::string *msg);

struct EnumJob;
// Kernel-side descriptor of one enumeration over [lo, hi) (capi.cpp).
EnumJob make_enum_job(const hp_structs *s, const void *d_ws, uint64_t lo, uint64_t hi,
                      uint16_t *out, int32_t *emin, uint64_t *desig, uint64_t *nondesign);

// Batched launches (capi.cpp).  The work list of `njobs` jobs is written
// into host[0 .. hp_batch_workspace_bytes(njobs)); order[njobs],
// start[njobs + 1] and groups[njobs] are scratch and launch groups supplied
// by the caller (nothing is allocated).
struct BatchGroup {
    int kb, item_lo, item_hi;   // product depth (blocked: 8 depth + 2 wide + unary, wide 0 none,
                                // 1 blocks of 1024, 2 blocks of 2048), its items
};
hp_status plan_batch(const hp_job *jobs, int njobs, int form, size_t ws_bytes, char *host,
                     int *order, int64_t *start, BatchGroup *groups, int *ngroups);

// Error plumbing (capi.cpp).
hp_status fail(hp_status st, const std::string &msg);

}  // namespace hpmap
