// Device-side job descriptors and kernel launchers of libhpmap (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hpmap {

// One enumeration job as the kernels see it.  Plain data, copied into kernel
// arguments (single launches) or into the batch work list (device memory).
struct EnumJob {
    const uint16_t *c2q;            // conformation -> class
    const uint8_t *pairs;           // K_pad x 2 pair table (rows >= K unused)
    const uint32_t *masks;          // n_conf x W contact bitmasks
    const int8_t *gemm_a;           // int8 contact matrix, MFMA A-operand order
    uint16_t *out;                  // phenotype per sequence, or null
    int32_t *emin;                  // ground-state energy per sequence, or null
    unsigned long long *desig;      // designability, += (or null)
    unsigned long long *nondesign;  // deleterious count, += (or null)
    uint64_t lo, hi;                // sequence range [lo, hi)
    int32_t N, K, W, KB;            // chain length, pairs, mask words, K_pad/32
    int32_t n_conf, n_tiles;        // conformations, 32-conformation tiles
};

// Work list of a batched launch, laid out in the batch workspace.
struct BatchHeader {
    uint32_t counter;     // next item to take (reset to 0 by a fill kernel)
    int32_t njobs;
    int32_t n_items;
    int32_t kb_max;
};

// Tile shape of the int8 form: sequence tiles of 32 per wave (T of them),
// NW waves per workgroup.
struct GemmShape {
    int T;
    int NW;
};

hipError_t launch_popcount(const EnumJob &j, hipStream_t st);
hipError_t launch_gemm(const EnumJob &j, GemmShape shape, hipStream_t st);
GemmShape default_gemm_shape(int KB);
uint64_t gemm_seqs_per_item(GemmShape shape);
// Batched persistent launch: header at d_ws, then EnumJob[njobs], then
// int64 item_start[njobs + 1].
hipError_t launch_gemm_batch(void *d_batch_ws, int kb_max, int n_items, hipStream_t st);
hipError_t launch_fill_u32(uint32_t *p, uint32_t value, uint64_t n, hipStream_t st);
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long value, uint64_t n,
                           hipStream_t st);

hipError_t launch_neighbors(const uint16_t *map, int N, int n_class, unsigned long long *neutral,
                            unsigned long long *deleterious, unsigned long long *other, int phi_q,
                            unsigned long long *phi_row, hipStream_t st);
hipError_t launch_components(const uint16_t *map, int N, uint32_t *labels, uint32_t *compsize,
                             uint32_t *ncomp, uint32_t *largest, int n_class, hipStream_t st);

}  // namespace hpmap
