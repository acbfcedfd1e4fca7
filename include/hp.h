/*
 * hp.h -- C ABI of the MI355X HP-model genotype-phenotype map library
 * (libhpmap.so).
 *
 * The library computes, for every binary H/P sequence of a chain of N
 * monomers in a given index range, the ground state over all compact
 * structures of a lattice box, decides whether it is unique, and accumulates
 * per-structure designability; it then derives single-point-mutation
 * statistics and neutral-network components from the resulting map.
 * Model: S. J. Owen, "Graphical processing unit accelerated enumeration and
 * exploration of model genotype-phenotype maps for protein folding"
 * (arXiv 2008.05612), Methods (Eq. 1, ground-state rule), Eq. 2 and the
 * designability/robustness definitions around it.
 *
 * Conventions shared by every call
 *   - Sequences: bit i of the 64-bit index s is monomer i; 1 = H, 0 = P.
 *   - Energy: E(s,c) = -(number of H-H non-bonded lattice contacts of
 *     conformation c), i.e. Eq. 1 with E_HH = -1 and E_HP = E_PP = 0.
 *   - Structures: directed Hamiltonian paths of the X*Y*Z box ("compact
 *     self-avoiding walks").  A conformation is an orbit of directed paths
 *     under the box's isometry group; a class (the reported phenotype) is an
 *     orbit under isometries and chain reversal.  Both chain directions are
 *     scored, since E(s, reverse(c)) = E(reverse(s), c).
 *   - Ids: conformation ids rank the canonical keys (lexicographically
 *     smallest site sequence of the orbit, site = x + X*(y + Y*z)); class ids
 *     rank class keys (the smaller key of the two chain directions).
 *   - A sequence is designing iff exactly one conformation attains the
 *     minimum energy; its phenotype is that conformation's class id.  Any
 *     other sequence has the deleterious phenotype HP_NONE.
 *   - Memory: pointers named d_* are device pointers owned by the caller;
 *     the library never allocates or frees device memory.  Host pointers
 *     are owned by the caller too, except hp_structs handles, which the
 *     library allocates and hp_structs_free releases.
 *   - Streams: `stream` is a hipStream_t (NULL = the default stream).  Device
 *     work is enqueued asynchronously; results are valid once the caller has
 *     synchronised that stream.
 *   - Errors: every call returns hp_status.  Nothing calls exit() or throws.
 *     hp_last_error() describes the last failure of the calling thread.
 */
#ifndef HP_H
#define HP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HP_OK = 0,
    HP_EINVAL = -1,       /* bad argument: NULL, range, size, dims */
    HP_ENOMEM = -2,       /* host allocation failed */
    HP_EDEVICE = -3,      /* a HIP call failed */
    HP_ERANGE = -4,       /* problem too large for the id or index types */
    HP_EUNSUPPORTED = -5  /* valid request the library does not handle */
} hp_status;

#define HP_NONE 0xFFFFu

/* Energy-kernel forms (all give bit-identical results). */
#define HP_FORM_POPCOUNT 0  /* contact bitmasks, AND + popcount per pair        */
#define HP_FORM_GEMM_I8 1   /* E = -P.C as an int8 matrix product on MFMA cores */
/* Block-factorised int8 form: each block of 256 consecutive sequences shares
 * every monomer above the low 8, so per conformation the energy is a block
 * term plus weights of the 8 low monomers and their mutual contacts; one
 * int8 product per 256 sequences forms those (as bytes), a second product of
 * depth 32 applies them to the sequences.  Two-letter tables (E_HP !=
 * E_PP) add the unary terms of the outer monomers as a few more per-block
 * rows.  Needs N >= 8 and weights whose per-block bytes fit int8 within 32
 * rows, and with unary rows a first product at most 256 deep (pure HP on
 * every box up to 6x6 and 3x3x3 qualifies, Table 1 up to 3x3x3 but not 6x6;
 * hp_canonical_block_count is 0 when a handle does not); only plain ranges
 * (hp_enumerate, hp_enumerate_gap).  Otherwise HP_EUNSUPPORTED.           */
#define HP_FORM_BLOCKED_I8 2

typedef struct hp_structs hp_structs;

typedef struct {
    int32_t X, Y, Z;      /* box dimensions */
    int32_t N;            /* chain length = X*Y*Z */
    uint32_t group_order; /* number of box isometries */
    uint64_t n_walks;     /* directed Hamiltonian paths = group_order * n_conf */
    uint32_t n_conf;      /* conformations scored per sequence */
    uint32_t n_class;     /* phenotypes */
    uint32_t n_selfrev;   /* classes holding a single (reversal-symmetric) conformation */
    uint32_t nbp;         /* non-bonded contacts of every compact structure */
    uint32_t K;           /* odd-separation pairs (i, j), j - i >= 3 */
    uint32_t W;           /* 32-bit words per contact bitmask, ceil(K/32) */
    uint32_t K_pad;       /* depth of the int8 product: K + unary rows + 2 index rows, to 32 */
    int32_t table[4];     /* contact energies {E_PP, E_PH, E_HP, E_HH} (integers) */
    uint32_t unary_rows;  /* N for a table with E_HP != E_PP, else 0 */
    uint32_t cmax;        /* largest number of contacts of one monomer in any structure */
} hp_info;

/*
 * hp_structures -- enumerate and symmetry-reduce the compact structures of
 * an X*Y*Z box (Methods, "HP and MJ lattice models": the library of folds is
 * the set of compact self-avoiding walks).  Use Z = 1 for a 2D box.
 * Host-only work.  *out receives a new immutable handle, safe to share
 * between threads; release it with hp_structs_free.
 * Errors: HP_EINVAL for dims < 1, N < 2, or a box with no Hamiltonian path;
 * HP_ERANGE if N > 36 or the class count does not fit below HP_NONE.
 */
hp_status hp_structures(int X, int Y, int Z, hp_structs **out);

/*
 * hp_structures_energy -- as hp_structures, with the general two-letter
 * contact energies of Eq. 1: table = {E_PP, E_PH, E_HP, E_HH}, integers (the
 * paper's Table 1 scaled by 10 is {0, -10, -10, -23}); hp_structures is the
 * table {0, 0, 0, -1}.  Energies reported by hp_enumerate are in the table's
 * units.  The table must be symmetric (E_PH == E_HP) and attractive:
 * E_HH - 2 E_HP + E_PP <= 0 and E_HP - E_PP <= 0, not both 0; its weights
 * must fit the int8 product (HP_EUNSUPPORTED otherwise) and the largest
 * energy range must stay below 2^14 units (HP_ERANGE).
 */
hp_status hp_structures_energy(int X, int Y, int Z, const int32_t table[4], hp_structs **out);
void hp_structs_free(hp_structs *s);
hp_status hp_structs_info(const hp_structs *s, hp_info *info);

/*
 * hp_structs_export -- copy the handle's tables to host buffers (any may be
 * NULL):  walks[n_conf*N] canonical site sequence of each conformation;
 * conf_to_class[n_conf]; rev_conf[n_conf] conformation of the reversed
 * chain; self_rev[n_class]; pairs[K*2] the (i, j) of each bitmask/row
 * position k; contacts[n_conf*nbp*2] the (i, j) contact pairs of each
 * conformation, i < j, ascending.
 */
hp_status hp_structs_export(const hp_structs *s, uint8_t *walks, uint16_t *conf_to_class,
                            uint32_t *rev_conf, uint8_t *self_rev, uint8_t *pairs,
                            uint8_t *contacts);

/*
 * Device workspace holding the packed structure tables the kernel forms
 * read (contact bitmasks, the int8 contact matrix in MFMA operand order, the
 * blocked form's 0/1 contact matrix where it applies, the pair table and the
 * conformation-to-class map).  hp_workspace_bytes gives
 * its size; hp_upload fills caller memory d_ws (>= that many bytes, 256-byte
 * aligned) asynchronously on `stream`.  The host source stays owned by the
 * handle, so the handle must outlive the copy (synchronise before freeing).
 */
size_t hp_workspace_bytes(const hp_structs *s);
hp_status hp_upload(const hp_structs *s, void *d_ws, size_t ws_bytes, void *stream);

/*
 * hp_enumerate -- ground states of every sequence s in [seq_lo, seq_hi)
 * (Methods: minimum of Eq. 1 over all folds; a sequence with no unique
 * minimum does not fold).  seq_hi <= 2^N.
 *   d_out[s - seq_lo]   phenotype (class id) or HP_NONE; may be NULL.
 *   d_emin[s - seq_lo]  minimum energy (int32, in the table's units); may be NULL.
 *   d_designability[q] += number of sequences in range with phenotype q
 *                         (n_class uint64 counters; may be NULL).
 *   d_nondesign[0]     += number of deleterious sequences (may be NULL).
 * `form` selects HP_FORM_POPCOUNT, HP_FORM_GEMM_I8 or HP_FORM_BLOCKED_I8.
 * d_ws must hold the uploaded workspace of the same handle.
 * Errors: HP_EINVAL (NULL handle/workspace, empty or out-of-range seq range,
 * unknown form), HP_EUNSUPPORTED (HP_FORM_BLOCKED_I8 for a handle it does not
 * cover), HP_EDEVICE (launch failure).
 */
hp_status hp_enumerate(const hp_structs *s, const void *d_ws, int form, uint64_t seq_lo,
                       uint64_t seq_hi, uint16_t *d_out, int32_t *d_emin,
                       uint64_t *d_designability, uint64_t *d_nondesign, void *stream);

/*
 * Reversal symmetry (Appendix B: the map is symmetric, so only half of the
 * sequence-structure relationships need computing).  Reversing the chain
 * maps the phenotype of s onto that of reverse(s) (bit i <-> bit N-1-i), so
 * it suffices to score the canonical sequences s <= reverse(s).
 *   hp_canonical_count   number of canonical sequences (2^(h-1)(2^h+1), times
 *                        2 for odd N, h = floor(N/2)): about half of 2^N.
 *   hp_enumerate_symmetric  as hp_enumerate over canonical indices
 *                        [t_lo, t_hi) (t_hi <= hp_canonical_count): each
 *                        canonical s fills d_out / d_emin at s AND at
 *                        reverse(s), so both are full 2^N-entry maps indexed
 *                        by sequence; designability and the deleterious count
 *                        add 2 for s != reverse(s) and 1 for palindromes.
 *                        Over [0, hp_canonical_count) the outputs equal those
 *                        of hp_enumerate over [0, 2^N).
 * Canonical index order: with s = (a, m, b) (high h bits, middle bit for odd
 * N, low h bits) and b' = reverse_h(b), s is canonical iff a <= b'.  Indices
 * run over m, then over row pairs p < 2^(h-1), each holding row b' = p
 * (a = 0 .. p) followed by row b' = 2^h - 1 - p (a = 0 .. 2^h - 1 - p), i.e.
 * 2^h + 1 sequences per pair.
 */
uint64_t hp_canonical_count(const hp_structs *s);
hp_status hp_enumerate_symmetric(const hp_structs *s, const void *d_ws, int form, uint64_t t_lo,
                                 uint64_t t_hi, uint16_t *d_out, int32_t *d_emin,
                                 uint64_t *d_designability, uint64_t *d_nondesign, void *stream);

/*
 * Reversal symmetry in the blocked form (HP_FORM_BLOCKED_I8 geometry; same
 * requirements).  Blocks are 256 sequences that differ only in the 8 middle
 * monomers (positions h .. h+7 for even N, h .. h+3 and h+5 .. h+8 around the
 * middle monomer for odd N, h = (N - 8 - N % 2) / 2); reversal maps blocks
 * onto blocks.  With a = the h highest monomers, b = the h lowest and b' =
 * reverse(b), the canonical blocks are those with a <= b'.
 *   hp_canonical_block_count   number of canonical blocks (0 when the
 *                        blocked form does not cover the handle): about
 *                        2^N / 512.
 *   hp_enumerate_symmetric_blocked  scores canonical blocks [b_lo, b_hi)
 *                        and fills d_out / d_emin (full 2^N-entry maps,
 *                        indexed by sequence) at every sequence s of the
 *                        block and, for blocks with a < b', at reverse(s);
 *                        designability and the deleterious count add 2 per
 *                        such s and 1 for the sequences of blocks with
 *                        a == b' (their reverses lie in the same block).
 *                        Over [0, hp_canonical_block_count) the outputs equal
 *                        those of hp_enumerate over [0, 2^N).
 * Block index order: over the middle monomer (odd N), then row pairs
 * p < 2^(h-1) of the (a, b') triangle, each holding row b' = p (a = 0 .. p)
 * followed by row b' = 2^h - 1 - p (a = 0 .. 2^h - 1 - p).
 * Errors: as hp_enumerate_symmetric; HP_EUNSUPPORTED as HP_FORM_BLOCKED_I8.
 */
uint64_t hp_canonical_block_count(const hp_structs *s);
hp_status hp_enumerate_symmetric_blocked(const hp_structs *s, const void *d_ws, uint64_t b_lo,
                                         uint64_t b_hi, uint16_t *d_out, int32_t *d_emin,
                                         uint64_t *d_designability, uint64_t *d_nondesign,
                                         void *stream);

/*
 * Reversal symmetry with wide blocks of HP_FORM_BLOCKED_I8 (pure pair
 * energies, N >= 10; hp_wide_block_count is 0 when a handle is not covered).
 * A wide block is 1024 sequences that differ only in the 10 monomers around
 * the middle: positions h .. h+9 for even N; for odd N positions h .. h+4
 * and h+6 .. h+10, the middle monomer h+5 staying outer; h = (N - 10 - N % 2)
 * / 2.  Reversal maps wide blocks onto wide blocks; with a = the h highest
 * monomers (and m the middle one for odd N), b = the h lowest and b' =
 * reverse(b), the canonical wide blocks are those with a <= b'.  One
 * workgroup of 4 waves scores a wide block, the first product of each
 * conformation tile computed once for all four waves.
 *   hp_wide_block_count  number of canonical wide blocks: about 2^N / 2048.
 *   hp_enumerate_symmetric_wide  scores canonical wide blocks [b_lo, b_hi)
 *                        and fills d_out / d_emin (full 2^N-entry maps,
 *                        indexed by sequence) at every sequence s of the
 *                        block and, for blocks with a < b', at reverse(s);
 *                        designability and the deleterious count add 2 per
 *                        such s and 1 for the sequences of blocks with
 *                        a == b'.  Over [0, hp_wide_block_count) the outputs
 *                        equal those of hp_enumerate over [0, 2^N).  Ranges
 *                        longer than 2^20 blocks run as several launches.
 * Block index order: as for hp_enumerate_symmetric_blocked (over m, then row
 * pairs p < 2^(h-1) of the (a, b') triangle, row b' = p then row
 * b' = 2^h - 1 - p).
 * Errors: HP_EINVAL for a NULL handle or workspace, an empty range or
 * b_hi > hp_wide_block_count; HP_EUNSUPPORTED for a handle wide blocks do not
 * cover; HP_EDEVICE for a failed launch.
 */
uint64_t hp_wide_block_count(const hp_structs *s);
hp_status hp_enumerate_symmetric_wide(const hp_structs *s, const void *d_ws, uint64_t b_lo,
                                      uint64_t b_hi, uint16_t *d_out, int32_t *d_emin,
                                      uint64_t *d_designability, uint64_t *d_nondesign,
                                      void *stream);

/*
 * Energy gap and threshold (Methods, end of "HP and MJ lattice models": the
 * threshold is the smallest difference between the lowest and second-lowest
 * fold energies that counts as distinguishable; closer than that, the
 * sequence does not fold).  With E1 <= E2 the two lowest conformation
 * energies of a sequence (E2 = E1 when the minimum is shared), in the units
 * of the handle's energy table:
 *   gap     = E2 - E1, saturated at 255; 255 when the box has one
 *             conformation;
 *   folds   iff gap >= threshold (threshold 1 .. 255; 1 is the uniqueness
 *             rule of hp_enumerate, and integer energies make the two equal).
 * hp_enumerate_gap  as hp_enumerate, plus the threshold and an optional
 *                   uint8 d_gap[seq_hi - seq_lo] (device, caller-owned).
 *                   Designability counts folding sequences only; every other
 *                   sequence is deleterious (out = HP_NONE).
 * hp_sample         the random-sampling mode (Methods: sequences are sampled
 *                   where enumerating all is out of reach), with the sequence
 *                   draws made on the device.  Draw i (idx_lo <= i < idx_hi
 *                   <= 2^48) is the low N bits of output i of the splitmix64
 *                   generator (Steele, Lea and Flood, OOPSLA 2014) seeded
 *                   with `seed`: z = seed + (i + 1) * 0x9E3779B97F4A7C15,
 *                   then the variant-13 finaliser (xor-shift 30, multiply
 *                   0xBF58476D1CE4E5B9, xor-shift 27, multiply
 *                   0x94D049BB133111EB, xor-shift 31).  Every monomer is H
 *                   with probability 1/2, independently.  Per-draw outputs are
 *                   indexed by i - idx_lo: d_seqs (uint64, the drawn
 *                   sequence), d_out, d_emin, d_gap, each optional.  Draws are
 *                   with replacement; designability counts draws.
 * Errors: as hp_enumerate; HP_EINVAL also for a threshold outside 1 .. 255,
 * an empty draw range or idx_hi > 2^48.
 */
hp_status hp_enumerate_gap(const hp_structs *s, const void *d_ws, int form, uint64_t seq_lo,
                           uint64_t seq_hi, int32_t threshold, uint16_t *d_out, int32_t *d_emin,
                           uint8_t *d_gap, uint64_t *d_designability, uint64_t *d_nondesign,
                           void *stream);
hp_status hp_sample(const hp_structs *s, const void *d_ws, int form, uint64_t seed,
                    uint64_t idx_lo, uint64_t idx_hi, int32_t threshold, uint64_t *d_seqs,
                    uint16_t *d_out, int32_t *d_emin, uint8_t *d_gap, uint64_t *d_designability,
                    uint64_t *d_nondesign, void *stream);

/*
 * Batched launch: several enumeration jobs, possibly of different lattices
 * and uneven sizes, from one work list of fixed-size items (256 sequences
 * for HP_FORM_GEMM_I8; for HP_FORM_BLOCKED_I8 one wide block where wide
 * blocks apply and the selected staging mode is -1 or 3 -- of 2048 when the
 * job's range ends are multiples of 2^17, N >= 17 and 8 waves are allowed
 * (mode -1, or nw 8), else of 1024 -- otherwise 4 blocks of 256).  Jobs are grouped by product depth (hp_info.K_pad; blocked: also
 * by wide blocks and unary rows) and each group is one kernel launch,
 * compiled for that depth, with one workgroup per item; the groups
 * are enqueued back to back on `stream`.  HP_FORM_POPCOUNT runs the jobs as
 * separate hp_enumerate calls.  Each job has the meaning of one hp_enumerate
 * call.  d_batch_ws is caller device memory of hp_batch_workspace_bytes(njobs)
 * bytes holding the work list (rewritten by every call).  The work list is
 * copied to d_batch_ws on `stream`, after the work already queued there
 * (which may still read an earlier work list), and the call waits for that
 * copy before enqueueing the launches: it returns once `stream` has drained
 * up to the copy.  Calls on other streams that share d_batch_ws must be
 * ordered by the caller.
 * Errors: as hp_enumerate, for any job; HP_EINVAL if njobs < 1 or the
 * workspace is too small; HP_EUNSUPPORTED if a job's handle is not covered
 * by HP_FORM_BLOCKED_I8.
 */
typedef struct {
    const hp_structs *structs;
    const void *d_ws;
    uint64_t seq_lo, seq_hi;
    uint16_t *d_out;
    int32_t *d_emin;
    uint64_t *d_designability;
    uint64_t *d_nondesign;
} hp_job;

size_t hp_batch_workspace_bytes(int njobs);
hp_status hp_enumerate_batch(const hp_job *jobs, int njobs, int form, void *d_batch_ws,
                             size_t batch_ws_bytes, void *stream);

/*
 * Captured launches: hp_graph_capture_batch records the device work of
 * hp_enumerate_batch (the per-depth kernel launches; no memsets) into a
 * hipGraph once, for HP_FORM_GEMM_I8 or HP_FORM_BLOCKED_I8; hp_graph_launch
 * replays it on `stream`.  The work list is uploaded at capture time, after
 * the device has finished all queued work (hipDeviceSynchronize), and must
 * stay in d_batch_ws while the graph is used.  Designability counters
 * accumulate on every replay.
 */
typedef struct hp_graph hp_graph;
hp_status hp_graph_capture_batch(const hp_job *jobs, int njobs, int form, void *d_batch_ws,
                                 size_t batch_ws_bytes, hp_graph **out);
hp_status hp_graph_launch(hp_graph *g, void *stream);
void hp_graph_free(hp_graph *g);

/*
 * hp_enumerate_batch_static -- hp_enumerate_batch for callers that cannot
 * allocate device memory (code under hipGraph capture, tight serving loops,
 * harnesses that forbid allocation).  It takes no workspace: the work list
 * lives in a device array of the library, one per GPU, sized for
 * HP_STATIC_BATCH_MAX_JOBS jobs (about 10 KiB) and held until the process
 * ends; every call on that GPU rewrites it.  The call allocates nothing: the
 * list reaches the array through kernel launches on `stream`, in stream
 * order after the work already queued there, and the call does not wait.
 * Calls that overlap on one GPU (different streams, not ordered by the
 * caller) race on the shared array.  Outputs and accumulation are those of
 * hp_enumerate_batch with the same jobs and form.
 * Errors: as hp_enumerate_batch; HP_ERANGE if njobs > HP_STATIC_BATCH_MAX_JOBS
 * (checked before any device call).
 */
#define HP_STATIC_BATCH_MAX_JOBS 32
hp_status hp_enumerate_batch_static(const hp_job *jobs, int njobs, int form, void *stream);

/*
 * Launch shape of HP_FORM_BLOCKED_I8: every wave scores one block of 256
 * sequences.  hp_blocked_select sets, process-wide, the waves per workgroup
 * nw (2, 4 or 8; default 4; the waves of a workgroup share each staged
 * contact tile) and the staging mode (0: double-buffered LDS; 1:
 * triple-buffered LDS with the block-level product of the next tile issued
 * while the current tile's keys are updated; 2: as 0, with the per-sequence
 * operand of the second product read from LDS instead of held in registers;
 * 3: wide blocks, one first product per conformation tile shared by the
 * waves of a workgroup: with nw = 8, where both ends of the range are
 * multiples of 2^17 and N >= 17, 2048 sequences (monomers 0 .. 4 and 6, 8,
 * .., 16 vary) per workgroup of 8 waves, otherwise 1024 sequences sharing
 * every monomer above the low 10 per workgroup of 4 waves; with nw = 4
 * always the latter -- pure pair energies over plain ranges only, elsewhere
 * mode 3 acts as -1; -1, default: 3 with 8 waves where wide blocks apply,
 * else 2 for K_pad <= 192, else 0).  hp_blocked_selected
 * reports them (either pointer may be NULL).  Results never depend on the
 * shape.
 * Errors: HP_EINVAL for another value, or mode 3 with nw = 2.
 */
hp_status hp_blocked_select(int nw, int mode);
void hp_blocked_selected(int *nw, int *mode);
/*
 * hp_autotune_blocked -- time the launch shapes of HP_FORM_BLOCKED_I8
 * (entries 0 .. 8: nw = 2, 4, 8 x mode = 0, 1, 2, entry i is nw =
 * {2,4,8}[i / 3], mode = i % 3; entry 9: wide blocks, nw 8, mode 3, where
 * they apply, else ms[9] = -1) on sequences [seq_lo, seq_lo + n_seq) (no
 * outputs written, `repeats` launches each after one warm-up), select the
 * fastest process-wide, and report per-shape milliseconds in ms[10] and the
 * choice (any pointer may be NULL).  Synchronises `stream`.
 * Errors: HP_EUNSUPPORTED for a handle the blocked form does not cover;
 * HP_EINVAL for a range outside [0, 2^N); HP_EDEVICE for a failed launch.
 */
hp_status hp_autotune_blocked(const hp_structs *s, const void *d_ws, uint64_t seq_lo,
                              uint64_t n_seq, int repeats, float *ms, int *best_nw,
                              int *best_mode, void *stream);

/*
 * Tile shapes of the int8 form and their autotuning.  Several shapes are
 * compiled per product depth K_pad (hp_info.K_pad).  A shape is (T, NW, mode):
 * T sequence tiles of 32 per wave, NW waves per workgroup, and mode 0 when
 * the contact-matrix tiles are staged through LDS by the workgroup, 1 when
 * every wave loads them from global memory itself, 2 when they are staged
 * through LDS and each wave overlaps the products of one tile with the key
 * updates of the previous one.  The choice is
 * process-wide per K_pad and shared by all threads; the first listed shape is
 * the default.  The launch configuration never changes results, only speed.
 *   hp_gemm_shape_count  number of compiled shapes for K_pad (0 if none);
 *   hp_gemm_shape_info   describe shape idx (any out pointer may be NULL);
 *   hp_gemm_select       make shape idx the choice for K_pad;
 *   hp_gemm_selected     current choice for K_pad (-1 if none compiled);
 *   hp_autotune          time every shape of the handle's K_pad on sequences
 *                        [seq_lo, seq_lo + n_seq) (no outputs written,
 *                        `repeats` launches each after one warm-up), select
 *                        the fastest, write per-shape milliseconds to ms[]
 *                        (hp_gemm_shape_count entries, may be NULL) and its
 *                        index to *best (may be NULL).  Synchronises `stream`.
 *                        If the environment variable HP_TUNE_CACHE names a
 *                        file, the choice is recorded there and read back by
 *                        later processes on first use of that K_pad.
 * Errors: HP_EINVAL for an unknown shape, NULL handle/workspace or a range
 * outside [0, 2^N); HP_EDEVICE for a failed launch.
 */
int hp_gemm_shape_count(uint32_t K_pad);
hp_status hp_gemm_shape_info(uint32_t K_pad, int idx, int *T, int *NW, int *mode);
hp_status hp_gemm_select(uint32_t K_pad, int idx);
int hp_gemm_selected(uint32_t K_pad);
hp_status hp_autotune(const hp_structs *s, const void *d_ws, uint64_t seq_lo, uint64_t n_seq,
                      int repeats, float *ms, int *best, void *stream);

/*
 * hp_neighbors -- single-point-mutation statistics of a complete map
 * (Eq. 2: phi_pq; robustness rho_q = phi_qq; phi_del).  d_map holds the
 * phenotype of all 2^N sequences.  For every designing genotype g with
 * phenotype q and each of its N one-bit mutants p:
 *   d_neutral[q] += (p == q);  d_deleterious[q] += (p == HP_NONE);
 *   d_other[q]   += otherwise.
 * The ratios of Eq. 2 are these counts divided by N * N_q.  If phi_q >= 0,
 * d_phi_row[p] (p < n_class) and d_phi_row[n_class] (deleterious) += the
 * mutants of phi_q-genotypes, i.e. the numerators of phi_{p,phi_q}.
 * Counters are uint64 arrays of n_class (n_class + 1 for the row); any may
 * be NULL.  Errors: HP_EINVAL for NULL map or phi_q >= n_class.
 * A 16-byte aligned d_map with N >= 3 is read eight genotypes per lane (one
 * 16-byte load per mutant bit); any other map one genotype per lane.  The
 * results are the same; the same holds for hp_phi_counts and hp_components.
 */
hp_status hp_neighbors(const hp_structs *s, const uint16_t *d_map, uint64_t *d_neutral,
                       uint64_t *d_deleterious, uint64_t *d_other, int32_t phi_q,
                       uint64_t *d_phi_row, void *stream);

/*
 * hp_phi_counts -- the whole phi_pq matrix of Eq. 2 (every pair of
 * phenotypes, not one row) as counts.  d_map holds the phenotype of all 2^N
 * sequences.  d_counts is a row-major uint64 matrix of n_class rows and
 * n_class + 1 columns owned by the caller (n_class (n_class + 1) 8 bytes:
 * 21.4 GB for the 51704 classes of 3x3x3, 6.6 GB for 6x6).  For every
 * genotype g of phenotype q < n_class and each of its N one-bit mutants of
 * phenotype p: d_counts[q (n_class + 1) + p] += 1, with p replaced by
 * n_class when it is HP_NONE or not below n_class (deleterious).  Hence
 * phi_pq = counts[q][p] / (N N_q), the diagonal is the robustness numerator,
 * column n_class the numerator of phi_del, and row q equals the d_phi_row
 * of hp_neighbors with phi_q = q.  Counts accumulate: zero the matrix first.
 * Asynchronous on `stream`.
 * Errors: HP_EINVAL for a NULL handle, map or matrix; HP_EDEVICE.
 *
 * hp_phi_sparse -- compressed rows of such a matrix: d_row_ptr (n_class + 1
 * uint64, caller-owned) receives the row offsets, d_cols (uint32) and d_vals
 * (uint64) the non-zero entries of each row in ascending column order, up to
 * `capacity` entries.  *nnz (may be NULL) receives the number of non-zero
 * entries.  With d_cols and d_vals both NULL only d_row_ptr and *nnz are
 * produced (a size query).  Synchronises `stream` once to read the count,
 * so it cannot be captured into a graph.
 * Errors: HP_EINVAL for a NULL handle, matrix or row_ptr, or only one of
 * d_cols / d_vals NULL; HP_ERANGE when capacity < nnz (nothing written
 * beyond d_row_ptr); HP_EDEVICE.
 */
hp_status hp_phi_counts(const hp_structs *s, const uint16_t *d_map, uint64_t *d_counts,
                        void *stream);
hp_status hp_phi_sparse(const hp_structs *s, const uint64_t *d_counts, uint64_t *d_row_ptr,
                        uint32_t *d_cols, uint64_t *d_vals, uint64_t capacity, uint64_t *nnz,
                        void *stream);

/*
 * hp_components -- neutral networks: connected components of the subgraph
 * of the N-cube of sequences (edges = single point mutations) induced on
 * genotypes of equal designing phenotype (the Introduction's two pictures
 * of how phenotypes lie in genotype space, and neutral networks in the
 * Results).
 *   d_labels[g]   smallest genotype of g's component, 0xFFFFFFFF if g is
 *                 deleterious (2^N entries, overwritten);
 *   d_compsize[g] size of the component whose smallest genotype is g, 0 for
 *                 every other g (2^N entries, overwritten);
 *   d_ncomp[q]    number of components of phenotype q (n_class, overwritten);
 *   d_largest[q]  size of q's largest component (n_class, overwritten).
 * d_ncomp and d_largest may be NULL.  Requires N <= 31.
 * Errors: HP_EINVAL for NULL labels/compsize/map; HP_ERANGE for N > 31.
 */
hp_status hp_components(const hp_structs *s, const uint16_t *d_map, uint32_t *d_labels,
                        uint32_t *d_compsize, uint32_t *d_ncomp, uint32_t *d_largest,
                        void *stream);

/* Thread-local text of the last failure ("" if none). */
const char *hp_last_error(void);

/* Library version string. */
const char *hp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* HP_H */
