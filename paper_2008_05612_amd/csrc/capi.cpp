// C ABI of libhpmap: argument checking, error reporting, workspace upload,
// the sequence block loop, batched launches and their hipGraph capture.
// Every entry point returns hp_status; no call exits or throws across the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "hp_internal.h"
#include "kernels.h"

namespace hpmap {

namespace {
thread_local std::string g_last_error;

// Sequences per kernel launch of hp_enumerate; longer ranges are streamed as
// a loop of such blocks (the full 6x6 map is 64 blocks).
constexpr uint64_t kBlockSeqs = uint64_t(1) << 30;
constexpr uint64_t kMaxDraws = uint64_t(1) << 48;   // sampled-mode indices per seed

hp_status device_fail(hipError_t e, const char *what)
{
    return fail(HP_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

hp_status check_range(const hp_structs *s, const void *d_ws, uint64_t lo, uint64_t hi)
{
    if (!s)
        return fail(HP_EINVAL, "structures handle is NULL");
    if (!d_ws)
        return fail(HP_EINVAL, "workspace pointer is NULL");
    const uint64_t space = uint64_t(1) << s->N;
    if (lo >= hi)
        return fail(HP_EINVAL, "empty sequence range (seq_lo >= seq_hi)");
    if (hi > space)
        return fail(HP_EINVAL, "seq_hi exceeds 2^N");
    return HP_OK;
}

}  // namespace

// Work list of a batch, written into caller buffers (no allocation): jobs
// ordered by product depth (stable), items of gemm_batch_seqs_per_item()
// sequences (dense form) or of blk_batch_seqs_per_item() sequences in whole
// 256-sequence blocks (blocked form), and the item range of each depth.
hp_status plan_batch(const hp_job *jobs, int njobs, int form, size_t ws_bytes, char *host,
                     int *order, int64_t *start, BatchGroup *groups, int *ngroups)
{
    if (!jobs || njobs < 1)
        return fail(HP_EINVAL, "batch needs at least one job");
    if (ws_bytes < hp_batch_workspace_bytes(njobs))
        return fail(HP_EINVAL, "batch workspace too small");
    const bool blocked = form == HP_FORM_BLOCKED_I8;
    int kb_max = 1;
    for (int i = 0; i < njobs; ++i) {
        hp_status st = check_range(jobs[i].structs, jobs[i].d_ws, jobs[i].seq_lo, jobs[i].seq_hi);
        if (st != HP_OK)
            return st;
        if (blocked && !jobs[i].structs->blk_ok)
            return fail(HP_EUNSUPPORTED, "the blocked form needs N >= 8, per-block bytes "
                                         "within int8 and, with unary rows, depth <= 256");
        kb_max = std::max(kb_max, int(jobs[i].structs->K_pad / 32));
    }
    // blocked jobs group by depth, by whether they carry unary rows and by
    // the wide blocks they run as (0 none, 1 of 1024, 2 of 2048): key
    // 8 depth + 2 wide + unary
    auto wide_kind = [&](int i) {
        const hp_job &jb = jobs[i];
        return blk_batch_wide8(jb.structs, jb.seq_lo, jb.seq_hi) ? 2u
               : blk_batch_wide(jb.structs)                         ? 1u
                                                                    : 0u;
    };
    auto depth = [&](int i) {
        const hp_structs *t = jobs[i].structs;
        return int(blocked ? 8 * t->blk_KB + 2 * wide_kind(i) + (t->blk_coefB != 0 ? 1u : 0u)
                           : t->K_pad / 32);
    };
    // stable insertion sort by depth (batches hold a handful of jobs)
    for (int r = 0; r < njobs; ++r) {
        int k = r;
        while (k > 0 && depth(order[k - 1]) > depth(r)) {
            order[k] = order[k - 1];
            --k;
        }
        order[k] = r;
    }
    start[0] = 0;
    for (int r = 0; r < njobs; ++r) {
        const hp_job &jb = jobs[order[r]];
        uint64_t items;
        if (blocked && wide_kind(order[r]) == 2) {
            items = ((jb.seq_hi - jb.seq_lo) >> kWide11ChunkBits) << 6;
        } else if (blocked && blk_batch_wide(jb.structs)) {
            items = ((jb.seq_hi - 1) >> kWideBits) - (jb.seq_lo >> kWideBits) + 1;
        } else if (blocked) {
            const uint64_t nblk = ((jb.seq_hi - 1) >> kBlkBits) - (jb.seq_lo >> kBlkBits) + 1;
            const uint64_t per = blk_batch_seqs_per_item() >> kBlkBits;
            items = (nblk + per - 1) / per;
        } else {
            const uint64_t per = gemm_batch_seqs_per_item();
            items = (jb.seq_hi - jb.seq_lo + per - 1) / per;
        }
        start[r + 1] = start[r] + int64_t(items);
    }
    if (start[njobs] > INT32_MAX)
        return fail(HP_ERANGE, "batch has too many work items");
    std::memset(host, 0, hp_batch_workspace_bytes(njobs));
    BatchHeader hdr{};
    hdr.reserved = 0;
    hdr.njobs = njobs;
    hdr.n_items = int32_t(start[njobs]);
    hdr.kb_max = kb_max;
    std::memcpy(host, &hdr, sizeof(hdr));
    char *ej = host + sizeof(BatchHeader);
    int ng = 0;
    for (int r = 0; r < njobs; ++r) {
        const hp_job &jb = jobs[order[r]];
        const EnumJob j = make_enum_job(jb.structs, jb.d_ws, jb.seq_lo, jb.seq_hi, jb.d_out,
                                        jb.d_emin, jb.d_designability, jb.d_nondesign);
        std::memcpy(ej + sizeof(EnumJob) * r, &j, sizeof(EnumJob));
        const int kb = depth(order[r]);
        if (ng == 0 || groups[ng - 1].kb != kb)
            groups[ng++] = {kb, int(start[r]), int(start[r])};
        groups[ng - 1].item_hi = int(start[r + 1]);
    }
    std::memcpy(host + sizeof(BatchHeader) + sizeof(EnumJob) * njobs, start,
                sizeof(int64_t) * (njobs + 1));
    *ngroups = ng;
    return HP_OK;
}

// One launch per product depth of the plan, in order on `st`.
hipError_t launch_plan(const BatchGroup *groups, int ngroups, int form, void *d_batch_ws,
                       hipStream_t st)
{
    for (int i = 0; i < ngroups; ++i) {
        const BatchGroup &g = groups[i];
        if (g.item_hi <= g.item_lo)
            continue;
        hipError_t e = form == HP_FORM_BLOCKED_I8
                           ? launch_gemm_blk_batch(d_batch_ws, g.kb >> 3, (g.kb & 1) != 0,
                                                   (g.kb >> 1) & 3, g.item_lo, g.item_hi, st)
                           : launch_gemm_batch(d_batch_ws, g.kb, g.item_lo, g.item_hi, st);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

namespace {

// Host side of a batch plan: the work list bytes and the launch groups.
struct BatchPlan {
    std::vector<char> host;
    std::vector<int> order;
    std::vector<int64_t> start;
    std::vector<BatchGroup> groups;
    int ngroups = 0;

    hp_status make(const hp_job *jobs, int njobs, int form, size_t ws_bytes)
    {
        if (!jobs || njobs < 1)
            return fail(HP_EINVAL, "batch needs at least one job");
        host.assign(hp_batch_workspace_bytes(njobs), 0);
        order.assign(njobs, 0);
        start.assign(njobs + 1, 0);
        groups.assign(njobs, BatchGroup{});
        return plan_batch(jobs, njobs, form, ws_bytes, host.data(), order.data(), start.data(),
                          groups.data(), &ngroups);
    }
};

}  // namespace


// Block geometry fields of a job (the blocked form).
static void set_block_geometry(EnumJob &j, const hp_structs *s, bool canonical)
{
    const BlockGeometry g = block_geometry(s->N, canonical);
    j.blk_vmask = 0;
    j.blk_pos = 0;
    for (int x = 0; x < 8; ++x) {
        j.blk_vmask |= uint64_t(1) << g.pos[x];
        j.blk_pos |= uint64_t(g.pos[x]) << (8 * x);
    }
    j.blk_pp[0] = j.blk_pp[1] = j.blk_pp[2] = 0;
    for (int n = 0; n < g.npp; ++n)
        j.blk_pp[n / 8] |= uint64_t(g.pa[n] | (g.pb[n] << 4)) << (8 * (n % 8));
    j.blk_npp = g.npp;
    j.blk_KB = int32_t(s->blk_KB);
    j.blk_coefB = s->blk_coefB;
    j.blk_ngroups = s->blk_ngroups[canonical ? 1 : 0];
    for (int w = 0; w < 3; ++w)
        j.blk_grp[w] = s->blk_grp[canonical ? 1 : 0][w];
    j.half_bits = canonical ? g.half : s->N / 2;
    j.blk_s2 = j.gemm_b ? reinterpret_cast<const int8_t *>(j.gemm_b) +
                              (s->ws.blk_s2 - s->ws.gemm_b) + (canonical ? 8 * 64 * 16 : 0)
                        : nullptr;
}

EnumJob make_enum_job(const hp_structs *s, const void *d_ws, uint64_t lo, uint64_t hi, uint16_t *out,
                 int32_t *emin, uint64_t *desig, uint64_t *nondesign)
{
    const char *base = static_cast<const char *>(d_ws);
    EnumJob j{};
    j.c2q = reinterpret_cast<const uint16_t *>(base + s->ws.c2q);
    j.pairs = reinterpret_cast<const uint8_t *>(base + s->ws.pairs);
    j.masks = reinterpret_cast<const uint32_t *>(base + s->ws.masks);
    j.gemm_a = reinterpret_cast<const int8_t *>(base + s->ws.gemm_a);
    j.gemm_b = reinterpret_cast<const int8_t *>(base + s->ws.gemm_b);
    j.wide_s2 = s->wide_ok ? reinterpret_cast<const int8_t *>(base + s->ws.wide_s2) : nullptr;
    j.blk_shift = int32_t(s->blk_shift);
    j.blk_win_tiles = int32_t(s->blk_win_tiles);
    j.blk_coef = s->blk_coef;
    j.out = out;
    j.emin = emin;
    j.desig = reinterpret_cast<unsigned long long *>(desig);
    j.nondesign = reinterpret_cast<unsigned long long *>(nondesign);
    j.lo = lo;
    j.hi = hi;
    j.N = s->N;
    j.K = int32_t(s->K);
    j.W = int32_t(s->W);
    j.KB = int32_t(s->K_pad / 32);
    j.n_conf = int32_t(s->n_conf);
    j.n_tiles = int32_t((s->n_conf + kTileConf - 1) / kTileConf);
    j.U = int32_t(s->U);
    j.win_tiles = int32_t(s->win_tiles);
    j.win_shift = int32_t(s->win_shift);
    j.A = s->A;
    j.B = s->B;
    j.e0 = s->e0;
    j.planes = int32_t(s->planes);
    j.uw = int32_t(s->uw);
    j.MW = int32_t(s->MW);
    j.mode = kSeqPlain;
    j.threshold = 1;
    set_block_geometry(j, s, false);
    return j;
}

hp_status fail(hp_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

}  // namespace hpmap

struct hp_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

using namespace hpmap;

extern "C" {

const char *hp_last_error(void) { return g_last_error.c_str(); }

const char *hp_version(void) { return "hpmap 0.1 (gfx950)"; }

hp_status hp_structures(int X, int Y, int Z, hp_structs **out)
{
    static const int32_t pure_hp[4] = {0, 0, 0, -1};
    return hp_structures_energy(X, Y, Z, pure_hp, out);
}

hp_status hp_structures_energy(int X, int Y, int Z, const int32_t table[4], hp_structs **out)
{
    if (!out)
        return fail(HP_EINVAL, "out pointer is NULL");
    *out = nullptr;
    if (!table)
        return fail(HP_EINVAL, "energy table is NULL");
    hp_structs *s = new (std::nothrow) hp_structs();
    if (!s)
        return fail(HP_ENOMEM, "out of host memory");
    std::string msg;
    hp_status st;
    try {
        st = build_structures(X, Y, Z, table, s, &msg);
    } catch (const std::bad_alloc &) {
        st = HP_ENOMEM;
        msg = "out of host memory";
    }
    if (st != HP_OK) {
        delete s;
        return fail(st, msg);
    }
    *out = s;
    return HP_OK;
}

void hp_structs_free(hp_structs *s) { delete s; }

hp_status hp_structs_info(const hp_structs *s, hp_info *info)
{
    if (!s || !info)
        return fail(HP_EINVAL, "NULL argument");
    info->X = s->X;
    info->Y = s->Y;
    info->Z = s->Z;
    info->N = s->N;
    info->group_order = s->G;
    info->n_walks = s->n_walks;
    info->n_conf = s->n_conf;
    info->n_class = s->n_class;
    info->n_selfrev = s->n_selfrev;
    info->nbp = s->nbp;
    info->K = s->K;
    info->W = s->W;
    info->K_pad = s->K_pad;
    for (int q = 0; q < 4; ++q)
        info->table[q] = s->table[q];
    info->unary_rows = s->U;
    info->cmax = s->cmax;
    return HP_OK;
}

hp_status hp_structs_export(const hp_structs *s, uint8_t *walks, uint16_t *conf_to_class,
                            uint32_t *rev_conf, uint8_t *self_rev, uint8_t *pairs,
                            uint8_t *contacts)
{
    if (!s)
        return fail(HP_EINVAL, "structures handle is NULL");
    if (walks)
        std::memcpy(walks, s->walks.data(), s->walks.size());
    if (conf_to_class)
        std::memcpy(conf_to_class, s->c2q.data(), s->c2q.size() * 2);
    if (rev_conf)
        std::memcpy(rev_conf, s->rev_conf.data(), s->rev_conf.size() * 4);
    if (self_rev)
        std::memcpy(self_rev, s->self_rev.data(), s->self_rev.size());
    if (pairs)
        std::memcpy(pairs, s->pairs.data(), s->pairs.size());
    if (contacts)
        std::memcpy(contacts, s->contacts.data(), s->contacts.size());
    return HP_OK;
}

size_t hp_workspace_bytes(const hp_structs *s) { return s ? s->ws.total : 0; }

hp_status hp_upload(const hp_structs *s, void *d_ws, size_t ws_bytes, void *stream)
{
    if (!s || !d_ws)
        return fail(HP_EINVAL, "NULL argument");
    if (ws_bytes < s->ws.total)
        return fail(HP_EINVAL, "workspace smaller than hp_workspace_bytes()");
    if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0)
        return fail(HP_EINVAL, "workspace must be 256-byte aligned");
    hipStream_t st = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(d_ws);
    struct Part { size_t off; const void *src; size_t bytes; } parts[] = {
        {s->ws.c2q, s->c2q.data(), s->c2q.size() * 2},
        {s->ws.pairs, s->pair_rows.data(), s->pair_rows.size()},
        {s->ws.masks, s->masks.data(), s->masks.size() * 4},
        {s->ws.gemm_a, s->gemm_a.data(), s->gemm_a.size()},
        {s->ws.gemm_b, s->gemm_b.data(), s->gemm_b.size()},
        {s->ws.blk_s2, s->blk_s2.data(), s->blk_s2.size()},
        {s->ws.wide_s2, s->wide_s2.data(), s->wide_s2.size()},
    };
    for (const Part &p : parts) {
        if (!p.bytes)
            continue;
        hipError_t e = hipMemcpyAsync(base + p.off, p.src, p.bytes, hipMemcpyHostToDevice, st);
        if (e != hipSuccess)
            return device_fail(e, "hp_upload");
    }
    return HP_OK;
}

namespace {

// Options of one enumeration call beyond the plain map.
struct RunOpts {
    int mode = kSeqPlain;
    int threshold = 1;
    uint64_t seed = 0;
    uint8_t *gap = nullptr;
    uint64_t *seqs = nullptr;
};

// Launches [lo, hi) in blocks of kBlockSeqs indices.  Per-index outputs are
// offset by the block's position (plain and sampled modes); the designability
// counters accumulate.
hp_status run_blocks(const hp_structs *s, const void *d_ws, int form, uint64_t lo_all,
                     uint64_t hi_all, uint16_t *d_out, int32_t *d_emin, uint64_t *d_designability,
                     uint64_t *d_nondesign, const RunOpts &o, void *stream, const char *what)
{
    if (form != HP_FORM_POPCOUNT && form != HP_FORM_GEMM_I8 && form != HP_FORM_BLOCKED_I8)
        return fail(HP_EINVAL, "unknown kernel form");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const GemmVariant *var = nullptr;
    if (form == HP_FORM_GEMM_I8 && !(var = gemm_selected_variant(int(s->K_pad / 32))))
        return fail(HP_EUNSUPPORTED, "no compiled int8 kernel for this K_pad");
    if (form == HP_FORM_BLOCKED_I8) {
        if (o.mode != kSeqPlain)
            return fail(HP_EUNSUPPORTED, "the blocked form scores plain sequence ranges only");
        if (!s->blk_ok)
            return fail(HP_EUNSUPPORTED, "the blocked form needs N >= 8, per-block bytes "
                                         "within int8 and, with unary rows, depth <= 256");
    }
    for (uint64_t lo = lo_all; lo < hi_all;) {
        const uint64_t hi = hi_all - lo > kBlockSeqs ? lo + kBlockSeqs : hi_all;
        const uint64_t off = lo - lo_all;
        const bool local = o.mode != kSeqCanonical;   // canonical mode writes full-size maps
        EnumJob j = make_enum_job(s, d_ws, lo, hi, d_out && local ? d_out + off : d_out,
                                  d_emin && local ? d_emin + off : d_emin, d_designability,
                                  d_nondesign);
        j.mode = o.mode;
        j.threshold = o.threshold;
        j.seed = o.seed;
        j.gap = o.gap && local ? o.gap + off : o.gap;
        j.seqs = o.seqs ? o.seqs + off : nullptr;
        hipError_t e = form == HP_FORM_POPCOUNT ? launch_popcount(j, hs)
                       : form == HP_FORM_BLOCKED_I8 ? launch_gemm_blocked(j, blocked_selected_nw(), blocked_selected_mode(), hs)
                                                    : var->launch(j, hs);
        if (e != hipSuccess)
            return device_fail(e, what);
        lo = hi;
    }
    return HP_OK;
}

}  // namespace

hp_status hp_enumerate(const hp_structs *s, const void *d_ws, int form, uint64_t seq_lo,
                       uint64_t seq_hi, uint16_t *d_out, int32_t *d_emin,
                       uint64_t *d_designability, uint64_t *d_nondesign, void *stream)
{
    hp_status st = check_range(s, d_ws, seq_lo, seq_hi);
    if (st != HP_OK)
        return st;
    return run_blocks(s, d_ws, form, seq_lo, seq_hi, d_out, d_emin, d_designability, d_nondesign,
                      RunOpts{}, stream, "hp_enumerate launch");
}

hp_status hp_enumerate_gap(const hp_structs *s, const void *d_ws, int form, uint64_t seq_lo,
                           uint64_t seq_hi, int32_t threshold, uint16_t *d_out, int32_t *d_emin,
                           uint8_t *d_gap, uint64_t *d_designability, uint64_t *d_nondesign,
                           void *stream)
{
    hp_status st = check_range(s, d_ws, seq_lo, seq_hi);
    if (st != HP_OK)
        return st;
    if (threshold < 1 || threshold > 255)
        return fail(HP_EINVAL, "threshold must be in 1 .. 255");
    RunOpts o;
    o.threshold = threshold;
    o.gap = d_gap;
    return run_blocks(s, d_ws, form, seq_lo, seq_hi, d_out, d_emin, d_designability, d_nondesign,
                      o, stream, "hp_enumerate_gap launch");
}

hp_status hp_sample(const hp_structs *s, const void *d_ws, int form, uint64_t seed,
                    uint64_t idx_lo, uint64_t idx_hi, int32_t threshold, uint64_t *d_seqs,
                    uint16_t *d_out, int32_t *d_emin, uint8_t *d_gap, uint64_t *d_designability,
                    uint64_t *d_nondesign, void *stream)
{
    if (!s)
        return fail(HP_EINVAL, "structures handle is NULL");
    if (!d_ws)
        return fail(HP_EINVAL, "workspace pointer is NULL");
    if (idx_lo >= idx_hi)
        return fail(HP_EINVAL, "empty draw range (idx_lo >= idx_hi)");
    if (idx_hi > kMaxDraws)
        return fail(HP_EINVAL, "idx_hi exceeds 2^48 draws per seed");
    if (threshold < 1 || threshold > 255)
        return fail(HP_EINVAL, "threshold must be in 1 .. 255");
    RunOpts o;
    o.mode = kSeqSampled;
    o.threshold = threshold;
    o.seed = seed;
    o.gap = d_gap;
    o.seqs = d_seqs;
    return run_blocks(s, d_ws, form, idx_lo, idx_hi, d_out, d_emin, d_designability, d_nondesign,
                      o, stream, "hp_sample launch");
}

uint64_t hp_canonical_count(const hp_structs *s)
{
    if (!s)
        return 0;
    const uint64_t side = uint64_t(1) << (s->N / 2);
    return side * (side + 1) / 2 * (s->N % 2 ? 2 : 1);
}

hp_status hp_enumerate_symmetric(const hp_structs *s, const void *d_ws, int form, uint64_t t_lo,
                                 uint64_t t_hi, uint16_t *d_out, int32_t *d_emin,
                                 uint64_t *d_designability, uint64_t *d_nondesign, void *stream)
{
    if (!s)
        return fail(HP_EINVAL, "structures handle is NULL");
    if (!d_ws)
        return fail(HP_EINVAL, "workspace pointer is NULL");
    if (t_lo >= t_hi)
        return fail(HP_EINVAL, "empty canonical range (t_lo >= t_hi)");
    if (t_hi > hp_canonical_count(s))
        return fail(HP_EINVAL, "t_hi exceeds the number of canonical sequences");
    RunOpts o;
    o.mode = kSeqCanonical;
    return run_blocks(s, d_ws, form, t_lo, t_hi, d_out, d_emin, d_designability, d_nondesign, o,
                      stream, "hp_enumerate_symmetric launch");
}

uint64_t hp_canonical_block_count(const hp_structs *s)
{
    if (!s || !s->blk_ok)
        return 0;
    const int odd = s->N & 1;
    const int h = (s->N - kBlkBits - odd) / 2;
    const uint64_t tri = h ? (uint64_t(1) << (h - 1)) * ((uint64_t(1) << h) + 1) : 1;
    return tri * (odd ? 2 : 1);
}

hp_status hp_enumerate_symmetric_blocked(const hp_structs *s, const void *d_ws, uint64_t b_lo,
                                         uint64_t b_hi, uint16_t *d_out, int32_t *d_emin,
                                         uint64_t *d_designability, uint64_t *d_nondesign,
                                         void *stream)
{
    if (!s)
        return fail(HP_EINVAL, "structures handle is NULL");
    if (!d_ws)
        return fail(HP_EINVAL, "workspace pointer is NULL");
    if (!s->blk_ok)
        return fail(HP_EUNSUPPORTED, "the blocked form needs N >= 8, per-block bytes "
                                     "within int8 and, with unary rows, depth <= 256");
    if (b_lo >= b_hi)
        return fail(HP_EINVAL, "empty block range (b_lo >= b_hi)");
    if (b_hi > hp_canonical_block_count(s))
        return fail(HP_EINVAL, "b_hi exceeds the number of canonical blocks");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    constexpr uint64_t kChunk = kBlockSeqs >> kBlkBits;   // canonical blocks per launch
    for (uint64_t lo = b_lo; lo < b_hi;) {
        const uint64_t hi = b_hi - lo > kChunk ? lo + kChunk : b_hi;
        EnumJob j = make_enum_job(s, d_ws, lo, hi, d_out, d_emin, d_designability, d_nondesign);
        j.mode = kSeqCanonical;
        set_block_geometry(j, s, true);
        hipError_t e = launch_gemm_blocked(j, blocked_selected_nw(), blocked_selected_mode(), hs);
        if (e != hipSuccess)
            return device_fail(e, "hp_enumerate_symmetric_blocked launch");
        lo = hi;
    }
    return HP_OK;
}

uint64_t hp_wide_block_count(const hp_structs *s)
{
    if (!s || !s->wide_ok)
        return 0;
    const int odd = s->N & 1;
    const int h = (s->N - kWideBits - odd) / 2;
    const uint64_t tri = h ? (uint64_t(1) << (h - 1)) * ((uint64_t(1) << h) + 1) : 1;
    return tri * (odd ? 2 : 1);
}

hp_status hp_enumerate_symmetric_wide(const hp_structs *s, const void *d_ws, uint64_t b_lo,
                                      uint64_t b_hi, uint16_t *d_out, int32_t *d_emin,
                                      uint64_t *d_designability, uint64_t *d_nondesign,
                                      void *stream)
{
    if (!s)
        return fail(HP_EINVAL, "structures handle is NULL");
    if (!d_ws)
        return fail(HP_EINVAL, "workspace pointer is NULL");
    if (!s->wide_ok)
        return fail(HP_EUNSUPPORTED, "wide blocks need pure pair energies, N >= 10 and "
                                     "per-block bytes within int8");
    if (b_lo >= b_hi)
        return fail(HP_EINVAL, "empty block range (b_lo >= b_hi)");
    if (b_hi > hp_wide_block_count(s))
        return fail(HP_EINVAL, "b_hi exceeds the number of canonical wide blocks");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    constexpr uint64_t kChunk = kBlockSeqs >> kWideBits;   // canonical wide blocks per launch
    for (uint64_t lo = b_lo; lo < b_hi;) {
        const uint64_t hi = b_hi - lo > kChunk ? lo + kChunk : b_hi;
        EnumJob j = make_enum_job(s, d_ws, lo, hi, d_out, d_emin, d_designability, d_nondesign);
        j.mode = kSeqCanonical;
        j.half_bits = (s->N - kWideBits - (s->N & 1)) / 2;
        hipError_t e = launch_gemm_wide_canonical(j, hs);
        if (e != hipSuccess)
            return device_fail(e, "hp_enumerate_symmetric_wide launch");
        lo = hi;
    }
    return HP_OK;
}

size_t hp_batch_workspace_bytes(int njobs)
{
    if (njobs < 1)
        return 0;
    size_t b = sizeof(BatchHeader) + sizeof(EnumJob) * size_t(njobs) +
               sizeof(int64_t) * size_t(njobs + 1);
    return (b + 255) & ~size_t(255);
}

hp_status hp_enumerate_batch(const hp_job *jobs, int njobs, int form, void *d_batch_ws,
                             size_t batch_ws_bytes, void *stream)
{
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if (form == HP_FORM_POPCOUNT) {
        for (int i = 0; i < njobs && jobs; ++i) {
            hp_status st = hp_enumerate(jobs[i].structs, jobs[i].d_ws, form, jobs[i].seq_lo,
                                        jobs[i].seq_hi, jobs[i].d_out, jobs[i].d_emin,
                                        jobs[i].d_designability, jobs[i].d_nondesign, stream);
            if (st != HP_OK)
                return st;
        }
        return (jobs && njobs >= 1) ? HP_OK : fail(HP_EINVAL, "batch needs at least one job");
    }
    if (form != HP_FORM_GEMM_I8 && form != HP_FORM_BLOCKED_I8)
        return fail(HP_EINVAL, "unknown kernel form");
    if (!d_batch_ws)
        return fail(HP_EINVAL, "batch workspace is NULL");
    BatchPlan plan;
    hp_status st = plan.make(jobs, njobs, form, batch_ws_bytes);
    if (st != HP_OK)
        return st;
    // The upload is ordered on `stream` after the work already queued there
    // (an earlier batch may still read this workspace), and completes before
    // return, since the host plan is released then.
    hipError_t e = hipMemcpyAsync(d_batch_ws, plan.host.data(), plan.host.size(),
                                  hipMemcpyHostToDevice, hs);
    if (e == hipSuccess)
        e = hipStreamSynchronize(hs);
    if (e != hipSuccess)
        return device_fail(e, "batch upload");
    e = launch_plan(plan.groups.data(), plan.ngroups, form, d_batch_ws, hs);
    if (e != hipSuccess)
        return device_fail(e, "batch launch");
    return HP_OK;
}

hp_status hp_graph_capture_batch(const hp_job *jobs, int njobs, int form, void *d_batch_ws,
                                 size_t batch_ws_bytes, hp_graph **out)
{
    if (!out)
        return fail(HP_EINVAL, "out pointer is NULL");
    *out = nullptr;
    if (form != HP_FORM_GEMM_I8 && form != HP_FORM_BLOCKED_I8)
        return fail(HP_EUNSUPPORTED, "graph capture is provided for the int8 forms");
    if (!d_batch_ws)
        return fail(HP_EINVAL, "batch workspace is NULL");
    BatchPlan plan;
    hp_status st = plan.make(jobs, njobs, form, batch_ws_bytes);
    if (st != HP_OK)
        return st;
    // no stream to order on: wait for all work on the device, which may
    // still read this workspace, then upload
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess)
        e = hipMemcpy(d_batch_ws, plan.host.data(), plan.host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess)
        return device_fail(e, "batch upload");
    hipStream_t cap = nullptr;
    if ((e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess)
        return device_fail(e, "capture stream");
    hp_graph *g = new (std::nothrow) hp_graph();
    if (!g) {
        (void)hipStreamDestroy(cap);   // cleanup on the error path; its status adds nothing
        return fail(HP_ENOMEM, "out of host memory");
    }
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = launch_plan(plan.groups.data(), plan.ngroups, form, d_batch_ws, cap);
        e = hipStreamEndCapture(cap, &g->graph);
        if (le != hipSuccess)
            e = le;
    }
    if (e == hipSuccess)
        e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cap);   // the capture's own status decides the result
    if (e != hipSuccess) {
        hp_graph_free(g);
        return device_fail(e, "graph capture");
    }
    *out = g;
    return HP_OK;
}

hp_status hp_graph_launch(hp_graph *g, void *stream)
{
    if (!g || !g->exec)
        return fail(HP_EINVAL, "graph is NULL");
    hipError_t e = hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HP_OK : device_fail(e, "graph launch");
}

void hp_graph_free(hp_graph *g)
{
    if (!g)
        return;
    if (g->exec)
        (void)hipGraphExecDestroy(g->exec);   // release has no caller to report to
    if (g->graph)
        (void)hipGraphDestroy(g->graph);
    delete g;
}

hp_status hp_neighbors(const hp_structs *s, const uint16_t *d_map, uint64_t *d_neutral,
                       uint64_t *d_deleterious, uint64_t *d_other, int32_t phi_q,
                       uint64_t *d_phi_row, void *stream)
{
    if (!s || !d_map)
        return fail(HP_EINVAL, "NULL structures or map");
    if (phi_q >= int32_t(s->n_class))
        return fail(HP_EINVAL, "phi_q >= n_class");
    if (phi_q >= 0 && !d_phi_row)
        return fail(HP_EINVAL, "phi_q given without a phi row buffer");
    hipError_t e = launch_neighbors(d_map, s->N, int(s->n_class),
                                    reinterpret_cast<unsigned long long *>(d_neutral),
                                    reinterpret_cast<unsigned long long *>(d_deleterious),
                                    reinterpret_cast<unsigned long long *>(d_other), phi_q,
                                    phi_q >= 0 ? reinterpret_cast<unsigned long long *>(d_phi_row)
                                               : nullptr,
                                    static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HP_OK : device_fail(e, "hp_neighbors launch");
}

hp_status hp_phi_counts(const hp_structs *s, const uint16_t *d_map, uint64_t *d_counts,
                        void *stream)
{
    if (!s || !d_map || !d_counts)
        return fail(HP_EINVAL, "NULL structures, map or counts");
    hipError_t e = launch_phi_counts(d_map, s->N, int(s->n_class),
                                     reinterpret_cast<unsigned long long *>(d_counts),
                                     static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HP_OK : device_fail(e, "hp_phi_counts launch");
}

hp_status hp_phi_sparse(const hp_structs *s, const uint64_t *d_counts, uint64_t *d_row_ptr,
                        uint32_t *d_cols, uint64_t *d_vals, uint64_t capacity, uint64_t *nnz,
                        void *stream)
{
    if (!s || !d_counts || !d_row_ptr)
        return fail(HP_EINVAL, "NULL structures, counts or row_ptr");
    if ((d_cols == nullptr) != (d_vals == nullptr))
        return fail(HP_EINVAL, "give both cols and vals, or neither for a size query");
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const auto *counts = reinterpret_cast<const unsigned long long *>(d_counts);
    const int n_class = int(s->n_class);
    hipError_t e = launch_phi_row_ptr(counts, n_class, d_row_ptr, st);
    if (e != hipSuccess)
        return device_fail(e, "hp_phi_sparse row counts");
    uint64_t total = 0;
    e = hipMemcpyAsync(&total, d_row_ptr + n_class, sizeof(total), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e != hipSuccess)
        return device_fail(e, "hp_phi_sparse entry count");
    if (nnz)
        *nnz = total;
    if (!d_cols)
        return HP_OK;
    if (capacity < total)
        return fail(HP_ERANGE, "capacity is below the number of non-zero entries");
    e = launch_phi_compact(counts, n_class, d_row_ptr, d_cols, d_vals, st);
    return e == hipSuccess ? HP_OK : device_fail(e, "hp_phi_sparse compaction");
}

hp_status hp_components(const hp_structs *s, const uint16_t *d_map, uint32_t *d_labels,
                        uint32_t *d_compsize, uint32_t *d_ncomp, uint32_t *d_largest,
                        void *stream)
{
    if (!s || !d_map || !d_labels || !d_compsize)
        return fail(HP_EINVAL, "NULL structures, map, labels or compsize");
    if (s->N > 31)
        return fail(HP_ERANGE, "components need N <= 31 (32-bit labels)");
    hipError_t e = launch_components(d_map, s->N, d_labels, d_compsize, d_ncomp, d_largest,
                                     int(s->n_class), static_cast<hipStream_t>(stream));
    return e == hipSuccess ? HP_OK : device_fail(e, "hp_components launch");
}

}  // extern "C"
