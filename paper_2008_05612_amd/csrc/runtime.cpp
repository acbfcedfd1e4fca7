// Runtime pieces of libhpmap around the int8 kernels: the registry of compiled
// tile shapes, the process-wide shape choice per product depth (and the
// blocked form's waves per workgroup), the autotuner that times the shapes
// on the device, and its on-disk cache.
//
// Cache file (path in the HP_TUNE_CACHE environment variable, optional): one
// line per depth, "gfx950 <K_pad> <T> <NW> <mode>", written by hp_autotune and
// read the first time a depth is launched.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hp_internal.h"
#include "kernels.h"

namespace hpmap {

namespace {

struct Registry {
    std::vector<GemmVariant> by_kb[kMaxKB + 1];
    std::atomic<int> selected[kMaxKB + 1];
    std::once_flag cache_once;

    Registry()
    {
        for (auto &s : selected)
            s.store(0);
        int (*groups[])(const GemmVariant **) = {gemm_variants_kb1_4, gemm_variants_kb5,
                                                 gemm_variants_kb6_10, gemm_variants_kb11_12};
        for (auto g : groups) {
            const GemmVariant *v = nullptr;
            int n = g(&v);
            for (int i = 0; i < n; ++i)
                if (v[i].KB >= 1 && v[i].KB <= kMaxKB)
                    by_kb[v[i].KB].push_back(v[i]);
        }
    }
};

Registry &registry()
{
    static Registry r;
    return r;
}

int find_shape(int KB, int T, int NW, int mode)
{
    const auto &v = registry().by_kb[KB];
    for (size_t i = 0; i < v.size(); ++i)
        if (v[i].T == T && v[i].NW == NW && v[i].mode == mode)
            return int(i);
    return -1;
}

void load_cache()
{
    const char *path = std::getenv("HP_TUNE_CACHE");
    if (!path || !*path)
        return;
    FILE *f = std::fopen(path, "r");
    if (!f)
        return;
    char arch[32];
    int kpad, T, NW, mode;
    while (std::fscanf(f, "%31s %d %d %d %d", arch, &kpad, &T, &NW, &mode) == 5) {
        if (std::strcmp(arch, "gfx950") != 0 || kpad % 32 != 0)
            continue;
        const int KB = kpad / 32;
        if (KB < 1 || KB > kMaxKB)
            continue;
        const int idx = find_shape(KB, T, NW, mode);
        if (idx >= 0)
            registry().selected[KB].store(idx);
    }
    std::fclose(f);
}

void store_cache(int KB, const GemmVariant &v)
{
    const char *path = std::getenv("HP_TUNE_CACHE");
    if (!path || !*path)
        return;
    // keep other depths' lines, replace this depth's
    std::vector<std::string> keep;
    if (FILE *f = std::fopen(path, "r")) {
        char line[256];
        while (std::fgets(line, sizeof line, f)) {
            char arch[32];
            int kpad;
            if (std::sscanf(line, "%31s %d", arch, &kpad) == 2 && std::strcmp(arch, "gfx950") == 0 &&
                kpad == KB * 32)
                continue;
            keep.emplace_back(line);
        }
        std::fclose(f);
    }
    if (FILE *f = std::fopen(path, "w")) {
        for (const auto &l : keep)
            std::fputs(l.c_str(), f);
        std::fprintf(f, "gfx950 %d %d %d %d\n", KB * 32, v.T, v.NW, v.mode);
        std::fclose(f);
    }
}

}  // namespace

const GemmVariant *gemm_selected_variant(int KB)
{
    if (KB < 1 || KB > kMaxKB)
        return nullptr;
    Registry &r = registry();
    std::call_once(r.cache_once, load_cache);
    const auto &v = r.by_kb[KB];
    if (v.empty())
        return nullptr;
    int idx = r.selected[KB].load();
    if (idx < 0 || idx >= int(v.size()))
        idx = 0;
    return &v[idx];
}

namespace {
std::atomic<int> g_blocked_nw{4};     // waves per workgroup of the blocked form
std::atomic<int> g_blocked_mode{-1};  // its staging mode; -1: by product depth
}

int blocked_selected_nw() { return g_blocked_nw.load(); }
int blocked_selected_mode() { return g_blocked_mode.load(); }

}  // namespace hpmap

using namespace hpmap;

extern "C" {

hp_status hp_blocked_select(int nw, int mode)
{
    if (nw != 2 && nw != 4 && nw != 8)
        return fail(HP_EINVAL, "blocked form: waves per workgroup must be 2, 4 or 8");
    if (mode < -1 || mode > 3)
        return fail(HP_EINVAL, "blocked form: staging mode must be -1, 0, 1, 2 or 3");
    if (mode == 3 && nw != 4 && nw != 8)
        return fail(HP_EINVAL, "blocked form: wide blocks (mode 3) run 4 or 8 waves per workgroup");
    g_blocked_nw.store(nw);
    g_blocked_mode.store(mode);
    return HP_OK;
}

void hp_blocked_selected(int *nw, int *mode)
{
    if (nw)
        *nw = g_blocked_nw.load();
    if (mode)
        *mode = g_blocked_mode.load();
}

int hp_gemm_shape_count(uint32_t K_pad)
{
    if (K_pad % 32 != 0 || K_pad / 32 < 1 || K_pad / 32 > uint32_t(kMaxKB))
        return 0;
    return int(registry().by_kb[K_pad / 32].size());
}

hp_status hp_gemm_shape_info(uint32_t K_pad, int idx, int *T, int *NW, int *mode)
{
    const int n = hp_gemm_shape_count(K_pad);
    if (idx < 0 || idx >= n)
        return fail(HP_EINVAL, "no such tile shape for this K_pad");
    const GemmVariant &v = registry().by_kb[K_pad / 32][idx];
    if (T)
        *T = v.T;
    if (NW)
        *NW = v.NW;
    if (mode)
        *mode = v.mode;
    return HP_OK;
}

hp_status hp_gemm_select(uint32_t K_pad, int idx)
{
    const int n = hp_gemm_shape_count(K_pad);
    if (idx < 0 || idx >= n)
        return fail(HP_EINVAL, "no such tile shape for this K_pad");
    Registry &r = registry();
    std::call_once(r.cache_once, load_cache);
    r.selected[K_pad / 32].store(idx);
    return HP_OK;
}

int hp_gemm_selected(uint32_t K_pad)
{
    if (hp_gemm_shape_count(K_pad) == 0)
        return -1;
    Registry &r = registry();
    std::call_once(r.cache_once, load_cache);
    return r.selected[K_pad / 32].load();
}

hp_status hp_autotune(const hp_structs *s, const void *d_ws, uint64_t seq_lo, uint64_t n_seq,
                      int repeats, float *ms, int *best, void *stream)
{
    if (!s || !d_ws)
        return fail(HP_EINVAL, "NULL structures or workspace");
    if (n_seq == 0 || seq_lo + n_seq > (uint64_t(1) << s->N) || seq_lo + n_seq < seq_lo)
        return fail(HP_EINVAL, "tuning range outside [0, 2^N)");
    if (repeats < 1)
        repeats = 1;
    const int KB = int(s->K_pad / 32);
    const auto &vars = registry().by_kb[KB];
    if (vars.empty())
        return fail(HP_EUNSUPPORTED, "no compiled tile shape for this K_pad");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t err = hipEventCreate(&e0);
    if (err == hipSuccess)
        err = hipEventCreate(&e1);
    int best_idx = -1;
    float best_ms = 0.f;
    for (size_t i = 0; i < vars.size() && err == hipSuccess; ++i) {
        EnumJob j = make_enum_job(s, d_ws, seq_lo, seq_lo + n_seq, nullptr, nullptr, nullptr,
                                  nullptr);
        err = vars[i].launch(j, st);   // warm-up (code load, caches)
        if (err != hipSuccess)
            break;
        err = hipEventRecord(e0, st);
        for (int r = 0; r < repeats && err == hipSuccess; ++r)
            err = vars[i].launch(j, st);
        if (err == hipSuccess)
            err = hipEventRecord(e1, st);
        if (err == hipSuccess)
            err = hipEventSynchronize(e1);
        float t = 0.f;
        if (err == hipSuccess)
            err = hipEventElapsedTime(&t, e0, e1);
        t /= float(repeats);
        if (ms)
            ms[i] = t;
        if (err == hipSuccess && (best_idx < 0 || t < best_ms)) {
            best_idx = int(i);
            best_ms = t;
        }
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (err != hipSuccess)
        return fail(HP_EDEVICE, std::string("hp_autotune: ") + hipGetErrorString(err));
    Registry &r = registry();
    std::call_once(r.cache_once, load_cache);
    r.selected[KB].store(best_idx);
    store_cache(KB, vars[best_idx]);
    if (best)
        *best = best_idx;
    return HP_OK;
}

hp_status hp_autotune_blocked(const hp_structs *s, const void *d_ws, uint64_t seq_lo,
                              uint64_t n_seq, int repeats, float *ms, int *best_nw,
                              int *best_mode, void *stream)
{
    if (!s || !d_ws)
        return fail(HP_EINVAL, "NULL structures or workspace");
    if (!s->blk_ok)
        return fail(HP_EUNSUPPORTED, "the blocked form does not cover this handle");
    if (n_seq == 0 || seq_lo + n_seq > (uint64_t(1) << s->N) || seq_lo + n_seq < seq_lo)
        return fail(HP_EINVAL, "tuning range outside [0, 2^N)");
    if (repeats < 1)
        repeats = 1;
    static const int kNW[3] = {2, 4, 8};
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t err = hipEventCreate(&e0);
    if (err == hipSuccess)
        err = hipEventCreate(&e1);
    int bi = -1;
    float best_t = 0.f;
    EnumJob j = make_enum_job(s, d_ws, seq_lo, seq_lo + n_seq, nullptr, nullptr, nullptr, nullptr);
    for (int i = 0; i < 10 && err == hipSuccess; ++i) {
        // shapes 0 .. 8: nw x staging mode; shape 9: wide blocks, where they
        // apply (8 waves: blocks of 2048 where the range allows)
        const int nw = i < 9 ? kNW[i / 3] : 8, mode = i < 9 ? i % 3 : 3;
        if (i == 9 && !(s->wide_ok && j.blk_ngroups == 0 && j.blk_coefB == 0)) {
            if (ms)
                ms[i] = -1.f;
            continue;
        }
        err = launch_gemm_blocked(j, nw, mode, st);   // warm-up
        if (err == hipSuccess)
            err = hipEventRecord(e0, st);
        for (int r = 0; r < repeats && err == hipSuccess; ++r)
            err = launch_gemm_blocked(j, nw, mode, st);
        if (err == hipSuccess)
            err = hipEventRecord(e1, st);
        if (err == hipSuccess)
            err = hipEventSynchronize(e1);
        float t = 0.f;
        if (err == hipSuccess)
            err = hipEventElapsedTime(&t, e0, e1);
        t /= float(repeats);
        if (ms)
            ms[i] = t;
        if (err == hipSuccess && (bi < 0 || t < best_t)) {
            bi = i;
            best_t = t;
        }
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (err != hipSuccess)
        return fail(HP_EDEVICE, std::string("hp_autotune_blocked: ") + hipGetErrorString(err));
    const int bnw = bi < 9 ? kNW[bi / 3] : 8, bmode = bi < 9 ? bi % 3 : 3;
    g_blocked_nw.store(bnw);
    g_blocked_mode.store(bmode);
    if (best_nw)
        *best_nw = bnw;
    if (best_mode)
        *best_mode = bmode;
    return HP_OK;
}

}  // extern "C"
