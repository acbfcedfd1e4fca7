// Host side of hp_structures: compact-structure enumeration, symmetry
// reduction and packing of the tables the GPU kernels read.
//
// The structures of the model are the compact self-avoiding walks of a lattice
// box (Methods, "HP and MJ lattice models"), i.e. its directed Hamiltonian
// paths.  Each conformation (orbit under the box isometries) is produced once,
// as its lexicographically smallest member: the depth-first search keeps, for
// the current prefix, the set of isometries whose image of the prefix still
// equals the prefix, and abandons the prefix as soon as one image becomes
// smaller.  Because the search visits sites in ascending order, the surviving
// walks come out already sorted, so conformation ids are emission ranks.
//
// Pruning of prefixes that cannot be completed, both exact necessary
// conditions: (a) the unvisited sites plus the head are connected; (b) colour
// balance of the bipartite lattice.  Sets are 64-bit site masks.
#include <algorithm>
#include <array>
#include <atomic>
#include <cstring>
#include <thread>

#include "hp_internal.h"

namespace hpmap {
namespace {

using Perm = std::array<uint8_t, kMaxN>;

struct Box {
    int X, Y, Z, N;
    uint64_t full;
    uint64_t nbr[kMaxN];
    uint64_t colour_even;              // sites with x+y+z even
    uint64_t lo_x, hi_x, lo_y, hi_y, lo_z, hi_z;  // sites that may shift in each direction
    std::vector<Perm> group;
};

uint64_t bit(int s) { return uint64_t(1) << s; }

uint64_t dilate(const Box &b, uint64_t m)
{
    const int XY = b.X * b.Y;
    return ((m & b.hi_x) << 1) | ((m & b.lo_x) >> 1) | ((m & b.hi_y) << b.X) |
           ((m & b.lo_y) >> b.X) | ((m & b.hi_z) << XY) | ((m & b.lo_z) >> XY);
}

// Isometries from signed permutation matrices acting on doubled, centred
// coordinates u = 2x - (X-1); a matrix is kept when it maps the box onto
// itself, and duplicates (same action on the sites) are dropped.
std::vector<Perm> box_group(const Box &b)
{
    const int dims[3] = {b.X, b.Y, b.Z};
    std::vector<Perm> out;
    int perm[3] = {0, 1, 2};
    do {
        if (dims[perm[0]] != dims[0] || dims[perm[1]] != dims[1] || dims[perm[2]] != dims[2])
            continue;
        for (int signs = 0; signs < 8; ++signs) {
            Perm p{};
            for (int s = 0; s < b.N; ++s) {
                int c[3] = {s % b.X, (s / b.X) % b.Y, s / (b.X * b.Y)};
                int n[3];
                for (int a = 0; a < 3; ++a) {
                    int u = 2 * c[perm[a]] - (dims[a] - 1);
                    if (signs & (1 << a))
                        u = -u;
                    n[a] = (u + dims[a] - 1) / 2;
                }
                p[s] = static_cast<uint8_t>(n[0] + b.X * (n[1] + b.Y * n[2]));
            }
            bool dup = false;
            for (const Perm &q : out)
                dup = dup || std::equal(q.begin(), q.begin() + b.N, p.begin());
            if (!dup)
                out.push_back(p);
        }
    } while (std::next_permutation(perm, perm + 3));
    // identity first, so that it is always element 0 of the tied set
    for (size_t g = 0; g < out.size(); ++g) {
        bool id = true;
        for (int s = 0; s < b.N; ++s)
            id = id && out[g][s] == s;
        if (id) {
            std::swap(out[0], out[g]);
            break;
        }
    }
    return out;
}

Box make_box(int X, int Y, int Z)
{
    Box b{};
    b.X = X; b.Y = Y; b.Z = Z; b.N = X * Y * Z;
    b.full = (b.N == 64) ? ~uint64_t(0) : bit(b.N) - 1;
    for (int s = 0; s < b.N; ++s) {
        int x = s % X, y = (s / X) % Y, z = s / (X * Y);
        if ((x + y + z) % 2 == 0) b.colour_even |= bit(s);
        if (x > 0) b.lo_x |= bit(s);
        if (x < X - 1) b.hi_x |= bit(s);
        if (y > 0) b.lo_y |= bit(s);
        if (y < Y - 1) b.hi_y |= bit(s);
        if (z > 0) b.lo_z |= bit(s);
        if (z < Z - 1) b.hi_z |= bit(s);
    }
    for (int s = 0; s < b.N; ++s)
        b.nbr[s] = dilate(b, bit(s));
    b.group = box_group(b);
    return b;
}

struct Search {
    const Box *box;
    uint8_t path[kMaxN];
    std::vector<uint8_t> found;      // canonical walks, N bytes each
    uint64_t cap;                    // stop once this many canonical walks exist overall
    std::atomic<uint64_t> *counter;
    bool overflow = false;

    bool completable(uint64_t visited, int head) const
    {
        const Box &b = *box;
        uint64_t free = b.full & ~visited;
        if (!free)
            return true;
        uint64_t reach = bit(head);
        for (;;) {
            uint64_t next = (reach | dilate(b, reach)) & (free | bit(head));
            if (next == reach)
                break;
            reach = next;
        }
        if ((reach & free) != free)
            return false;
        int rem = __builtin_popcountll(free) + 1;
        bool head_even = (b.colour_even >> head) & 1;
        int same = __builtin_popcountll((head_even ? b.colour_even : ~b.colour_even) & free) + 1;
        return same == (rem + 1) / 2;
    }

    void dfs(int depth, uint64_t visited, uint64_t tied)
    {
        const Box &b = *box;
        if (overflow)
            return;
        if (depth == b.N) {
            found.insert(found.end(), path, path + b.N);
            if (counter->fetch_add(1) + 1 > cap)
                overflow = true;
            return;
        }
        int head = path[depth - 1];
        uint64_t cand = b.nbr[head] & ~visited;
        while (cand) {
            int v = __builtin_ctzll(cand);
            cand &= cand - 1;
            uint64_t t = tied, keep = 0;
            bool smaller = false;
            while (t) {
                int g = __builtin_ctzll(t);
                t &= t - 1;
                int w = b.group[g][v];
                if (w < v) { smaller = true; break; }
                if (w == v) keep |= bit(g);
            }
            if (smaller)
                continue;
            uint64_t nv = visited | bit(v);
            if (!completable(nv, v))
                continue;
            path[depth] = static_cast<uint8_t>(v);
            dfs(depth + 1, nv, keep);
        }
    }

    void from(int start)
    {
        const Box &b = *box;
        uint64_t tied = 0;
        for (size_t g = 0; g < b.group.size(); ++g) {
            int w = b.group[g][start];
            if (w < start)
                return;             // a symmetric start site is smaller
            if (w == start)
                tied |= bit(static_cast<int>(g));
        }
        if (!completable(bit(start), start))
            return;
        path[0] = static_cast<uint8_t>(start);
        dfs(1, bit(start), tied);
    }
};

int cmp_walk(const uint8_t *a, const uint8_t *b, int N) { return std::memcmp(a, b, N); }

void canonicalise(const Box &b, const uint8_t *walk, uint8_t *out)
{
    uint8_t img[kMaxN];
    bool first = true;
    for (const Perm &p : b.group) {
        for (int i = 0; i < b.N; ++i)
            img[i] = p[walk[i]];
        if (first || cmp_walk(img, out, b.N) < 0) {
            std::memcpy(out, img, b.N);
            first = false;
        }
    }
}

}  // namespace

BlockGeometry block_geometry(int N, bool canonical)
{
    BlockGeometry g{};
    const int odd = N & 1;
    g.half = canonical ? (N - kBlkBits - odd) / 2 : 0;
    for (int x = 0; x < 8; ++x)
        g.pos[x] = canonical ? g.half + x + (x >= 4 ? odd : 0) : x;
    g.npp = 0;
    if (!canonical) {
        for (int p = 0; p < kLow8NumPairs; ++p) {
            const int pr = p < 8 ? int((kLow8Pairs >> (8 * p)) & 0xffu) : kLow8Pair8;
            g.pa[p] = pr & 15;
            g.pb[p] = pr >> 4;
        }
        g.npp = kLow8NumPairs;
        return g;
    }
    for (int a = 0; a < 8; ++a)
        for (int b = a + 1; b < 8; ++b) {
            const int d = g.pos[b] - g.pos[a];
            if (d >= 3 && d % 2 == 1) {
                g.pa[g.npp] = a;
                g.pb[g.npp] = b;
                ++g.npp;
            }
        }
    return g;
}

hp_status build_structures(int X, int Y, int Z, const int32_t table[4], hp_structs *s,
                           std::string *msg)
{
    if (X < 1 || Y < 1 || Z < 1) {
        *msg = "box dimensions must be >= 1";
        return HP_EINVAL;
    }
    const long Nl = long(X) * Y * Z;
    if (Nl < 2) {
        *msg = "chain length X*Y*Z must be >= 2";
        return HP_EINVAL;
    }
    if (Nl > kMaxN) {
        *msg = "chain length X*Y*Z must be <= 36";
        return HP_ERANGE;
    }
    const Box box = make_box(X, Y, Z);
    const int N = box.N;

    // ---- enumeration, start sites spread over threads -------------------
    std::atomic<uint64_t> counter{0};
    std::vector<Search> per_start(N);
    const uint64_t cap = 2ull * 65535ull;   // beyond this the class ids cannot fit
    {
        unsigned nth = std::max(1u, std::min<unsigned>(std::thread::hardware_concurrency(), 32u));
        std::atomic<int> next{0};
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nth; ++t)
            th.emplace_back([&]() {
                for (;;) {
                    int st = next.fetch_add(1);
                    if (st >= N)
                        break;
                    Search &se = per_start[st];
                    se.box = &box;
                    se.cap = cap;
                    se.counter = &counter;
                    se.from(st);
                }
            });
        for (auto &t : th)
            t.join();
    }
    for (const Search &se : per_start)
        if (se.overflow) {
            *msg = "too many conformations for 16-bit class ids";
            return HP_ERANGE;
        }
    s->X = X; s->Y = Y; s->Z = Z; s->N = N;
    s->G = static_cast<uint32_t>(box.group.size());
    s->walks.clear();
    for (const Search &se : per_start)
        s->walks.insert(s->walks.end(), se.found.begin(), se.found.end());
    const uint32_t n_conf = static_cast<uint32_t>(s->walks.size() / N);
    if (n_conf == 0) {
        *msg = "box has no Hamiltonian path";
        return HP_EINVAL;
    }
    if (n_conf >= kMaxConf) {
        *msg = "too many conformations";
        return HP_ERANGE;
    }
    s->n_conf = n_conf;
    s->n_walks = uint64_t(n_conf) * s->G;

    // ---- reversal partners and classes -----------------------------------
    s->rev_conf.assign(n_conf, 0);
    {
        std::vector<std::thread> th;
        unsigned nth = std::max(1u, std::min<unsigned>(std::thread::hardware_concurrency(), 32u));
        for (unsigned t = 0; t < nth; ++t)
            th.emplace_back([&, t]() {
                uint8_t r[kMaxN], k[kMaxN];
                for (uint32_t c = t; c < n_conf; c += nth) {
                    const uint8_t *w = &s->walks[size_t(c) * N];
                    for (int i = 0; i < N; ++i)
                        r[i] = w[N - 1 - i];
                    canonicalise(box, r, k);
                    uint32_t lo = 0, hi = n_conf;
                    while (lo < hi) {
                        uint32_t mid = (lo + hi) / 2;
                        if (cmp_walk(&s->walks[size_t(mid) * N], k, N) < 0)
                            lo = mid + 1;
                        else
                            hi = mid;
                    }
                    bool ok = lo < n_conf && cmp_walk(&s->walks[size_t(lo) * N], k, N) == 0;
                    s->rev_conf[c] = ok ? lo : UINT32_MAX;
                }
            });
        for (auto &t : th)
            t.join();
    }
    for (uint32_t c = 0; c < n_conf; ++c)
        if (s->rev_conf[c] >= n_conf) {
            *msg = "internal: reversed walk not found";
            return HP_EINVAL;
        }
    s->c2q.assign(n_conf, 0);
    uint32_t n_class = 0, n_selfrev = 0;
    // a class is represented by its smaller conformation id, so numbering the
    // representatives in ascending order ranks the class keys
    for (uint32_t c = 0; c < n_conf; ++c) {
        uint32_t r = s->rev_conf[c];
        if (r >= c) {
            if (n_class >= HP_NONE) {
                *msg = "class count does not fit below HP_NONE";
                return HP_ERANGE;
            }
            s->c2q[c] = static_cast<uint16_t>(n_class);
            s->c2q[r] = static_cast<uint16_t>(n_class);
            n_selfrev += (r == c);
            ++n_class;
        }
    }
    s->n_class = n_class;
    s->n_selfrev = n_selfrev;
    s->self_rev.assign(n_class, 0);
    for (uint32_t c = 0; c < n_conf; ++c)
        if (s->rev_conf[c] == c)
            s->self_rev[s->c2q[c]] = 1;

    // ---- pair table: odd separations d >= 3, by d then i -----------------
    std::vector<int> pidx(size_t(N) * N, -1);
    s->pairs.clear();
    for (int d = 3; d < N; d += 2)
        for (int i = 0; i + d < N; ++i) {
            pidx[size_t(i) * N + i + d] = static_cast<int>(s->pairs.size() / 2);
            s->pairs.push_back(static_cast<uint8_t>(i));
            s->pairs.push_back(static_cast<uint8_t>(i + d));
        }
    s->K = static_cast<uint32_t>(s->pairs.size() / 2);
    s->W = std::max<uint32_t>(1, (s->K + 31) / 32);

    // ---- contacts and per-monomer contact counts -------------------------
    const int edges = (X - 1) * Y * Z + X * (Y - 1) * Z + X * Y * (Z - 1);
    s->nbp = static_cast<uint32_t>(edges - (N - 1));
    s->contacts.assign(size_t(n_conf) * s->nbp * 2, 0);
    std::vector<uint8_t> deg(size_t(n_conf) * N, 0);
    uint32_t cmax = 0;
    for (uint32_t c = 0; c < n_conf; ++c) {
        const uint8_t *w = &s->walks[size_t(c) * N];
        int pos[kMaxN];
        for (int i = 0; i < N; ++i)
            pos[w[i]] = i;
        uint32_t nc = 0;
        for (int i = 0; i < N; ++i) {
            uint64_t nb = box.nbr[w[i]];
            // partners j > i+1, ascending j
            int js[6], nj = 0;
            while (nb) {
                int site = __builtin_ctzll(nb);
                nb &= nb - 1;
                int j = pos[site];
                if (j > i + 1)
                    js[nj++] = j;
            }
            std::sort(js, js + nj);
            for (int q = 0; q < nj; ++q) {
                int j = js[q];
                if (nc >= s->nbp) {
                    *msg = "internal: contact count exceeds edges - bonds";
                    return HP_EINVAL;
                }
                if (pidx[size_t(i) * N + j] < 0) {
                    *msg = "internal: contact with even separation";
                    return HP_EINVAL;
                }
                s->contacts[(size_t(c) * s->nbp + nc) * 2] = static_cast<uint8_t>(i);
                s->contacts[(size_t(c) * s->nbp + nc) * 2 + 1] = static_cast<uint8_t>(j);
                ++nc;
                ++deg[size_t(c) * N + i];
                ++deg[size_t(c) * N + j];
            }
        }
        if (nc != s->nbp) {
            *msg = "internal: contact count differs from edges - bonds";
            return HP_EINVAL;
        }
        for (int i = 0; i < N; ++i)
            cmax = std::max<uint32_t>(cmax, deg[size_t(c) * N + i]);
    }
    s->cmax = cmax;

    // ---- energy model ------------------------------------------------------
    // Eq. 1 with a symmetric two-letter table sums, over contacts (i, j),
    // E_PP + (E_HP - E_PP)(h_i + h_j) + (E_HH - 2 E_HP + E_PP) h_i h_j, so
    // E = e0 - F with F = A n_HH + B sum_i h_i c_i, e0 = E_PP nbp,
    // A = -(E_HH - 2 E_HP + E_PP), B = -(E_HP - E_PP).
    for (int q = 0; q < 4; ++q)
        s->table[q] = table[q];
    if (table[1] != table[2]) {
        *msg = "contact table must be symmetric (E_PH == E_HP)";
        return HP_EINVAL;
    }
    const int64_t A = -(int64_t(table[3]) - 2 * int64_t(table[2]) + table[0]);
    const int64_t B = -(int64_t(table[2]) - table[0]);
    if (A < 0 || B < 0 || (A == 0 && B == 0)) {
        *msg = "only attractive tables are handled: need E_HH - 2 E_HP + E_PP <= 0 and "
               "E_HP - E_PP <= 0, not both zero";
        return HP_EUNSUPPORTED;
    }
    // int8 scale m: the largest power of two with A m <= 128 and B cmax m <= 128
    int m = 128;
    while (m >= 1 && (A * m > 128 || B * int64_t(cmax) * m > 128))
        m /= 2;
    if (m < 1) {
        *msg = "contact table too large for the int8 product";
        return HP_EUNSUPPORTED;
    }
    const int64_t fmax = A * s->nbp + 2 * B * s->nbp;
    if (fmax >= (int64_t(1) << 14)) {
        *msg = "contact table too large for 32-bit search keys";
        return HP_ERANGE;
    }
    s->A = int32_t(A);
    s->B = int32_t(B);
    s->e0 = table[0] * int32_t(s->nbp);
    s->U = B ? uint32_t(N) : 0u;
    int shift = 7;
    while ((1 << shift) < 128 * m)
        ++shift;
    s->win_shift = uint32_t(shift);
    s->win_tiles = uint32_t(((1 << shift) - 1) / kTileConf);
    s->K_pad = ((s->K + s->U + 2 + 31) / 32) * 32;
    if (s->K_pad / 32 > uint32_t(kMaxKB)) {
        *msg = "product depth exceeds the compiled kernels";
        return HP_EUNSUPPORTED;
    }
    s->planes = 0;
    if (B)
        while ((1u << s->planes) <= cmax)
            ++s->planes;
    s->uw = N > 32 ? 2 : 1;
    s->MW = s->W + s->planes * s->uw;

    // ---- contact bitmasks and the int8 contact matrix ----------------------
    s->masks.assign(size_t(n_conf) * s->MW, 0);
    const uint32_t KB = s->K_pad / 32;
    const uint32_t n_tiles = (n_conf + kTileConf - 1) / kTileConf;
    const uint32_t wconf = s->win_tiles * kTileConf;
    s->gemm_a.assign(size_t(n_tiles) * KB * 1024, 0);
    auto a_byte = [&](uint32_t c, uint32_t k) -> int8_t & {
        uint32_t t = c / kTileConf, col = c % kTileConf;
        uint32_t kb = k / 32, kk = k % 32;
        uint32_t lane = col + 32 * (kk / 16);
        return s->gemm_a[((size_t(t) * KB + kb) * 64 + lane) * 16 + kk % 16];
    };
    for (uint32_t c = 0; c < n_conf; ++c) {
        uint32_t *mask = &s->masks[size_t(c) * s->MW];
        for (uint32_t q = 0; q < s->nbp; ++q) {
            const int i = s->contacts[(size_t(c) * s->nbp + q) * 2];
            const int j = s->contacts[(size_t(c) * s->nbp + q) * 2 + 1];
            const int k = pidx[size_t(i) * N + j];
            mask[k / 32] |= 1u << (k % 32);
            a_byte(c, k) = static_cast<int8_t>(-A * m);
        }
        for (uint32_t i = 0; i < s->U; ++i) {
            const uint32_t ci = deg[size_t(c) * N + i];
            a_byte(c, s->K + i) = static_cast<int8_t>(-B * int64_t(ci) * m);
            for (uint32_t b = 0; b < s->planes; ++b)
                if ((ci >> b) & 1u)
                    mask[s->W + b * s->uw + i / 32] |= 1u << (i % 32);
        }
        // index rows: key low bits = position of c inside its window, plus 1;
        // padding columns keep all-zero rows, i.e. key 0 = "no conformation"
        const uint32_t idx1 = c % wconf + 1;
        a_byte(c, s->K + s->U) = static_cast<int8_t>(idx1 & 127);
        a_byte(c, s->K + s->U + 1) = static_cast<int8_t>(-static_cast<int>(idx1 >> 7));
    }

    // ---- blocked int8 form ----------------------------------------------------
    // For a block of sequences sharing every monomer outside 8 varying ones,
    // F = base + sum_v h_v w_v + sum_{varying pairs} A C_vv' h_v h_v'
    // + sum_{outer i} B h_i c_i: base counts the A-weighted contacts between
    // outer monomers, w_v = A (contacts of v with outer H) + B c_v, and the
    // unary terms of outer monomers (two-letter tables, B > 0) are split into
    // groups, one row each.  Stage one multiplies block-dependent weights
    // into this 0/1 contact matrix to produce, per conformation, the int8
    // bytes -m2 base, -m2 w_v, -m2 A C_vv', -m2 B (sum of c_i h_i over a
    // group) and the two window index bytes; stage two multiplies them with
    // the per-sequence indicators -128 (1, h_v, h_v h_v', 1) and (1, -128),
    // giving the key 128 m2 F + u.  m2 is the largest power of two keeping
    // every byte of both block geometries within int8 (bounds taken over all
    // conformations with every outer monomer H) and the rows within 32.
    s->blk_ok = false;
    s->gemm_b.clear();
    if (N >= kBlkBits && s->nbp > 0) {
        // contacts of monomer i in conformation c
        std::vector<uint8_t> cc(size_t(n_conf) * N, 0);
        for (uint32_t c = 0; c < n_conf; ++c)
            for (uint32_t q = 0; q < s->nbp; ++q)
                for (int e = 0; e < 2; ++e)
                    ++cc[size_t(c) * N + s->contacts[(size_t(c) * s->nbp + q) * 2 + e]];
        auto max_sum = [&](const std::vector<int> &mono) {   // max_c sum of c_i over mono
            int best = 0;
            for (uint32_t c = 0; c < n_conf; ++c) {
                int t = 0;
                for (int i : mono)
                    t += cc[size_t(c) * N + i];
                best = std::max(best, t);
            }
            return best;
        };
        int maxw[2] = {0, 0};
        std::vector<int> outer[2];
        for (int g = 0; g < 2; ++g) {
            const BlockGeometry geo = block_geometry(N, g == 1);
            bool vary[64] = {};
            for (int x = 0; x < 8; ++x)
                vary[geo.pos[x]] = true;
            for (int i = 0; i < N; ++i)
                if (!vary[i])
                    outer[g].push_back(i);
            for (int x = 0; x < 8; ++x) {
                const int v = geo.pos[x];
                for (uint32_t c = 0; c < n_conf; ++c) {
                    int with_outer = 0;
                    for (uint32_t q = 0; q < s->nbp; ++q) {
                        const int a = s->contacts[(size_t(c) * s->nbp + q) * 2];
                        const int b = s->contacts[(size_t(c) * s->nbp + q) * 2 + 1];
                        with_outer += (a == v && !vary[b]) || (b == v && !vary[a]);
                    }
                    maxw[g] = std::max(maxw[g], int(A * with_outer + B * cc[size_t(c) * N + v]));
                }
            }
        }
        int m2 = 64;
        int ngroups[2] = {0, 0};
        uint64_t grp[2][3];
        for (; m2 >= 1; m2 /= 2) {
            bool fit = int64_t(m2) * A * s->nbp <= 128 && m2 * (A + B) <= 128 &&
                       2 * m2 * B <= 128 && m2 * std::max(maxw[0], maxw[1]) <= 128;
            for (int g = 0; g < 2 && fit; ++g) {
                // unary groups: consecutive outer monomers while m2 B max sum <= 128
                ngroups[g] = 0;
                grp[g][0] = grp[g][1] = grp[g][2] = ~uint64_t(0);   // 15: no group
                if (B > 0) {
                    std::vector<int> cur;
                    for (int i : outer[g]) {
                        cur.push_back(i);
                        if (int64_t(m2) * B * max_sum(cur) > 128) {
                            cur.assign(1, i);
                            ++ngroups[g];
                            if (int64_t(m2) * B * max_sum(cur) > 128) {
                                fit = false;
                                break;
                            }
                        }
                        const int gid = ngroups[g];
                        grp[g][i / 16] &= ~(uint64_t(15) << (4 * (i % 16)));
                        grp[g][i / 16] |= uint64_t(gid & 15) << (4 * (i % 16));
                    }
                    if (!cur.empty())
                        ++ngroups[g];
                }
                const int npp = block_geometry(N, g == 1).npp;
                fit = fit && ngroups[g] <= 14 && 9 + npp + ngroups[g] + 2 <= 32;
            }
            if (fit)
                break;
        }
        const uint32_t bkb = (s->K + 2 + 31) / 32;
        const uint32_t kb_cap = B > 0 ? uint32_t(kBlkUnaryMaxKB) : uint32_t(kMaxKB);
        if (m2 >= 1 && bkb <= kb_cap) {
            int bshift = 7;
            while ((1 << bshift) < 128 * m2)
                ++bshift;
            s->blk_ok = true;
            s->blk_KB = bkb;
            s->blk_shift = uint32_t(bshift);
            s->blk_win_tiles = uint32_t(((1 << bshift) - 1) / kTileConf);
            s->blk_coef = int32_t(m2 * A);
            s->blk_coefB = int32_t(m2 * B);
            for (int g = 0; g < 2; ++g) {
                s->blk_ngroups[g] = ngroups[g];
                for (int w = 0; w < 3; ++w)
                    s->blk_grp[g][w] = grp[g][w];
            }
            const uint32_t bconf = s->blk_win_tiles * kTileConf;
            s->gemm_b.assign(size_t(n_tiles) * bkb * 1024, 0);
            auto b_byte = [&](uint32_t c, uint32_t k) -> int8_t & {
                uint32_t t = c / kTileConf, col = c % kTileConf;
                uint32_t kb = k / 32, kk = k % 32;
                uint32_t lane = col + 32 * (kk / 16);
                return s->gemm_b[((size_t(t) * bkb + kb) * 64 + lane) * 16 + kk % 16];
            };
            for (uint32_t c = 0; c < n_conf; ++c) {
                for (uint32_t q = 0; q < s->nbp; ++q) {
                    const int i = s->contacts[(size_t(c) * s->nbp + q) * 2];
                    const int j = s->contacts[(size_t(c) * s->nbp + q) * 2 + 1];
                    b_byte(c, pidx[size_t(i) * N + j]) = 1;
                }
                const uint32_t u = c % bconf + 1;
                b_byte(c, s->K) = static_cast<int8_t>(u & 127);
                b_byte(c, s->K + 1) = static_cast<int8_t>(u >> 7);
            }
        }
    }

    // Per-sequence operand of the second product, for both block geometries:
    // 8 sequence tiles x 64 lanes x 16 bytes in MFMA operand order.  Lane l
    // holds block sequence x = 32 t + (l & 31); its byte q carries the
    // indicator of the virtual row m = 8 (q / 4) + 4 (l / 32) + q % 4 (the
    // row the first product's result register q holds in that lane):
    // m = 0 the block term (-128), 1 .. 8 the weight of varying monomer m-1
    // (-128 h), then one row per varying pair (-128 h_a h_b), one per unary
    // group (-128), then the two index bytes (1 and -128).
    s->blk_s2.clear();
    if (s->blk_ok) {
        s->blk_s2.assign(2 * 8 * 64 * 16, 0);
        for (int g = 0; g < 2; ++g) {
            const BlockGeometry geo = block_geometry(N, g == 1);
            const int row_un = 9 + geo.npp;
            const int row_idx = row_un + s->blk_ngroups[g];
            for (int t = 0; t < 8; ++t)
                for (int lane = 0; lane < 64; ++lane) {
                    const int x = 32 * t + (lane & 31), half = lane >> 5;
                    for (int q = 0; q < 16; ++q) {
                        const int m = 8 * (q / 4) + 4 * half + q % 4;
                        int v = 0;
                        if (m == 0)
                            v = -128;
                        else if (m < 9)
                            v = ((x >> (m - 1)) & 1) ? -128 : 0;
                        else if (m < row_un)
                            v = ((x >> geo.pa[m - 9]) & (x >> geo.pb[m - 9]) & 1) ? -128 : 0;
                        else if (m < row_idx)
                            v = -128;
                        else if (m == row_idx)
                            v = 1;
                        else if (m == row_idx + 1)
                            v = -128;
                        s->blk_s2[((size_t(g) * 8 + t) * 64 + lane) * 16 + q] = static_cast<int8_t>(v);
                    }
                }
        }
    }

    // Wide blocks (pure pair energies), three geometries: plain (the low 10
    // monomers vary), reversal-canonical (the 10 around the middle) and
    // plain 11 (monomers 0 .. 4 and 6, 8, .., 16; N >= 17), see
    // hp_internal.h.  Wave w of the workgroup holds the 256 sequences whose
    // varying monomers above the low 8 are the bits of w (4 waves, or 8 for
    // plain 11).  Same first-product matrix and key scale as above; the
    // virtual rows are m = 0 the block term, 1 .. nb the weight of varying
    // monomer m - 1, then the 16 varying pairs (kLow10Pairs, kMid10OddPairs
    // for odd N canonical, kW11Pairs), then the two index bytes.  Lane l of
    // tile t of wave w holds block sequence x = 256 w + 32 t + (l & 31) and
    // its byte q the indicator of row m = 8 (q / 4) + 4 (l / 32) + q % 4.
    s->wide_ok = false;
    s->wide_s2.clear();
    const int wodd = N & 1;
    const int whalf = N >= kWideBits ? (N - kWideBits - wodd) / 2 : 0;
    const int n_geom = N >= kWide11ChunkBits ? 3 : 2;
    auto wide_nb = [&](int g) { return g == 2 ? kWide11Bits : kWideBits; };
    auto wide_pos = [&](int g, int x) {
        return g == 0 ? x : g == 1 ? whalf + x + (x >= 5 ? wodd : 0) : (x < 5 ? x : 2 * x - 4);
    };
    auto wide_pair = [&](int g, int p) {
        const uint64_t w = g == 2 ? (p < 8 ? kW11Pairs0 : kW11Pairs1)
                           : (g == 1 && wodd) ? (p < 8 ? kMid10OddPairs0 : kMid10OddPairs1)
                                              : (p < 8 ? kLow10Pairs0 : kLow10Pairs1);
        return int((w >> (8 * (p & 7))) & 0xffu);
    };
    if (s->blk_ok && B == 0 && N >= kWideBits) {
        int maxw = 0;   // largest weight of a varying monomer (all outer monomers H)
        for (int g = 0; g < n_geom; ++g) {
            bool vary[64] = {};
            for (int x = 0; x < wide_nb(g); ++x)
                vary[wide_pos(g, x)] = true;
            for (int x = 0; x < wide_nb(g); ++x) {
                const int v = wide_pos(g, x);
                for (uint32_t c = 0; c < n_conf; ++c) {
                    int with_outer = 0;
                    for (uint32_t q = 0; q < s->nbp; ++q) {
                        const int a = s->contacts[(size_t(c) * s->nbp + q) * 2];
                        const int b = s->contacts[(size_t(c) * s->nbp + q) * 2 + 1];
                        with_outer += (a == v && !vary[b]) || (b == v && !vary[a]);
                    }
                    maxw = std::max(maxw, int(A) * with_outer);
                }
            }
        }
        s->wide_ok = int64_t(s->blk_coef) * maxw <= 128;
    }
    if (s->wide_ok) {
        const int n_waves = n_geom == 3 ? 4 + 4 + kWide11Waves : 4 + 4;
        s->wide_s2.assign(size_t(n_waves) * 8 * 64 * 16, 0);
        for (int slot = 0; slot < n_waves; ++slot) {
            const int g = slot < 4 ? 0 : slot < 8 ? 1 : 2;
            const int w = slot < 8 ? slot & 3 : slot - 8;
            const int row_vv = 1 + wide_nb(g), row_idx = row_vv + 16;
            for (int t = 0; t < 8; ++t)
                for (int lane = 0; lane < 64; ++lane) {
                    const int x = 256 * w + 32 * t + (lane & 31), half = lane >> 5;
                    for (int q = 0; q < 16; ++q) {
                        const int m = 8 * (q / 4) + 4 * half + q % 4;
                        int v = 0;
                        if (m == 0) {
                            v = -128;
                        } else if (m < row_vv) {
                            v = ((x >> (m - 1)) & 1) ? -128 : 0;
                        } else if (m < row_idx) {
                            const int pr = wide_pair(g, m - row_vv);
                            v = ((x >> (pr & 15)) & (x >> (pr >> 4)) & 1) ? -128 : 0;
                        } else if (m == row_idx) {
                            v = 1;
                        } else if (m == row_idx + 1) {
                            v = -128;
                        }
                        s->wide_s2[((size_t(slot) * 8 + t) * 64 + lane) * 16 + q] =
                            static_cast<int8_t>(v);
                    }
                }
        }
    }

    // pair table for the popcount form, 4 bytes per row (i, j, 0, 0)
    s->pair_rows.assign(size_t(s->K_pad) * 4, 0);
    for (uint32_t k = 0; k < s->K_pad; ++k) {
        uint8_t *r = &s->pair_rows[size_t(k) * 4];
        r[0] = k < s->K ? s->pairs[2 * k] : 63;
        r[1] = k < s->K ? s->pairs[2 * k + 1] : 63;
    }

    // ---- workspace layout ---------------------------------------------------
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    WsLayout &L = s->ws;
    L.c2q = 0;
    L.pairs = up(L.c2q + size_t(n_conf) * 2);
    L.masks = up(L.pairs + s->pair_rows.size());
    L.gemm_a = up(L.masks + s->masks.size() * 4);
    L.gemm_b = up(L.gemm_a + s->gemm_a.size());
    L.blk_s2 = up(L.gemm_b + s->gemm_b.size());
    L.wide_s2 = up(L.blk_s2 + s->blk_s2.size());
    L.total = up(L.wide_s2 + s->wide_s2.size());
    return HP_OK;
}

}  // namespace hpmap
