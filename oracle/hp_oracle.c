/*
 * hp_oracle.c -- plain, slow CPU oracle for the HP-model genotype-phenotype map.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU path and imports nothing from it.
 *
 * Everything here is integer arithmetic and follows the definitions of the
 * paper directly, with no blocking, bit tricks or reordering:
 *
 *   - Structures are the compact self-avoiding walks of a lattice box, i.e.
 *     the directed Hamiltonian paths of the box's nearest-neighbour graph
 *     (Methods, "HP and MJ lattice models").
 *   - The energy of sequence s on walk w is the contact Hamiltonian of Eq. 1
 *     specialised to pure HP: each non-bonded lattice contact (i,j) adds
 *     -h_i*h_j, h_i = 1 for H and 0 for P.  Bit i of s is monomer i.
 *   - A sequence folds (is designing) iff exactly one conformation attains the
 *     minimum energy; otherwise it has the deleterious phenotype (Methods,
 *     end of "HP and MJ lattice models"; the min/second-min test of the GPU
 *     listing in Appendix C).
 *   - With an energy threshold (Methods, same passage) a sequence folds iff the
 *     second-lowest conformation energy exceeds the lowest by at least the
 *     threshold; threshold 1 with integer energies is the uniqueness rule.
 *     Random sequences for the sampling mode come from a published
 *     counter-based generator (splitmix64).
 *   - Designability N_q, the neighbourhood counts behind phi_pq, robustness and
 *     phi_del (Eq. 2 and the text around it), and neutral-network components
 *     are plain counts over the 2^N hypercube of sequences.
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - A conformation is an orbit of directed walks under the box isometry
 *     group G; a class (the reported phenotype) is an orbit under G x chain
 *     reversal.  Both chain directions are scored.
 *   - Conformation ids are ranks of canonical keys (lexicographically smallest
 *     site sequence in the orbit); class ids are ranks of class keys
 *     (min of the two directions' keys).  The deleterious phenotype is 0xFFFF.
 *   - Neutral-network components are labelled by their smallest member.
 *
 * Parity status: every function here is pinned by tests (paper counts, closed
 * forms, invariants, independent brute force on tiny lattices); none is
 * "parity unpinned".
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXN 64
#define OR_NONE 0xFFFFu

/* ------------------------------------------------------------------------ */
/* Lattice box: site id sigma(x,y,z) = x + X*(y + Y*z).                      */
/* ------------------------------------------------------------------------ */

static void site_xyz(int X, int Y, int s, int *x, int *y, int *z)
{
    *x = s % X;
    *y = (s / X) % Y;
    *z = s / (X * Y);
}

static int lattice_adjacent(int X, int Y, int a, int b)
{
    int ax, ay, az, bx, by, bz;
    site_xyz(X, Y, a, &ax, &ay, &az);
    site_xyz(X, Y, b, &bx, &by, &bz);
    int d = abs(ax - bx) + abs(ay - by) + abs(az - bz);
    return d == 1;
}

/* ------------------------------------------------------------------------ */
/* Depth-first enumeration of all directed Hamiltonian paths.                */
/* ------------------------------------------------------------------------ */

typedef void (*leaf_fn)(const uint8_t *path, int N, void *ctx);

typedef struct {
    int X, Y, Z, N;
    int prune;
    int deg[OR_MAXN];
    int nbr[OR_MAXN][6];        /* lattice neighbours of each site, ascending */
    uint8_t path[OR_MAXN];
    uint8_t used[OR_MAXN];
    long count;
    leaf_fn leaf;
    void *ctx;
} walker;

/* Necessary conditions for a Hamiltonian completion from `head`:
 *  (a) the head together with every unvisited site forms a connected set;
 *  (b) colour balance: the lattice is bipartite (colour = parity of x+y+z),
 *      so a path through these R sites that starts on the head's colour
 *      holds ceil(R/2) sites of that colour.                              */
static int colour(const walker *w, int s)
{
    int x = s % w->X, y = (s / w->X) % w->Y, z = s / (w->X * w->Y);
    return (x + y + z) & 1;
}

static int rest_connected(walker *w, int head, int depth)
{
    uint8_t seen[OR_MAXN];
    int stack[OR_MAXN];
    int sp = 0, reached = 0, same = 1;
    int hc = colour(w, head);
    memset(seen, 0, sizeof(seen));
    stack[sp++] = head;
    seen[head] = 1;
    while (sp > 0) {
        int a = stack[--sp];
        for (int k = 0; k < w->deg[a]; k++) {
            int b = w->nbr[a][k];
            if (!w->used[b] && !seen[b]) {
                seen[b] = 1;
                reached++;
                same += colour(w, b) == hc;
                stack[sp++] = b;
            }
        }
    }
    int R = w->N - depth + 1;
    return reached == w->N - depth && same == (R + 1) / 2;
}

static void dfs(walker *w, int depth)
{
    if (depth == w->N) {
        w->count++;
        if (w->leaf)
            w->leaf(w->path, w->N, w->ctx);
        return;
    }
    int head = w->path[depth - 1];
    for (int k = 0; k < w->deg[head]; k++) {
        int b = w->nbr[head][k];
        if (w->used[b])
            continue;
        w->used[b] = 1;
        w->path[depth] = (uint8_t)b;
        if (!w->prune || rest_connected(w, b, depth + 1))
            dfs(w, depth + 1);
        w->used[b] = 0;
    }
}

static void walker_init(walker *w, int X, int Y, int Z, int prune, leaf_fn leaf, void *ctx)
{
    memset(w, 0, sizeof(*w));
    w->X = X; w->Y = Y; w->Z = Z; w->N = X * Y * Z;
    w->prune = prune;
    w->leaf = leaf;
    w->ctx = ctx;
    for (int a = 0; a < w->N; a++)
        for (int b = 0; b < w->N; b++)
            if (lattice_adjacent(X, Y, a, b))
                w->nbr[a][w->deg[a]++] = b;
}

static long walk_from(walker *w, int start)
{
    w->count = 0;
    w->used[start] = 1;
    w->path[0] = (uint8_t)start;
    if (!w->prune || rest_connected(w, start, 1))
        dfs(w, 1);
    w->used[start] = 0;
    return w->count;
}

/* Serial walk over all start sites in ascending order (DFS order). */
static long walk_all(int X, int Y, int Z, int prune, leaf_fn leaf, void *ctx)
{
    walker w;
    walker_init(&w, X, Y, Z, prune, leaf, ctx);
    long total = 0;
    for (int start = 0; start < w.N; start++)
        total += walk_from(&w, start);
    return total;
}

/* Same set of walks, start sites spread over threads; `leaf` must be
 * thread-safe and must not depend on the order of the walks.           */
static long walk_all_par(int X, int Y, int Z, leaf_fn leaf, void *ctx)
{
    int N = X * Y * Z;
    long total = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total)
    for (int start = 0; start < N; start++) {
        walker w;
        walker_init(&w, X, Y, Z, 1, leaf, ctx);
        total += walk_from(&w, start);
    }
    return total;
}

typedef struct { uint8_t *out; long cap; long n; } collect_ctx;

static void collect_leaf(const uint8_t *path, int N, void *vctx)
{
    collect_ctx *c = (collect_ctx *)vctx;
    if (c->n < c->cap)
        memcpy(c->out + (size_t)c->n * N, path, (size_t)N);
    c->n++;
}

/* All directed Hamiltonian paths of the X*Y*Z box, each as N site ids, in
 * DFS order.  Returns the total count; writes at most `cap` walks.  `prune`
 * switches the connectivity test on (the result must not depend on it).   */
long or_walks(int X, int Y, int Z, int prune, uint8_t *out, long cap)
{
    collect_ctx c = { out, out ? cap : 0, 0 };
    return walk_all(X, Y, Z, prune, collect_leaf, &c);
}

/* ------------------------------------------------------------------------ */
/* Isometry group of the box.                                                */
/* ------------------------------------------------------------------------ */

/* Writes each distinct isometry as a site permutation (N bytes: image of
 * site s at [g*N + s]) and returns |G|.  Isometries are axis permutations
 * that keep the box dimensions, composed with per-axis reflections;
 * maps that act identically on the sites are counted once.               */
int or_group(int X, int Y, int Z, uint8_t *perms)
{
    static const int axis_perms[6][3] = {
        {0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int dims[3] = {X, Y, Z};
    int N = X * Y * Z;
    int G = 0;
    uint8_t cand[OR_MAXN];
    for (int p = 0; p < 6; p++) {
        const int *pa = axis_perms[p];
        /* new coordinate a takes old coordinate pa[a]; needs equal lengths */
        if (dims[pa[0]] != X || dims[pa[1]] != Y || dims[pa[2]] != Z)
            continue;
        for (int refl = 0; refl < 8; refl++) {
            for (int s = 0; s < N; s++) {
                int c[3];
                site_xyz(X, Y, s, &c[0], &c[1], &c[2]);
                int n[3];
                for (int a = 0; a < 3; a++) {
                    n[a] = c[pa[a]];
                    if (refl & (1 << a))
                        n[a] = dims[a] - 1 - n[a];
                }
                cand[s] = (uint8_t)(n[0] + X * (n[1] + Y * n[2]));
            }
            int dup = 0;
            for (int g = 0; g < G && !dup; g++)
                dup = memcmp(perms + (size_t)g * N, cand, (size_t)N) == 0;
            if (!dup) {
                memcpy(perms + (size_t)G * N, cand, (size_t)N);
                G++;
            }
        }
    }
    return G;
}

/* Canonical key of a walk: the lexicographically smallest of its images
 * (g(w_0), ..., g(w_{N-1})) over all g in G.                               */
static void canon_key(const uint8_t *perms, int G, int N, const uint8_t *walk, uint8_t *key)
{
    for (int i = 0; i < N; i++)
        key[i] = perms[walk[i]];            /* image under the first isometry */
    for (int g = 1; g < G; g++) {
        const uint8_t *pg = perms + (size_t)g * N;
        /* compare the image under g with the best so far, element by element */
        int i = 0;
        while (i < N && pg[walk[i]] == key[i])
            i++;
        if (i < N && pg[walk[i]] < key[i])
            for (; i < N; i++)
                key[i] = pg[walk[i]];
    }
}

static void reversed(const uint8_t *walk, int N, uint8_t *out)
{
    for (int i = 0; i < N; i++)
        out[i] = walk[N - 1 - i];
}

/* Public wrapper used by tests. */
void or_canonical_key(int X, int Y, int Z, const uint8_t *walk, uint8_t *key)
{
    uint8_t perms[48 * OR_MAXN];
    int G = or_group(X, Y, Z, perms);
    canon_key(perms, G, X * Y * Z, walk, key);
}

/* ------------------------------------------------------------------------ */
/* Conformations and classes.                                                */
/* ------------------------------------------------------------------------ */

static int g_cmp_n; /* key length for qsort; set before each sort */
static int cmp_keys(const void *a, const void *b)
{
    return memcmp(a, b, (size_t)g_cmp_n);
}

typedef struct {
    const uint8_t *perms;
    int G;
    uint8_t *keys;
    long cap;
    long n;
} key_ctx;

static void key_leaf(const uint8_t *path, int N, void *vctx)
{
    key_ctx *c = (key_ctx *)vctx;
    long slot;
#pragma omp atomic capture
    slot = c->n++;
    if (slot < c->cap)
        canon_key(c->perms, c->G, N, path, c->keys + (size_t)slot * N);
}

static long sort_unique(uint8_t *keys, long n, int N)
{
    g_cmp_n = N;
    qsort(keys, (size_t)n, (size_t)N, cmp_keys);
    long m = 0;
    for (long i = 0; i < n; i++) {
        if (m == 0 || memcmp(keys + (size_t)(m - 1) * N, keys + (size_t)i * N, (size_t)N) != 0) {
            if (m != i)
                memmove(keys + (size_t)m * N, keys + (size_t)i * N, (size_t)N);
            m++;
        }
    }
    return m;
}

/* Number of directed walks of the box (pruned DFS). */
long or_count_walks(int X, int Y, int Z)
{
    return walk_all_par(X, Y, Z, NULL, NULL);
}

/* Conformations of the box: the sorted, distinct canonical keys of all
 * directed walks.  `scratch` must hold (number of directed walks) * N bytes;
 * the first n_conf keys are left in it, ascending.  Returns n_conf, or -1
 * if scratch is too small.                                                  */
long or_conformations(int X, int Y, int Z, uint8_t *scratch, long scratch_walks)
{
    uint8_t perms[48 * OR_MAXN];
    int N = X * Y * Z;
    key_ctx c;
    c.perms = perms;
    c.G = or_group(X, Y, Z, perms);
    c.keys = scratch;
    c.cap = scratch_walks;
    c.n = 0;
    walk_all_par(X, Y, Z, key_leaf, &c);
    if (c.n > scratch_walks)
        return -1;
    return sort_unique(scratch, c.n, N);
}

static long find_key(const uint8_t *keys, long n, int N, const uint8_t *k)
{
    long lo = 0, hi = n;
    while (lo < hi) {
        long mid = (lo + hi) / 2;
        int c = memcmp(keys + (size_t)mid * N, k, (size_t)N);
        if (c == 0)
            return mid;
        if (c < 0)
            lo = mid + 1;
        else
            hi = mid;
    }
    return -1;
}

/* Classes: for each conformation key k, the class key is
 * min(k, canon(reverse(k))).  Class ids are the ranks of the distinct class
 * keys.  Writes conf_to_class[n_conf], rev_conf[n_conf] (the conformation
 * of the reversed chain) and self_rev per class; returns n_class.
 * `class_keys` needs n_conf * N bytes of room.                              */
long or_classes(int X, int Y, int Z, const uint8_t *conf_keys, long n_conf,
                int32_t *conf_to_class, int32_t *rev_conf, uint8_t *self_rev,
                uint8_t *class_keys)
{
    uint8_t perms[48 * OR_MAXN];
    int N = X * Y * Z;
    int G = or_group(X, Y, Z, perms);
    uint8_t r[OR_MAXN], rk[OR_MAXN];
    for (long c = 0; c < n_conf; c++) {
        const uint8_t *k = conf_keys + (size_t)c * N;
        reversed(k, N, r);
        canon_key(perms, G, N, r, rk);
        rev_conf[c] = (int32_t)find_key(conf_keys, n_conf, N, rk);
        const uint8_t *ck = memcmp(k, rk, (size_t)N) <= 0 ? k : rk;
        memcpy(class_keys + (size_t)c * N, ck, (size_t)N);
    }
    long n_class = sort_unique(class_keys, n_conf, N);
    for (long c = 0; c < n_conf; c++) {
        const uint8_t *k = conf_keys + (size_t)c * N;
        reversed(k, N, r);
        canon_key(perms, G, N, r, rk);
        const uint8_t *ck = memcmp(k, rk, (size_t)N) <= 0 ? k : rk;
        conf_to_class[c] = (int32_t)find_key(class_keys, n_class, N, ck);
    }
    for (long q = 0; q < n_class; q++)
        self_rev[q] = 0;
    for (long c = 0; c < n_conf; c++)
        if (rev_conf[c] == c)
            self_rev[conf_to_class[c]] = 1;
    return n_class;
}

/* Contacts of a walk: pairs (i,j), i<j, j-i >= 2, whose sites are lattice
 * neighbours (Delta of Eq. 1).  Writes pairs as (i,j) bytes; returns count. */
int or_contacts(int X, int Y, int Z, const uint8_t *walk, uint8_t *pairs)
{
    int N = X * Y * Z;
    int n = 0;
    for (int i = 0; i < N; i++)
        for (int j = i + 2; j < N; j++)
            if (lattice_adjacent(X, Y, walk[i], walk[j])) {
                pairs[2 * n] = (uint8_t)i;
                pairs[2 * n + 1] = (uint8_t)j;
                n++;
            }
    return n;
}

/* Contacts of every conformation key: writes ct_off[n_conf+1] (pair units)
 * and the pairs; `pairs` needs n_conf * N * N * 2 bytes at most.          */
long or_all_contacts(int X, int Y, int Z, const uint8_t *keys, long n_conf,
                     int32_t *ct_off, uint8_t *pairs)
{
    int N = X * Y * Z;
    long total = 0;
    ct_off[0] = 0;
    for (long c = 0; c < n_conf; c++) {
        total += or_contacts(X, Y, Z, keys + (size_t)c * N, pairs + 2 * (size_t)total);
        ct_off[c + 1] = (int32_t)total;
    }
    return total;
}

/* ------------------------------------------------------------------------ */
/* Energies and ground states.                                               */
/* ------------------------------------------------------------------------ */

static int monomer(uint64_t s, int i) { return (int)((s >> i) & 1u); }

/* E(s,w) = -sum over contacts (i,j) of h_i*h_j, from an explicit list. */
int or_energy(uint64_t s, int ncontacts, const uint8_t *pairs)
{
    int e = 0;
    for (int k = 0; k < ncontacts; k++)
        e -= monomer(s, pairs[2 * k]) * monomer(s, pairs[2 * k + 1]);
    return e;
}

/* Eq. 1 with a general two-letter contact table: each contact (i,j) adds
 * table[2*h_i + h_j]  (table = {E_PP, E_PH, E_HP, E_HH}, integers, e.g. the
 * paper's Table 1 scaled by 10: {0, -10, -10, -23}).                       */
int or_energy_table(uint64_t s, int ncontacts, const uint8_t *pairs, const int32_t *table)
{
    int e = 0;
    for (int k = 0; k < ncontacts; k++)
        e += table[2 * monomer(s, pairs[2 * k]) + monomer(s, pairs[2 * k + 1])];
    return e;
}

/* Ground states with a contact table (see or_energy_table); otherwise as
 * or_ground_states below.                                                   */
void or_ground_states_table(long n_conf, const int32_t *ct_off, const uint8_t *pairs,
                            const int32_t *conf_to_class, const int32_t *table,
                            uint64_t lo, uint64_t hi, uint16_t *out, int32_t *emin,
                            uint64_t *designability, uint64_t *nondesign)
{
    long count = (long)(hi - lo);
    uint16_t *res = out ? out : (uint16_t *)malloc(sizeof(uint16_t) * (size_t)(count > 0 ? count : 1));
#pragma omp parallel for schedule(dynamic, 64)
    for (long t = 0; t < count; t++) {
        uint64_t s = lo + (uint64_t)t;
        int best = 0;
        long nbest = 0;
        long arg = -1;
        for (long c = 0; c < n_conf; c++) {
            int e = or_energy_table(s, ct_off[c + 1] - ct_off[c], pairs + 2 * (size_t)ct_off[c],
                                    table);
            if (nbest == 0 || e < best) {
                best = e;
                nbest = 1;
                arg = c;
            } else if (e == best) {
                nbest++;
            }
        }
        if (emin)
            emin[t] = best;
        res[t] = (nbest == 1) ? (uint16_t)conf_to_class[arg] : (uint16_t)OR_NONE;
    }
    for (long t = 0; t < count; t++) {
        if (res[t] == OR_NONE) {
            if (nondesign)
                (*nondesign)++;
        } else if (designability) {
            designability[res[t]]++;
        }
    }
    if (!out)
        free(res);
}

/* Energy gap and threshold (Methods, end of "HP and MJ lattice models": a
 * threshold sets the smallest energy difference between the lowest and the
 * second-lowest fold that counts as distinguishable; a sequence whose two
 * lowest folds lie closer than that does not fold).  For each listed
 * sequence seqs[t], with E1 <= E2 the two smallest energies over all
 * conformations (E2 = E1 when the minimum is shared):
 *   emin[t] = E1;  gap[t] = min(E2 - E1, 255), or 255 with one conformation;
 *   out[t]  = class of the minimiser if E2 - E1 >= threshold, else 0xFFFF.
 * threshold = 1 is the plain uniqueness rule.  Energies use the contact
 * table {E_PP, E_PH, E_HP, E_HH} (or_energy_table).  designability[q] and
 * *nondesign are incremented (+=).  Any output pointer may be NULL.        */
void or_ground_states_gap(long n_conf, const int32_t *ct_off, const uint8_t *pairs,
                          const int32_t *conf_to_class, const int32_t *table,
                          const uint64_t *seqs, long count, int threshold, uint16_t *out,
                          int32_t *emin, uint8_t *gap, uint64_t *designability,
                          uint64_t *nondesign)
{
    uint16_t *res = out ? out : (uint16_t *)malloc(sizeof(uint16_t) * (size_t)(count > 0 ? count : 1));
#pragma omp parallel for schedule(dynamic, 64)
    for (long t = 0; t < count; t++) {
        uint64_t s = seqs[t];
        long e1 = 0, e2 = 0;      /* valid once 1 and 2 conformations are seen */
        long seen = 0;
        long arg = -1;
        for (long c = 0; c < n_conf; c++) {
            long e = or_energy_table(s, ct_off[c + 1] - ct_off[c], pairs + 2 * (size_t)ct_off[c],
                                     table);
            if (seen == 0 || e < e1) {
                e2 = e1;
                e1 = e;
                arg = c;
            } else if (seen == 1 || e < e2) {
                e2 = e;
            }
            seen++;
        }
        long g = seen >= 2 ? e2 - e1 : 255;
        if (g > 255)
            g = 255;
        if (emin)
            emin[t] = (int32_t)e1;
        if (gap)
            gap[t] = (uint8_t)g;
        res[t] = (seen >= 1 && g >= threshold) ? (uint16_t)conf_to_class[arg] : (uint16_t)OR_NONE;
    }
    for (long t = 0; t < count; t++) {
        if (res[t] == OR_NONE) {
            if (nondesign)
                (*nondesign)++;
        } else if (designability) {
            designability[res[t]]++;
        }
    }
    if (!out)
        free(res);
}

/* Random sequences for the sampling mode (Methods: where enumerating every
 * sequence is out of reach, sequences with independent equiprobable H/P
 * monomers are drawn instead).  The draws come from splitmix64 (Steele, Lea
 * and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014),
 * used as a counter-based generator: draw i of the stream seeded with x is
 * mix(x + (i + 1) * 0x9E3779B97F4A7C15) with the variant-13 mixing function
 * z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
 * z *= 0x94D049BB133111EB; z ^= z >> 31.  Sample i is the low N bits of
 * draw i, i.e. N independent fair coin flips.                              */
uint64_t or_splitmix64(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * UINT64_C(0x9E3779B97F4A7C15);
    z ^= z >> 30;
    z *= UINT64_C(0xBF58476D1CE4E5B9);
    z ^= z >> 27;
    z *= UINT64_C(0x94D049BB133111EB);
    z ^= z >> 31;
    return z;
}

void or_sample_sequences(uint64_t seed, uint64_t lo, uint64_t hi, int N, uint64_t *out)
{
    uint64_t mask = N >= 64 ? ~UINT64_C(0) : ((UINT64_C(1) << N) - 1);
    for (uint64_t i = lo; i < hi; i++)
        out[i - lo] = or_splitmix64(seed, i) & mask;
}

/* Ground states for every sequence s in [lo, hi):
 *   emin[s-lo] = min over conformations of E(s,c);
 *   out[s-lo]  = class of the unique minimising conformation, or 0xFFFF when
 *                two or more conformations share the minimum.
 * Conformation c has contacts pairs[ct_off[c] .. ct_off[c+1]) (pair units).
 * designability[q] and *nondesign are incremented (+=), never cleared.
 * Any output pointer may be NULL.  OpenMP spreads sequences over threads;
 * each sequence is computed exactly as in the serial loop.                 */
void or_ground_states(long n_conf, const int32_t *ct_off, const uint8_t *pairs,
                      const int32_t *conf_to_class, uint64_t lo, uint64_t hi,
                      uint16_t *out, int32_t *emin, uint64_t *designability,
                      uint64_t *nondesign)
{
    long count = (long)(hi - lo);
    uint16_t *res = out ? out : (uint16_t *)malloc(sizeof(uint16_t) * (size_t)(count > 0 ? count : 1));
#pragma omp parallel for schedule(dynamic, 64)
    for (long t = 0; t < count; t++) {
        uint64_t s = lo + (uint64_t)t;
        int best = 1;      /* above every energy, all of which are <= 0 */
        long nbest = 0;
        long arg = -1;
        for (long c = 0; c < n_conf; c++) {
            int e = or_energy(s, ct_off[c + 1] - ct_off[c], pairs + 2 * (size_t)ct_off[c]);
            if (e < best) {
                best = e;
                nbest = 1;
                arg = c;
            } else if (e == best) {
                nbest++;
            }
        }
        if (emin)
            emin[t] = best;
        res[t] = (nbest == 1) ? (uint16_t)conf_to_class[arg] : (uint16_t)OR_NONE;
    }
    for (long t = 0; t < count; t++) {
        if (res[t] == OR_NONE) {
            if (nondesign)
                (*nondesign)++;
        } else if (designability) {
            designability[res[t]]++;
        }
    }
    if (!out)
        free(res);
}

/* Brute-force ground states over ALL directed walks (no symmetry
 * reduction): a sequence is designing iff all minimising walks have the same
 * canonical key.  The phenotype is the rank of that conformation's class key
 * in `class_keys` (n_class keys, ascending).  For tiny boxes only.         */
void or_ground_states_brute(int X, int Y, int Z, const uint8_t *class_keys, long n_class,
                            uint64_t lo, uint64_t hi, uint16_t *out, int32_t *emin)
{
    int N = X * Y * Z;
    long nw = or_count_walks(X, Y, Z);
    uint8_t *walks = (uint8_t *)malloc((size_t)nw * N);
    or_walks(X, Y, Z, 0, walks, nw);
    uint8_t perms[48 * OR_MAXN];
    int G = or_group(X, Y, Z, perms);
    uint8_t *wkeys = (uint8_t *)malloc((size_t)nw * N);
    int *nct = (int *)malloc(sizeof(int) * (size_t)nw);
    uint8_t *wpairs = (uint8_t *)malloc((size_t)nw * 2 * (size_t)N * N);
    for (long w = 0; w < nw; w++) {
        canon_key(perms, G, N, walks + (size_t)w * N, wkeys + (size_t)w * N);
        nct[w] = or_contacts(X, Y, Z, walks + (size_t)w * N, wpairs + (size_t)w * 2 * N * N);
    }
    long count = (long)(hi - lo);
#pragma omp parallel for schedule(dynamic, 16)
    for (long t = 0; t < count; t++) {
        uint64_t s = lo + (uint64_t)t;
        int best = 1;
        for (long w = 0; w < nw; w++) {
            int e = or_energy(s, nct[w], wpairs + (size_t)w * 2 * N * N);
            if (e < best)
                best = e;
        }
        long first = -1;
        int same = 1;
        for (long w = 0; w < nw; w++) {
            int e = or_energy(s, nct[w], wpairs + (size_t)w * 2 * N * N);
            if (e != best)
                continue;
            if (first < 0)
                first = w;
            else if (memcmp(wkeys + (size_t)w * N, wkeys + (size_t)first * N, (size_t)N) != 0)
                same = 0;
        }
        if (emin)
            emin[t] = best;
        uint16_t ph = OR_NONE;
        if (same) {
            uint8_t r[OR_MAXN], rk[OR_MAXN];
            const uint8_t *k = wkeys + (size_t)first * N;
            reversed(k, N, r);
            canon_key(perms, G, N, r, rk);
            const uint8_t *ck = memcmp(k, rk, (size_t)N) <= 0 ? k : rk;
            ph = (uint16_t)find_key(class_keys, n_class, N, ck);
        }
        out[t] = ph;
    }
    free(walks);
    free(wkeys);
    free(nct);
    free(wpairs);
}

/* ------------------------------------------------------------------------ */
/* Single-point-mutation neighbourhood (Eq. 2) and neutral networks.         */
/* ------------------------------------------------------------------------ */

/* For every designing genotype g (phenotype q = map[g] < n_class) and every
 * one of its N one-bit mutants p = map[g ^ (1<<i)]:
 *   neutral[q]++ if p == q; deleterious[q]++ if p is 0xFFFF; other[q]++ else.
 * If phi_q >= 0, phi_row[p] (p < n_class) or phi_row[n_class] (deleterious:
 * 0xFFFF, or an id that is not a phenotype) counts the mutants of
 * phi_q-genotypes.  Ids at or beyond n_class are not phenotypes (Eq. 2 sums
 * over the genotypes of a phenotype), so such genotypes have no counters, as
 * in or_phi_counts.  All counters are += .                                  */
void or_neighbors(int N, const uint16_t *map, long n_class, uint64_t *neutral,
                  uint64_t *deleterious, uint64_t *other, int phi_q, uint64_t *phi_row)
{
    uint64_t total = (uint64_t)1 << N;
    for (uint64_t g = 0; g < total; g++) {
        uint16_t q = map[g];
        if (q == OR_NONE || (long)q >= n_class)
            continue;
        for (int i = 0; i < N; i++) {
            uint16_t p = map[g ^ ((uint64_t)1 << i)];
            if (p == q)
                neutral[q]++;
            else if (p == OR_NONE)
                deleterious[q]++;
            else
                other[q]++;
            if (phi_q >= 0 && q == (uint16_t)phi_q)
                phi_row[(p == OR_NONE || (long)p >= n_class) ? n_class : (long)p]++;
        }
    }
}

/* The whole matrix behind phi_pq (Eq. 2): phi_pq is the mean, over the N_q
 * genotypes g of phenotype q, of the fraction of g's N single-point mutants
 * whose phenotype is p.  counts[q * (n_class + 1) + p] receives the number of
 * (genotype of q, mutant of phenotype p) pairs, so phi_pq = counts / (N N_q);
 * column n_class counts deleterious mutants (phi_del).  Genotypes whose id is
 * not a phenotype (0xFFFF or >= n_class) have no row; such mutant ids go to
 * the deleterious column.  counts has n_class rows; all entries are += .    */
void or_phi_counts(int N, const uint16_t *map, long n_class, uint64_t *counts)
{
    uint64_t total = (uint64_t)1 << N;
    for (uint64_t g = 0; g < total; g++) {
        long q = map[g];
        if (q >= n_class)
            continue;
        for (int i = 0; i < N; i++) {
            long p = map[g ^ ((uint64_t)1 << i)];
            if (p >= n_class)
                p = n_class;
            counts[(uint64_t)q * (uint64_t)(n_class + 1) + (uint64_t)p]++;
        }
    }
}

/* Connected components of the subgraph of the N-cube induced on genotypes of
 * equal (designing) phenotype.  labels[g] = smallest genotype of g's
 * component; 0xFFFFFFFF for deleterious genotypes.  Breadth-first search
 * started from each unlabelled genotype in ascending order.                */
void or_components(int N, const uint16_t *map, uint32_t *labels)
{
    uint64_t total = (uint64_t)1 << N;
    uint32_t *queue = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)total);
    for (uint64_t g = 0; g < total; g++)
        labels[g] = 0xFFFFFFFFu;
    for (uint64_t g = 0; g < total; g++) {
        if (map[g] == OR_NONE || labels[g] != 0xFFFFFFFFu)
            continue;
        uint64_t head = 0, tail = 0;
        labels[g] = (uint32_t)g;
        queue[tail++] = (uint32_t)g;
        while (head < tail) {
            uint32_t a = queue[head++];
            for (int i = 0; i < N; i++) {
                uint32_t b = a ^ (1u << i);
                if (map[b] == map[g] && labels[b] == 0xFFFFFFFFu) {
                    labels[b] = (uint32_t)g;
                    queue[tail++] = b;
                }
            }
        }
    }
    free(queue);
}

/* Number of OpenMP threads the oracle's parallel loops use (1 without
 * OpenMP). */
int or_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Set the number of OpenMP threads later parallel loops use (no effect
 * without OpenMP); results do not depend on it. */
void or_set_num_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}
