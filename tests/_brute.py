"""Pure-Python restatement of the model's definitions for tiny lattice boxes.

Written independently of the C oracle (no shared code) so that the oracle can be
pinned against something other than itself: walks by recursion over coordinate
tuples, the box isometries from signed axis permutations, energies from
Eq. 1 with H=1/P=0, and the unique-minimum rule for the phenotype.
Only practical for N <= 12.
"""
from __future__ import annotations

import itertools

NONE = 0xFFFF


def sites(X, Y, Z):
    return [(x, y, z) for z in range(Z) for y in range(Y) for x in range(X)]


def sid(c, X, Y):
    return c[0] + X * (c[1] + Y * c[2])


def adjacent(a, b):
    return sum(abs(p - q) for p, q in zip(a, b)) == 1


def directed_walks(X, Y, Z):
    pts = sites(X, Y, Z)
    N = len(pts)
    out = []

    def rec(path, used):
        if len(path) == N:
            out.append(tuple(sid(p, X, Y) for p in path))
            return
        h = path[-1]
        for q in pts:
            if q not in used and adjacent(h, q):
                used.add(q)
                path.append(q)
                rec(path, used)
                path.pop()
                used.discard(q)

    for p in pts:
        rec([p], {p})
    return out


def isometries(X, Y, Z):
    dims = (X, Y, Z)
    pts = sites(X, Y, Z)
    maps = set()
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            img = []
            ok = True
            for c in pts:
                n = []
                for a in range(3):
                    v = c[perm[a]] * signs[a]
                    if signs[a] < 0:
                        v += dims[a] - 1
                    if not (0 <= v < dims[a]):
                        ok = False
                    n.append(v)
                img.append(tuple(n))
            if ok and sorted(img) == sorted(pts):
                m = [0] * len(pts)
                for c, n in zip(pts, img):
                    m[sid(c, X, Y)] = sid(n, X, Y)
                maps.add(tuple(m))
    return sorted(maps)


def contacts(walk, X, Y):
    N = len(walk)

    def xyz(s):
        return (s % X, (s // X) % Y, s // (X * Y))

    return {(i, j) for i in range(N) for j in range(i + 2, N) if adjacent(xyz(walk[i]), xyz(walk[j]))}


def energy(s, cts, table=None):
    if table is None:
        return -sum(((s >> i) & 1) * ((s >> j) & 1) for i, j in cts)
    return sum(table[2 * ((s >> i) & 1) + ((s >> j) & 1)] for i, j in cts)


def model(X, Y, Z, table=None):
    """Conformations, classes and the full phenotype map of a tiny box."""
    walks = directed_walks(X, Y, Z)
    G = isometries(X, Y, Z)
    N = X * Y * Z

    def key(w):
        return min(tuple(g[s] for s in w) for g in G)

    wkey = {w: key(w) for w in walks}
    conf_keys = sorted(set(wkey.values()))

    def class_key(k):
        return min(k, key(tuple(reversed(k))))

    class_keys = sorted({class_key(k) for k in conf_keys})
    cidx = {k: i for i, k in enumerate(class_keys)}
    wct = {w: contacts(w, X, Y) for w in walks}
    phen = []
    emin = []
    for s in range(1 << N):
        es = {w: energy(s, wct[w], table) for w in walks}
        m = min(es.values())
        winners = {wkey[w] for w in walks if es[w] == m}
        emin.append(m)
        phen.append(cidx[class_key(next(iter(winners)))] if len(winners) == 1 else NONE)
    return {
        "walks": walks,
        "G": G,
        "conf_keys": conf_keys,
        "class_keys": class_keys,
        "conf_contacts": [contacts(k, X, Y) for k in conf_keys],
        "phen": phen,
        "emin": emin,
    }


def gap_model(X, Y, Z, seqs, threshold=1, table=None):
    """Energy gap and thresholded phenotype of each listed sequence, scoring
    every directed walk: conformation energies are grouped by orbit key and
    sorted; gap = second - first (255 with one conformation, capped at 255)."""
    walks = directed_walks(X, Y, Z)
    G = isometries(X, Y, Z)

    def key(w):
        return min(tuple(g[s] for s in w) for g in G)

    wkey = {w: key(w) for w in walks}

    def class_key(k):
        return min(k, key(tuple(reversed(k))))

    class_keys = sorted({class_key(k) for k in wkey.values()})
    cidx = {k: i for i, k in enumerate(class_keys)}
    wct = {w: contacts(w, X, Y) for w in walks}
    res = []
    for s in seqs:
        conf_e = {}
        for w in walks:
            e = energy(s, wct[w], table)
            assert conf_e.setdefault(wkey[w], e) == e   # isometries keep the contacts
        ranked = sorted(conf_e.items(), key=lambda kv: kv[1])
        gap = 255 if len(ranked) < 2 else min(ranked[1][1] - ranked[0][1], 255)
        phen = cidx[class_key(ranked[0][0])] if gap >= threshold else NONE
        res.append((phen, ranked[0][1], gap))
    return res


def hamiltonian_path_count(X, Y, Z):
    """Directed Hamiltonian paths by dynamic programming over visited sets
    (an algorithm unrelated to depth-first search)."""
    import numpy as np

    pts = sites(X, Y, Z)
    N = len(pts)
    nb = [[sid(q, X, Y) for q in pts if adjacent(p, q)] for p in pts]
    full = (1 << N) - 1
    dp = np.zeros((1 << N, N), dtype=np.int64)
    for v in range(N):
        dp[1 << v, v] = 1
    masks = np.arange(1 << N, dtype=np.int64)
    pc = np.array([bin(m).count("1") for m in range(1 << N)])
    for k in range(1, N):
        layer = masks[pc == k]
        for v in range(N):
            has_v = layer[(layer >> v) & 1 == 1]
            for u in nb[v]:
                sel = has_v[(has_v >> u) & 1 == 0]
                dp[sel | (1 << u), u] += dp[sel, v]
    return int(dp[full].sum())
