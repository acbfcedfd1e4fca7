"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every check uses a printed count
from the paper, a closed form, an invariant, or an independent brute force
(``tests/_brute.py``, pure Python) on tiny lattices.
"""
import os

import numpy as np
import pytest

import oracle
from tests import _brute

GOLD = os.path.join(os.path.dirname(__file__), "golden")
NONE = 0xFFFF


def _paper_counts():
    rows = {}
    for line in open(os.path.join(GOLD, "paper_counts.txt")):
        if line.startswith("#") or not line.strip():
            continue
        lat, qty, val = line.split()[:3]
        rows[(lat, qty)] = int(val)
    return rows


def _edges(X, Y, Z):
    return (X - 1) * Y * Z + X * (Y - 1) * Z + X * Y * (Z - 1)


TINY = [(2, 2, 1), (2, 3, 1), (3, 3, 1), (2, 2, 2), (3, 4, 1), (2, 2, 3)]


# --------------------------------------------------------------------------
# Structure enumeration
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dims", TINY + [(4, 4, 1), (3, 5, 1), (2, 3, 3)])
def test_walk_count_matches_subset_dp(dims):
    # dynamic programming over visited sets counts directed Hamiltonian paths
    # by a method that shares nothing with depth-first search
    assert oracle.count_walks(*dims) == _brute.hamiltonian_path_count(*dims)


@pytest.mark.parametrize("dims", TINY + [(4, 4, 1)])
def test_pruning_does_not_change_the_walk_set(dims):
    a = {tuple(w) for w in oracle.walks(*dims, prune=True).tolist()}
    b = {tuple(w) for w in oracle.walks(*dims, prune=False).tolist()}
    assert a == b and len(a) == oracle.count_walks(*dims)


@pytest.mark.parametrize("dims", TINY)
def test_walks_and_group_match_python_brute_force(dims):
    ref = _brute.directed_walks(*dims)
    got = [tuple(w) for w in oracle.walks(*dims).tolist()]
    assert sorted(got) == sorted(ref)
    G = {tuple(g) for g in oracle.group(*dims).tolist()}
    assert G == set(_brute.isometries(*dims))


@pytest.mark.parametrize("dims,order", [((2, 2, 1), 8), ((2, 3, 1), 4), ((3, 3, 1), 8),
                                        ((6, 6, 1), 8), ((2, 3, 4), 8), ((3, 3, 3), 48),
                                        ((5, 5, 1), 8)])
def test_group_order_and_isometry(dims, order):
    X, Y, Z = dims
    G = oracle.group(*dims)
    assert G.shape[0] == order
    N = X * Y * Z
    xyz = [(s % X, (s // X) % Y, s // (X * Y)) for s in range(N)]
    for g in G:
        assert sorted(g.tolist()) == list(range(N))
        for a in range(N):
            for b in range(N):
                assert _brute.adjacent(xyz[a], xyz[b]) == _brute.adjacent(xyz[g[a]], xyz[g[b]])


@pytest.mark.parametrize("dims", TINY + [(4, 4, 1), (5, 5, 1)])
def test_closed_forms_small(dims):
    _check_closed_forms(oracle.structures(*dims))


def _check_closed_forms(st):
    X, Y, Z = st.dims
    N = st.N
    # only the identity fixes a directed Hamiltonian path, so every orbit has |G| walks
    assert st.n_walks == st.G * st.n_conf
    # reversal pairs conformations; self-reverse ones are their own class
    assert st.n_class == (st.n_conf + int(st.self_rev.sum())) // 2
    assert np.array_equal(st.rev_conf[st.rev_conf], np.arange(st.n_conf))
    assert np.array_equal(st.conf_to_class[st.rev_conf], st.conf_to_class)
    # every compact walk uses N-1 lattice edges as bonds, the rest are contacts
    nbp = _edges(X, Y, Z) - (N - 1)
    assert np.all(np.diff(st.ct_off) == nbp)
    d = st.pairs[:, 1].astype(int) - st.pairs[:, 0].astype(int)
    assert np.all(d >= 3) and np.all(d % 2 == 1)   # bipartite lattice
    # keys ascending and distinct
    k = st.conf_keys.astype(np.int64)
    assert all(tuple(k[i]) < tuple(k[i + 1]) for i in range(min(len(k) - 1, 2000)))


def test_paper_counts_6x6():
    pc = _paper_counts()
    st = oracle.structures(6, 6, 1)
    assert st.n_conf == pc[("6x6", "n_conf")]
    assert np.all(np.diff(st.ct_off) == pc[("6x6", "nbp")])
    _check_closed_forms(st)


def test_paper_counts_3x3x3():
    pc = _paper_counts()
    st = oracle.structures(3, 3, 3)
    assert st.n_class == pc[("3x3x3", "n_class")]
    _check_closed_forms(st)


@pytest.mark.parametrize("dims", TINY)
def test_structures_match_python_brute_force(dims):
    ref = _brute.model(*dims) if np.prod(dims) <= 9 else None
    st = oracle.structures(*dims)
    if ref is None:
        walks = _brute.directed_walks(*dims)
        G = _brute.isometries(*dims)
        keys = sorted({min(tuple(g[s] for s in w) for g in G) for w in walks})
        assert [tuple(x) for x in st.conf_keys.tolist()] == keys
        return
    assert [tuple(x) for x in st.conf_keys.tolist()] == ref["conf_keys"]
    assert [tuple(x) for x in st.class_keys.tolist()] == ref["class_keys"]
    assert st.contact_sets() == ref["conf_contacts"]


# --------------------------------------------------------------------------
# Hand-derived tiny lattices
# --------------------------------------------------------------------------

def test_2x2_single_conformation_designs_everything():
    # one conformation: the unique minimum is always attained by it (E <= 0),
    # so all 16 sequences design class 0
    st = oracle.structures(2, 2, 1)
    assert st.n_conf == 1 and st.n_class == 1
    assert st.contact_sets() == [{(0, 3)}]
    gs = oracle.ground_states(st)
    assert gs.designability.tolist() == [16] and gs.nondesign == 0


def test_2x3_hand_derived():
    st = oracle.structures(2, 3, 1)
    # four conformations: S (corner to opposite corner), U (corner to adjacent
    # corner), J (corner to middle) and J' = R(J)
    sets = st.contact_sets()
    assert sorted(map(sorted, sets)) == sorted(map(sorted, [
        {(0, 3), (2, 5)}, {(0, 5), (1, 4)}, {(0, 5), (2, 5)}, {(0, 3), (0, 5)}]))
    gs = oracle.ground_states(st)
    by_set = {}
    for c, s in enumerate(sets):
        by_set[frozenset(s)] = st.conf_to_class[c]
    qS = by_set[frozenset({(0, 3), (2, 5)})]
    qU = by_set[frozenset({(0, 5), (1, 4)})]
    qJ = by_set[frozenset({(0, 5), (2, 5)})]
    assert by_set[frozenset({(0, 3), (0, 5)})] == qJ
    d = gs.designability
    # U designs when h1 h4 = 1 and h0 h5 = 1 but not both other contacts...
    # counted by hand: U 9, J-class 6 (3 per direction), S 0, rest deleterious
    assert (int(d[qU]), int(d[qJ]), int(d[qS]), gs.nondesign) == (9, 6, 0, 49)
    # h = (1,.,0,1,.,1) with h1 h4 = 0 designs J' only (both directions scored)
    s = 0b101001  # H at 0, 3, 5
    assert gs.out[s] == qJ


def test_3x3_hand_derived_examples():
    st = oracle.structures(3, 3, 1)
    assert st.n_conf == 5 and st.n_class == 3
    gs = oracle.ground_states(st)
    sets = st.contact_sets()
    si = sets.index({(0, 7), (1, 8), (3, 8), (5, 8)})        # spiral into the centre
    so = sets.index({(0, 3), (0, 5), (0, 7), (1, 8)})        # its reverse
    assert st.conf_to_class[si] == st.conf_to_class[so]
    # H at {1,3,8}: energies SI -2, SO -1, snake -1, C1 0, C2 -1 -> designs SI
    s = (1 << 1) | (1 << 3) | (1 << 8)
    assert gs.emin[s] == -2 and gs.out[s] == st.conf_to_class[si]
    # its reverse, H at {0,5,7}, designs SO: the same class
    assert gs.out[(1 << 0) | (1 << 5) | (1 << 7)] == st.conf_to_class[si]
    # H at {0,7}: SI, SO and C1 all reach -1 -> deleterious
    assert gs.out[(1 << 0) | (1 << 7)] == NONE


# --------------------------------------------------------------------------
# Energies and ground states
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dims", [(2, 2, 1), (2, 3, 1), (3, 3, 1), (2, 2, 2)])
def test_ground_states_match_python_brute_force(dims):
    ref = _brute.model(*dims)
    st = oracle.structures(*dims)
    gs = oracle.ground_states(st)
    assert gs.out.tolist() == ref["phen"]
    assert gs.emin.tolist() == ref["emin"]


@pytest.mark.parametrize("dims", [(2, 2, 1), (2, 3, 1), (3, 3, 1), (2, 2, 2), (3, 4, 1),
                                  (2, 2, 3), (4, 4, 1)])
def test_reduced_equals_all_walks(dims):
    st = oracle.structures(*dims)
    gs = oracle.ground_states(st)
    out_b, emin_b = oracle.ground_states_brute(st)
    assert np.array_equal(gs.out, out_b)
    assert np.array_equal(gs.emin, emin_b)


def _rev_bits(s, N):
    return int(format(s, "0%db" % N)[::-1], 2)


@pytest.mark.parametrize("dims", [(4, 4, 1), (3, 4, 1), (2, 2, 3)])
def test_energy_closed_forms(dims):
    st = oracle.structures(*dims)
    N = st.N
    nbp = int(st.ct_off[1] - st.ct_off[0])
    allh = (1 << N) - 1
    even = sum(1 << i for i in range(0, N, 2))
    odd = sum(1 << i for i in range(1, N, 2))
    rng = np.random.default_rng(7)
    for c in range(st.n_conf):
        pc = st.pairs[st.ct_off[c]:st.ct_off[c + 1]]
        assert oracle.energy(allh, pc) == -nbp
        assert oracle.energy(even, pc) == 0 and oracle.energy(odd, pc) == 0
        for s in rng.integers(0, 1 << N, 8).tolist():
            e = oracle.energy(s, pc)
            assert -nbp <= e <= 0
            # reversing the chain of the structure is reversing the sequence
            rc = st.rev_conf[c]
            prc = st.pairs[st.ct_off[rc]:st.ct_off[rc + 1]]
            assert oracle.energy(_rev_bits(s, N), pc) == oracle.energy(s, prc)
            # the energy counts H-H contacts exactly
            assert e == -sum(((s >> i) & 1) & ((s >> j) & 1) for i, j in pc.tolist())


def _check_map_invariants(st, gs, N):
    assert int(gs.designability.sum()) + gs.nondesign == 1 << N
    idx = np.arange(1 << N, dtype=np.int64)
    rev = np.zeros_like(idx)
    for i in range(N):
        rev |= ((idx >> i) & 1) << (N - 1 - i)
    assert np.array_equal(gs.out[rev], gs.out)
    assert np.array_equal(gs.emin[rev], gs.emin)
    odd_classes = st.self_rev == 0
    assert np.all(gs.designability[odd_classes] % 2 == 0)
    even = sum(1 << i for i in range(0, N, 2))
    odd = sum(1 << i for i in range(1, N, 2))
    pure = (idx & odd == 0) | (idx & even == 0)
    if st.n_conf >= 2:
        assert np.all(gs.out[pure] == NONE)
    counts = np.bincount(gs.out[gs.out != NONE], minlength=st.n_class)
    assert np.array_equal(counts, gs.designability)


@pytest.mark.parametrize("dims", [(3, 3, 1), (3, 4, 1), (4, 4, 1), (2, 2, 3), (2, 3, 3)])
def test_map_invariants(dims):
    st = oracle.structures(*dims)
    gs = oracle.ground_states(st)
    _check_map_invariants(st, gs, st.N)


def test_windows_compose():
    st = oracle.structures(4, 4, 1)
    full = oracle.ground_states(st)
    a = oracle.ground_states(st, 0, 12345)
    b = oracle.ground_states(st, 12345, 1 << 16)
    assert np.array_equal(np.concatenate([a.out, b.out]), full.out)
    assert np.array_equal(a.designability + b.designability, full.designability)
    assert a.nondesign + b.nondesign == full.nondesign


# --------------------------------------------------------------------------
# Neighbourhood counts and neutral networks
# --------------------------------------------------------------------------

def _py_neighbors(N, phen, n_class, phi_q):
    neu = np.zeros(n_class, np.uint64)
    dele = np.zeros(n_class, np.uint64)
    oth = np.zeros(n_class, np.uint64)
    row = np.zeros(n_class + 1, np.uint64)
    phen = np.asarray(phen)
    g = np.arange(1 << N)
    q = phen
    des = q != NONE
    for i in range(N):
        p = phen[g ^ (1 << i)]
        m = des & (p == q)
        np.add.at(neu, q[m], 1)
        m = des & (p == NONE)
        np.add.at(dele, q[m], 1)
        m = des & (p != q) & (p != NONE)
        np.add.at(oth, q[m], 1)
        sel = q == phi_q
        pp = np.where(p[sel] == NONE, n_class, p[sel])
        np.add.at(row, pp, 1)
    return neu, dele, oth, row


@pytest.mark.parametrize("dims", [(3, 3, 1), (4, 4, 1), (2, 2, 3)])
def test_neighbors_match_python(dims):
    st = oracle.structures(*dims)
    gs = oracle.ground_states(st)
    top = int(np.argmax(gs.designability))
    nb = oracle.neighbors(st.N, gs.out, st.n_class, phi_q=top)
    neu, dele, oth, row = _py_neighbors(st.N, gs.out, st.n_class, top)
    assert np.array_equal(nb.neutral, neu)
    assert np.array_equal(nb.deleterious, dele)
    assert np.array_equal(nb.other, oth)
    assert np.array_equal(nb.phi_row, row)
    # each neutral edge is seen from both ends; every mutant is one of the three kinds
    assert np.all(nb.neutral % 2 == 0)
    assert np.array_equal(nb.neutral + nb.deleterious + nb.other,
                          st.N * gs.designability.astype(np.uint64))
    assert int(row.sum()) == st.N * int(gs.designability[top])
    assert int(row[top]) == int(nb.neutral[top])


def test_neighbors_ids_beyond_n_class():
    """Ids at or beyond n_class are not phenotypes: such genotypes have no
    counters, and as mutants they count as 'other' in the three counters and
    in the deleterious column of the phi row (like 0xFFFF), the column the
    phi matrix uses for them.  Brute force with plain loops on a 2^10 map."""
    N, n_class = 10, 6
    rng = np.random.default_rng(5)
    phen = rng.integers(0, n_class + 3, 1 << N).astype(np.uint16)
    phen[rng.random(1 << N) < 0.2] = NONE
    q0 = int(phen[phen < n_class][0])
    neu = np.zeros(n_class, np.uint64); dele = np.zeros_like(neu); oth = np.zeros_like(neu)
    row = np.zeros(n_class + 1, np.uint64)
    for g in range(1 << N):
        q = int(phen[g])
        if q >= n_class:          # 0xFFFF included
            continue
        for i in range(N):
            p = int(phen[g ^ (1 << i)])
            if p == q:
                neu[q] += 1
            elif p == NONE:
                dele[q] += 1
            else:
                oth[q] += 1
            if q == q0:
                row[n_class if p >= n_class else p] += 1
    nb = oracle.neighbors(N, phen, n_class, phi_q=q0)
    assert np.array_equal(nb.neutral, neu)
    assert np.array_equal(nb.deleterious, dele)
    assert np.array_equal(nb.other, oth)
    assert np.array_equal(nb.phi_row, row)
    assert np.array_equal(oracle.phi_counts(N, phen, n_class)[q0], row)


def _py_components(N, phen):
    lab = [0xFFFFFFFF] * (1 << N)
    for g in range(1 << N):
        if phen[g] == NONE or lab[g] != 0xFFFFFFFF:
            continue
        comp = {g}
        stack = [g]
        while stack:
            a = stack.pop()
            for i in range(N):
                b = a ^ (1 << i)
                if phen[b] == phen[g] and b not in comp:
                    comp.add(b)
                    stack.append(b)
        m = min(comp)
        for b in comp:
            lab[b] = m
    return np.array(lab, dtype=np.uint32)


@pytest.mark.parametrize("dims", [(3, 3, 1), (3, 4, 1), (4, 4, 1)])
def test_components_match_python(dims):
    st = oracle.structures(*dims)
    gs = oracle.ground_states(st)
    lab = oracle.components(st.N, gs.out)
    ref = _py_components(st.N, gs.out.tolist())
    assert np.array_equal(lab, ref)
    des = gs.out != NONE
    sizes = np.bincount(gs.out[des], minlength=st.n_class)
    assert np.array_equal(sizes, gs.designability)
    # every label is a member of its own component and the smallest one
    assert np.all(lab[des] <= np.arange(1 << st.N)[des])
    assert np.all(gs.out[lab[des]] == gs.out[des])


# --------------------------------------------------------------------------
# Two-letter contact tables (Table 1 of the paper, scaled by 10)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dims", [(2, 2, 1), (2, 3, 1), (3, 3, 1), (2, 2, 2)])
def test_table_ground_states_match_python_brute_force(dims):
    ref = _brute.model(*dims, table=oracle.HP1996_X10)
    st = oracle.structures(*dims)
    gs = oracle.ground_states(st, table=oracle.HP1996_X10)
    assert gs.out.tolist() == ref["phen"]
    assert gs.emin.tolist() == ref["emin"]


def test_pure_hp_table_is_the_default():
    st = oracle.structures(4, 4, 1)
    a = oracle.ground_states(st)
    b = oracle.ground_states(st, table=oracle.PURE_HP)
    assert np.array_equal(a.out, b.out) and np.array_equal(a.emin, b.emin)


@pytest.mark.parametrize("dims", [(4, 4, 1), (2, 2, 3)])
def test_table_energy_decomposition(dims):
    # any symmetric two-letter table: E = a n_HH + b sum_i h_i c_i + E_PP NBP
    # with a = E_HH - 2 E_HP + E_PP, b = E_HP - E_PP, c_i = contacts of i
    st = oracle.structures(*dims)
    rng = np.random.default_rng(11)
    for table in (oracle.HP1996_X10, (3, -5, -5, -17), (-2, 4, 4, -9)):
        e_pp, e_ph, e_hp, e_hh = table
        a, b = e_hh - 2 * e_hp + e_pp, e_hp - e_pp
        for c in range(0, st.n_conf, max(1, st.n_conf // 40)):
            pc = st.pairs[st.ct_off[c]:st.ct_off[c + 1]]
            deg = np.zeros(st.N, int)
            for i, j in pc.tolist():
                deg[i] += 1
                deg[j] += 1
            for s in rng.integers(0, 1 << st.N, 6).tolist():
                h = [(s >> i) & 1 for i in range(st.N)]
                n_hh = sum(h[i] * h[j] for i, j in pc.tolist())
                want = a * n_hh + b * sum(h[i] * deg[i] for i in range(st.N)) + e_pp * len(pc)
                assert oracle.energy_table(s, pc, table) == want


def test_hp1996_map_invariants():
    st = oracle.structures(3, 4, 1)
    gs = oracle.ground_states(st, table=oracle.HP1996_X10)
    _check_map_invariants_table(st, gs, st.N)


def _check_map_invariants_table(st, gs, N):
    assert int(gs.designability.sum()) + gs.nondesign == 1 << N
    idx = np.arange(1 << N, dtype=np.int64)
    rev = np.zeros_like(idx)
    for i in range(N):
        rev |= ((idx >> i) & 1) << (N - 1 - i)
    assert np.array_equal(gs.out[rev], gs.out)
    assert np.all(gs.designability[st.self_rev == 0] % 2 == 0)


# --------------------------------------------------------------------------
# Energy gap, threshold and random sampling
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dims", [(2, 2, 1), (2, 3, 1), (3, 3, 1), (2, 2, 2)])
@pytest.mark.parametrize("table,thresholds", [(None, (1, 2, 3)),
                                              (oracle.HP1996_X10, (1, 7, 10, 13, 30))])
def test_gap_matches_python_brute_force(dims, table, thresholds):
    st = oracle.structures(*dims)
    seqs = list(range(1 << st.N))
    for thr in thresholds:
        ref = _brute.gap_model(*dims, seqs, thr, table)
        g = oracle.ground_states_gap(st, seqs, thr, table)
        assert g.out.tolist() == [r[0] for r in ref]
        assert g.emin.tolist() == [r[1] for r in ref]
        assert g.gap.tolist() == [r[2] for r in ref]


def test_gap_matches_python_brute_force_3x4_sample():
    st = oracle.structures(3, 4, 1)
    seqs = np.random.default_rng(5).integers(0, 1 << st.N, 200).tolist()
    for table, thr in ((None, 2), (oracle.HP1996_X10, 10)):
        ref = _brute.gap_model(3, 4, 1, seqs, thr, table)
        g = oracle.ground_states_gap(st, seqs, thr, table)
        assert [tuple(x) for x in zip(g.out.tolist(), g.emin.tolist(), g.gap.tolist())] == ref


def test_gap_hand_derived_3x3():
    # H at {1,3,8}: energies SI -2, SO -1, SN -1, C1 0, C2 -1 -> gap 1;
    # H at {0,7}: three-way tie at -1 -> gap 0; 2x2 has one conformation.
    st = oracle.structures(3, 3, 1)
    g = oracle.ground_states_gap(st, [266, 129], threshold=1)
    assert g.gap.tolist() == [1, 0] and g.emin.tolist() == [-2, -1]
    assert g.out[0] != oracle.NONE and g.out[1] == oracle.NONE
    g2 = oracle.ground_states_gap(st, [266], threshold=2)
    assert g2.out[0] == oracle.NONE and g2.nondesign == 1
    one = oracle.ground_states_gap(oracle.structures(2, 2, 1), range(16), threshold=255)
    assert np.all(one.gap == 255) and np.all(one.out == 0)


@pytest.mark.parametrize("dims", [(4, 4, 1), (2, 2, 3)])
def test_gap_closed_forms_and_threshold_monotone(dims):
    st = oracle.structures(*dims)
    N = st.N
    seqs = np.arange(1 << N, dtype=np.uint64)
    nbp = st.ct_off[1] - st.ct_off[0]
    base = oracle.ground_states(st)
    prev = None
    for thr in range(1, 6):
        g = oracle.ground_states_gap(st, seqs, thr)
        # threshold 1 is the uniqueness rule (the map pinned above)
        if thr == 1:
            assert np.array_equal(g.out, base.out) and np.array_equal(g.emin, base.emin)
        assert np.array_equal(g.out != oracle.NONE, g.gap >= thr)
        assert np.all(g.gap <= nbp)
        assert int(g.designability.sum()) + g.nondesign == 1 << N
        if prev is not None:
            assert np.all(g.designability <= prev.designability)
            kept = g.out != oracle.NONE
            assert np.array_equal(g.out[kept], prev.out[kept])
        prev = g
    # all-H and parity-pure sequences tie every conformation: gap 0
    even = sum(1 << i for i in range(0, N, 2))
    odd = sum(1 << i for i in range(1, N, 2))
    g = oracle.ground_states_gap(st, [(1 << N) - 1, even, odd, 0])
    assert g.gap.tolist() == [0, 0, 0, 0]
    assert g.emin[0] == -nbp


def test_splitmix64_published_values():
    path = os.path.join(os.path.dirname(__file__), "golden", "splitmix64.txt")
    rows = [line.split() for line in open(path) if line.strip() and not line.startswith("#")]
    assert len(rows) == 3
    for i, v in rows:
        assert oracle.splitmix64(0, int(i)) == int(v, 16)


def test_sampled_sequences_are_fair_coin_flips():
    N = 36
    seqs = oracle.sample_sequences(0x2008056120, 0, 1 << 16, N)
    assert seqs.dtype == np.uint64 and np.all(seqs < (1 << N))
    assert np.array_equal(seqs[100:200], oracle.sample_sequences(0x2008056120, 100, 200, N))
    n = seqs.shape[0]
    for i in range(N):
        ones = int(((seqs >> np.uint64(i)) & np.uint64(1)).sum())
        assert abs(ones - n / 2) < 5 * np.sqrt(n / 4), i
    # different seeds give different streams; no repeats among 2^16 36-bit draws is
    # expected (birthday bound 2^32 / 2^36 = 1/16 chance of one)
    assert len(np.unique(seqs)) >= n - 2
    other = oracle.sample_sequences(1, 0, 1 << 10, N)
    assert not np.array_equal(other, seqs[:1 << 10])


# --------------------------------------------------------------------------
# The full phi_pq matrix (Eq. 2 for every pair of phenotypes)
# --------------------------------------------------------------------------

def test_phi_counts_hand_example():
    # N = 2: genotypes 0, 1, 2, 3 with phenotypes q0, q0, q1, deleterious.
    # 0 -> {1: q0, 2: q1}; 1 -> {0: q0, 3: del}; 2 -> {3: del, 0: q0}.
    c = oracle.phi_counts(2, np.array([0, 0, 1, NONE], np.uint16), 2)
    assert c.tolist() == [[2, 1, 1], [1, 0, 1]]
    # an id that is not a phenotype (5 >= n_class) has no row and counts as
    # a deleterious mutant
    c = oracle.phi_counts(2, np.array([0, 5, 1, NONE], np.uint16), 2)
    assert c.tolist() == [[0, 1, 1], [1, 0, 1]]


@pytest.mark.parametrize("N", [1, 5, 10])
def test_phi_counts_closed_forms(N):
    n = 1 << N
    # one phenotype everywhere: every mutation is neutral
    c = oracle.phi_counts(N, np.zeros(n, np.uint16), 1)
    assert c.tolist() == [[N * n, 0]]
    # nothing folds: no rows carry counts
    assert not oracle.phi_counts(N, np.full(n, NONE, np.uint16), 3).any()
    # phenotype = parity of the number of H: every mutation flips it
    par = np.array([bin(g).count("1") & 1 for g in range(n)], np.uint16)
    c = oracle.phi_counts(N, par, 2)
    assert c.tolist() == [[0, N * n // 2, 0], [N * n // 2, 0, 0]]


def test_phi_counts_brute_force_random_maps():
    rng = np.random.default_rng(11)
    for N, n_class in ((4, 3), (7, 5), (8, 40)):
        # ids beyond n_class and the deleterious id mixed in
        phen = rng.integers(0, n_class + 2, 1 << N).astype(np.uint16)
        phen[rng.random(1 << N) < 0.3] = NONE
        want = {}
        for g in range(1 << N):
            if phen[g] >= n_class:
                continue
            for i in range(N):
                p = int(phen[g ^ (1 << i)])
                key = (int(phen[g]), p if p < n_class else n_class)
                want[key] = want.get(key, 0) + 1
        got = oracle.phi_counts(N, phen, n_class)
        assert got.shape == (n_class, n_class + 1)
        nz = {(int(q), int(p)): int(got[q, p]) for q, p in zip(*np.nonzero(got))}
        assert nz == want


@pytest.mark.parametrize("dims", [(2, 3, 1), (3, 3, 1), (4, 4, 1), (2, 2, 3)])
def test_phi_counts_invariants(dims):
    st = oracle.structures(*dims)
    gs = oracle.ground_states(st)
    n = st.n_class
    c = oracle.phi_counts(st.N, gs.out, n)
    nb = oracle.neighbors(st.N, gs.out, n)
    # a single-point mutation is its own inverse: q -> p links equal p -> q links
    assert np.array_equal(c[:, :n], c[:, :n].T)
    # every genotype of q has N mutants
    assert np.array_equal(c.sum(axis=1), st.N * gs.designability.astype(np.uint64))
    # the diagonal is the robustness numerator, the last column phi_del's
    assert np.array_equal(np.diag(c[:, :n]), nb.neutral)
    assert np.array_equal(c[:, n], nb.deleterious)
    assert np.array_equal(c[:, :n].sum(axis=1) - np.diag(c[:, :n]), nb.other)
    for q in range(n):
        row = oracle.neighbors(st.N, gs.out, n, phi_q=q).phi_row
        assert np.array_equal(c[q], row)
