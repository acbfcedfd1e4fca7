"""Host-side checks of libhpmap that need no GPU.

- every entry point declared in include/hp.h is exported by the library;
- hp_structures (the product's own enumerator) reproduces the oracle's
  conformations, ids, classes and contact sets exactly;
- argument validation returns the documented error codes before any device
  call is made.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2008_05612_amd as hp
from paper_2008_05612_amd import _binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(hp.library_path()):
        from paper_2008_05612_amd import build
        build.build()
    return hp.library()


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "hp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hp_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert "hp_enumerate" in names and "hp_components" in names and "hp_neighbors" in names
    handle = ctypes.CDLL(hp.library_path())
    for n in names:
        assert hasattr(handle, n), n


def test_version_and_no_error(lib):
    assert b"gfx950" in lib.hp_version()


DIMS = [(2, 2, 1), (2, 3, 1), (3, 3, 1), (2, 2, 2), (3, 4, 1), (2, 2, 3), (4, 4, 1),
        (3, 5, 1), (5, 5, 1), (2, 3, 3), (2, 4, 3), (1, 5, 1), (1, 2, 1)]


def _compare(dims):
    st = oracle.structures(*dims)
    s = hp.Structures(*dims)
    ex = s.export()
    assert s.N == st.N and s.group_order == st.G
    assert s.n_conf == st.n_conf and s.n_class == st.n_class
    assert s.n_walks == st.n_walks
    assert s.n_selfrev == int(st.self_rev.sum())
    assert np.array_equal(ex["walks"], st.conf_keys)
    assert np.array_equal(ex["conf_to_class"].astype(np.int64), st.conf_to_class.astype(np.int64))
    assert np.array_equal(ex["rev_conf"].astype(np.int64), st.rev_conf.astype(np.int64))
    assert np.array_equal(ex["self_rev"], st.self_rev)
    nbp = s.nbp
    if st.n_conf:
        assert np.all(np.diff(st.ct_off) == nbp)
    got = ex["contacts"].reshape(-1, 2)
    ref = st.pairs.reshape(-1, 2)
    # both list each conformation's contacts ascending by (i, j)
    ref_sorted = np.concatenate([np.array(sorted(map(tuple, ref[st.ct_off[c]:st.ct_off[c + 1]].tolist())),
                                          dtype=np.uint8).reshape(-1, 2) for c in range(st.n_conf)]) \
        if nbp else np.zeros((0, 2), np.uint8)
    assert np.array_equal(got, ref_sorted)
    # pair table: all odd separations >= 3, each exactly once
    pairs = ex["pairs"].astype(int)
    N = st.N
    want = {(i, j) for i in range(N) for j in range(i + 3, N) if (j - i) % 2 == 1}
    assert len(pairs) == s.K == len(want) and set(map(tuple, pairs.tolist())) == want
    assert s.W == max(1, (s.K + 31) // 32)
    assert s.K_pad % 32 == 0 and s.K_pad >= s.K + 2 and s.K_pad - 32 < s.K + 2
    return s


@pytest.mark.parametrize("dims", DIMS)
def test_structures_match_oracle(lib, dims):
    _compare(dims)


@pytest.mark.parametrize("dims", [(6, 6, 1), (3, 3, 3), (2, 3, 4)])
def test_structures_match_oracle_config_lattices(lib, dims):
    s = _compare(dims)
    if dims == (6, 6, 1):
        assert s.n_conf == 57337 and s.nbp == 25 and s.K == 289 and s.K_pad == 320
    if dims == (3, 3, 3):
        assert s.n_class == 51704 and s.nbp == 28 and s.K == 156 and s.K_pad == 160


def _status(fn, *args):
    return fn(*args)


def test_argument_errors(lib):
    h = ctypes.c_void_p()
    assert lib.hp_structures(0, 1, 1, ctypes.byref(h)) == -1
    assert lib.hp_structures(1, 1, 1, ctypes.byref(h)) == -1
    assert lib.hp_structures(7, 7, 1, ctypes.byref(h)) == -4     # N > 36
    assert lib.hp_structures(4, 4, 1, None) == -1
    assert b"NULL" in lib.hp_last_error()
    s = hp.Structures(4, 4, 1)
    fake_ws = ctypes.c_void_p(256)   # never dereferenced: validation fails first
    # empty range, range beyond 2^N, unknown form, NULL handle/workspace
    assert lib.hp_enumerate(s.handle, fake_ws, 1, 5, 5, None, None, None, None, None) == -1
    assert lib.hp_enumerate(s.handle, fake_ws, 1, 0, (1 << 16) + 1, None, None, None, None,
                            None) == -1
    assert lib.hp_enumerate(s.handle, fake_ws, 7, 0, 16, None, None, None, None, None) == -1
    assert lib.hp_enumerate(None, fake_ws, 1, 0, 16, None, None, None, None, None) == -1
    assert lib.hp_enumerate(s.handle, None, 1, 0, 16, None, None, None, None, None) == -1
    assert lib.hp_neighbors(s.handle, None, None, None, None, -1, None, None) == -1
    assert lib.hp_neighbors(s.handle, fake_ws, None, None, None, s.n_class, None, None) == -1
    assert lib.hp_components(s.handle, fake_ws, None, None, None, None, None) == -1
    # phi matrix: NULL handle, map, matrix or row_ptr; cols without vals
    assert lib.hp_phi_counts(None, fake_ws, fake_ws, None) == -1
    assert lib.hp_phi_counts(s.handle, None, fake_ws, None) == -1
    assert lib.hp_phi_counts(s.handle, fake_ws, None, None) == -1
    assert lib.hp_phi_sparse(None, fake_ws, fake_ws, None, None, 0, None, None) == -1
    assert lib.hp_phi_sparse(s.handle, None, fake_ws, None, None, 0, None, None) == -1
    assert lib.hp_phi_sparse(s.handle, fake_ws, None, None, None, 0, None, None) == -1
    assert lib.hp_phi_sparse(s.handle, fake_ws, fake_ws, fake_ws, None, 8, None, None) == -1
    assert lib.hp_phi_sparse(s.handle, fake_ws, fake_ws, None, fake_ws, 8, None, None) == -1
    big = hp.Structures(6, 6, 1)
    assert lib.hp_components(big.handle, fake_ws, fake_ws, fake_ws, None, None, None) == -4
    # energy-gap threshold outside 1 .. 255; sampling: empty draw range, idx_hi > 2^48
    assert lib.hp_enumerate_gap(s.handle, fake_ws, 1, 0, 16, 0, None, None, None, None, None,
                                None) == -1
    assert lib.hp_enumerate_gap(s.handle, fake_ws, 1, 0, 16, 256, None, None, None, None, None,
                                None) == -1
    assert lib.hp_sample(s.handle, fake_ws, 1, 5, 9, 9, 1, None, None, None, None, None, None,
                         None) == -1
    assert lib.hp_sample(s.handle, fake_ws, 1, 5, 0, (1 << 48) + 1, 1, None, None, None, None,
                         None, None, None) == -1
    assert lib.hp_sample(s.handle, fake_ws, 1, 5, 0, 16, 0, None, None, None, None, None, None,
                         None) == -1
    assert lib.hp_sample(s.handle, fake_ws, 9, 5, 0, 16, 1, None, None, None, None, None, None,
                         None) == -1
    # blocked form: plain ranges with N >= 8 and per-block bytes within int8 only
    assert lib.hp_enumerate_symmetric(s.handle, fake_ws, 2, 0, 16, None, None, None, None,
                                      None) == -5
    assert lib.hp_sample(s.handle, fake_ws, 2, 5, 0, 16, 1, None, None, None, None, None, None,
                         None) == -5
    tiny = hp.Structures(2, 3, 1)
    assert lib.hp_enumerate(tiny.handle, fake_ws, 2, 0, 16, None, None, None, None, None) == -5
    # unary weight 25: a monomer with 5 contacts alone fills a byte, so the
    # unary rows of 3x3x3 exceed the 32 rows of the first product
    heavy = hp.Structures(3, 3, 3, table=(0, -25, -25, -57))
    assert lib.hp_enumerate(heavy.handle, fake_ws, 2, 0, 16, None, None, None, None, None) == -5
    assert lib.hp_enumerate(s.handle, fake_ws, 3, 0, 16, None, None, None, None, None) == -1
    assert lib.hp_blocked_select(3, 0) == -1 and lib.hp_blocked_select(4, 4) == -1
    assert lib.hp_blocked_select(2, 3) == -1      # wide blocks run 4 or 8 waves per workgroup
    assert lib.hp_blocked_select(16, 3) == -1 and lib.hp_blocked_select(16, -1) == -1
    assert lib.hp_blocked_select(8, 3) == 0 and hp.hp_blocked_selected() == (8, 3)
    assert lib.hp_blocked_select(4, -1) == 0
    assert lib.hp_autotune_blocked(tiny.handle, fake_ws, 0, 16, 1, None, None, None, None) == -5
    assert lib.hp_autotune_blocked(s.handle, fake_ws, 0, (1 << 16) + 1, 1, None, None, None,
                                   None) == -1
    assert hp.hp_blocked_selected() == (4, -1)
    assert lib.hp_upload(s.handle, fake_ws, 10, None) == -1
    assert lib.hp_upload(s.handle, ctypes.c_void_p(257), 1 << 30, None) == -1
    assert lib.hp_batch_workspace_bytes(0) == 0
    assert lib.hp_enumerate_batch(None, 0, 1, fake_ws, 1 << 20, None) == -1
    jobs = (_binding._Job * 1)()
    jobs[0] = _binding._Job(s.handle.value, 256, 0, 16, None, None, None, None)
    assert lib.hp_enumerate_batch(jobs, 1, 1, fake_ws, 8, None) == -1     # workspace too small
    jobs[0] = _binding._Job(s.handle.value, 256, 16, 16, None, None, None, None)
    assert lib.hp_enumerate_batch(jobs, 1, 1, fake_ws, 1 << 20, None) == -1   # empty job
    g = ctypes.c_void_p()
    assert lib.hp_graph_capture_batch(jobs, 1, 0, fake_ws, 1 << 20, ctypes.byref(g)) == -5
    tiny = hp.Structures(2, 2, 1)      # N < 8: not covered by the blocked form
    jobs[0] = _binding._Job(tiny.handle.value, 256, 0, 16, None, None, None, None)
    assert lib.hp_enumerate_batch(jobs, 1, 2, fake_ws, 1 << 20, None) == -5
    assert lib.hp_graph_capture_batch(jobs, 1, 2, fake_ws, 1 << 20, ctypes.byref(g)) == -5
    # the batch without allocation: its argument checks come before any device call
    assert lib.hp_enumerate_batch_static(None, 0, 1, None) == -1
    many = (_binding._Job * 33)()
    assert lib.hp_enumerate_batch_static(many, 33, 1, None) == -4
    assert b"at most 32" in lib.hp_last_error()
    jobs[0] = _binding._Job(s.handle.value, 256, 16, 16, None, None, None, None)
    assert lib.hp_enumerate_batch_static(jobs, 1, 1, None) == -1     # empty job
    assert lib.hp_enumerate_batch_static(jobs, 1, 5, None) == -1     # unknown form
    jobs[0] = _binding._Job(tiny.handle.value, 256, 0, 16, None, None, None, None)
    assert lib.hp_enumerate_batch_static(jobs, 1, 2, None) == -5


def test_workspace_layout(lib):
    s = hp.Structures(3, 3, 3)
    n = lib.hp_workspace_bytes(s.handle)
    n_tiles = (s.n_conf + 31) // 32
    assert n >= s.n_conf * 2 + s.n_conf * s.W * 4 + n_tiles * 32 * s.K_pad
    assert n % 256 == 0


def test_energy_table_structures(lib):
    import oracle
    for dims in [(3, 3, 3), (6, 6, 1), (4, 4, 1)]:
        st = oracle.structures(*dims)
        s = hp.Structures(*dims, table=(0, -10, -10, -23))
        ref = hp.Structures(*dims)
        assert s.table == (0, -10, -10, -23) and ref.table == (0, 0, 0, -1)
        assert s.unary_rows == s.N and ref.unary_rows == 0
        assert s.K_pad == ((s.K + s.N + 2 + 31) // 32) * 32
        deg = np.zeros((st.n_conf, st.N), int)
        for c in range(st.n_conf):
            for i, j in st.pairs[st.ct_off[c]:st.ct_off[c + 1]].tolist():
                deg[c, i] += 1
                deg[c, j] += 1
        assert s.cmax == deg.max()
        assert np.array_equal(s.export()["contacts"], ref.export()["contacts"])
    h = ctypes.c_void_p()
    bad = (ctypes.c_int32 * 4)(0, -10, -11, -23)         # asymmetric
    assert lib.hp_structures_energy(3, 3, 1, bad, ctypes.byref(h)) == -1
    rep = (ctypes.c_int32 * 4)(0, 5, 5, -1)              # repulsive H-P contacts
    assert lib.hp_structures_energy(3, 3, 1, rep, ctypes.byref(h)) == -5
    big = (ctypes.c_int32 * 4)(0, -100, -100, -300)       # weights beyond int8
    assert lib.hp_structures_energy(3, 3, 3, big, ctypes.byref(h)) == -5
    assert lib.hp_structures_energy(3, 3, 1, None, ctypes.byref(h)) == -1


def test_canonical_block_count(lib):
    # reversal maps blocks (a, m, b) -> (rev b, m, rev a); count the blocks with
    # a <= rev(b) by brute force and check they cover 2^N sequences once
    for dims in [(2, 2, 2), (3, 3, 1), (3, 4, 1), (2, 2, 3), (4, 4, 1), (3, 5, 1), (2, 3, 3)]:
        s = hp.Structures(*dims)
        N = s.N
        odd = N & 1
        h = (N - 8 - odd) // 2
        rev = lambda x: int(format(x, "0%db" % h)[::-1], 2) if h else 0  # noqa: E731
        canon = diag = 0
        for m in range(2 if odd else 1):
            for a in range(1 << h):
                for b in range(1 << h):
                    if a <= rev(b):
                        canon += 1
                        diag += a == rev(b)
        assert hp.hp_canonical_block_count(s) == canon, dims
        assert 256 * (2 * (canon - diag) + diag) == 1 << N
    assert hp.hp_canonical_block_count(hp.Structures(3, 3, 3)) == 262656
    assert hp.hp_canonical_block_count(hp.Structures(2, 3, 1)) == 0
    assert hp.hp_canonical_block_count(hp.Structures(3, 3, 3, table=(0, -10, -10, -23))) == 262656
    assert hp.hp_canonical_block_count(hp.Structures(3, 3, 3, table=(0, -25, -25, -57))) == 0


def test_low10_pair_list_is_every_odd_pair():
    # the wide block geometry's pair list (shared by host tables and kernel)
    src = open(os.path.join(ROOT, "paper_2008_05612_amd", "csrc", "hp_internal.h")).read()
    words = [int(re.search(r"kLow10Pairs%d = (0x[0-9a-f]+)ull" % i, src).group(1), 16)
             for i in (0, 1)]
    n = int(re.search(r"kLow10NumPairs = (\d+);", src).group(1))
    got = [((words[p // 8] >> (8 * (p % 8))) & 15, ((words[p // 8] >> (8 * (p % 8))) >> 4) & 15)
           for p in range(16)]
    want = [(a, b) for a in range(10) for b in range(a + 1, 10) if (b - a) >= 3 and (b - a) % 2]
    assert n == 16 and sorted(got) == want and len(set(got)) == 16
    # 1 block row, 10 weights, 16 pair rows and 2 index rows fit the 32 rows
    assert 1 + 10 + n + 2 <= 32


def test_mid10_odd_pair_list_is_every_odd_pair():
    # canonical wide blocks of odd N: x-indices 0 .. 4 sit at offsets 0 .. 4,
    # 5 .. 9 at offsets 6 .. 10 (the middle monomer stays outer)
    src = open(os.path.join(ROOT, "paper_2008_05612_amd", "csrc", "hp_internal.h")).read()
    words = [int(re.search(r"kMid10OddPairs%d = (0x[0-9a-f]+)ull" % i, src).group(1), 16)
             for i in (0, 1)]
    got = [((words[p // 8] >> (8 * (p % 8))) & 15, ((words[p // 8] >> (8 * (p % 8))) >> 4) & 15)
           for p in range(16)]
    off = [x + (x >= 5) for x in range(10)]
    want = [(a, b) for a in range(10) for b in range(a + 1, 10)
            if off[b] - off[a] >= 3 and (off[b] - off[a]) % 2]
    assert sorted(got) == want and len(set(got)) == 16


def test_wide11_pair_list_is_every_odd_pair():
    # 2048-sequence wide blocks: x-indices 0 .. 4 at monomers 0 .. 4, 5 .. 10
    # at the even monomers 6 .. 16; a chunk of 2^17 sequences holds 64 blocks
    src = open(os.path.join(ROOT, "paper_2008_05612_amd", "csrc", "hp_internal.h")).read()
    words = [int(re.search(r"kW11Pairs%d = (0x[0-9A-Fa-f]+)ull" % i, src).group(1), 16)
             for i in (0, 1)]
    got = [((words[p // 8] >> (8 * (p % 8))) & 15, ((words[p // 8] >> (8 * (p % 8))) >> 4) & 15)
           for p in range(16)]
    pos = [x if x < 5 else 2 * x - 4 for x in range(11)]
    want = [(a, b) for a in range(11) for b in range(a + 1, 11)
            if pos[b] - pos[a] >= 3 and (pos[b] - pos[a]) % 2]
    real = [pr for pr in got if (pos[pr[1]] - pos[pr[0]]) % 2]
    pad = [pr for pr in got if not (pos[pr[1]] - pos[pr[0]]) % 2]
    assert sorted(real) == want and len(set(real)) == 14
    # the two padding pairs have equal parity: never in contact, rows stay zero
    assert len(pad) == 2 and all(a < b for a, b in pad)
    assert 1 + 11 + 16 + 2 <= 32
    # varying and outer monomers of a chunk partition monomers 0 .. 16
    outer = [5 + 2 * k for k in range(6)]
    assert sorted(pos + outer) == list(range(17))
    assert int(re.search(r"kWide11ChunkBits = (\d+);", src).group(1)) == 17


def test_wide_block_count(lib):
    # wide blocks vary the 10 monomers around the middle; reversal maps block
    # (a, m, b) -> (rev b, m, rev a): count a <= rev(b) by brute force and
    # check that the blocks and their reverses cover 2^N sequences once
    for dims in [(2, 5, 1), (3, 4, 1), (2, 2, 3), (4, 4, 1), (3, 5, 1), (2, 2, 4), (2, 3, 3)]:
        s = hp.Structures(*dims)
        N = s.N
        odd = N & 1
        h = (N - 10 - odd) // 2
        rev = lambda x: int(format(x, "0%db" % h)[::-1], 2) if h else 0  # noqa: E731
        canon = diag = 0
        for m in range(2 if odd else 1):
            for a in range(1 << h):
                for b in range(1 << h):
                    if a <= rev(b):
                        canon += 1
                        diag += a == rev(b)
        assert hp.hp_wide_block_count(s) == canon, dims
        assert 1024 * (2 * (canon - diag) + diag) == 1 << N
    assert hp.hp_wide_block_count(hp.Structures(3, 3, 3)) == 65792
    assert hp.hp_wide_block_count(hp.Structures(6, 6, 1)) == 33558528
    assert hp.hp_wide_block_count(hp.Structures(3, 3, 1)) == 0          # N < 10
    assert hp.hp_wide_block_count(hp.Structures(3, 3, 3, table=(0, -10, -10, -23))) == 0
    fake_ws = ctypes.c_void_p(256)
    s = hp.Structures(4, 4, 1)
    assert lib.hp_enumerate_symmetric_wide(s.handle, fake_ws, 5, 5, None, None, None, None,
                                           None) == -1
    assert lib.hp_enumerate_symmetric_wide(s.handle, fake_ws, 0, 137, None, None, None, None,
                                           None) == -1
    assert lib.hp_enumerate_symmetric_wide(s.handle, None, 0, 1, None, None, None, None,
                                           None) == -1
    t = hp.Structures(3, 3, 3, table=(0, -10, -10, -23))
    assert lib.hp_enumerate_symmetric_wide(t.handle, fake_ws, 0, 1, None, None, None, None,
                                           None) == -5


def test_low8_pair_list_is_every_odd_pair():
    # the plain block geometry's pair list (shared by host tables and kernel)
    # holds exactly the pairs of the low 8 monomers with odd separation >= 3
    src = open(os.path.join(ROOT, "paper_2008_05612_amd", "csrc", "hp_internal.h")).read()
    c = int(re.search(r"kLow8Pairs = (0x[0-9a-f]+)ull", src).group(1), 16)
    last = int(re.search(r"kLow8Pair8 = (0x[0-9a-f]+);", src).group(1), 16)
    n = int(re.search(r"kLow8NumPairs = (\d+);", src).group(1))
    got = [((c >> (8 * p)) & 15, ((c >> (8 * p)) >> 4) & 15) for p in range(8)]
    got.append((last & 15, last >> 4))
    want = [(a, b) for a in range(8) for b in range(a + 1, 8) if (b - a) >= 3 and (b - a) % 2]
    assert n == 9 and sorted(got) == want and len(set(got)) == 9
