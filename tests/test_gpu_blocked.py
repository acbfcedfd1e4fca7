"""GPU parity of the block-factorised int8 form (HP_FORM_BLOCKED_I8) against
the oracle, bit-exact: full maps of every small box it covers (N >= 8),
ragged and unaligned ranges (blocks of 256 sequences cut by the range), oracle
windows on the configuration lattices, the energy-gap threshold, a pure pair
table with weight 3, and the full 3x3x3 map in the benchmark's launch
configuration, equal to the dense int8 form's map."""
import numpy as np
import pytest

import oracle
import paper_2008_05612_amd as hp
from tests.conftest import gpu_available
from tests.test_gpu_enumerate import _assert_equal, _full_map_invariants, _oracle, _windows, run

pytestmark = pytest.mark.gpu
BLK = hp.FORM_BLOCKED_I8


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("dims", [(3, 3, 1), (2, 2, 2), (3, 4, 1), (2, 2, 3), (4, 4, 1),
                                  (3, 5, 1), (2, 3, 3)])
def test_blocked_full_small_lattices(dims):
    N = dims[0] * dims[1] * dims[2]
    _assert_equal(run(dims, BLK, 0, 1 << N), _oracle(dims, 0, 1 << N))


@pytest.mark.parametrize("lo,hi", [(0, 1), (3, 1000), (511, 513), (255, 257), (40000, 65536),
                                   (1, 65535), (256, 512), (65280, 65536)])
def test_blocked_ragged_ranges_4x4(lo, hi):
    _assert_equal(run((4, 4, 1), BLK, lo, hi), _oracle((4, 4, 1), lo, hi))


@pytest.mark.parametrize("dims,size", [((5, 5, 1), 3001), ((2, 3, 4), 777), ((3, 3, 3), 1111),
                                       ((6, 6, 1), 1200)])
def test_blocked_config_lattice_windows(dims, size):
    N = dims[0] * dims[1] * dims[2]
    for lo, hi in _windows(N, size, 0x2008056120 + N):
        _assert_equal(run(dims, BLK, lo, hi), _oracle(dims, lo, hi))


@pytest.mark.parametrize("dims", [(5, 5, 1), (2, 3, 4)])
def test_blocked_full_map_equals_popcount(dims):
    import torch
    o2, d2, n2 = _full_map_invariants(dims, BLK)
    o0, d0, n0 = _full_map_invariants(dims, hp.FORM_POPCOUNT)
    assert torch.equal(o0, o2)
    assert np.array_equal(d0, d2) and n0 == n2


def test_blocked_full_3x3x3_map():
    """All 2^27 sequences in one call (the benchmark's launch configuration):
    invariants, equality with the dense int8 form's map, oracle samples."""
    import torch
    o2, d2, n2 = _full_map_invariants((3, 3, 3), BLK)
    o1, d1, n1 = _full_map_invariants((3, 3, 3), hp.FORM_GEMM_I8)
    assert torch.equal(o1, o2)
    assert np.array_equal(d1, d2) and n1 == n2
    del o1
    rng = np.random.default_rng(2708)
    st = oracle.structures(3, 3, 3)
    for lo in [int(x) for x in rng.integers(0, (1 << 27) - 64, 6)]:
        gs = oracle.ground_states(st, lo, lo + 64)
        assert np.array_equal(o2[lo:lo + 64].cpu().numpy().view(np.uint16), gs.out)


@pytest.mark.parametrize("dims,lo,hi,thresholds", [((4, 4, 1), 0, 1 << 16, (1, 2, 3)),
                                                   ((3, 3, 3), 70001, 73002, (2,)),
                                                   ((6, 6, 1), (1 << 35) + 99, (1 << 35) + 1299,
                                                    (3,))])
def test_blocked_gap_threshold(dims, lo, hi, thresholds):
    import torch
    s = hp.Structures(*dims)
    ws = s.workspace()
    st = oracle.structures(*dims)
    seqs = np.arange(lo, hi, dtype=np.uint64)
    n = hi - lo
    for thr in thresholds:
        ref = oracle.ground_states_gap(st, seqs, thr)
        o = torch.empty(n, dtype=torch.int16, device="cuda")
        e = torch.empty(n, dtype=torch.int32, device="cuda")
        g = torch.empty(n, dtype=torch.uint8, device="cuda")
        d = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
        nd = torch.zeros(1, dtype=torch.int64, device="cuda")
        print("blocked gap", dims, lo, hi, thr, flush=True)
        hp.hp_enumerate_gap(s, ws, BLK, lo, hi, thr, o, e, g, d, nd)
        torch.cuda.synchronize()
        assert np.array_equal(o.cpu().numpy().view(np.uint16), ref.out)
        assert np.array_equal(e.cpu().numpy(), ref.emin)
        assert np.array_equal(g.cpu().numpy(), ref.gap)
        assert np.array_equal(d.cpu().numpy().view(np.uint64), ref.designability)
        assert int(nd.item()) == ref.nondesign


@pytest.mark.parametrize("dims,lo,hi", [((4, 4, 1), 0, 1 << 16), ((3, 3, 3), 5000, 7100)])
def test_blocked_pair_table_weight_three(dims, lo, hi):
    import torch
    table = (0, 0, 0, -3)          # E_HH = -3: pair weight A = 3, no unary rows
    s = hp.Structures(*dims, table=table)
    assert s.unary_rows == 0
    ws = s.workspace()
    n = hi - lo
    o = torch.empty(n, dtype=torch.int16, device="cuda")
    e = torch.empty(n, dtype=torch.int32, device="cuda")
    d = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
    nd = torch.zeros(1, dtype=torch.int64, device="cuda")
    hp.hp_enumerate(s, ws, BLK, lo, hi, o, e, d, nd)
    torch.cuda.synchronize()
    gs = oracle.ground_states(oracle.structures(*dims), lo, hi, table=table)
    _assert_equal({"out": o.cpu().numpy().view(np.uint16), "emin": e.cpu().numpy(),
                   "desig": d.cpu().numpy().view(np.uint64), "nondesign": int(nd.item())}, gs)


@pytest.mark.parametrize("nw,mode", [(2, 0), (4, 0), (8, 0), (2, 1), (4, 1), (8, 1), (2, 2), (4, 2),
                                     (8, 2), (4, 3), (8, 3)])
def test_blocked_every_launch_shape(nw, mode):
    keep = hp.hp_blocked_selected()
    try:
        hp.hp_blocked_select(nw, mode)
        print("blocked shape", nw, mode, flush=True)
        for dims, lo, hi in [((4, 4, 1), 0, 1 << 16), ((3, 3, 1), 0, 512), ((3, 3, 3), 12345, 14470),
                             ((6, 6, 1), (1 << 36) - 1500, 1 << 36), ((2, 3, 4), 77, 1077)]:
            _assert_equal(run(dims, BLK, lo, hi), _oracle(dims, lo, hi))
    finally:
        hp.hp_blocked_select(*keep)


# ---------------------------------------------------------------------------
# reversal-canonical blocks (hp_enumerate_symmetric_blocked)
# ---------------------------------------------------------------------------

def _rev(s, N):
    return int(format(s, "0%db" % N)[::-1], 2)


def canonical_block_sequences(N, t):
    """Sequences of canonical block t as the header documents the order
    (test-side restatement): returns (list of sequences, diagonal flag)."""
    odd = N & 1
    h = (N - 8 - odd) // 2
    side = 1 << h
    span = side + 1
    per_m = (side >> 1) * span if h else 1
    m, r = divmod(t, per_m)
    p = r // span if h else 0
    o = r - p * span
    first = o <= p
    bp = p if first else side - 1 - p
    a = o if first else o - p - 1
    b = _rev(bp, h) if h else 0
    pos = [h + x + (odd if x >= 4 else 0) for x in range(8)]
    outer = (a << (h + 8 + odd)) | (m << (h + 4)) | b
    seqs = [outer | sum(((x >> k) & 1) << pos[k] for k in range(8)) for x in range(256)]
    return seqs, a == bp


def _sym_run(dims, b_lo, b_hi, out=None, emin=None):
    import torch
    s = hp.Structures(*dims)
    ws = s.workspace()
    n = 1 << s.N
    if out is None:
        out = torch.full((n,), -7, dtype=torch.int16, device="cuda")
        emin = torch.full((n,), 99, dtype=torch.int32, device="cuda")
    d = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
    nd = torch.zeros(1, dtype=torch.int64, device="cuda")
    print("symmetric blocked", dims, b_lo, b_hi, flush=True)
    hp.hp_enumerate_symmetric_blocked(s, ws, b_lo, b_hi, out, emin, d, nd)
    torch.cuda.synchronize()
    return s, out, emin, d, nd


@pytest.mark.parametrize("dims", [(2, 2, 2), (3, 3, 1), (3, 4, 1), (2, 2, 3), (4, 4, 1), (3, 5, 1),
                                  (2, 3, 3)])
def test_symmetric_blocked_full_small_maps(dims):
    s = hp.Structures(*dims)
    nb = hp.hp_canonical_block_count(s)
    s, out, emin, d, nd = _sym_run(dims, 0, nb)
    N = s.N
    _assert_equal({"out": out.cpu().numpy().view(np.uint16), "emin": emin.cpu().numpy(),
                   "desig": d.cpu().numpy().view(np.uint64), "nondesign": int(nd.item())},
                  _oracle(dims, 0, 1 << N))


def test_symmetric_blocked_full_3x3x3_equals_plain():
    import torch
    s = hp.Structures(3, 3, 3)
    nb = hp.hp_canonical_block_count(s)
    assert nb == 262656
    third = nb // 3 + 17
    s, out, emin, d, nd = _sym_run((3, 3, 3), 0, third)
    d2 = torch.zeros_like(d)
    nd2 = torch.zeros_like(nd)
    hp.hp_enumerate_symmetric_blocked(s, s.workspace(), third, nb, out, emin, d2, nd2)
    o1, d1, n1 = _full_map_invariants((3, 3, 3), BLK)
    assert torch.equal(out, o1)
    assert np.array_equal((d + d2).cpu().numpy().view(np.uint64), d1)
    assert int(nd.item()) + int(nd2.item()) == n1


@pytest.mark.parametrize("dims", [(6, 6, 1), (3, 3, 3), (5, 5, 1)])
def test_symmetric_blocked_windows_match_oracle(dims):
    import torch
    s = hp.Structures(*dims)
    N = s.N
    nb = hp.hp_canonical_block_count(s)
    st = oracle.structures(*dims)
    rng = np.random.default_rng(0x5EB + N)
    big = N > 30     # 6x6: the uint16 map alone is 137 GB; no energies, no full scan
    out = torch.empty((1 << N,), dtype=torch.int16, device="cuda")
    emin = None if big else torch.empty((1 << N,), dtype=torch.int32, device="cuda")
    for b0 in [0, nb - 3] + [int(x) for x in rng.integers(0, nb - 3, 2)]:
        out.fill_(-7)
        if emin is not None:
            emin.fill_(99)
        _sym_run(dims, b0, b0 + 3, out, emin)
        seqs, revs = [], []
        for t in range(b0, b0 + 3):
            sq, diag = canonical_block_sequences(N, t)
            seqs += sq
            if not diag:
                revs += [_rev(x, N) for x in sq]
        ref = oracle.ground_states_gap(st, seqs)
        idx = torch.tensor(seqs, dtype=torch.int64, device="cuda")
        assert np.array_equal(out[idx].cpu().numpy().view(np.uint16), ref.out)
        if emin is not None:
            assert np.array_equal(emin[idx].cpu().numpy(), ref.emin)
        if revs:
            ridx = torch.tensor(revs, dtype=torch.int64, device="cuda")
            rref = oracle.ground_states_gap(st, revs)
            assert np.array_equal(out[ridx].cpu().numpy().view(np.uint16), rref.out)
        # nothing outside the scored blocks and their reverses was written
        if not big:
            touched = int((out != -7).sum().item())
            assert touched == len(set(seqs) | set(revs))


def test_autotune_blocked_selects_a_shape_and_keeps_results():
    keep = hp.hp_blocked_selected()
    try:
        s = hp.Structures(5, 5, 1)
        (nw, mode), ms = hp.hp_autotune_blocked(s, s.workspace(), 0, 1 << 18, repeats=1)
        assert (nw, mode) == hp.hp_blocked_selected()
        assert len(ms) == 10 and min(ms) > 0       # wide blocks apply to 5x5
        assert (nw, mode) in [(2, 0), (2, 1), (2, 2), (4, 0), (4, 1), (4, 2), (8, 0), (8, 1),
                              (8, 2), (8, 3)]
        assert ms[9 if mode == 3 else [2, 4, 8].index(nw) * 3 + mode] == min(ms)
        _assert_equal(run((5, 5, 1), BLK, 777, 777 + 5000), _oracle((5, 5, 1), 777, 777 + 5000))
    finally:
        hp.hp_blocked_select(*keep)


# ---------------------------------------------------------------------------
# wide blocks (staging mode 3) on 4 waves: 1024 sequences per workgroup,
# first product shared by the waves
# ---------------------------------------------------------------------------

@pytest.fixture()
def wide():
    keep = hp.hp_blocked_selected()
    hp.hp_blocked_select(4, 3)
    yield
    hp.hp_blocked_select(*keep)


@pytest.mark.parametrize("dims", [(3, 4, 1), (4, 4, 1), (3, 5, 1), (2, 3, 3), (2, 2, 4)])
def test_wide_full_small_lattices(wide, dims):
    N = dims[0] * dims[1] * dims[2]
    _assert_equal(run(dims, BLK, 0, 1 << N), _oracle(dims, 0, 1 << N))


@pytest.mark.parametrize("lo,hi", [(0, 1), (3, 1000), (1023, 1025), (1000, 3100), (40000, 65536),
                                   (1, 65535), (1024, 2048), (64512, 65536)])
def test_wide_ragged_ranges_4x4(wide, lo, hi):
    _assert_equal(run((4, 4, 1), BLK, lo, hi), _oracle((4, 4, 1), lo, hi))


@pytest.mark.parametrize("dims,size", [((5, 5, 1), 3001), ((2, 3, 4), 2777), ((3, 3, 3), 2111),
                                       ((6, 6, 1), 2200)])
def test_wide_config_lattice_windows(wide, dims, size):
    N = dims[0] * dims[1] * dims[2]
    for lo, hi in _windows(N, size, 0x2008056121 + N):
        _assert_equal(run(dims, BLK, lo, hi), _oracle(dims, lo, hi))


@pytest.mark.parametrize("dims,lo,hi,thresholds", [((4, 4, 1), 0, 1 << 16, (1, 2, 3)),
                                                   ((3, 3, 3), 777, 777 + 3000, (2, 4))])
def test_wide_gap_threshold(wide, dims, lo, hi, thresholds):
    import torch
    s = hp.Structures(*dims)
    ws = s.workspace()
    st = oracle.structures(*dims)
    for th in thresholds:
        o = torch.full((hi - lo,), -7, dtype=torch.int16, device="cuda")
        g = torch.zeros(hi - lo, dtype=torch.uint8, device="cuda")
        hp.hp_enumerate_gap(s, ws, BLK, lo, hi, th, o, None, g)
        torch.cuda.synchronize()
        gs = oracle.ground_states_gap(st, np.arange(lo, hi, dtype=np.uint64), threshold=th)
        assert np.array_equal(o.cpu().numpy().view(np.uint16), gs.out), th
        assert np.array_equal(g.cpu().numpy(), gs.gap), th


@pytest.mark.parametrize("dims", [(5, 5, 1), (2, 3, 4)])
def test_wide_full_map_equals_popcount(wide, dims):
    import torch
    o2, d2, n2 = _full_map_invariants(dims, BLK)
    o0, d0, n0 = _full_map_invariants(dims, hp.FORM_POPCOUNT)
    assert torch.equal(o0, o2)
    assert np.array_equal(d0, d2) and n0 == n2


# ---------------------------------------------------------------------------
# wide blocks of 2048 sequences (8 waves; the default, or nw 8 with mode 3):
# plain ranges whose ends are multiples of 2^17 on lattices with N >= 17
# ---------------------------------------------------------------------------

C17 = 1 << 17


@pytest.fixture()
def wide8():
    keep = hp.hp_blocked_selected()
    hp.hp_blocked_select(8, 3)
    yield
    hp.hp_blocked_select(*keep)


@pytest.mark.parametrize("dims,lo,hi", [((5, 5, 1), C17, 3 * C17), ((2, 3, 4), 0, C17),
                                        ((4, 5, 1), 5 * C17, 7 * C17),
                                        ((2, 9, 1), 0, 2 * C17), ((3, 6, 1), 0, 2 * C17)])
def test_wide8_chunks_match_oracle(wide8, dims, lo, hi):
    """2^17-sequence chunks (64 blocks of 2048 each) against the oracle, every
    sequence; 2x9 (2 conformation tiles) and 3x6 (6) have fewer tiles than a
    workgroup has waves, so only a partial group runs and some waves compute
    no first product (whole maps, N = 18)."""
    _assert_equal(run(dims, BLK, lo, hi), _oracle(dims, lo, hi))


@pytest.mark.parametrize("dims,lo,hi", [((2, 3, 4), 3 * C17, 9 * C17),
                                        ((3, 3, 3), 37 * C17, 41 * C17),
                                        ((6, 6, 1), (1 << 35) - C17, (1 << 35) + C17)])
def test_wide8_chunks_equal_popcount(wide8, dims, lo, hi):
    """Several chunks (6x6: across the middle of the sequence space, K_pad 320)
    equal the popcount form's map, energies and histogram bit for bit, and
    the same range cut one sequence short (blocks of 1024) agrees too."""
    a = run(dims, BLK, lo, hi)
    b = run(dims, hp.FORM_POPCOUNT, lo, hi)
    for k in ("out", "emin", "desig"):
        assert np.array_equal(a[k], b[k]), k
    assert a["nondesign"] == b["nondesign"]
    c = run(dims, BLK, lo + 1, hi)
    assert np.array_equal(c["out"], a["out"][1:]) and np.array_equal(c["emin"], a["emin"][1:])


def test_wide8_gap_threshold(wide8):
    import torch
    dims, lo, hi = (5, 5, 1), 4 * C17, 6 * C17
    s = hp.Structures(*dims)
    ws = s.workspace()
    st = oracle.structures(*dims)
    for th in (2, 3):
        o = torch.full((hi - lo,), -7, dtype=torch.int16, device="cuda")
        g = torch.zeros(hi - lo, dtype=torch.uint8, device="cuda")
        print("gap", dims, lo, hi, th, flush=True)
        hp.hp_enumerate_gap(s, ws, BLK, lo, hi, th, o, None, g)
        torch.cuda.synchronize()
        gs = oracle.ground_states_gap(st, np.arange(lo, hi, dtype=np.uint64), threshold=th)
        assert np.array_equal(o.cpu().numpy().view(np.uint16), gs.out), th
        assert np.array_equal(g.cpu().numpy(), gs.gap), th


def test_wide8_full_3x3x3_map_equals_4_waves(wide8):
    """The full 3x3x3 map with 8-wave blocks of 2048 equals the 4-wave
    blocks' map and histogram bit for bit."""
    import torch
    o8, d8, n8 = _full_map_invariants((3, 3, 3), BLK)
    hp.hp_blocked_select(4, 3)
    o4, d4, n4 = _full_map_invariants((3, 3, 3), BLK)
    assert torch.equal(o8, o4)
    assert np.array_equal(d8, d4) and n8 == n4


@pytest.mark.parametrize("dims", [(3, 4, 1), (4, 4, 1), (2, 3, 3)])
def test_wide8_selection_on_canonical_blocks(wide8, dims):
    """With 8 waves selected, reversal-canonical blocks keep their own
    geometry: the symmetric map still equals the oracle's."""
    s = hp.Structures(*dims)
    nb = hp.hp_canonical_block_count(s)
    s, out, emin, d, nd = _sym_run(dims, 0, nb)
    _assert_equal({"out": out.cpu().numpy().view(np.uint16), "emin": emin.cpu().numpy(),
                   "desig": d.cpu().numpy().view(np.uint64), "nondesign": int(nd.item())},
                  _oracle(dims, 0, 1 << s.N))
