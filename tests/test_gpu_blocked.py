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


@pytest.mark.parametrize("nw,mode", [(2, 0), (4, 0), (8, 0), (2, 1), (4, 1), (8, 1)])
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
