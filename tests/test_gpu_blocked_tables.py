"""GPU parity of the block-factorised int8 form with two-letter contact
tables (unary terms, E_HP != E_PP) against the oracle, bit-exact: full small
maps, oracle windows on the configuration lattices up to 3x3x3 (Table 1
energies and a second table; 6x6 stays on the dense form), the energy-gap
threshold, every selectable launch shape (tables run one shape), reversal-
canonical blocks, mixed batches, and the full 3x3x3 map with Table 1
energies equal to the dense int8 form's map."""
import numpy as np
import pytest

import oracle
import paper_2008_05612_amd as hp
from tests.conftest import gpu_available
from tests.test_gpu_blocked import _rev, canonical_block_sequences
from tests.test_gpu_enumerate import _windows

pytestmark = pytest.mark.gpu
BLK = hp.FORM_BLOCKED_I8
HP1996 = oracle.HP1996_X10        # Table 1 x 10: E_PP, E_PH, E_HP, E_HH
T2 = (0, -1, -1, -3)              # pair weight 1, unary weight 1
_cache = {}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def test_tables_deep_products_stay_on_the_dense_form():
    # with unary rows the blocked form takes first products up to depth 256;
    # 6x6 (K = 289) with Table 1 runs in the dense int8 form
    s, ws = _get((6, 6, 1), HP1996)
    assert hp.hp_canonical_block_count(s) == 0
    with pytest.raises(hp.HPError) as e:
        hp.hp_enumerate(s, ws, BLK, 0, 256)
    assert e.value.status == -5


def _get(dims, table):
    key = (dims, table)
    if key not in _cache:
        s = hp.Structures(*dims, table=table)
        _cache[key] = (s, s.workspace())
    return _cache[key]


def _run(dims, table, lo, hi, form=BLK):
    import torch
    s, ws = _get(dims, table)
    n = hi - lo
    o = torch.full((n,), -7, dtype=torch.int16, device="cuda")
    e = torch.full((n,), 99, dtype=torch.int32, device="cuda")
    d = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
    nd = torch.zeros(1, dtype=torch.int64, device="cuda")
    print("blocked table", dims, table, lo, hi, flush=True)
    hp.hp_enumerate(s, ws, form, lo, hi, o, e, d, nd)
    torch.cuda.synchronize()
    return o.cpu().numpy().view(np.uint16), e.cpu().numpy(), d.cpu().numpy().view(np.uint64), \
        int(nd.item())


def _check(got, dims, table, lo, hi):
    gs = oracle.ground_states(oracle.structures(*dims), lo, hi, table=table)
    o, e, d, nd = got
    assert np.array_equal(o, gs.out)
    assert np.array_equal(e, gs.emin)
    assert np.array_equal(d, gs.designability)
    assert nd == gs.nondesign


@pytest.mark.parametrize("table", [HP1996, T2])
@pytest.mark.parametrize("dims", [(3, 3, 1), (2, 2, 2), (3, 4, 1), (2, 2, 3), (4, 4, 1),
                                  (3, 5, 1), (2, 3, 3)])
def test_tables_full_small_lattices(dims, table):
    s, _ = _get(dims, table)
    assert s.unary_rows > 0 and hp.hp_canonical_block_count(s) > 0
    N = s.N
    _check(_run(dims, table, 0, 1 << N), dims, table, 0, 1 << N)


@pytest.mark.parametrize("table", [HP1996, T2])
@pytest.mark.parametrize("dims,size", [((5, 5, 1), 2001), ((2, 3, 4), 777), ((3, 3, 3), 1111)])
def test_tables_config_lattice_windows(dims, size, table):
    N = dims[0] * dims[1] * dims[2]
    for lo, hi in _windows(N, size, 0x1996 + N):
        _check(_run(dims, table, lo, hi), dims, table, lo, hi)


@pytest.mark.parametrize("dims,lo,hi,thresholds", [((4, 4, 1), 0, 1 << 16, (1, 10, 23)),
                                                   ((3, 3, 3), 90001, 92002, (3, 13))])
def test_tables_gap_threshold(dims, lo, hi, thresholds):
    import torch
    s, ws = _get(dims, HP1996)
    st = oracle.structures(*dims)
    seqs = np.arange(lo, hi, dtype=np.uint64)
    n = hi - lo
    for thr in thresholds:
        ref = oracle.ground_states_gap(st, seqs, thr, table=HP1996)
        o = torch.empty(n, dtype=torch.int16, device="cuda")
        e = torch.empty(n, dtype=torch.int32, device="cuda")
        g = torch.empty(n, dtype=torch.uint8, device="cuda")
        d = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
        nd = torch.zeros(1, dtype=torch.int64, device="cuda")
        print("blocked table gap", dims, lo, hi, thr, flush=True)
        hp.hp_enumerate_gap(s, ws, BLK, lo, hi, thr, o, e, g, d, nd)
        torch.cuda.synchronize()
        assert np.array_equal(o.cpu().numpy().view(np.uint16), ref.out)
        assert np.array_equal(e.cpu().numpy(), ref.emin)
        assert np.array_equal(g.cpu().numpy(), ref.gap)
        assert np.array_equal(d.cpu().numpy().view(np.uint64), ref.designability)
        assert int(nd.item()) == ref.nondesign


@pytest.mark.parametrize("nw,mode", [(2, 0), (4, 0), (8, 0), (2, 1), (4, 1), (8, 1), (2, 2), (4, 2),
                                     (8, 2), (8, 3)])
def test_tables_every_launch_shape(nw, mode):
    keep = hp.hp_blocked_selected()
    try:
        hp.hp_blocked_select(nw, mode)
        for dims, lo, hi in [((4, 4, 1), 0, 1 << 16), ((3, 3, 3), 12345, 14470),
                             ((2, 3, 4), (1 << 24) - 1100, 1 << 24)]:
            _check(_run(dims, HP1996, lo, hi), dims, HP1996, lo, hi)
    finally:
        hp.hp_blocked_select(*keep)


def _sym(dims, table, b_lo, b_hi, out, emin):
    import torch
    s, ws = _get(dims, table)
    d = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
    nd = torch.zeros(1, dtype=torch.int64, device="cuda")
    print("symmetric blocked table", dims, b_lo, b_hi, flush=True)
    hp.hp_enumerate_symmetric_blocked(s, ws, b_lo, b_hi, out, emin, d, nd)
    torch.cuda.synchronize()
    return d.cpu().numpy().view(np.uint64), int(nd.item())


@pytest.mark.parametrize("dims", [(3, 3, 1), (2, 2, 3), (4, 4, 1), (3, 5, 1), (2, 3, 3)])
def test_tables_symmetric_blocked_full_small_maps(dims):
    import torch
    s, _ = _get(dims, HP1996)
    n = 1 << s.N
    out = torch.full((n,), -7, dtype=torch.int16, device="cuda")
    emin = torch.full((n,), 99, dtype=torch.int32, device="cuda")
    d, nd = _sym(dims, HP1996, 0, hp.hp_canonical_block_count(s), out, emin)
    _check((out.cpu().numpy().view(np.uint16), emin.cpu().numpy(), d, nd), dims, HP1996, 0, n)


@pytest.mark.parametrize("dims", [(3, 3, 3), (5, 5, 1)])
def test_tables_symmetric_blocked_windows(dims):
    import torch
    s, _ = _get(dims, HP1996)
    N = s.N
    nb = hp.hp_canonical_block_count(s)
    st = oracle.structures(*dims)
    out = torch.full((1 << N,), -7, dtype=torch.int16, device="cuda")
    rng = np.random.default_rng(0x96 + N)
    for b0 in [0, nb - 2] + [int(x) for x in rng.integers(0, nb - 2, 2)]:
        _sym(dims, HP1996, b0, b0 + 2, out, None)
        seqs, revs = [], []
        for t in range(b0, b0 + 2):
            sq, diag = canonical_block_sequences(N, t)
            seqs += sq
            if not diag:
                revs += [_rev(x, N) for x in sq]
        idx = torch.tensor(seqs + revs, dtype=torch.int64, device="cuda")
        ref = oracle.ground_states_gap(st, seqs + revs, table=HP1996)
        assert np.array_equal(out[idx].cpu().numpy().view(np.uint16), ref.out)


def test_tables_batch():
    import torch
    specs = [((4, 4, 1), HP1996, 0, 1 << 16), ((3, 3, 3), HP1996, 5000, 9100),
             ((2, 3, 4), T2, 333, 3333), ((3, 3, 3), None, 100, 2200)]
    jobs, outs = [], []
    for dims, table, lo, hi in specs:
        s, ws = _get(dims, table)
        o = torch.full((hi - lo,), -7, dtype=torch.int16, device="cuda")
        d = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
        jobs.append(hp.Job(s, ws, lo, hi, o, None, d, None))
        outs.append((dims, table, lo, hi, o, d))
    bws = torch.zeros(hp._binding.batch_workspace_bytes(len(jobs)), dtype=torch.uint8,
                      device="cuda")
    print("blocked table batch", flush=True)
    hp.hp_enumerate_batch(jobs, BLK, bws)
    torch.cuda.synchronize()
    for dims, table, lo, hi, o, d in outs:
        gs = oracle.ground_states(oracle.structures(*dims), lo, hi, table=table)
        assert np.array_equal(o.cpu().numpy().view(np.uint16), gs.out)
        assert np.array_equal(d.cpu().numpy().view(np.uint64), gs.designability)


def test_tables_full_3x3x3_equals_dense():
    """All 2^27 sequences with Table 1 energies: the blocked and the dense
    int8 forms give the same map, energies and histogram."""
    import torch
    s, ws = _get((3, 3, 3), HP1996)
    total = 1 << 27
    res = []
    for form in (BLK, hp.FORM_GEMM_I8):
        o = torch.empty(total, dtype=torch.int16, device="cuda")
        e = torch.empty(total, dtype=torch.int32, device="cuda")
        d = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
        nd = torch.zeros(1, dtype=torch.int64, device="cuda")
        print("HP1996 3x3x3 full map form", form, flush=True)
        hp.hp_enumerate(s, ws, form, 0, total, o, e, d, nd)
        torch.cuda.synchronize()
        res.append((o, e, d, int(nd.item())))
    (o1, e1, d1, n1), (o2, e2, d2, n2) = res
    assert torch.equal(o1, o2) and torch.equal(e1, e2) and torch.equal(d1, d2) and n1 == n2
    assert int(d1.sum().item()) + n1 == total
    # the paper's counts (Results): 47449 designable folds, 4.76 % designing
    assert int((d1 > 0).sum().item()) == 47449
    assert abs(100.0 * int(d1.sum().item()) / total - 4.76) < 0.005
