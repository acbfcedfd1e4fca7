"""GPU parity of hp_enumerate (both kernel forms) against the CPU oracle.

Every check is bit-exact: phenotype ids, minimum energies, designability and
the deleterious count.  Small lattices are compared over all 2^N sequences;
the configuration lattices (5x5, 2x3x4, 3x3x3, 6x6) over oracle windows at
fixed and seeded offsets, with ragged window sizes, and the full maps through
invariants that hold at any size.
"""
import numpy as np
import pytest

import oracle
import paper_2008_05612_amd as hp
from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu

FORMS = [hp.FORM_POPCOUNT, hp.FORM_GEMM_I8]
NONE = 0xFFFF

_structs = {}


def _get(dims):
    if dims not in _structs:
        print("structures", dims, flush=True)
        s = hp.Structures(*dims)
        _structs[dims] = (s, s.workspace())
    return _structs[dims]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def run(dims, form, lo, hi, out=True, emin=True):
    import torch
    s, ws = _get(dims)
    n = hi - lo
    o = torch.full((n,), -7, dtype=torch.int16, device="cuda") if out else None
    e = torch.full((n,), 99, dtype=torch.int32, device="cuda") if emin else None
    d = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
    nd = torch.zeros(1, dtype=torch.int64, device="cuda")
    print("enumerate", dims, "form", form, "range", lo, hi, flush=True)
    hp.hp_enumerate(s, ws, form, lo, hi, o, e, d, nd)
    torch.cuda.synchronize()
    res = {
        "out": o.cpu().numpy().view(np.uint16) if out else None,
        "emin": e.cpu().numpy() if emin else None,
        "desig": d.cpu().numpy().view(np.uint64),
        "nondesign": int(nd.item()),
    }
    return res


def _oracle(dims, lo, hi):
    st = oracle.structures(*dims)
    return oracle.ground_states(st, lo, hi)


def _assert_equal(res, gs):
    assert np.array_equal(res["out"], gs.out)
    assert np.array_equal(res["emin"], gs.emin)
    assert np.array_equal(res["desig"], gs.designability)
    assert res["nondesign"] == gs.nondesign


SMALL = [(1, 2, 1), (2, 2, 1), (2, 3, 1), (3, 3, 1), (1, 5, 1), (2, 2, 2), (3, 4, 1),
         (2, 2, 3), (4, 4, 1), (3, 5, 1), (2, 3, 3)]


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("dims", SMALL)
def test_full_small_lattices(dims, form):
    N = dims[0] * dims[1] * dims[2]
    res = run(dims, form, 0, 1 << N)
    _assert_equal(res, _oracle(dims, 0, 1 << N))


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("lo,hi", [(0, 1), (3, 1000), (511, 513), (40000, 65536), (1, 65535)])
def test_ragged_ranges_4x4(form, lo, hi):
    res = run((4, 4, 1), form, lo, hi)
    _assert_equal(res, _oracle((4, 4, 1), lo, hi))


def _windows(N, size, seed):
    rng = np.random.default_rng(seed)
    top = 1 << N
    offs = [0, top - size, top // 2 - size // 2]
    offs += [int(x) for x in rng.integers(0, top - size, 3)]
    return [(o, o + size) for o in offs]


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("dims,size", [((5, 5, 1), 3001), ((2, 3, 4), 777), ((3, 3, 3), 1111),
                                       ((6, 6, 1), 1200)])
def test_config_lattice_windows(dims, size, form):
    N = dims[0] * dims[1] * dims[2]
    for lo, hi in _windows(N, size, 0x2008056120 + N):
        res = run(dims, form, lo, hi)
        _assert_equal(res, _oracle(dims, lo, hi))


def test_accumulation_across_calls():
    import torch
    s, ws = _get((4, 4, 1))
    d = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
    nd = torch.zeros(1, dtype=torch.int64, device="cuda")
    for lo, hi in [(0, 1000), (1000, 40000), (40000, 65536)]:
        hp.hp_enumerate(s, ws, hp.FORM_GEMM_I8, lo, hi, None, None, d, nd)
    torch.cuda.synchronize()
    gs = _oracle((4, 4, 1), 0, 1 << 16)
    assert np.array_equal(d.cpu().numpy().view(np.uint64), gs.designability)
    assert int(nd.item()) == gs.nondesign


def _bitrev(idx, N):
    import torch
    r = torch.zeros_like(idx)
    for i in range(N):
        r |= ((idx >> i) & 1) << (N - 1 - i)
    return r


def _full_map_invariants(dims, form):
    """Run the full map on the GPU and check what holds at any size."""
    import torch
    s, ws = _get(dims)
    N = s.N
    total = 1 << N
    out = torch.empty(total, dtype=torch.int16, device="cuda")
    d = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
    nd = torch.zeros(1, dtype=torch.int64, device="cuda")
    print("full map", dims, "form", form, flush=True)
    hp.hp_enumerate(s, ws, form, 0, total, out, None, d, nd)
    torch.cuda.synchronize()
    desig = d.cpu().numpy().view(np.uint64)
    nondes = int(nd.item())
    assert int(desig.sum()) + nondes == total
    ex = s.export()
    assert np.all(desig[ex["self_rev"] == 0] % 2 == 0)
    idx = torch.arange(total, device="cuda", dtype=torch.int64)
    assert torch.equal(out[_bitrev(idx, N)], out)
    # parity-pure sequences tie on E = 0 whenever there are two conformations
    even = sum(1 << i for i in range(0, N, 2))
    odd = sum(1 << i for i in range(1, N, 2))
    pure = ((idx & odd) == 0) | ((idx & even) == 0)
    assert bool((out[pure] == -1).all())
    counts = torch.bincount(out.to(torch.int64) & 0xFFFF, minlength=NONE + 1)[:s.n_class]
    assert np.array_equal(counts.cpu().numpy().astype(np.uint64), desig)
    return out, desig, nondes


@pytest.mark.parametrize("dims", [(5, 5, 1), (2, 3, 4)])
def test_full_map_forms_agree(dims):
    o1, d1, n1 = _full_map_invariants(dims, hp.FORM_GEMM_I8)
    o0, d0, n0 = _full_map_invariants(dims, hp.FORM_POPCOUNT)
    import torch
    assert torch.equal(o0, o1)
    assert np.array_equal(d0, d1) and n0 == n1


def test_full_3x3x3_map_gemm():
    """The 3x3x3 map at full size, in the launch configuration the benchmark
    times: invariants over all 2^27 sequences plus oracle samples."""
    out, desig, nondes = _full_map_invariants((3, 3, 3), hp.FORM_GEMM_I8)
    rng = np.random.default_rng(27)
    st = oracle.structures(3, 3, 3)
    for lo in [int(x) for x in rng.integers(0, (1 << 27) - 64, 6)]:
        gs = oracle.ground_states(st, lo, lo + 64)
        assert np.array_equal(out[lo:lo + 64].cpu().numpy().view(np.uint16), gs.out)


HP1996_X10 = (0, -10, -10, -23)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("dims", [(2, 2, 1), (2, 3, 1), (3, 3, 1), (2, 2, 2), (3, 4, 1),
                                  (4, 4, 1), (2, 3, 3)])
def test_table_full_small_lattices(dims, form):
    import torch
    N = dims[0] * dims[1] * dims[2]
    s = hp.Structures(*dims, table=HP1996_X10)
    ws = s.workspace()
    n = 1 << N
    o = torch.empty(n, dtype=torch.int16, device="cuda")
    e = torch.empty(n, dtype=torch.int32, device="cuda")
    d = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
    nd = torch.zeros(1, dtype=torch.int64, device="cuda")
    hp.hp_enumerate(s, ws, form, 0, n, o, e, d, nd)
    torch.cuda.synchronize()
    gs = oracle.ground_states(oracle.structures(*dims), 0, n, table=HP1996_X10)
    _assert_equal({"out": o.cpu().numpy().view(np.uint16), "emin": e.cpu().numpy(),
                   "desig": d.cpu().numpy().view(np.uint64), "nondesign": int(nd.item())}, gs)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("dims,size", [((3, 3, 3), 1000), ((6, 6, 1), 900), ((2, 3, 4), 700)])
def test_table_config_windows(dims, size, form):
    import torch
    N = dims[0] * dims[1] * dims[2]
    s = hp.Structures(*dims, table=HP1996_X10)
    ws = s.workspace()
    st = oracle.structures(*dims)
    for lo, hi in _windows(N, size, 1996 + N)[:4]:
        n = hi - lo
        o = torch.empty(n, dtype=torch.int16, device="cuda")
        e = torch.empty(n, dtype=torch.int32, device="cuda")
        d = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
        nd = torch.zeros(1, dtype=torch.int64, device="cuda")
        print("table window", dims, form, lo, hi, flush=True)
        hp.hp_enumerate(s, ws, form, lo, hi, o, e, d, nd)
        torch.cuda.synchronize()
        gs = oracle.ground_states(st, lo, hi, table=HP1996_X10)
        _assert_equal({"out": o.cpu().numpy().view(np.uint16), "emin": e.cpu().numpy(),
                       "desig": d.cpu().numpy().view(np.uint64), "nondesign": int(nd.item())}, gs)
