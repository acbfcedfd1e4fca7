"""Reversal-symmetric enumeration (hp_enumerate_symmetric) against the oracle
and against the plain enumeration: only canonical sequences s <= reverse(s)
are scored, and each fills the map at s and at reverse(s)."""
import numpy as np
import pytest

import oracle
import paper_2008_05612_amd as hp
from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu
HP1996_X10 = (0, -10, -10, -23)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def _rev(x, n):
    return int(format(x, "0%db" % n)[::-1], 2) if n else 0


def _full_symmetric(s, ws, form):
    import torch
    n = 1 << s.N
    o = torch.full((n,), -7, dtype=torch.int16, device="cuda")
    e = torch.full((n,), 99, dtype=torch.int32, device="cuda")
    d = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
    nd = torch.zeros(1, dtype=torch.int64, device="cuda")
    cnt = hp.hp_canonical_count(s)
    # two calls with a ragged split, to exercise accumulation across ranges
    cut = cnt // 3 + 7 if cnt > 20 else cnt
    hp.hp_enumerate_symmetric(s, ws, form, 0, cut, o, e, d, nd)
    if cut < cnt:
        hp.hp_enumerate_symmetric(s, ws, form, cut, cnt, o, e, d, nd)
    torch.cuda.synchronize()
    return (o.cpu().numpy().view(np.uint16), e.cpu().numpy(), d.cpu().numpy().view(np.uint64),
            int(nd.item()))


@pytest.mark.parametrize("table", [None, HP1996_X10])
@pytest.mark.parametrize("form", [hp.FORM_POPCOUNT, hp.FORM_GEMM_I8])
@pytest.mark.parametrize("dims", [(1, 2, 1), (2, 2, 1), (2, 3, 1), (3, 3, 1), (1, 5, 1), (2, 2, 2),
                                  (3, 4, 1), (2, 2, 3), (4, 4, 1), (3, 5, 1), (2, 3, 3)])
def test_symmetric_full_map_matches_oracle(dims, form, table):
    s = hp.Structures(*dims, table=table)
    N = s.N
    side = 1 << (N // 2)
    assert hp.hp_canonical_count(s) == side * (side + 1) // 2 * (2 if N % 2 else 1)
    o, e, d, nd = _full_symmetric(s, s.workspace(), form)
    gs = oracle.ground_states(oracle.structures(*dims), table=table)
    assert np.array_equal(o, gs.out)
    assert np.array_equal(e, gs.emin)
    assert np.array_equal(d, gs.designability)
    assert nd == gs.nondesign


@pytest.mark.parametrize("form", [hp.FORM_POPCOUNT, hp.FORM_GEMM_I8])
def test_symmetric_full_5x5_equals_plain(form):
    import torch
    s = hp.Structures(5, 5, 1)
    ws = s.workspace()
    n = 1 << 25
    o1 = torch.empty(n, dtype=torch.int16, device="cuda")
    d1 = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
    nd1 = torch.zeros(1, dtype=torch.int64, device="cuda")
    hp.hp_enumerate(s, ws, form, 0, n, o1, None, d1, nd1)
    o2, e2, d2, nd2 = _full_symmetric(s, ws, form)
    assert np.array_equal(o1.cpu().numpy().view(np.uint16), o2)
    assert np.array_equal(d1.cpu().numpy().view(np.uint64), d2)
    assert int(nd1.item()) == nd2


@pytest.mark.parametrize("dims", [(3, 3, 3), (6, 6, 1)])
def test_symmetric_windows_match_oracle(dims):
    """Canonical-index windows of the config lattices: every s written (and
    its reverse) against the oracle, sequence by sequence."""
    import torch
    s = hp.Structures(*dims)
    ws = s.workspace()
    N = s.N
    cnt = hp.hp_canonical_count(s)
    st = oracle.structures(*dims)
    rng = np.random.default_rng(0x2008056120)
    for t0 in [0, cnt - 97] + [int(x) for x in rng.integers(0, cnt - 97, 2)]:
        d = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
        nd = torch.zeros(1, dtype=torch.int64, device="cuda")
        print("symmetric window", dims, t0, flush=True)
        if N <= 30:
            o = torch.full((1 << N,), -7, dtype=torch.int16, device="cuda")
            hp.hp_enumerate_symmetric(s, ws, hp.FORM_GEMM_I8, t0, t0 + 97, o, None, d, nd)
            torch.cuda.synchronize()
            written = torch.nonzero(o != -7).flatten().cpu().numpy().tolist()
            oh = o.cpu().numpy().view(np.uint16)
        else:
            # a full 2^36 map is too large for a unit test: counts only
            hp.hp_enumerate_symmetric(s, ws, hp.FORM_GEMM_I8, t0, t0 + 97, None, None, d, nd)
            torch.cuda.synchronize()
            written, oh = None, None
        want = np.zeros(s.n_class, np.uint64)
        want_nd = 0
        seqs = _canonical(N, t0, t0 + 97)
        for sq in seqs:
            gs = oracle.ground_states(st, sq, sq + 1)
            w = 1 if _rev(sq, N) == sq else 2
            if gs.out[0] == 0xFFFF:
                want_nd += w
            else:
                want[gs.out[0]] += w
            if oh is not None:
                assert oh[sq] == gs.out[0] and oh[_rev(sq, N)] == gs.out[0], sq
        if written is not None:
            assert sorted(written) == sorted({x for sq in seqs for x in (sq, _rev(sq, N))})
        assert np.array_equal(d.cpu().numpy().view(np.uint64), want)
        assert int(nd.item()) == want_nd


def _canonical(N, t_lo, t_hi):
    """Canonical sequences at indices [t_lo, t_hi), in the documented order:
    middle bit; then row pairs p < 2^(h-1), each listing row b' = p (a in
    [0, p]) and then row b' = 2^h - 1 - p (a in [0, 2^h - 1 - p]); s has high
    half a, middle bit m and low half reverse(b').  Whole rows before t_lo
    are skipped by their length."""
    h = N // 2
    mid = N & 1
    side = 1 << h
    rows = [0] if h == 0 else [r for p in range(side // 2) for r in (p, side - 1 - p)]
    out = []
    t = 0
    for m in range(2 if mid else 1):
        for bp in rows:
            if t + bp + 1 <= t_lo:
                t += bp + 1
                continue
            for a in range(bp + 1):
                if t_lo <= t < t_hi:
                    out.append((a << (h + mid)) | (m << h) | _rev(bp, h))
                t += 1
                if t >= t_hi:
                    return out
    return out
