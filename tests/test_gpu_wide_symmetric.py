"""Reversal-canonical wide blocks (hp_enumerate_symmetric_wide): 1024
sequences per block varying in the 10 monomers around the middle, each block
written at its sequences and, off the diagonal, at their reverses.  Bit-exact
against the oracle: full maps of small boxes, the full 3x3x3 map (equal to
the plain map and to the oracle's fixture), block windows on the
configuration lattices, with nothing written outside the scored blocks."""
import numpy as np
import pytest

import oracle
import paper_2008_05612_amd as hp
from tests import _golden333 as g333
from tests._canon import canonical_wide_block_sequences
from tests.conftest import gpu_available
from tests.test_gpu_enumerate import _assert_equal, _full_map_invariants, _oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def _rev(s, N):
    return int(format(s, "0%db" % N)[::-1], 2)


def wide_block_sequences(N, t):
    seqs, diag = canonical_wide_block_sequences(N, t)
    return [int(x) for x in seqs], diag


def _run(dims, b_lo, b_hi, out=None, emin=None):
    import torch
    s = hp.Structures(*dims)
    ws = s.workspace()
    n = 1 << s.N
    if out is None:
        out = torch.full((n,), -7, dtype=torch.int16, device="cuda")
        emin = torch.full((n,), 99, dtype=torch.int32, device="cuda")
    d = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
    nd = torch.zeros(1, dtype=torch.int64, device="cuda")
    print("symmetric wide", dims, b_lo, b_hi, flush=True)
    hp.hp_enumerate_symmetric_wide(s, ws, b_lo, b_hi, out, emin, d, nd)
    torch.cuda.synchronize()
    return s, out, emin, d, nd


@pytest.mark.parametrize("dims", [(2, 5, 1), (3, 4, 1), (2, 2, 3), (4, 4, 1), (3, 5, 1),
                                  (2, 2, 4), (2, 3, 3)])
def test_wide_symmetric_full_small_maps(dims):
    s = hp.Structures(*dims)
    nb = hp.hp_wide_block_count(s)
    assert nb > 0
    s, out, emin, d, nd = _run(dims, 0, nb)
    _assert_equal({"out": out.cpu().numpy().view(np.uint16), "emin": emin.cpu().numpy(),
                   "desig": d.cpu().numpy().view(np.uint64), "nondesign": int(nd.item())},
                  _oracle(dims, 0, 1 << s.N))


def test_wide_symmetric_full_3x3x3_equals_plain_and_oracle():
    import torch
    s = hp.Structures(3, 3, 3)
    nb = hp.hp_wide_block_count(s)
    assert nb == 65792
    third = nb // 3 + 17
    s, out, emin, d, nd = _run((3, 3, 3), 0, third)
    d2 = torch.zeros_like(d)
    nd2 = torch.zeros_like(nd)
    hp.hp_enumerate_symmetric_wide(s, s.workspace(), third, nb, out, emin, d2, nd2)
    o1, d1, n1 = _full_map_invariants((3, 3, 3), hp.FORM_BLOCKED_I8)
    assert torch.equal(out, o1)
    assert np.array_equal((d + d2).cpu().numpy().view(np.uint64), d1)
    assert int(nd.item()) + int(nd2.item()) == n1
    n, bad, full = g333.compare(out)
    print("oracle chunks compared %d, mismatching %s, whole map %s" % (n, bad, full), flush=True)
    assert not bad and full is not False


@pytest.mark.parametrize("dims", [(6, 6, 1), (3, 3, 3), (5, 5, 1)])
def test_wide_symmetric_windows_match_oracle(dims):
    import torch
    s = hp.Structures(*dims)
    N = s.N
    nb = hp.hp_wide_block_count(s)
    st = oracle.structures(*dims)
    rng = np.random.default_rng(0x5EC + N)
    big = N > 30     # 6x6: the uint16 map alone is 137 GB; no energies, no full scan
    out = torch.empty((1 << N,), dtype=torch.int16, device="cuda")
    emin = None if big else torch.empty((1 << N,), dtype=torch.int32, device="cuda")
    for b0 in [0, nb - 2] + [int(x) for x in rng.integers(0, nb - 2, 2)]:
        out.fill_(-7)
        if emin is not None:
            emin.fill_(99)
        _run(dims, b0, b0 + 2, out, emin)
        seqs, revs = [], []
        for t in range(b0, b0 + 2):
            sq, diag = wide_block_sequences(N, t)
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
