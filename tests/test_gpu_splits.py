"""Ranges longer than one launch: the library's own splitting.

hp_enumerate, hp_enumerate_gap and hp_sample cut a range into launches of
2^30 indices counted from the range's start, offsetting every per-index
output; hp_enumerate_symmetric_blocked cuts a canonical-block range into
launches of 2^22 blocks, hp_enumerate_symmetric_wide a wide-block range into
launches of 2^20 blocks.  Each test hands the library ONE range that crosses
such a cut (not 256-aligned, so the blocked form also meets ragged blocks on
both sides of it) and checks oracle windows at the start, on both sides of
the cut and at the end, plus the count invariant over the whole range.
"""
import numpy as np
import pytest

import oracle
import paper_2008_05612_amd as hp
from tests._canon import canonical_block_sequences, canonical_wide_block_sequences
from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu
CUT = 1 << 30          # indices per launch of hp_enumerate / _gap / hp_sample
BLK_CUT = 1 << 22      # canonical blocks per launch of hp_enumerate_symmetric_blocked
W = 1024               # oracle window
LO = (1 << 33) + 100   # range start (6x6), not a multiple of 256
LEN = CUT + 4 * W + 37


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def six():
    s = hp.Structures(6, 6, 1)
    return s, s.workspace(), oracle.structures(6, 6, 1)


def _windows():
    """Offsets (relative to the range start) of the oracle windows: start,
    both sides of the cut, end."""
    return [0, CUT - W, CUT, LEN - W]


@pytest.mark.parametrize("form", [hp.FORM_BLOCKED_I8, hp.FORM_GEMM_I8])
def test_enumerate_across_the_launch_cut(six, form):
    import torch
    s, ws, st = six
    out = torch.full((LEN,), -2, dtype=torch.int16, device="cuda")
    emin = torch.full((LEN,), 99, dtype=torch.int32, device="cuda")
    d = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
    nd = torch.zeros(1, dtype=torch.int64, device="cuda")
    print("6x6 [%d, %d) form %d" % (LO, LO + LEN, form), flush=True)
    hp.hp_enumerate(s, ws, form, LO, LO + LEN, out, emin, d, nd)
    torch.cuda.synchronize()
    assert int(d.sum().item()) + int(nd.item()) == LEN
    assert not bool((out == -2).any())
    for off in _windows():
        gs = oracle.ground_states(st, LO + off, LO + off + W)
        assert np.array_equal(out[off:off + W].cpu().numpy().view(np.uint16), gs.out), off
        assert np.array_equal(emin[off:off + W].cpu().numpy(), gs.emin), off


def test_gap_across_the_launch_cut(six):
    import torch
    s, ws, st = six
    out = torch.full((LEN,), -2, dtype=torch.int16, device="cuda")
    gap = torch.zeros(LEN, dtype=torch.uint8, device="cuda")
    d = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
    nd = torch.zeros(1, dtype=torch.int64, device="cuda")
    print("6x6 gap, threshold 2, [%d, %d)" % (LO, LO + LEN), flush=True)
    hp.hp_enumerate_gap(s, ws, hp.FORM_BLOCKED_I8, LO, LO + LEN, 2, out, None, gap, d, nd)
    torch.cuda.synchronize()
    assert int(d.sum().item()) + int(nd.item()) == LEN
    for off in _windows():
        seqs = np.arange(LO + off, LO + off + W, dtype=np.uint64)
        gs = oracle.ground_states_gap(st, seqs, threshold=2)
        assert np.array_equal(out[off:off + W].cpu().numpy().view(np.uint16), gs.out), off
        assert np.array_equal(gap[off:off + W].cpu().numpy(), gs.gap), off


def test_sample_across_the_launch_cut(six):
    import torch
    s, ws, st = six
    seed = 0x2008056120
    lo = 12345
    seqs = torch.zeros(LEN, dtype=torch.int64, device="cuda")
    out = torch.full((LEN,), -2, dtype=torch.int16, device="cuda")
    d = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
    nd = torch.zeros(1, dtype=torch.int64, device="cuda")
    print("6x6 sampling, draws [%d, %d)" % (lo, lo + LEN), flush=True)
    hp.hp_sample(s, ws, hp.FORM_GEMM_I8, seed, lo, lo + LEN, 1, seqs, out, None, None, d, nd)
    torch.cuda.synchronize()
    assert int(d.sum().item()) + int(nd.item()) == LEN
    for off in _windows():
        want = oracle.sample_sequences(seed, lo + off, lo + off + W, 36)
        got = seqs[off:off + W].cpu().numpy().view(np.uint64)
        assert np.array_equal(got, want), off
        gs = oracle.ground_states_gap(st, want, threshold=1)
        assert np.array_equal(out[off:off + W].cpu().numpy().view(np.uint16), gs.out), off


def test_symmetric_blocked_across_the_launch_cut(six):
    """Canonical blocks [B, B + 2^22 + 600) in one call (cut at B + 2^22)
    against the same range in calls of 2^21 blocks that cross nothing; the
    two blocks at the cut against the oracle.  These calls write no map (a
    canonical-block map is full size, 137 GB for 6x6): the counts carry the
    comparison, each sequence counted with its reverse unless its block is
    its own reverse."""
    import torch
    s, ws, st = six
    b_lo = 12345
    b_hi = b_lo + BLK_CUT + 600
    cut = b_lo + BLK_CUT
    d1 = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
    nd1 = torch.zeros(1, dtype=torch.int64, device="cuda")
    print("6x6 canonical blocks [%d, %d) in one call" % (b_lo, b_hi), flush=True)
    hp.hp_enumerate_symmetric_blocked(s, ws, b_lo, b_hi, None, None, d1, nd1)
    d2 = torch.zeros_like(d1)
    nd2 = torch.zeros_like(nd1)
    for b in range(b_lo, b_hi, BLK_CUT // 2):
        hp.hp_enumerate_symmetric_blocked(s, ws, b, min(b + BLK_CUT // 2, b_hi), None, None,
                                          d2, nd2)
    torch.cuda.synchronize()
    assert torch.equal(d1, d2) and torch.equal(nd1, nd2)
    assert int(d1.sum().item()) + int(nd1.item()) <= 2 * 256 * (b_hi - b_lo)
    want = np.zeros(s.n_class, dtype=np.uint64)
    want_nd = 0
    for t in (cut - 1, cut):
        seqs, diag = canonical_block_sequences(36, t)
        gs = oracle.ground_states_gap(st, seqs, threshold=1)
        w = 1 if diag else 2
        want += np.bincount(gs.out[gs.out != oracle.NONE], minlength=s.n_class).astype(
            np.uint64) * np.uint64(w)
        want_nd += int((gs.out == oracle.NONE).sum()) * w
    d3 = torch.zeros_like(d1)
    nd3 = torch.zeros_like(nd1)
    hp.hp_enumerate_symmetric_blocked(s, ws, cut - 1, cut + 1, None, None, d3, nd3)
    torch.cuda.synchronize()
    assert np.array_equal(d3.cpu().numpy().view(np.uint64), want)
    assert int(nd3.item()) == want_nd


def test_symmetric_wide_across_the_launch_cut(six):
    """Canonical wide blocks [B, B + 2^20 + 300) in one call (cut at
    B + 2^20) against calls of 2^19 blocks; the two wide blocks at the cut
    against the oracle (counts only, as above)."""
    import torch
    s, ws, st = six
    cut_n = 1 << 20
    b_lo = 4321
    b_hi = b_lo + cut_n + 300
    cut = b_lo + cut_n
    d1 = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
    nd1 = torch.zeros(1, dtype=torch.int64, device="cuda")
    print("6x6 canonical wide blocks [%d, %d) in one call" % (b_lo, b_hi), flush=True)
    hp.hp_enumerate_symmetric_wide(s, ws, b_lo, b_hi, None, None, d1, nd1)
    d2 = torch.zeros_like(d1)
    nd2 = torch.zeros_like(nd1)
    for b in range(b_lo, b_hi, cut_n // 2):
        hp.hp_enumerate_symmetric_wide(s, ws, b, min(b + cut_n // 2, b_hi), None, None, d2, nd2)
    torch.cuda.synchronize()
    assert torch.equal(d1, d2) and torch.equal(nd1, nd2)
    want = np.zeros(s.n_class, dtype=np.uint64)
    want_nd = 0
    for t in (cut - 1, cut):
        seqs, diag = canonical_wide_block_sequences(36, t)
        gs = oracle.ground_states_gap(st, seqs, threshold=1)
        w = 1 if diag else 2
        want += np.bincount(gs.out[gs.out != oracle.NONE], minlength=s.n_class).astype(
            np.uint64) * np.uint64(w)
        want_nd += int((gs.out == oracle.NONE).sum()) * w
    d3 = torch.zeros_like(d1)
    nd3 = torch.zeros_like(nd1)
    hp.hp_enumerate_symmetric_wide(s, ws, cut - 1, cut + 1, None, None, d3, nd3)
    torch.cuda.synchronize()
    assert np.array_equal(d3.cpu().numpy().view(np.uint64), want)
    assert int(nd3.item()) == want_nd
