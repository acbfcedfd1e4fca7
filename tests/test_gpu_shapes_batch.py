"""Every compiled tile shape of the int8 form, the persistent batched launch
and its hipGraph replay, all bit-exact against the oracle."""
import numpy as np
import pytest

import oracle
import paper_2008_05612_amd as hp
from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


_structs = {}


def _get(dims):
    if dims not in _structs:
        s = hp.Structures(*dims)
        _structs[dims] = (s, s.workspace())
    return _structs[dims]


def _alloc(s, n):
    import torch
    return (torch.full((n,), -7, dtype=torch.int16, device="cuda"),
            torch.full((n,), 99, dtype=torch.int32, device="cuda"),
            torch.zeros(s.n_class, dtype=torch.int64, device="cuda"),
            torch.zeros(1, dtype=torch.int64, device="cuda"))


def _host(o, e, d, nd):
    return (o.cpu().numpy().view(np.uint16), e.cpu().numpy(), d.cpu().numpy().view(np.uint64),
            int(nd.item()))


def _check(res, gs):
    o, e, d, nd = res
    assert np.array_equal(o, gs.out)
    assert np.array_equal(e, gs.emin)
    assert np.array_equal(d, gs.designability)
    assert nd == gs.nondesign


# one lattice per product depth, with a window that spans several workgroups
# and ends in a ragged tail
SHAPE_CASES = [((2, 2, 1), 0, 16), ((3, 4, 1), 0, 4096), ((4, 4, 1), 0, 65536),
               ((2, 3, 3), 1234, 1234 + 70001), ((2, 3, 4), 5000, 5000 + 3001),
               ((5, 5, 1), 77, 77 + 20001), ((3, 3, 3), 99999, 99999 + 2500),
               ((6, 6, 1), (1 << 36) - 3001, 1 << 36)]


@pytest.mark.parametrize("dims,lo,hi", SHAPE_CASES)
def test_every_shape_bit_exact(dims, lo, hi):
    import torch
    s, ws = _get(dims)
    gs = oracle.ground_states(oracle.structures(*dims), lo, hi)
    shapes = hp.hp_gemm_shapes(s.K_pad)
    assert shapes, "no compiled shape for K_pad %d" % s.K_pad
    keep = hp.hp_gemm_selected(s.K_pad)
    try:
        for idx, shape in enumerate(shapes):
            print("shape", dims, s.K_pad, idx, shape, flush=True)
            hp.hp_gemm_select(s.K_pad, idx)
            bufs = _alloc(s, hi - lo)
            hp.hp_enumerate(s, ws, hp.FORM_GEMM_I8, lo, hi, *bufs)
            torch.cuda.synchronize()
            _check(_host(*bufs), gs)
    finally:
        hp.hp_gemm_select(s.K_pad, keep)


def test_autotune_selects_a_shape():
    import torch
    s, ws = _get((5, 5, 1))
    keep = hp.hp_gemm_selected(s.K_pad)
    best, ms = hp.hp_autotune(s, ws, 0, 1 << 16, repeats=1)
    assert 0 <= best < len(ms) and all(m > 0 for m in ms)
    assert hp.hp_gemm_selected(s.K_pad) == best
    assert ms[best] == min(ms)
    hp.hp_gemm_select(s.K_pad, keep)
    torch.cuda.synchronize()


BATCH = [((4, 4, 1), 0, 1 << 16), ((5, 5, 1), 3, 3 + 50001), ((2, 3, 4), 1 << 20, (1 << 20) + 4099),
         ((3, 3, 3), 12345, 12345 + 2048), ((2, 2, 1), 0, 16), ((4, 4, 1), 100, 7000)]


# the blocked form needs N >= 8: the 2x2 job is left out; ranges cut blocks
BATCH_BLOCKED = [((4, 4, 1), 0, 1 << 16), ((5, 5, 1), 3, 3 + 50001),
                 ((2, 3, 4), (1 << 20) + 7, (1 << 20) + 4099), ((3, 3, 3), 12345, 12345 + 2048),
                 ((4, 4, 1), 100, 7000), ((6, 6, 1), (1 << 35) - 1000, (1 << 35) + 777)]


def _batch_jobs(batch=None):
    jobs, bufs = [], []
    for dims, lo, hi in (BATCH if batch is None else batch):
        s, ws = _get(dims)
        b = _alloc(s, hi - lo)
        bufs.append(b)
        jobs.append(hp.Job(s, ws, lo, hi, *b))
    return jobs, bufs


# blocked batches run wide blocks by default (every job here has N >= 10);
# with a per-wave staging mode selected they run blocks of 256
@pytest.mark.parametrize("form,shape", [(hp.FORM_GEMM_I8, None), (hp.FORM_BLOCKED_I8, None),
                                        (hp.FORM_BLOCKED_I8, (4, 2)), (hp.FORM_BLOCKED_I8, (8, 3))])
def test_batch_matches_oracle(form, shape):
    import torch
    batch = BATCH if form == hp.FORM_GEMM_I8 else BATCH_BLOCKED
    keep = hp.hp_blocked_selected()
    try:
        if shape:
            hp.hp_blocked_select(*shape)
        jobs, bufs = _batch_jobs(batch)
        bws = torch.zeros(hp._binding.batch_workspace_bytes(len(jobs)), dtype=torch.uint8,
                          device="cuda")
        print("batch of", len(jobs), "form", form, "shape", shape, flush=True)
        hp.hp_enumerate_batch(jobs, form, bws)
        torch.cuda.synchronize()
    finally:
        hp.hp_blocked_select(*keep)
    for (dims, lo, hi), b in zip(batch, bufs):
        _check(_host(*b), oracle.ground_states(oracle.structures(*dims), lo, hi))


def test_batch_popcount_form_matches_oracle():
    import torch
    jobs, bufs = _batch_jobs()
    bws = torch.zeros(hp._binding.batch_workspace_bytes(len(jobs)), dtype=torch.uint8,
                      device="cuda")
    hp.hp_enumerate_batch(jobs, hp.FORM_POPCOUNT, bws)
    torch.cuda.synchronize()
    for (dims, lo, hi), b in zip(BATCH, bufs):
        _check(_host(*b), oracle.ground_states(oracle.structures(*dims), lo, hi))


@pytest.mark.parametrize("form", [hp.FORM_GEMM_I8, hp.FORM_BLOCKED_I8])
def test_graph_replays_match_eager(form):
    import torch
    batch = BATCH if form == hp.FORM_GEMM_I8 else BATCH_BLOCKED
    jobs, bufs = _batch_jobs(batch)
    bws = torch.zeros(hp._binding.batch_workspace_bytes(len(jobs)), dtype=torch.uint8,
                      device="cuda")
    g = hp.hp_graph_capture_batch(jobs, form, bws)
    refs = [oracle.ground_states(oracle.structures(*dims), lo, hi) for dims, lo, hi in batch]
    for replay in range(1, 4):
        for o, e, d, nd in bufs:      # outputs overwritten; counters keep accumulating
            o.fill_(-7)
            e.fill_(99)
        print("graph replay", replay, flush=True)
        g.launch()
        torch.cuda.synchronize()
        # unrelated eager work between replays
        x = torch.arange(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        assert int(x.item()) == (1 << 20) * ((1 << 20) - 1) // 2
        for b, gs in zip(bufs, refs):
            o, e, d, nd = _host(*b)
            assert np.array_equal(o, gs.out) and np.array_equal(e, gs.emin)
            assert np.array_equal(d, gs.designability * np.uint64(replay))
            assert nd == gs.nondesign * replay
