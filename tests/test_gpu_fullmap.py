"""Full-map driver: checkpoint/resume, and the full 6x6 map.

The 6x6 map (2^36 sequences x 57337 conformations, 137 GB resident; the
blocked form over reversal-canonical wide blocks, in steps of 2^33
sequences, so that every step crosses the library's own launch cuts at 2^30
sequences).  Its parity
checks: every entry written and the sum invariant over all 2^36 sequences,
the symmetry invariant on a large random sample, oracle windows at both ends
and at seeded offsets, the oracle on the blocks on both sides of launch
cuts, and the popcount form on sampled windows.
"""
import json

import numpy as np
import pytest

import oracle
import paper_2008_05612_amd as hp
from paper_2008_05612_amd import fullmap
from tests._canon import (canonical_block_sequences, canonical_wide_block_sequences,
                          reverse_bits)
from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


class _Stop(Exception):
    pass


def test_checkpoint_resume_is_identical(tmp_path):
    dims = (4, 4, 1)
    ref = fullmap.run(dims, block_bits=12, keep_map=False, progress=lambda m: None)
    ck = str(tmp_path / "ck.json")
    seen = []

    def stop_after_five(msg):
        seen.append(msg)
        if len(seen) == 5:
            raise _Stop()

    with pytest.raises(_Stop):
        fullmap.run(dims, block_bits=12, keep_map=False, checkpoint=ck, progress=stop_after_five)
    assert json.load(open(ck))["next_block"] == 5
    res = fullmap.run(dims, block_bits=12, keep_map=False, checkpoint=ck,
                      progress=lambda m: None)
    assert res["resumed_at_block"] == 5
    assert np.array_equal(res["_designability"], ref["_designability"])
    assert res["nondesign"] == ref["nondesign"]
    gs = oracle.ground_states(oracle.structures(*dims))
    assert np.array_equal(ref["_designability"], gs.designability)


@pytest.mark.parametrize("form", [None, hp.FORM_GEMM_I8, hp.FORM_POPCOUNT])
def test_checkpoint_resume_symmetric(tmp_path, form):
    dims = (4, 4, 1)
    ref = fullmap.run(dims, block_bits=10, keep_map=False, progress=lambda m: None)
    ck = str(tmp_path / "cks.json")
    seen = []

    def stop_after_two(msg):
        seen.append(msg)
        if len(seen) == 2:
            raise _Stop()

    with pytest.raises(_Stop):
        fullmap.run(dims, form=form, block_bits=10, keep_map=False, checkpoint=ck,
                    symmetric=True, progress=stop_after_two)
    res = fullmap.run(dims, form=form, block_bits=10, keep_map=False, checkpoint=ck,
                      symmetric=True, progress=lambda m: None)
    assert res["resumed_at_block"] == 2 and res["scored_sequences"] < 1 << 16
    assert res["form"] == {None: "blocked_i8", hp.FORM_GEMM_I8: "gemm_i8",
                           hp.FORM_POPCOUNT: "popcount"}[form]
    assert np.array_equal(res["_designability"], ref["_designability"])
    assert res["nondesign"] == ref["nondesign"]


def test_full_6x6_map():
    import torch
    res = fullmap.run((6, 6, 1), neighbors=True, symmetric=True, block_bits=33, fill=-2,
                      progress=lambda m: print(m, flush=True))
    pub = {k: v for k, v in res.items() if not k.startswith("_") and k != "map"}
    print(json.dumps(pub), flush=True)
    out = res["map"]
    s = res["_structs"]
    N = 36
    d = res["_designability"]
    assert res["sum_check"] and res["neighbor_sum_check"]
    assert res["unwritten"] == 0
    assert np.all(d[s.export()["self_rev"] == 0] % 2 == 0)
    neu = res["_counts"][0]
    assert np.all(neu % 2 == 0)
    # reversal symmetry on 2^26 random sequences
    g = torch.Generator(device="cuda").manual_seed(0x2008056120)
    idx = torch.randint(0, 1 << N, (1 << 26,), device="cuda", generator=g, dtype=torch.int64)
    rev = torch.zeros_like(idx)
    for i in range(N):
        rev |= ((idx >> i) & 1) << (N - 1 - i)
    assert torch.equal(out[idx], out[rev])
    # oracle windows
    st = oracle.structures(6, 6, 1)
    rng = np.random.default_rng(0x2008056120)
    offs = [0, (1 << N) - 4096] + [int(x) for x in rng.integers(0, (1 << N) - 4096, 4)]
    for lo in offs:
        gs = oracle.ground_states(st, lo, lo + 4096)
        assert np.array_equal(out[lo:lo + 4096].cpu().numpy().view(np.uint16), gs.out), lo
    # the blocks on both sides of launch cuts (2^30 sequences per launch:
    # 2^20 wide blocks or 2^22 blocks of 256)
    wide = res["geometry"] == "wide"
    cut = 1 << (20 if wide else 22)
    block_seqs = canonical_wide_block_sequences if wide else canonical_block_sequences
    for t in cut - 1, cut, 5 * cut - 1, 5 * cut:
        seqs, diag = block_seqs(N, t)
        gs = oracle.ground_states_gap(st, seqs, threshold=1)
        idx = torch.from_numpy(seqs.view(np.int64)).cuda()
        ridx = torch.from_numpy(reverse_bits(seqs, N).view(np.int64)).cuda()
        assert np.array_equal(out[idx].cpu().numpy().view(np.uint16), gs.out), t
        assert np.array_equal(out[ridx].cpu().numpy().view(np.uint16), gs.out), t
    # popcount form on sampled windows of the resident map
    for lo in offs[:3]:
        o2 = torch.empty(1 << 20, dtype=torch.int16, device="cuda")
        lo2 = min(lo, (1 << N) - (1 << 20))
        hp.hp_enumerate(s, s.workspace(), hp.FORM_POPCOUNT, lo2, lo2 + (1 << 20), o2)
        torch.cuda.synchronize()
        assert torch.equal(o2, out[lo2:lo2 + (1 << 20)])
