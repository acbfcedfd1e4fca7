"""The full pure-HP 3x3x3 map (all 2^27 sequences x 103346 conformations) in
all three kernel forms (the blocked form in its per-wave and its wide
launch shapes), against the CPU oracle's full map.

The oracle's map is a committed fixture (tests/golden/pure_hp_3x3x3_map.txt,
written by tests/golden/make_pure_hp_3x3x3.py from the oracle alone): SHA-256
hashes of the phenotypes of every chunk of 2^20 reversal-canonical
sequences, and, once every chunk is done, of the whole map and of the
designability histogram.  Each form's map must match every chunk the fixture
holds, the three forms must agree entry by entry, and the counts must sum to
2^27.
"""
import numpy as np
import pytest

import paper_2008_05612_amd as hp
from tests import _golden333 as g333
from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu
# form and, for the blocked form, its launch shape (waves, staging mode):
# per-wave blocks, wide blocks of 1024 on 4 waves, of 2048 on 8 waves, and the
# default shape (the benchmark's)
FORMS = {"blocked_i8": (hp.FORM_BLOCKED_I8, (4, 2)), "blocked_i8_wide": (hp.FORM_BLOCKED_I8, (4, 3)),
         "blocked_i8_wide8": (hp.FORM_BLOCKED_I8, (8, 3)), "blocked_i8_default": (hp.FORM_BLOCKED_I8, (4, -1)),
         "gemm_i8": (hp.FORM_GEMM_I8, None), "popcount": (hp.FORM_POPCOUNT, None)}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def full_maps():
    import torch
    s = hp.Structures(3, 3, 3)
    ws = s.workspace()
    total = 1 << 27
    res = {}
    keep = hp.hp_blocked_selected()
    try:
        for name, (form, shape) in FORMS.items():
            if shape:
                hp.hp_blocked_select(*shape)
            out = torch.full((total,), -2, dtype=torch.int16, device="cuda")
            d = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
            nd = torch.zeros(1, dtype=torch.int64, device="cuda")
            print("3x3x3 full map, form", name, flush=True)
            hp.hp_enumerate(s, ws, form, 0, total, out, None, d, nd)
            torch.cuda.synchronize()
            res[name] = (out, d.cpu().numpy().view(np.uint64), int(nd.item()))
    finally:
        hp.hp_blocked_select(*keep)
    return s, res, g333.canonical_sequences()


@pytest.mark.parametrize("name", list(FORMS))
def test_full_map_matches_the_oracle(full_maps, name):
    s, res, canon = full_maps
    out, d, nd = res[name]
    assert int(d.sum()) + nd == 1 << 27
    chunks, whole = g333.load()
    if not chunks:
        pytest.skip("the oracle's fixture holds no chunk yet")
    n, bad, full = g333.compare(out, canon)
    print("%s: %d oracle chunks compared, mismatching %s, whole map %s"
          % (name, n, bad, full), flush=True)
    assert not bad
    if full is not None:
        assert full
        assert g333.designability_sha(d) == whole["designability_sha256"]
        assert nd == int(whole["nondesign"])


def test_three_forms_agree(full_maps):
    import torch
    s, res, canon = full_maps
    ref = res["blocked_i8"]
    assert not bool((ref[0] == -2).any())
    for name in ("blocked_i8_wide", "blocked_i8_wide8", "blocked_i8_default", "gemm_i8", "popcount"):
        assert torch.equal(res[name][0], ref[0]), name
        assert np.array_equal(res[name][1], ref[1]), name
        assert res[name][2] == ref[2], name
