"""The mixed batch at its full sizes: one captured hipGraph over the complete
4x4 (2^16), 5x5 (2^25), 2x3x4 (2^24) and 3x3x3 (2^27) maps, in the dense and
blocked int8 forms, then the neutral-network union-find on the 3x3x3 job.

References: the 4x4 map from the oracle; the 5x5 and 2x3x4 maps from the
popcount form (separate launches) plus oracle windows at seeded offsets; the
3x3x3 map from the oracle's committed full map (tests/golden/
pure_hp_3x3x3_map.txt, per chunk of reversal-canonical sequences).  Every
job's counts must sum to its sequence count.
"""
import numpy as np
import pytest

import oracle
import paper_2008_05612_amd as hp
from tests import _golden333 as g333
from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu
JOBS = [(4, 4, 1), (5, 5, 1), (2, 3, 4), (3, 3, 3)]
NONE = 0xFFFF


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


_st = {}


def _structs(dims):
    if dims not in _st:
        s = hp.Structures(*dims)
        _st[dims] = (s, s.workspace())
    return _st[dims]


@pytest.fixture(scope="module")
def popcount_maps():
    import torch
    res = {}
    for dims in JOBS[1:3]:
        s, ws = _structs(dims)
        out = torch.empty(1 << s.N, dtype=torch.int16, device="cuda")
        hp.hp_enumerate(s, ws, hp.FORM_POPCOUNT, 0, 1 << s.N, out)
        res[dims] = out
    torch.cuda.synchronize()
    return res


@pytest.fixture(scope="module")
def canon():
    return g333.canonical_sequences()


@pytest.mark.parametrize("form", [hp.FORM_BLOCKED_I8, hp.FORM_GEMM_I8])
def test_full_mixed_batch_graph(form, popcount_maps, canon):
    import torch
    jobs, bufs = [], []
    for dims in JOBS:
        s, ws = _structs(dims)
        n = 1 << s.N
        b = (torch.full((n,), -2, dtype=torch.int16, device="cuda"),
             torch.zeros(s.n_class, dtype=torch.int64, device="cuda"),
             torch.zeros(1, dtype=torch.int64, device="cuda"))
        bufs.append(b)
        jobs.append(hp.Job(s, ws, 0, n, b[0], None, b[1], b[2]))
    bws = torch.zeros(hp._binding.batch_workspace_bytes(len(jobs)), dtype=torch.uint8,
                      device="cuda")
    print("full mixed batch, form %d: capture" % form, flush=True)
    g = hp.hp_graph_capture_batch(jobs, form, bws)
    print("replay", flush=True)
    g.launch()
    torch.cuda.synchronize()
    for dims, (out, d, nd) in zip(JOBS, bufs):
        s, _ = _structs(dims)
        assert int(d.sum().item()) + int(nd.item()) == 1 << s.N, dims
        assert not bool((out == -2).any()), dims
    # 4x4: the oracle's whole map
    o44, d44, nd44 = bufs[0]
    gs = oracle.ground_states(oracle.structures(4, 4, 1))
    assert np.array_equal(o44.cpu().numpy().view(np.uint16), gs.out)
    assert np.array_equal(d44.cpu().numpy().view(np.uint64), gs.designability)
    # 5x5 and 2x3x4: the popcount form's whole maps, and oracle windows
    rng = np.random.default_rng(0x2008056120)
    for dims, (out, d, nd) in zip(JOBS[1:3], bufs[1:3]):
        assert torch.equal(out, popcount_maps[dims]), dims
        st = oracle.structures(*dims)
        for lo in [0, (1 << st.N) - 512] + [int(x) for x in rng.integers(0, (1 << st.N) - 512, 2)]:
            w = oracle.ground_states(st, lo, lo + 512)
            assert np.array_equal(out[lo:lo + 512].cpu().numpy().view(np.uint16), w.out), (dims, lo)
    # 3x3x3: the oracle's full map, chunk by chunk
    o333, d333, nd333 = bufs[3]
    n, bad, full = g333.compare(o333, canon)
    print("3x3x3 job: %d oracle chunks compared, mismatching %s, whole map %s"
          % (n, bad, full), flush=True)
    assert n > 0 and not bad and full is not False
    # then the neutral networks of the 3x3x3 job
    s, _ = _structs((3, 3, 3))
    total = 1 << 27
    labels = torch.empty(total, dtype=torch.int32, device="cuda")
    size = torch.empty(total, dtype=torch.int32, device="cuda")
    ncomp = torch.empty(s.n_class, dtype=torch.int32, device="cuda")
    largest = torch.empty(s.n_class, dtype=torch.int32, device="cuda")
    print("components of the 3x3x3 job", flush=True)
    hp.hp_components(s, o333, labels, size, ncomp, largest)
    torch.cuda.synchronize()
    o = o333.cpu().numpy().view(np.uint16)
    lab = labels.cpu().numpy().view(np.uint32)
    sz = size.cpu().numpy().view(np.uint32)
    desig = d333.cpu().numpy().view(np.uint64)
    des = o != NONE
    idx = np.arange(total, dtype=np.uint32)
    roots = des & (lab == idx)
    per_class = np.zeros(s.n_class, np.uint64)
    np.add.at(per_class, o[roots], sz[roots].astype(np.uint64))
    assert np.array_equal(per_class, desig)
    assert np.array_equal(np.bincount(o[roots], minlength=s.n_class),
                          ncomp.cpu().numpy().astype(np.int64))
    assert np.all(lab[des] <= idx[des]) and np.all(o[lab[des]] == o[des])
    assert np.all(lab[~des] == 0xFFFFFFFF)
    # every neutral single-point mutation stays inside one component
    gidx = torch.arange(total, dtype=torch.int64, device="cuda")
    gdes = o333 != -1
    for i in range(27):
        nb = gidx ^ (1 << i)
        same = gdes & (o333[nb] == o333)
        assert torch.equal(labels[same], labels[nb[same]]), i
