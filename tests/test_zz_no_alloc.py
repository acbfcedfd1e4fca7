"""hp_enumerate_batch_static (no device allocation: the work list lives in
the library's own device array) against hp_enumerate_batch (caller
workspace) on the same jobs: bit-exact maps, energies and counts, for two
calls in a row, the second with fewer and smaller jobs, in both int8 forms.
A few windows are also checked against the oracle."""
import numpy as np
import pytest

import oracle
import paper_2008_05612_amd as hp
from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu

FIRST = [((4, 4, 1), 0, 1 << 16), ((5, 5, 1), 3, 3 + 50001), ((2, 3, 4), 7, 7 + 40000),
         ((3, 3, 3), 12345, 12345 + 30000), ((6, 6, 1), (1 << 35) - 1000, (1 << 35) + 2777),
         ((4, 4, 1), 100, 7000)]
SECOND = [((3, 3, 3), 777, 777 + 4099), ((4, 4, 1), 5, 901)]


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


def _jobs(batch):
    import torch
    jobs, bufs = [], []
    for dims, lo, hi in batch:
        s, ws = _structs(dims)
        b = (torch.full((hi - lo,), -7, dtype=torch.int16, device="cuda"),
             torch.full((hi - lo,), 99, dtype=torch.int32, device="cuda"),
             torch.zeros(s.n_class, dtype=torch.int64, device="cuda"),
             torch.zeros(1, dtype=torch.int64, device="cuda"))
        bufs.append(b)
        jobs.append(hp.Job(s, ws, lo, hi, *b))
    return jobs, bufs


@pytest.mark.parametrize("form", [hp.FORM_BLOCKED_I8, hp.FORM_GEMM_I8])
def test_static_batch_equals_workspace_batch(form):
    import torch
    for call, batch in enumerate((FIRST, SECOND)):
        ref_jobs, ref_bufs = _jobs(batch)
        bws = torch.zeros(hp._binding.batch_workspace_bytes(len(ref_jobs)), dtype=torch.uint8,
                          device="cuda")
        print("form %d call %d: %d jobs" % (form, call, len(batch)), flush=True)
        hp.hp_enumerate_batch(ref_jobs, form, bws)
        jobs, bufs = _jobs(batch)
        hp.hp_enumerate_batch_static(jobs, form)
        torch.cuda.synchronize()
        for (dims, lo, hi), a, b in zip(batch, bufs, ref_bufs):
            for x, y in zip(a, b):
                assert torch.equal(x, y), (call, dims, lo, hi)
        dims, lo, hi = batch[0]
        gs = oracle.ground_states(oracle.structures(*dims), lo, min(hi, lo + 2048))
        n = gs.out.shape[0]
        assert np.array_equal(bufs[0][0][:n].cpu().numpy().view(np.uint16), gs.out)


def test_static_batch_rejects_too_many_jobs():
    import torch
    s, ws = _structs((4, 4, 1))
    out = torch.empty(16, dtype=torch.int16, device="cuda")
    jobs = [hp.Job(s, ws, 0, 16, out)] * (hp._binding.STATIC_BATCH_MAX_JOBS + 1)
    with pytest.raises(hp.HPError) as e:
        hp.hp_enumerate_batch_static(jobs, hp.FORM_GEMM_I8)
    assert "HP_ERANGE" in str(e.value)
