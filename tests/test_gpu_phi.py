"""GPU parity of the whole phi_pq matrix (hp_phi_counts, hp_phi_sparse)
against the CPU oracle.

Real maps: the oracle enumerates its own map, the GPU its own (the two maps
are checked equal elsewhere).  Synthetic maps: seeded random phenotype ids,
including the deleterious id and ids at or beyond n_class, shared by both
sides.  Counts must agree exactly; the compressed rows must equal the
non-zero pattern of the oracle's dense matrix, columns ascending.
"""
import numpy as np
import pytest

import oracle
import paper_2008_05612_amd as hp
from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu
NONE = 0xFFFF


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def _gpu_counts(s, dmap):
    import torch
    c = torch.zeros((s.n_class, s.n_class + 1), dtype=torch.int64, device="cuda")
    print("phi counts", s.dims, flush=True)
    hp.hp_phi_counts(s, dmap, c)
    torch.cuda.synchronize()
    return c


def _gpu_sparse(s, c):
    import torch
    rp = torch.empty(s.n_class + 1, dtype=torch.int64, device="cuda")
    nnz = hp.hp_phi_sparse(s, c, rp)
    cols = torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda")
    vals = torch.empty(max(nnz, 1), dtype=torch.int64, device="cuda")
    assert hp.hp_phi_sparse(s, c, rp, cols, vals) == nnz
    torch.cuda.synchronize()
    return (rp.cpu().numpy().view(np.uint64), cols[:nnz].cpu().numpy().view(np.uint32),
            vals[:nnz].cpu().numpy().view(np.uint64))


def _check_sparse(dense, rp, cols, vals):
    q, p = np.nonzero(dense)   # row-major order: rows, then ascending columns
    assert int(rp[-1]) == len(q)
    assert np.array_equal(rp, np.concatenate([[0], np.cumsum(np.bincount(
        q, minlength=dense.shape[0]))]).astype(np.uint64))
    assert np.array_equal(cols, p.astype(np.uint32))
    assert np.array_equal(vals, dense[q, p])


@pytest.mark.parametrize("dims", [(3, 3, 1), (2, 2, 3), (4, 4, 1), (3, 5, 1), (4, 5, 1)])
def test_phi_matrix_real_maps(dims):
    import torch
    st = oracle.structures(*dims)
    gs = oracle.ground_states(st)
    want = oracle.phi_counts(st.N, gs.out, st.n_class)
    s = hp.Structures(*dims)
    assert s.n_class == st.n_class
    out = torch.empty(1 << s.N, dtype=torch.int16, device="cuda")
    hp.hp_enumerate(s, s.workspace(), hp.FORM_GEMM_I8, 0, 1 << s.N, out)
    c = _gpu_counts(s, out)
    got = c.cpu().numpy().view(np.uint64)
    assert np.array_equal(got, want)
    _check_sparse(want, *_gpu_sparse(s, c))


@pytest.mark.parametrize("dims,none_frac,extra", [
    ((4, 4, 1), 0.0, 0), ((4, 4, 1), 0.5, 3), ((2, 3, 3), 0.9, 2), ((4, 5, 1), 0.3, 1)])
def test_phi_matrix_synthetic_maps(dims, none_frac, extra):
    import torch
    s = hp.Structures(*dims)
    rng = np.random.default_rng(1000 * s.N + int(10 * none_frac))
    # few distinct ids so that every row has entries; ids n_class .. n_class
    # + extra - 1 are not phenotypes
    ids = rng.integers(0, s.n_class, 40)
    phen = ids[rng.integers(0, 40, 1 << s.N)].astype(np.uint16)
    if extra:
        sel = rng.random(1 << s.N) < 0.05
        phen[sel] = (s.n_class + rng.integers(0, extra, int(sel.sum()))).astype(np.uint16)
    phen[rng.random(1 << s.N) < none_frac] = NONE
    want = oracle.phi_counts(s.N, phen, s.n_class)
    dmap = torch.from_numpy(phen.view(np.int16)).cuda()
    c = _gpu_counts(s, dmap)
    assert np.array_equal(c.cpu().numpy().view(np.uint64), want)
    _check_sparse(want, *_gpu_sparse(s, c))


def test_phi_matrix_degenerate_maps():
    import torch
    s = hp.Structures(3, 3, 1)
    n = 1 << s.N
    # nothing folds: zero matrix, empty rows
    c = _gpu_counts(s, torch.full((n,), -1, dtype=torch.int16, device="cuda"))
    assert not c.any()
    rp, cols, vals = _gpu_sparse(s, c)
    assert not rp.any() and len(cols) == 0
    # one phenotype everywhere: every mutation neutral
    c = _gpu_counts(s, torch.zeros(n, dtype=torch.int16, device="cuda"))
    want = np.zeros((s.n_class, s.n_class + 1), np.uint64)
    want[0, 0] = s.N * n
    assert np.array_equal(c.cpu().numpy().view(np.uint64), want)
    # accumulation: a second call adds
    hp.hp_phi_counts(s, torch.zeros(n, dtype=torch.int16, device="cuda"), c)
    torch.cuda.synchronize()
    assert int(c[0, 0]) == 2 * s.N * n


def test_phi_sparse_capacity():
    import torch
    st = oracle.structures(4, 4, 1)
    gs = oracle.ground_states(st)
    s = hp.Structures(4, 4, 1)
    dmap = torch.from_numpy(gs.out.view(np.int16)).cuda()
    c = _gpu_counts(s, dmap)
    rp = torch.empty(s.n_class + 1, dtype=torch.int64, device="cuda")
    nnz = hp.hp_phi_sparse(s, c, rp)
    assert nnz == int(np.count_nonzero(oracle.phi_counts(st.N, gs.out, st.n_class)))
    small = torch.empty(nnz - 1, dtype=torch.int32, device="cuda")
    smallv = torch.empty(nnz - 1, dtype=torch.int64, device="cuda")
    with pytest.raises(hp.HPError) as e:
        hp.hp_phi_sparse(s, c, rp, small, smallv)
    assert e.value.status == -4
