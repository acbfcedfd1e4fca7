"""GPU parity of hp_neighbors and hp_components against the CPU oracle.

The oracle computes its own phenotype map (never the GPU's) and its own
neighbour counts and breadth-first-search components; the GPU gets the map it
computed itself through hp_enumerate.  Since both maps are checked equal
elsewhere, equal outputs here test the network kernels.  The 3x3x3 map is
checked at full size by invariants.
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


def _gpu_map(dims):
    import torch
    s = hp.Structures(*dims)
    ws = s.workspace()
    total = 1 << s.N
    out = torch.empty(total, dtype=torch.int16, device="cuda")
    hp.hp_enumerate(s, ws, hp.FORM_GEMM_I8, 0, total, out)
    return s, out


def _gpu_network(s, out, phi_q):
    import torch
    total = 1 << s.N
    z = lambda n: torch.zeros(n, dtype=torch.int64, device="cuda")  # noqa: E731
    neu, dele, oth, row = z(s.n_class), z(s.n_class), z(s.n_class), z(s.n_class + 1)
    print("neighbors", s.dims, flush=True)
    hp.hp_neighbors(s, out, neu, dele, oth, phi_q, row)
    labels = torch.empty(total, dtype=torch.int32, device="cuda")
    size = torch.empty(total, dtype=torch.int32, device="cuda")
    ncomp = torch.empty(s.n_class, dtype=torch.int32, device="cuda")
    largest = torch.empty(s.n_class, dtype=torch.int32, device="cuda")
    print("components", s.dims, flush=True)
    hp.hp_components(s, out, labels, size, ncomp, largest)
    torch.cuda.synchronize()
    u64 = lambda t: t.cpu().numpy().view(np.uint64)  # noqa: E731
    u32 = lambda t: t.cpu().numpy().view(np.uint32)  # noqa: E731
    return (u64(neu), u64(dele), u64(oth), u64(row), u32(labels), u32(size), u32(ncomp),
            u32(largest))


@pytest.mark.parametrize("dims", [(3, 3, 1), (3, 4, 1), (2, 2, 3), (4, 4, 1), (3, 5, 1),
                                  (4, 5, 1)])
def test_network_matches_oracle(dims):
    st = oracle.structures(*dims)
    gs = oracle.ground_states(st)
    top = int(np.argmax(gs.designability))
    s, out = _gpu_map(dims)
    neu, dele, oth, row, labels, size, ncomp, largest = _gpu_network(s, out, top)
    nb = oracle.neighbors(st.N, gs.out, st.n_class, phi_q=top)
    assert np.array_equal(neu, nb.neutral)
    assert np.array_equal(dele, nb.deleterious)
    assert np.array_equal(oth, nb.other)
    assert np.array_equal(row, nb.phi_row)
    lab = oracle.components(st.N, gs.out)
    assert np.array_equal(labels, lab)
    des = gs.out != NONE
    ref_size = np.bincount(lab[des], minlength=1 << st.N).astype(np.uint32)
    assert np.array_equal(size, ref_size)
    roots = des & (lab == np.arange(1 << st.N, dtype=np.uint32))
    ref_ncomp = np.bincount(gs.out[roots], minlength=st.n_class)
    assert np.array_equal(ncomp.astype(np.int64), ref_ncomp)
    ref_largest = np.zeros(st.n_class, np.uint32)
    np.maximum.at(ref_largest, gs.out[roots], ref_size[roots])
    assert np.array_equal(largest, ref_largest)


def test_network_3x3x3_full_invariants():
    s, out = _gpu_map((3, 3, 3))
    import torch
    d = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
    hp.hp_enumerate(s, s.workspace(), hp.FORM_GEMM_I8, 0, 1 << 27, None, None, d, None)
    top = int(torch.argmax(d).item())
    neu, dele, oth, row, labels, size, ncomp, largest = _gpu_network(s, out, top)
    desig = d.cpu().numpy().view(np.uint64)
    assert np.all(neu % 2 == 0)
    assert np.array_equal(neu + dele + oth, np.uint64(27) * desig)
    assert int(row.sum()) == 27 * int(desig[top]) and row[top] == neu[top]
    # components partition each phenotype's genotypes
    per_class = np.zeros(s.n_class, np.uint64)
    o = out.cpu().numpy().view(np.uint16)
    roots = (o != NONE) & (labels == np.arange(1 << 27, dtype=np.uint32))
    np.add.at(per_class, o[roots], size[roots].astype(np.uint64))
    assert np.array_equal(per_class, desig)
    assert np.all((ncomp > 0) == (desig > 0))
    des = o != NONE
    assert np.all(labels[des] <= np.arange(1 << 27, dtype=np.uint32)[des])
    assert np.all(o[labels[des]] == o[des])
    assert np.all(labels[~des] == 0xFFFFFFFF)


@pytest.mark.parametrize("dims,none_frac,extra,offset", [
    ((4, 4, 1), 0.3, 2, 0), ((4, 4, 1), 0.3, 2, 1), ((2, 3, 3), 0.6, 0, 0),
    ((2, 3, 3), 0.6, 0, 3), ((4, 5, 1), 0.1, 1, 0), ((4, 5, 1), 0.1, 1, 5)])
def test_network_synthetic_maps_both_layouts(dims, none_frac, extra, offset):
    """Seeded synthetic maps (few distinct ids so that neutral networks are
    large, deleterious genotypes, ids at or beyond n_class that are not
    phenotypes) read from a 16-byte aligned buffer (eight genotypes per lane)
    and from a buffer offset by `offset` genotypes (one genotype per lane):
    neighbour counts, phi row, phi matrix and component labels all equal the
    oracle's."""
    import torch
    s = hp.Structures(*dims)
    n = 1 << s.N
    rng = np.random.default_rng(7919 * s.N + 13 * offset + int(10 * none_frac))
    ids = rng.integers(0, s.n_class, 12)
    phen = ids[rng.integers(0, 12, n)].astype(np.uint16)
    if extra:
        sel = rng.random(n) < 0.03
        phen[sel] = (s.n_class + rng.integers(0, extra, int(sel.sum()))).astype(np.uint16)
    phen[rng.random(n) < none_frac] = NONE
    buf = torch.zeros(n + 16, dtype=torch.int16, device="cuda")
    view = buf[offset:offset + n]
    view.copy_(torch.from_numpy(phen.view(np.int16)))
    assert (view.data_ptr() % 16 == 0) == (offset % 8 == 0)
    top = int(ids[0])
    neu, dele, oth, row, labels, size, ncomp, largest = _gpu_network(s, view, top)
    nb = oracle.neighbors(s.N, phen, s.n_class, phi_q=top)
    assert np.array_equal(neu, nb.neutral)
    assert np.array_equal(dele, nb.deleterious)
    assert np.array_equal(oth, nb.other)
    assert np.array_equal(row, nb.phi_row)
    lab = oracle.components(s.N, phen)
    assert np.array_equal(labels, lab)
    des = phen != NONE
    assert np.array_equal(size, np.bincount(lab[des], minlength=n).astype(np.uint32))
    c = torch.zeros((s.n_class, s.n_class + 1), dtype=torch.int64, device="cuda")
    hp.hp_phi_counts(s, view, c)
    torch.cuda.synchronize()
    assert np.array_equal(c.cpu().numpy().view(np.uint64), oracle.phi_counts(s.N, phen, s.n_class))
