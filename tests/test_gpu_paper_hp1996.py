"""The full 3x3x3 map with the paper's HP contact table (Table 1, scaled by
10) against every number the paper prints for it.

Phenotype denominators are the designable phenotypes (47449).  The paper's
N_s counts the sequences of one conformation (its histogram covers half of
sequence space); classes here hold both chain directions.  Two printed
statistics are not reproduced at their printed precision (the mean share of
other non-deleterious neighbours, and the share of phenotypes whose
robustness lies above the null model); they are strict expected failures,
so a change that made them agree would be noticed.  The oracle is not
involved: these are the paper's own values.
"""
import os

import numpy as np
import pytest

import paper_2008_05612_amd as hp
from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_hp1996_3x3x3.txt")
HP1996_X10 = (0, -10, -10, -23)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def _golden(unreproduced=False):
    """Rows of the golden file: the asserted ones, or (unreproduced=True)
    the ones marked as not reproduced."""
    rows = {}
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        if (len(f) > 3 and f[3] == "unreproduced") == unreproduced:
            rows[f[0]] = (float(f[1]), float(f[2]))
    return rows


@pytest.fixture(scope="module")
def hp1996_map():
    import torch
    s = hp.Structures(3, 3, 3, table=HP1996_X10)
    ws = s.workspace()
    total = 1 << 27
    out = torch.empty(total, dtype=torch.int16, device="cuda")
    d = torch.zeros(s.n_class, dtype=torch.int64, device="cuda")
    nd = torch.zeros(1, dtype=torch.int64, device="cuda")
    print("HP1996 3x3x3 full map", flush=True)
    hp.hp_enumerate(s, ws, hp.FORM_GEMM_I8, 0, total, out, None, d, nd)
    torch.cuda.synchronize()
    desig = d.cpu().numpy().view(np.uint64)
    top = int(desig.argmax())
    z = lambda n: torch.zeros(n, dtype=torch.int64, device="cuda")  # noqa: E731
    neu, dele, oth, row = z(s.n_class), z(s.n_class), z(s.n_class), z(s.n_class + 1)
    hp.hp_neighbors(s, out, neu, dele, oth, top, row)
    torch.cuda.synchronize()
    u = lambda t: t.cpu().numpy().view(np.uint64)  # noqa: E731
    return s, desig, int(nd.item()), top, u(neu), u(dele), u(oth), u(row), out


def _near(name, got, gold):
    val, prec = gold[name]
    print("%-26s paper %-10g got %.6g" % (name, val, got), flush=True)
    assert abs(got - val) <= prec + 1e-12, name


def test_counts_match_the_paper(hp1996_map):
    s, desig, nondes, top, *_ = hp1996_map
    g = _golden()
    total = 1 << 27
    assert int(desig.sum()) + nondes == total
    _near("n_class", s.n_class, g)
    _near("undesignable_classes", int((desig == 0).sum()), g)
    _near("designable_classes", int((desig > 0).sum()), g)
    _near("designing_percent", 100.0 * float(desig.sum()) / total, g)
    _near("deleterious_percent", 100.0 * nondes / total, g)
    # The paper's N_s counts the sequences of one fold over half of sequence
    # space (Appendix B: the map is symmetric, so only half was computed),
    # i.e. per conformation; a class of two conformations c, R(c) holds twice
    # that, a self-reverse class exactly that.
    per_conf = desig // np.where(s.export()["self_rev"] == 1, 1, 2).astype(np.uint64)
    print("top class designability %d (self-reverse %d), per conformation %d"
          % (desig[top], s.export()["self_rev"][top], per_conf.max()), flush=True)
    _near("top_designability", int(per_conf.max()), g)


def test_neighbourhood_statistics_match_the_paper(hp1996_map):
    s, desig, nondes, top, neu, dele, oth, row, _ = hp1996_map
    g = _golden()
    N = 27
    des = desig > 0
    nq = desig[des].astype(np.float64)
    connected = int((row[:s.n_class][des] > 0).sum()) - 1    # other than the top fold itself
    print("connected to top: %d of %d designable (%.3f%%), of %d folds (%.3f%%)"
          % (connected, des.sum(), 100.0 * connected / des.sum(), s.n_class,
             100.0 * connected / s.n_class), flush=True)
    _near("connected_to_top_percent", 100.0 * connected / float(des.sum()), g)
    _near("mean_phi_del", float((dele[des] / (N * nq)).mean()), g)
    iso = int((oth[des] == 0).sum())
    _near("isolated_phenotypes", iso, g)
    _near("isolated_percent", 100.0 * iso / float(des.sum()), g)
    _near("connected_percent", 100.0 * (1 - iso / float(des.sum())), g)


@pytest.mark.xfail(strict=True, reason="printed 4.0 %; the map gives 4.07 %")
def test_mean_other_share_not_reproduced(hp1996_map):
    s, desig, nondes, top, neu, dele, oth, row, _ = hp1996_map
    des = desig > 0
    nq = desig[des].astype(np.float64)
    _near("mean_other_percent", 100.0 * float((oth[des] / (27 * nq)).mean()),
          _golden(unreproduced=True))


@pytest.mark.xfail(strict=True, reason="printed 43.6 %; every null-model reading tried gives "
                                       "far more")
def test_robust_above_null_not_reproduced(hp1996_map):
    s, desig, nondes, top, neu, dele, oth, row, _ = hp1996_map
    N, total = 27, float(1 << 27)
    des = desig > 0
    nq = desig[des].astype(np.float64)
    rho = neu[des] / (N * nq)
    self_rev = s.export()["self_rev"][des] == 1
    readings = {
        "frequency N_q / 2^N": nq / total,
        "frequency among designing sequences": nq / float(desig.sum()),
        "frequency per conformation": nq / np.where(self_rev, 1.0, 2.0) / total,
    }
    for name, null in readings.items():
        print("robust above null, %s: %.2f%% of designable phenotypes, %.2f%% of all folds"
              % (name, 100.0 * float((rho > null).mean()),
                 100.0 * float((rho > null).sum()) / s.n_class), flush=True)
    _near("robust_above_null_percent", 100.0 * float((rho > nq / total).mean()),
          _golden(unreproduced=True))


def test_full_phi_matrix_matches_the_paper(hp1996_map):
    """All 51704 x 51705 counts of Eq. 2 (21.4 GB dense on the device), then
    compressed rows: the paper's neighbourhood numbers and the invariants of
    the whole matrix."""
    import torch
    s, desig, nondes, top, neu, dele, oth, row, out = hp1996_map
    g = _golden()
    n, N = s.n_class, 27
    c = torch.zeros((n, n + 1), dtype=torch.int64, device="cuda")
    print("phi matrix %d x %d" % (n, n + 1), flush=True)
    hp.hp_phi_counts(s, out, c)
    rp = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    nnz = hp.hp_phi_sparse(s, c, rp)
    cols = torch.empty(nnz, dtype=torch.int32, device="cuda")
    vals = torch.empty(nnz, dtype=torch.int64, device="cuda")
    hp.hp_phi_sparse(s, c, rp, cols, vals)
    top_dense = c[top].cpu().numpy().view(np.uint64)
    del c
    torch.cuda.synchronize()
    rp = rp.cpu().numpy().astype(np.int64)
    p = cols.cpu().numpy().astype(np.int64)
    v = vals.cpu().numpy().view(np.uint64)
    q = np.repeat(np.arange(n), np.diff(rp))
    print("non-zero entries %d" % nnz, flush=True)
    # the row of the top fold is hp_neighbors' phi row
    assert np.array_equal(top_dense, row)
    # every genotype has N mutants; diagonal, deleterious column and the rest
    assert np.array_equal(np.bincount(q, weights=v, minlength=n).astype(np.uint64),
                          N * desig.astype(np.uint64))
    diag = q == p
    assert np.array_equal(np.bincount(q[diag], weights=v[diag], minlength=n).astype(np.uint64), neu)
    dcol = p == n
    assert np.array_equal(np.bincount(q[dcol], weights=v[dcol], minlength=n).astype(np.uint64),
                          dele)
    off = ~diag & ~dcol
    assert np.array_equal(np.bincount(q[off], weights=v[off], minlength=n).astype(np.uint64), oth)
    # single-point mutation is an involution: the q -> p and p -> q links match
    k1 = q[off] * n + p[off]
    k2 = p[off] * n + q[off]
    o2 = np.argsort(k2, kind="stable")
    assert np.array_equal(k1, k2[o2]) and np.array_equal(v[off], v[off][o2])
    # the paper's numbers, now read from the whole matrix
    des = desig > 0
    linked = np.bincount(q[off], minlength=n) > 0
    iso = int((des & ~linked).sum())
    _near("isolated_phenotypes", iso, g)
    _near("connected_percent", 100.0 * (1 - iso / float(des.sum())), g)
    _near("connected_to_top_percent", 100.0 * int((q[off] == top).sum()) / float(des.sum()), g)
