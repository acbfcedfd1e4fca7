"""CPU oracle for the HP-model genotype-phenotype map -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (``paper_2008_05612_amd``)
never imports, links or executes anything here, and this package imports
nothing from it.

The arithmetic lives in ``hp_oracle.c`` (plain C, optional OpenMP over
sequences); this module only builds it with gcc and marshals numpy arrays.
Every quantity is an integer; see the C file's header for the definitions it
follows (Methods: Eq. 1 and the ground-state rule; Eq. 2 for the neighbourhood
statistics).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
NONE = 0xFFFF

_lib = None


def build(force: bool = False) -> str:
    """Compile hp_oracle.c into liboracle.so (gcc -O2 -fopenmp)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i32p = ctypes.POINTER(ctypes.c_int32)
        u16p = ctypes.POINTER(ctypes.c_uint16)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        c_int, c_long, c_u64 = ctypes.c_int, ctypes.c_long, ctypes.c_uint64
        sig = {
            "or_walks": (c_long, [c_int, c_int, c_int, c_int, u8p, c_long]),
            "or_count_walks": (c_long, [c_int, c_int, c_int]),
            "or_group": (c_int, [c_int, c_int, c_int, u8p]),
            "or_canonical_key": (None, [c_int, c_int, c_int, u8p, u8p]),
            "or_conformations": (c_long, [c_int, c_int, c_int, u8p, c_long]),
            "or_classes": (c_long, [c_int, c_int, c_int, u8p, c_long, i32p, i32p, u8p, u8p]),
            "or_contacts": (c_int, [c_int, c_int, c_int, u8p, u8p]),
            "or_all_contacts": (c_long, [c_int, c_int, c_int, u8p, c_long, i32p, u8p]),
            "or_energy": (c_int, [c_u64, c_int, u8p]),
            "or_energy_table": (c_int, [c_u64, c_int, u8p, i32p]),
            "or_ground_states_table": (None, [c_long, i32p, u8p, i32p, i32p, c_u64, c_u64, u16p,
                                              i32p, u64p, u64p]),
            "or_ground_states": (None, [c_long, i32p, u8p, i32p, c_u64, c_u64, u16p, i32p,
                                        u64p, u64p]),
            "or_ground_states_brute": (None, [c_int, c_int, c_int, u8p, c_long, c_u64, c_u64,
                                              u16p, i32p]),
            "or_ground_states_gap": (None, [c_long, i32p, u8p, i32p, i32p, u64p, c_long, c_int,
                                            u16p, i32p, u8p, u64p, u64p]),
            "or_splitmix64": (c_u64, [c_u64, c_u64]),
            "or_sample_sequences": (None, [c_u64, c_u64, c_u64, c_int, u64p]),
            "or_neighbors": (None, [c_int, u16p, c_long, u64p, u64p, u64p, c_int, u64p]),
            "or_phi_counts": (None, [c_int, u16p, c_long, u64p]),
            "or_components": (None, [c_int, u16p, u32p]),
            "or_num_threads": (c_int, []),
            "or_set_num_threads": (None, [c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray, ct):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ct))


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (results never change)."""
    lib().or_set_num_threads(int(n))


def count_walks(X: int, Y: int, Z: int = 1) -> int:
    return int(lib().or_count_walks(X, Y, Z))


def walks(X: int, Y: int, Z: int = 1, prune: bool = True) -> np.ndarray:
    """All directed Hamiltonian paths of the box, shape (n_walks, N), uint8 site ids."""
    N = X * Y * Z
    n = count_walks(X, Y, Z)
    out = np.zeros((max(n, 1), N), dtype=np.uint8)
    got = lib().or_walks(X, Y, Z, int(prune), _p(out, ctypes.c_uint8), n)
    return out[:got]


def group(X: int, Y: int, Z: int = 1) -> np.ndarray:
    """Isometries of the box as site permutations, shape (|G|, N)."""
    N = X * Y * Z
    buf = np.zeros((48, N), dtype=np.uint8)
    G = lib().or_group(X, Y, Z, _p(buf, ctypes.c_uint8))
    return buf[:G].copy()


def canonical_key(X: int, Y: int, Z: int, walk) -> np.ndarray:
    w = np.ascontiguousarray(np.asarray(walk, dtype=np.uint8))
    key = np.zeros_like(w)
    lib().or_canonical_key(X, Y, Z, _p(w, ctypes.c_uint8), _p(key, ctypes.c_uint8))
    return key


def contacts(X: int, Y: int, Z: int, walk) -> np.ndarray:
    """Contact pairs (i, j) of one walk, shape (n, 2)."""
    N = X * Y * Z
    w = np.ascontiguousarray(np.asarray(walk, dtype=np.uint8))
    buf = np.zeros((N * N, 2), dtype=np.uint8)
    n = lib().or_contacts(X, Y, Z, _p(w, ctypes.c_uint8), _p(buf, ctypes.c_uint8))
    return buf[:n].copy()


@dataclass
class Structures:
    """Symmetry-reduced structure set of one box, as the oracle defines it."""
    dims: tuple
    N: int
    n_walks: int
    G: int
    conf_keys: np.ndarray        # (n_conf, N) uint8, ascending
    conf_to_class: np.ndarray    # (n_conf,) int32
    rev_conf: np.ndarray         # (n_conf,) int32: conformation of the reversed chain
    class_keys: np.ndarray       # (n_class, N) uint8, ascending
    self_rev: np.ndarray         # (n_class,) uint8
    ct_off: np.ndarray           # (n_conf+1,) int32, offsets into pairs (pair units)
    pairs: np.ndarray            # (total contacts, 2) uint8
    _flat: dict = field(default_factory=dict, repr=False)

    @property
    def n_conf(self) -> int:
        return int(self.conf_keys.shape[0])

    @property
    def n_class(self) -> int:
        return int(self.class_keys.shape[0])

    def contact_sets(self):
        return [set(map(tuple, self.pairs[self.ct_off[c]:self.ct_off[c + 1]].tolist()))
                for c in range(self.n_conf)]


_cache: dict = {}


def structures(X: int, Y: int, Z: int = 1) -> Structures:
    key = (X, Y, Z)
    if key in _cache:
        return _cache[key]
    N = X * Y * Z
    nw = count_walks(X, Y, Z)
    scratch = np.zeros((max(nw, 1), N), dtype=np.uint8)
    n_conf = lib().or_conformations(X, Y, Z, _p(scratch, ctypes.c_uint8), nw)
    assert n_conf >= 0
    conf_keys = scratch[:n_conf].copy()
    del scratch
    c2q = np.zeros(n_conf, dtype=np.int32)
    rev = np.zeros(n_conf, dtype=np.int32)
    srev = np.zeros(max(n_conf, 1), dtype=np.uint8)
    ckeys = np.zeros((max(n_conf, 1), N), dtype=np.uint8)
    n_class = lib().or_classes(X, Y, Z, _p(conf_keys, ctypes.c_uint8), n_conf, _p(c2q, ctypes.c_int32),
                               _p(rev, ctypes.c_int32), _p(srev, ctypes.c_uint8),
                               _p(ckeys, ctypes.c_uint8))
    ct_off = np.zeros(n_conf + 1, dtype=np.int32)
    pbuf = np.zeros((max(n_conf, 1) * N * N // 2 + 1, 2), dtype=np.uint8)
    tot = lib().or_all_contacts(X, Y, Z, _p(conf_keys, ctypes.c_uint8), n_conf,
                                _p(ct_off, ctypes.c_int32), _p(pbuf, ctypes.c_uint8))
    pairs = np.ascontiguousarray(pbuf[:tot])
    del pbuf
    G = group(X, Y, Z).shape[0]
    st = Structures((X, Y, Z), N, nw, G, conf_keys, c2q, rev, ckeys[:n_class].copy(),
                    srev[:n_class].copy(), ct_off, pairs)
    _cache[key] = st
    return st


def energy(s: int, pairs) -> int:
    p = np.ascontiguousarray(np.asarray(pairs, dtype=np.uint8).reshape(-1, 2))
    return int(lib().or_energy(int(s), p.shape[0], _p(p, ctypes.c_uint8)))


@dataclass
class GroundStates:
    out: np.ndarray             # uint16 phenotype (class id or 0xFFFF) per sequence
    emin: np.ndarray            # int32 minimum energy per sequence
    designability: np.ndarray   # uint64 per class
    nondesign: int


# Table 1 of the paper (E_HH = -2.3, E_HP = E_PH = -1, E_PP = 0), scaled by 10,
# as {E_PP, E_PH, E_HP, E_HH}.
HP1996_X10 = (0, -10, -10, -23)
PURE_HP = (0, 0, 0, -1)


def energy_table(s: int, pairs, table) -> int:
    p = np.ascontiguousarray(np.asarray(pairs, dtype=np.uint8).reshape(-1, 2))
    t = np.ascontiguousarray(np.asarray(table, dtype=np.int32))
    return int(lib().or_energy_table(int(s), p.shape[0], _p(p, ctypes.c_uint8),
                                     _p(t, ctypes.c_int32)))


def ground_states(st: Structures, lo: int = 0, hi: int | None = None,
                  table=None) -> GroundStates:
    """Ground states of every sequence in [lo, hi) against all conformations;
    `table` = {E_PP, E_PH, E_HP, E_HH} (integers) or None for pure HP."""
    if hi is None:
        hi = 1 << st.N
    if table is not None:
        n = hi - lo
        out = np.zeros(max(n, 1), dtype=np.uint16)
        emin = np.zeros(max(n, 1), dtype=np.int32)
        desig = np.zeros(max(st.n_class, 1), dtype=np.uint64)
        nond = np.zeros(1, dtype=np.uint64)
        t = np.ascontiguousarray(np.asarray(table, dtype=np.int32))
        lib().or_ground_states_table(st.n_conf, _p(st.ct_off, ctypes.c_int32),
                                     _p(st.pairs, ctypes.c_uint8),
                                     _p(st.conf_to_class, ctypes.c_int32), _p(t, ctypes.c_int32),
                                     lo, hi, _p(out, ctypes.c_uint16), _p(emin, ctypes.c_int32),
                                     _p(desig, ctypes.c_uint64), _p(nond, ctypes.c_uint64))
        return GroundStates(out[:n], emin[:n], desig[:st.n_class], int(nond[0]))
    n = hi - lo
    out = np.zeros(max(n, 1), dtype=np.uint16)
    emin = np.zeros(max(n, 1), dtype=np.int32)
    desig = np.zeros(max(st.n_class, 1), dtype=np.uint64)
    nond = np.zeros(1, dtype=np.uint64)
    lib().or_ground_states(st.n_conf, _p(st.ct_off, ctypes.c_int32), _p(st.pairs, ctypes.c_uint8),
                           _p(st.conf_to_class, ctypes.c_int32), lo, hi, _p(out, ctypes.c_uint16),
                           _p(emin, ctypes.c_int32), _p(desig, ctypes.c_uint64),
                           _p(nond, ctypes.c_uint64))
    return GroundStates(out[:n], emin[:n], desig[:st.n_class], int(nond[0]))


@dataclass
class GapStates:
    out: np.ndarray             # uint16 phenotype per listed sequence
    emin: np.ndarray            # int32 lowest energy
    gap: np.ndarray             # uint8 second-lowest minus lowest energy, saturated at 255
    designability: np.ndarray   # uint64 per class
    nondesign: int


def ground_states_gap(st: Structures, seqs, threshold: int = 1, table=None) -> GapStates:
    """Lowest energy, energy gap and thresholded phenotype of each sequence
    in `seqs` (any order, repeats allowed); `table` as in ground_states."""
    q = np.ascontiguousarray(np.asarray(seqs, dtype=np.uint64).reshape(-1))
    n = q.shape[0]
    out = np.zeros(max(n, 1), dtype=np.uint16)
    emin = np.zeros(max(n, 1), dtype=np.int32)
    gap = np.zeros(max(n, 1), dtype=np.uint8)
    desig = np.zeros(max(st.n_class, 1), dtype=np.uint64)
    nond = np.zeros(1, dtype=np.uint64)
    t = np.ascontiguousarray(np.asarray(PURE_HP if table is None else table, dtype=np.int32))
    if n:
        lib().or_ground_states_gap(st.n_conf, _p(st.ct_off, ctypes.c_int32),
                                   _p(st.pairs, ctypes.c_uint8),
                                   _p(st.conf_to_class, ctypes.c_int32), _p(t, ctypes.c_int32),
                                   _p(q, ctypes.c_uint64), n, int(threshold),
                                   _p(out, ctypes.c_uint16), _p(emin, ctypes.c_int32),
                                   _p(gap, ctypes.c_uint8), _p(desig, ctypes.c_uint64),
                                   _p(nond, ctypes.c_uint64))
    return GapStates(out[:n], emin[:n], gap[:n], desig[:st.n_class], int(nond[0]))


def splitmix64(seed: int, i: int) -> int:
    """Draw i (0-based) of the splitmix64 stream seeded with `seed`."""
    return int(lib().or_splitmix64(seed & (2**64 - 1), i))


def sample_sequences(seed: int, lo: int, hi: int, N: int) -> np.ndarray:
    """Random sequences lo .. hi-1 of the sampling mode (uint64, low N bits)."""
    out = np.zeros(max(hi - lo, 1), dtype=np.uint64)
    if hi > lo:
        lib().or_sample_sequences(seed & (2**64 - 1), lo, hi, N, _p(out, ctypes.c_uint64))
    return out[:hi - lo]


def ground_states_brute(st: Structures, lo: int = 0, hi: int | None = None):
    """Ground states over all directed walks, no reduction (tiny boxes only)."""
    if hi is None:
        hi = 1 << st.N
    n = hi - lo
    out = np.zeros(max(n, 1), dtype=np.uint16)
    emin = np.zeros(max(n, 1), dtype=np.int32)
    X, Y, Z = st.dims
    lib().or_ground_states_brute(X, Y, Z, _p(st.class_keys, ctypes.c_uint8), st.n_class, lo, hi,
                                 _p(out, ctypes.c_uint16), _p(emin, ctypes.c_int32))
    return out[:n], emin[:n]


@dataclass
class Neighbors:
    neutral: np.ndarray
    deleterious: np.ndarray
    other: np.ndarray
    phi_row: np.ndarray | None


def neighbors(N: int, phen: np.ndarray, n_class: int, phi_q: int = -1) -> Neighbors:
    m = np.ascontiguousarray(phen, dtype=np.uint16)
    assert m.shape[0] == 1 << N
    neu = np.zeros(max(n_class, 1), dtype=np.uint64)
    dele = np.zeros_like(neu)
    oth = np.zeros_like(neu)
    row = np.zeros(n_class + 1, dtype=np.uint64)
    lib().or_neighbors(N, _p(m, ctypes.c_uint16), n_class, _p(neu, ctypes.c_uint64),
                       _p(dele, ctypes.c_uint64), _p(oth, ctypes.c_uint64), phi_q,
                       _p(row, ctypes.c_uint64))
    return Neighbors(neu[:n_class], dele[:n_class], oth[:n_class], row if phi_q >= 0 else None)


def phi_counts(N: int, phen: np.ndarray, n_class: int) -> np.ndarray:
    """Numerators of phi_pq (Eq. 2) for every class pair: a uint64 matrix of
    n_class rows (phenotype q of the genotype) and n_class + 1 columns
    (phenotype p of the single-point mutant; column n_class = deleterious).
    phi_pq = counts[q, p] / (N * N_q)."""
    m = np.ascontiguousarray(phen, dtype=np.uint16)
    assert m.shape[0] == 1 << N
    c = np.zeros((max(n_class, 1), n_class + 1), dtype=np.uint64)
    lib().or_phi_counts(N, _p(m, ctypes.c_uint16), n_class, _p(c, ctypes.c_uint64))
    return c[:n_class]


def components(N: int, phen: np.ndarray) -> np.ndarray:
    """Min-index component labels (uint32; 0xFFFFFFFF for deleterious)."""
    m = np.ascontiguousarray(phen, dtype=np.uint16)
    assert m.shape[0] == 1 << N and N <= 31
    lab = np.zeros(1 << N, dtype=np.uint32)
    lib().or_components(N, _p(m, ctypes.c_uint16), _p(lab, ctypes.c_uint32))
    return lab
