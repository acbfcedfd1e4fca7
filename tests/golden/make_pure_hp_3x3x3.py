"""Write the oracle's full pure-HP 3x3x3 map as a golden fixture.

Calls only the CPU oracle (``oracle/``) and numpy; nothing here touches the
GPU path.  The result, ``pure_hp_3x3x3_map.txt`` beside this script, pins the
GPU forms' full 3x3x3 map (all 2^27 sequences against all 103346
conformations, pure HP contact energy, Methods: Eq. 1 and the ground-state
rule) sequence by sequence.

Only the reversal-canonical sequences (s <= rev(s), rev = reading the chain
from its other end) are scored.  The rest of the map follows exactly:
E(rev s, c) = E(s, R c) for the reversed conformation R c, and R maps the
conformations onto themselves and keeps each class, so phenotype(rev s) =
phenotype(s) (Appendix B: the map is symmetric under chain reversal).  The
oracle's own tests pin that identity on every small box.

The canonical sequences, in ascending order, are cut into chunks of 2^20.
Each chunk is scored by ``oracle.ground_states_gap`` (threshold 1 is the
plain uniqueness rule) and checkpointed, so the run can be stopped and
resumed; chunks are taken in bit-reversed order so that a partial run covers
the whole sequence space.  The fixture lists, per finished chunk, the SHA-256
of its phenotypes (uint16 little-endian, canonical order) and its weighted
designing count; once every chunk is done it adds the hash of the whole
2^27 map and of the designability histogram.

Usage:  python tests/golden/make_pure_hp_3x3x3.py --ckpt DIR [--threads T]
        [--max-chunks K]   (K chunks this call; the fixture is rewritten
        after every chunk)
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402

N = 27
CHUNK = 1 << 20
FIXTURE = os.path.join(HERE, "pure_hp_3x3x3_map.txt")
NONE = 0xFFFF


def reverse_bits(s: np.ndarray, n: int) -> np.ndarray:
    """rev(s): bit i of the result is bit n-1-i of s (uint64 array)."""
    s = s.astype(np.uint64)
    r = np.zeros_like(s)
    for i in range(n):
        r |= ((s >> np.uint64(i)) & np.uint64(1)) << np.uint64(n - 1 - i)
    return r


def canonical_sequences(n: int = N) -> np.ndarray:
    """All s in [0, 2^n) with s <= rev(s), ascending (uint64)."""
    parts = []
    step = 1 << 24
    for lo in range(0, 1 << n, step):
        s = np.arange(lo, min(lo + step, 1 << n), dtype=np.uint64)
        parts.append(s[s <= reverse_bits(s, n)])
    return np.concatenate(parts)


def chunk_order(n_chunks: int) -> list:
    bits = max(1, (n_chunks - 1).bit_length())
    rev = lambda c: int(format(c, "0%db" % bits)[::-1], 2)  # noqa: E731
    return sorted(range(n_chunks), key=rev)


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).astype(a.dtype.newbyteorder("<")).tobytes()).hexdigest()


def write_fixture(canon, ckpt, n_chunks, n_class):
    done = {}
    for c in range(n_chunks):
        p = os.path.join(ckpt, "chunk_%03d.npy" % c)
        if os.path.exists(p):
            done[c] = np.load(p)
    lines = [
        "# Full pure-HP 3x3x3 map from the CPU oracle (tests/golden/make_pure_hp_3x3x3.py).",
        "# E = -(number of H-H contacts), all 103346 conformations, uniqueness rule",
        "# (Methods: Eq. 1 and the ground-state rule; Appendix B for the reversal symmetry).",
        "# Reversal-canonical sequences (s <= rev s) ascending, in chunks of %d." % CHUNK,
        "# chunk <c> <first canonical index> <count> <sha256 of uint16 LE phenotypes> "
        "<designing sequences counted with their reverses>",
        "n_canonical %d" % canon.size,
        "n_chunks %d" % n_chunks,
    ]
    for c in sorted(done):
        lo = c * CHUNK
        out = done[c]
        s = canon[lo:lo + out.size]
        w = np.where(s == reverse_bits(s, N), 1, 2)
        lines.append("chunk %d %d %d %s %d" % (c, lo, out.size, sha(out),
                                              int(w[out != NONE].sum())))
    if len(done) == n_chunks:
        full = np.empty(1 << N, dtype=np.uint16)
        outc = np.concatenate([done[c] for c in range(n_chunks)])
        full[canon] = outc
        full[reverse_bits(canon, N)] = outc
        desig = np.bincount(full[full != NONE], minlength=n_class).astype(np.uint64)
        nond = int((full == NONE).sum())
        assert int(desig.sum()) + nond == 1 << N
        top = np.argsort(-desig.astype(np.int64), kind="stable")[:10]
        lines += [
            "map_sha256 %s" % sha(full),
            "designability_sha256 %s" % sha(desig),
            "nondesign %d" % nond,
            "designing %d" % int(desig.sum()),
            "designable_classes %d" % int((desig > 0).sum()),
            "top_classes " + " ".join("%d:%d" % (q, int(desig[q])) for q in top),
        ]
    tmp = FIXTURE + ".tmp"
    with open(tmp, "w") as f:
        f.write("\n".join(lines) + "\n")
    os.replace(tmp, FIXTURE)
    return len(done)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--ckpt", required=True)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--max-chunks", type=int, default=1 << 30)
    a = ap.parse_args()
    os.makedirs(a.ckpt, exist_ok=True)
    if a.threads:
        oracle.set_num_threads(a.threads)
    st = oracle.structures(3, 3, 3)
    canon = canonical_sequences()
    n_chunks = (canon.size + CHUNK - 1) // CHUNK
    ran = 0
    for c in chunk_order(n_chunks):
        p = os.path.join(a.ckpt, "chunk_%03d.npy" % c)
        if os.path.exists(p):
            continue
        if ran >= a.max_chunks:
            break
        t0 = time.time()
        seqs = canon[c * CHUNK:(c + 1) * CHUNK]
        g = oracle.ground_states_gap(st, seqs, threshold=1)
        np.save(p + ".tmp.npy", g.out)
        os.replace(p + ".tmp.npy", p)
        ran += 1
        k = write_fixture(canon, a.ckpt, n_chunks, st.n_class)
        print("chunk %d: %d sequences in %.0f s; %d of %d chunks done" %
              (c, seqs.size, time.time() - t0, k, n_chunks), flush=True)
    write_fixture(canon, a.ckpt, n_chunks, st.n_class)


if __name__ == "__main__":
    main()
