"""Comparison of a device-resident full 3x3x3 pure-HP map with the oracle's
fixture ``tests/golden/pure_hp_3x3x3_map.txt`` (written by
``tests/golden/make_pure_hp_3x3x3.py``, which calls only the oracle).

The fixture lists, per finished chunk of 2^20 reversal-canonical sequences
(s <= rev(s), ascending), the SHA-256 of their phenotypes; once complete it
also holds the hash of the whole map.  The canonical list is rebuilt here on
the device with torch (index bookkeeping only).
"""
from __future__ import annotations

import hashlib
import os

import numpy as np

FIXTURE = os.path.join(os.path.dirname(__file__), "golden", "pure_hp_3x3x3_map.txt")
N = 27
CHUNK = 1 << 20


def load():
    """(chunks, whole): chunks maps chunk index -> (first, count, sha256,
    designing); whole holds the full-map fields when every chunk is done."""
    chunks, whole = {}, {}
    if not os.path.exists(FIXTURE):
        return chunks, whole
    for line in open(FIXTURE):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "chunk":
            chunks[int(f[1])] = (int(f[2]), int(f[3]), f[4], int(f[5]))
        else:
            whole[f[0]] = f[1:] if len(f) > 2 else f[1]
    return chunks, whole


def canonical_sequences(device="cuda"):
    """All s in [0, 2^27) with s <= rev(s), ascending, as an int64 tensor."""
    import torch
    s = torch.arange(1 << N, dtype=torch.int64, device=device)
    r = torch.zeros_like(s)
    for i in range(N):
        r |= ((s >> i) & 1) << (N - 1 - i)
    return torch.nonzero(s <= r).flatten()


def _sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).astype(a.dtype.newbyteorder("<")).tobytes()).hexdigest()


def designability_sha(d: np.ndarray) -> str:
    """Hash of a uint64 designability histogram, as the fixture stores it."""
    return _sha(np.asarray(d, dtype=np.uint64))


def compare(out, canon=None):
    """Compare the device map `out` (int16/uint16 view, 2^27 entries) with
    every chunk of the fixture.  Returns (chunks checked, mismatching chunk
    indices, full-map hash result or None when the fixture is partial)."""
    chunks, whole = load()
    if canon is None:
        canon = canonical_sequences(out.device)
    bad = []
    for c, (first, count, sha, _) in sorted(chunks.items()):
        got = out[canon[first:first + count]].cpu().numpy().view(np.uint16)
        if _sha(got) != sha:
            bad.append(c)
    full = None
    if "map_sha256" in whole:
        full = _sha(out.cpu().numpy().view(np.uint16)) == whole["map_sha256"]
    return len(chunks), bad, full
