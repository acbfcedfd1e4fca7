"""Reversal bookkeeping shared by the GPU tests: the sequences of a
canonical block of the blocked form (blocks of 256) or of a canonical wide
block (1024), and bit reversal (index arithmetic only; nothing of the
method's energies)."""
import numpy as np


def reverse_bits(s, n):
    """rev(s): bit i of the result is bit n-1-i of s (uint64 array)."""
    s = np.asarray(s, dtype=np.uint64)
    r = np.zeros_like(s)
    for i in range(n):
        r |= ((s >> np.uint64(i)) & np.uint64(1)) << np.uint64(n - 1 - i)
    return r


def canonical_block_sequences(N, t):
    """The 256 sequences of canonical block t (even N) and whether the block
    is its own reverse, from the block index order stated for
    hp_enumerate_symmetric_blocked: row pairs p of the (a, b') triangle of
    2^h + 1 blocks each, row b' = p (a = 0 .. p) then row b' = 2^h - 1 - p;
    b = reverse_h(b'); the 8 middle monomers h .. h+7 vary."""
    assert N % 2 == 0
    h = (N - 8) // 2
    side = 1 << h
    p, o = divmod(t, side + 1)
    if o <= p:
        bp, a = p, o
    else:
        bp, a = side - 1 - p, o - p - 1
    b = int(reverse_bits(np.array([bp], dtype=np.uint64), h)[0])
    x = np.arange(256, dtype=np.uint64)
    return (np.uint64(a) << np.uint64(h + 8)) | (x << np.uint64(h)) | np.uint64(b), a == bp


def canonical_wide_block_sequences(N, t):
    """The 1024 sequences of canonical wide block t and whether the block is
    its own reverse, from the block index order stated for
    hp_enumerate_symmetric_wide: h = (N - 10 - N % 2) / 2 outer monomers on
    each side (a high, b low, and for odd N the middle monomer m between the
    two groups of 5 varying monomers), index over m, then row pairs p of the
    (a, b') triangle; b = reverse_h(b')."""
    odd = N & 1
    h = (N - 10 - odd) // 2
    side = 1 << h
    span = side + 1
    per_m = (side >> 1) * span if h else 1
    m, r = divmod(t, per_m)
    p = r // span if h else 0
    o = r - p * span
    if o <= p:
        bp, a = p, o
    else:
        bp, a = side - 1 - p, o - p - 1
    b = int(reverse_bits(np.array([bp], dtype=np.uint64), h)[0]) if h else 0
    x = np.arange(1024, dtype=np.uint64)
    outer = (a << (h + 10 + odd)) | (m << (h + 5)) | b
    seqs = np.full(1024, outer, dtype=np.uint64)
    for k in range(10):
        pos = h + k + (odd if k >= 5 else 0)
        seqs |= ((x >> np.uint64(k)) & np.uint64(1)) << np.uint64(pos)
    return seqs, a == bp
