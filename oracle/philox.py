"""Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC'11), written from its published definition.

Round function on counter (c0, c1, c2, c3) with key (k0, k1):
    (hi0, lo0) = mulhilo32(0xD2511F53, c0)
    (hi1, lo1) = mulhilo32(0xCD9E8D57, c2)
    c' = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)
and the key is bumped by the Weyl constants (0x9E3779B9, 0xBB67AE85)
between rounds; ten rounds.

Shot-bit convention (the paper is silent: it used Stim's own generator).
A Clifford fragment variant with 64-bit id ``vid`` draws, for shot ``s`` and
measurement index ``a`` (position in the fragment's measured set), the bit
    bit (a & 31) of word (s & 3) of
    philox(counter = (a >> 5, s >> 2, lo32(vid), hi32(vid)),
           key     = (lo32(seed), hi32(seed))).
The bit is consumed only when measurement ``a`` is random; a random outcome
equals its bit.
"""
from __future__ import annotations

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Return the four 32-bit output words for counter ``ctr`` and key ``key``."""
    c0, c1, c2, c3 = (int(v) & MASK for v in ctr)
    k0, k1 = (int(v) & MASK for v in key)
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 32, p0 & MASK
        hi1, lo1 = p1 >> 32, p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK, lo1, (hi0 ^ c3 ^ k1) & MASK, lo0
    return (c0, c1, c2, c3)


def shot_bit(seed: int, vid: int, shot: int, a: int) -> int:
    """Bit drawn for measurement index ``a`` of shot ``shot`` of variant ``vid``."""
    out = philox4x32_10((a >> 5, shot >> 2, vid & MASK, (vid >> 32) & MASK),
                        (seed & MASK, (seed >> 32) & MASK))
    return (out[shot & 3] >> (a & 31)) & 1


def variant_id(circuit: int, fragment: int, variant: int) -> int:
    """64-bit variant id: circuit in bits 40.., fragment in bits 32..39,
    variant index in bits 0..31."""
    return (circuit << 40) | (fragment << 32) | variant
