"""Philox4x64-10 counter-based generator, written from its published definition.

Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3"
(SC'11), Section 4 (the Philox family): a 4x64-bit counter and a 2x64-bit key
go through 10 rounds.  Each round multiplies words 0 and 2 by two fixed odd
constants, exchanges the 128-bit products' halves with the other words XORed
with the round key, and the key is bumped by the two Weyl constants between
rounds.  Python integers keep every step exact.

Test infrastructure only (see ``oracle/__init__.py``).
"""
from __future__ import annotations

from typing import Sequence, Tuple

MASK64 = (1 << 64) - 1
# Multipliers and Weyl key increments of Philox4x64 (Salmon et al., Table 2).
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15  # golden ratio
PHILOX_W1 = 0xBB67AE8584CAA73B  # sqrt(3) - 1


def philox4x64_10(counter: Sequence[int], key: Sequence[int]) -> Tuple[int, int, int, int]:
    """One Philox4x64-10 block: counter (4 words), key (2 words) -> 4 words."""
    x0, x1, x2, x3 = (int(c) & MASK64 for c in counter)
    k0, k1 = (int(k) & MASK64 for k in key)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
        p0 = PHILOX_M0 * x0
        p1 = PHILOX_M1 * x2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return x0, x1, x2, x3


def mulhi64(a: int, n: int) -> int:
    """floor(a * n / 2^64): maps a uniform 64-bit word onto [0, n)."""
    return (int(a) * int(n)) >> 64
