"""Limb codec: the radix-2^32 ("limb-based big-integer") representation.

Follows the radix representation of Section 4.1 ("The Radix Representation"):
a = sum_j a_j W^j with W = 2^32, and the storage format of Section 5.1
("Representation Overview"): 32-bit limbs.  A polynomial is stored limb-major,
uint32[L][N]: entry [i][j] is limb i (i = 0 least significant) of coefficient j.
"""
from __future__ import annotations

import numpy as np


def nlimbs(bits: int) -> int:
    """Number of 32-bit limbs of a ``bits``-bit value."""
    return (bits + 31) // 32


def int_to_limbs(x: int, L: int) -> list[int]:
    """Little-endian base-2^32 digits of 0 <= x < 2^(32L)."""
    if x < 0 or x >> (32 * L):
        raise ValueError("value does not fit in the limb count")
    return [(x >> (32 * i)) & 0xFFFFFFFF for i in range(L)]


def limbs_to_int(limbs) -> int:
    """sum_i limbs[i] * 2^(32 i)."""
    return sum(int(w) << (32 * i) for i, w in enumerate(limbs))


def poly_from_limbs(arr: np.ndarray) -> list[int]:
    """uint32[L][N] limb-major array -> list of N non-negative integers."""
    arr = np.ascontiguousarray(arr, dtype=np.uint32)
    L, N = arr.shape
    raw = np.ascontiguousarray(arr.T).astype("<u4").tobytes()
    w = 4 * L
    return [int.from_bytes(raw[j * w:(j + 1) * w], "little") for j in range(N)]


def poly_to_limbs(coeffs, L: int) -> np.ndarray:
    """List of N integers in [0, 2^(32L)) -> uint32[L][N] limb-major array."""
    w = 4 * L
    raw = b"".join(int(c).to_bytes(w, "little") for c in coeffs)
    return np.frombuffer(raw, dtype="<u4").reshape(len(coeffs), L).T.astype(np.uint32).copy()
