"""Seeded synthetic inputs for the non-RNS CKKS/BGV homomorphic multiplication.

This module only draws random numbers and lays them out in the container formats
the rest of the code consumes.  It performs none of the scheme's arithmetic (no
ring products, reductions, encodings or roundings), so that the CPU oracle and
the GPU library can both take their inputs from it without sharing any part of
the computation under test.

Every generator takes an explicit ``numpy.random.Generator``.  ``streams(c)``
derives the four independent generators used for workload ``c``:
``[keys, messages, encryption noise, schedule]`` from ``SeedSequence(1000*c)``.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "streams", "uniform_limbs", "hwt", "zo", "dg", "unit_disk", "uniform_mod",
    "nlimbs",
]


def streams(c: int):
    """Four independent generators [keys, messages, noise, schedule] for workload c."""
    return [np.random.default_rng(s) for s in np.random.SeedSequence(1000 * c).spawn(4)]


def nlimbs(bits: int) -> int:
    """Number of 32-bit words that hold a ``bits``-bit unsigned value."""
    return (bits + 31) // 32


def uniform_limbs(rng: np.random.Generator, bits: int, n: int, count: int | None = None) -> np.ndarray:
    """Uniform values in [0, 2**bits), laid out limb-major as uint32[(count,) L, n].

    Limb 0 holds the least significant 32 bits; bits at positions >= ``bits`` are zero.
    """
    L = nlimbs(bits)
    shape = (L, n) if count is None else (count, L, n)
    out = rng.integers(0, 1 << 32, size=shape, dtype=np.uint64).astype(np.uint32)
    top = bits - 32 * (L - 1)
    if top < 32:
        out[..., L - 1, :] &= np.uint32((1 << top) - 1)
    return out


def hwt(rng: np.random.Generator, n: int, h: int) -> np.ndarray:
    """Ternary vector with exactly ``h`` nonzero entries, each +1 or -1 with probability 1/2."""
    out = np.zeros(n, dtype=np.int64)
    pos = rng.choice(n, size=h, replace=False)
    out[pos] = np.where(rng.integers(0, 2, size=h) == 0, 1, -1)
    return out


def zo(rng: np.random.Generator, n: int) -> np.ndarray:
    """Ternary vector: 0 with probability 1/2, +1 and -1 with probability 1/4 each."""
    u = rng.integers(0, 4, size=n)
    return np.select([u == 0, u == 1], [1, -1], 0).astype(np.int64)


def dg(rng: np.random.Generator, n: int, sigma: float) -> np.ndarray:
    """Rounded Gaussian: nearest integer to N(0, sigma^2), no tail cut."""
    return np.rint(rng.normal(0.0, sigma, size=n)).astype(np.int64)


def unit_disk(rng: np.random.Generator, n: int) -> np.ndarray:
    """Complex values uniform in the closed unit disk (radius sqrt(U), angle 2*pi*U')."""
    r = np.sqrt(rng.random(n))
    th = 2.0 * np.pi * rng.random(n)
    return r * np.exp(1j * th)


def uniform_mod(rng: np.random.Generator, n: int, t: int) -> np.ndarray:
    """Integers uniform in [0, t)."""
    return rng.integers(0, t, size=n, dtype=np.int64)
