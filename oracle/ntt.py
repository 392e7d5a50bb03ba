"""Negacyclic number-theoretic transform over Z_q (Section 2.3).

* ``ntt_definition`` / ``intt_definition``: Eq. (negacyclic_ntt) and
  Eq. (negacyclic_intt) evaluated term by term, O(N^2).
* ``ntt_fast`` / ``intt_fast``: the same maps by the textbook radix-2 recursion of a
  cyclic DFT: since psi^((2i+1)j) = psi^j * omega^(ij) with omega = psi^2, the
  negacyclic transform of a is the cyclic DFT (root omega) of the twisted vector
  a_j psi^j (the twist of Section 5.1); the inverse is
  N^-1 psi^-i * (cyclic DFT with root omega^-1).  The cyclic DFT splits even and odd
  indices: F_i = E_(i mod N/2) + w^i O_(i mod N/2).  Uses numpy int64; every
  product is of two values below 2^31, so below 2^62, and exact.
* ``is_prime`` / ``root_of_unity``: helpers to pick an NTT-friendly (q, psi)
  pair for the checks, q = 1 (mod 2N) as the section requires.
"""
from __future__ import annotations

import numpy as np


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 3.3e24 (fixed witness set)."""
    if n < 2:
        return False
    small = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41)
    for p in small:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def root_of_unity(q: int, order: int) -> int:
    """Smallest g in Z_q^* whose power (q-1)/order has exact multiplicative order ``order``
    (order a power of two); returns that power, a primitive order-th root of unity."""
    if (q - 1) % order:
        raise ValueError("order does not divide q-1")
    for g in range(2, q):
        r = pow(g, (q - 1) // order, q)
        if pow(r, order // 2, q) == q - 1:
            return r
    raise ValueError("no root found")


def ntt_definition(a, q: int, psi: int) -> list[int]:
    """Eq. (negacyclic_ntt): abar_i = sum_j a_j psi^((2i+1) j) mod q."""
    N = len(a)
    pw = [pow(psi, e, q) for e in range(2 * N)]       # psi has order 2N
    return [sum(int(a[j]) * pw[((2 * i + 1) * j) % (2 * N)] for j in range(N)) % q
            for i in range(N)]


def intt_definition(abar, q: int, psi: int) -> list[int]:
    """Eq. (negacyclic_intt): a_i = N^-1 psi^-i sum_j abar_j omega^(-ij) mod q, omega = psi^2."""
    N = len(abar)
    omega = psi * psi % q
    winv = pow(omega, -1, q)
    wp = [pow(winv, e, q) for e in range(N)]           # omega has order N
    ninv = pow(N, -1, q)
    psinv = pow(psi, -1, q)
    out = []
    for i in range(N):
        s = sum(int(abar[j]) * wp[(i * j) % N] for j in range(N)) % q
        out.append(ninv * pow(psinv, i, q) * s % q)
    return out


def _cyclic_dft(x: np.ndarray, w: int, q: int) -> np.ndarray:
    """F_i = sum_j x_j w^(ij) mod q for a power-of-two length, by even/odd recursion."""
    n = x.shape[0]
    if n == 1:
        return x.copy()
    w2 = w * w % q
    E = _cyclic_dft(x[0::2], w2, q)
    O = _cyclic_dft(x[1::2], w2, q)
    half = n // 2
    wi = np.array([pow(w, i, q) for i in range(n)], dtype=np.int64) if n <= 64 else _powers(w, n, q)
    idx = np.arange(n) % half
    return (E[idx] + (wi * O[idx]) % q) % q


def _powers(w: int, n: int, q: int) -> np.ndarray:
    """[w^0, w^1, ..., w^(n-1)] mod q."""
    out = np.empty(n, dtype=np.int64)
    x = 1
    for i in range(n):
        out[i] = x
        x = x * w % q
    return out


def ntt_fast(a, q: int, psi: int) -> list[int]:
    """Eq. (negacyclic_ntt) via twist by psi^j and a cyclic DFT with root omega = psi^2."""
    if q >= 1 << 31:
        raise ValueError("int64 recursion needs q < 2^31")
    N = len(a)
    x = (np.asarray([int(v) % q for v in a], dtype=np.int64) * _powers(psi, N, q)) % q
    return [int(v) for v in _cyclic_dft(x, psi * psi % q, q)]


def intt_fast(abar, q: int, psi: int) -> list[int]:
    """Eq. (negacyclic_intt) via a cyclic DFT with root omega^-1, then N^-1 psi^-i."""
    if q >= 1 << 31:
        raise ValueError("int64 recursion needs q < 2^31")
    N = len(abar)
    x = np.asarray([int(v) % q for v in abar], dtype=np.int64)
    y = _cyclic_dft(x, pow(psi * psi % q, -1, q), q)
    scale = (_powers(pow(psi, -1, q), N, q) * pow(N, -1, q)) % q
    return [int(v) for v in (y * scale) % q]
