"""Galois automorphisms and key switching: slot rotation and conjugation
(test infrastructure).

Section 2.5 permutes slots with the automorphisms kappa_k: x -> x^k; Section 6.2
("Cryptographic Key Management") generates rotation keys for SIMD slot rotations
and conjugation keys for complex conjugation, and its operation list has
``leftrotate`` and ``conjugate`` (Table tab:homomorphic_latency times both).  The
paper gives no formulas; the definitions below are the HEAAN ones it defers to, on
the ring and with the readings (R1-R7) of ``scheme``:

G1  kappa_g(a)(X) = a(X^g) in Z_m[X]/(X^N+1), g odd: coefficient i moves to
    position i g mod 2N, negated when that position is >= N (X^N = -1).
G2  Rotation of the slots by r to the left uses g = 5^r mod 2N: slot j, the value
    at the root zeta^(5^j), then holds what slot j + r held.  Conjugation uses
    g = 2N - 1 (that is, -1): the coefficients are integers, so the value at
    zeta^-r is the complex conjugate of the value at zeta^r.
G3  The switching key for kappa_g is (b', a') over P Q_top,
    b' = [-a' s + e' + P kappa_g(s)]_(P Q_top) (BGV: t e'), made at the top level like
    the relinearization key (R2) and used mod P Q_l.
G4  Key switch of (c0, c1) at level logq: u = kappa_g(c1) in [0, Q_l) (the
    representative choice of R3),
        c0' = [kappa_g(c0) + R(u b')]_(Q_l),   c1' = [R(u a')]_(Q_l),
    R the division by P of R4 (CKKS) / R5 (BGV).  The result decrypts under s to
    kappa_g of the input's phase plus the switching noise; scale and gamma are kept.
"""
from __future__ import annotations

from dataclasses import dataclass

from . import ring
from .scheme import BGV, Ciphertext, _err, divide_round


def automorphism(a, g: int, modulus: int | None = None) -> list[int]:
    """G1: kappa_g(a), optionally reduced mod ``modulus``."""
    N = len(a)
    if g % 2 == 0:
        raise ValueError("g must be odd")
    out = [0] * N
    for i, v in enumerate(a):
        k = (i * g) % (2 * N)
        if k < N:
            out[k] += int(v)
        else:
            out[k - N] -= int(v)
    if modulus is not None:
        out = [x % modulus for x in out]
    return out


def rotation_element(r: int, N: int) -> int:
    """G2: the Galois element of a left rotation by r slots."""
    return pow(5, r, 2 * N)


def conjugation_element(N: int) -> int:
    """G2: the Galois element of complex conjugation."""
    return 2 * N - 1


@dataclass
class GaloisKey:
    """G3: switching key (b', a') for kappa_g, coefficients in [0, 2^(logP + logQ))."""
    b: list
    a: list
    g: int
    logN: int
    logQ: int
    logP: int
    scheme: str = "ckks"
    t: int = 0


def keygen_galois(s, a, e, g: int, logQ: int, logP: int, scheme: str = "ckks", t: int = 0) -> GaloisKey:
    """G3: b' = [-a' s + e' + P kappa_g(s)]_(P Q), a' uniform in [0, P Q)."""
    PQ = 1 << (logP + logQ)
    P = 1 << logP
    N = len(s)
    As = ring.ring_mul(a, s, PQ)
    ks = automorphism(s, g)
    ee = _err(e, scheme, t)
    b = [(-As[i] + ee[i] + P * ks[i]) % PQ for i in range(N)]
    return GaloisKey(b=b, a=[int(x) % PQ for x in a], g=g, logN=N.bit_length() - 1, logQ=logQ, logP=logP,
                     scheme=scheme, t=t)


def key_switch(ct: Ciphertext, key: GaloisKey) -> Ciphertext:
    """G4: kappa_g applied to the ciphertext, switched back to the secret s."""
    if ct.logq > key.logQ:
        raise ValueError("ciphertext level above the key level")
    Q = 1 << ct.logq
    PQ = 1 << (key.logP + ct.logq)
    u = automorphism(ct.c1, key.g, Q)
    v = automorphism(ct.c0, key.g, Q)
    B = [x % PQ for x in key.b]
    A = [x % PQ for x in key.a]
    k0 = ring.ring_mul(u, B, PQ)
    k1 = ring.ring_mul(u, A, PQ)
    c0 = [(v[i] + divide_round(k0[i], key.logP, ct.scheme, ct.t)) % Q for i in range(len(v))]
    c1 = [divide_round(k1[i], key.logP, ct.scheme, ct.t) % Q for i in range(len(v))]
    return Ciphertext(c0=c0, c1=c1, logN=ct.logN, logq=ct.logq, logp=ct.logp, scheme=ct.scheme, t=ct.t,
                      gamma=ct.gamma)


def leftrotate(ct: Ciphertext, r: int, key: GaloisKey) -> Ciphertext:
    """G2 + G4: slots rotated left by r (the key must be the one for 5^r)."""
    if key.g != rotation_element(r, 1 << ct.logN):
        raise ValueError("key is not the rotation key for this amount")
    return key_switch(ct, key)


def conjugate(ct: Ciphertext, key: GaloisKey) -> Ciphertext:
    """G2 + G4: complex conjugation of the slots (the key must be the one for -1)."""
    if key.g != conjugation_element(1 << ct.logN):
        raise ValueError("key is not the conjugation key")
    return key_switch(ct, key)
