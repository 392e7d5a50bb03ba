"""Non-RNS CKKS / BGV homomorphic multiplication, HEAAN-style parameterization.

The paper builds on the original (non-RNS) CKKS of HEAAN: a ciphertext carries
logp (scale), logq (modulus size) and logs (slots) (Section 6), the modulus chain
is a bit count that ``rescaleBy`` lowers by any number of bits (Section 3.2 and
the operation list of Section 6.2), and multiplication is followed by
relinearization with an evaluation key (Section 6.2, key management).  The paper
prints no equations for these operations; this module writes out the readings
below, which are the definitions every other implementation is checked against.

R1  Q_l = 2^logq; "mod Q_l" keeps the low logq bits.  P = 2^logP.
R2  One evaluation key per (scheme, N) at the top modulus: (b', a') over P*Q_top,
    b' = [-a' s + e' + P s^2]_(P Q_top).  A level-l ciphertext uses it mod P*Q_l.
R3  Relinearization multiplies the representative of d2 in [0, Q_l).
R4  CKKS divisions by 2^k round half up on the representative in [0, m):
    floor((x + 2^(k-1)) / 2^k).
R5  BGV divisions by 2^k are t-corrected:
    floor(x / 2^k) + [[ [x]_(2^k) * (2^-k mod t) ]]_t, with [[.]]_t centered in (-t/2, t/2].
    The message picks up the factor 2^-k mod t, tracked in gamma.
R6  Relinearization rounding, then the addition, then the rescale rounding.
R7  Centered reduction of Section 5.1 ("Signed Representation Handling"):
    x > m/2 maps to x - m, so the centered range is (-m/2, m/2].
R8  Errors and the ternary terms are scaled by t in BGV; gamma = 1 at encryption.
R9  CKKS encoding: canonical embedding with slots ordered by powers of 5, sparse
    packing with gap N/(2n), coefficients rounded half up after scaling by 2^logp.

All randomness (secret, uniform masks, errors, encryption ternaries) is passed in.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import ring

CKKS = "ckks"
BGV = "bgv"


def center(x: int, m: int) -> int:
    """R7: representative of x mod m in (-m/2, m/2]."""
    x %= m
    return x - m if 2 * x > m else x


@dataclass
class Ciphertext:
    """(c0, c1) with coefficients in [0, 2^logq)."""
    c0: list
    c1: list
    logN: int
    logq: int
    logp: int = 0
    scheme: str = CKKS
    t: int = 0
    gamma: int = 1


@dataclass
class EvalKey:
    """Relinearization key (b', a') with coefficients in [0, 2^(logP + logQ))."""
    b: list
    a: list
    logN: int
    logQ: int
    logP: int
    scheme: str = CKKS
    t: int = 0


@dataclass
class PublicKey:
    b: list
    a: list
    logN: int
    logQ: int
    scheme: str = CKKS
    t: int = 0


def _err(e, scheme: str, t: int):
    return [int(x) * (t if scheme == BGV else 1) for x in e]


def keygen_public(s, a, e, logQ: int, scheme: str = CKKS, t: int = 0) -> PublicKey:
    """pk = (b, a), b = [-a s + e]_Q (BGV: t e), a uniform in [0, Q)."""
    Q = 1 << logQ
    N = len(s)
    As = ring.ring_mul(a, s, Q)
    ee = _err(e, scheme, t)
    b = [(-As[i] + ee[i]) % Q for i in range(N)]
    return PublicKey(b=b, a=[int(x) % Q for x in a], logN=N.bit_length() - 1, logQ=logQ,
                     scheme=scheme, t=t)


def keygen_relin(s, a, e, logQ: int, logP: int, scheme: str = CKKS, t: int = 0) -> EvalKey:
    """R2: evk = (b', a'), b' = [-a' s + e' + P s^2]_(P Q) (BGV: t e'), a' uniform in [0, P Q)."""
    PQ = 1 << (logP + logQ)
    P = 1 << logP
    N = len(s)
    s2 = ring.negacyclic_schoolbook(s, s) if N <= 64 else ring.negacyclic_kronecker(s, s, PQ)
    As = ring.ring_mul(a, s, PQ)
    ee = _err(e, scheme, t)
    b = [(-As[i] + ee[i] + P * s2[i]) % PQ for i in range(N)]
    return EvalKey(b=b, a=[int(x) % PQ for x in a], logN=N.bit_length() - 1, logQ=logQ,
                   logP=logP, scheme=scheme, t=t)


# ---------------------------------------------------------------- CKKS encoding (R9)

def _slot_exponents(n: int) -> list[int]:
    """r_j = 5^j mod 4n for j < n."""
    M = 4 * n
    r, out = 1, []
    for _ in range(n):
        out.append(r)
        r = r * 5 % M
    return out


def ckks_encode_direct(z, N: int, logp: int) -> list[int]:
    """u_k = (1/n) Re(sum_j z_j zeta^(-r_j k)), zeta = exp(2 pi i / 4n), k < 2n;
    m_(k gap) = floor(2^logp u_k + 1/2).  O(n^2); for small n."""
    z = np.asarray(z, dtype=np.complex128)
    n = z.shape[0]
    gap = N // (2 * n)
    r = np.asarray(_slot_exponents(n), dtype=np.int64)
    k = np.arange(2 * n, dtype=np.int64)
    E = np.exp(-2j * np.pi * ((np.outer(k, r)) % (4 * n)) / (4 * n))
    u = (E @ z).real / n
    m = [0] * N
    for kk in range(2 * n):
        m[kk * gap] = int(np.floor(u[kk] * 2.0 ** logp + 0.5))
    return m


def ckks_encode(z, N: int, logp: int) -> list[int]:
    """Same map as ``ckks_encode_direct`` through one length-2n FFT: the values at the
    odd powers zeta^(2s+1) are W_s (z_j at r_j, conj(z_j) at 4n - r_j), and
    u_k zeta^k is their inverse DFT with root omega = zeta^2."""
    z = np.asarray(z, dtype=np.complex128)
    n = z.shape[0]
    gap = N // (2 * n)
    W = np.zeros(2 * n, dtype=np.complex128)
    for j, r in enumerate(_slot_exponents(n)):
        W[(r - 1) // 2] = z[j]
        W[(4 * n - r - 1) // 2] = np.conj(z[j])
    x = np.fft.fft(W) / (2 * n)
    k = np.arange(2 * n)
    u = (x * np.exp(-2j * np.pi * k / (4 * n))).real
    m = [0] * N
    scaled = np.floor(u * 2.0 ** logp + 0.5)
    for kk in range(2 * n):
        m[kk * gap] = int(scaled[kk])
    return m


def ckks_decode(mu, n: int, logp: int) -> np.ndarray:
    """z_j = 2^-logp sum_(k<2n) mu_(k gap) zeta^(r_j k) for centered integer mu."""
    N = len(mu)
    gap = N // (2 * n)
    x = np.array([float(mu[k * gap]) for k in range(2 * n)], dtype=np.float64)
    x = x * np.exp(2j * np.pi * np.arange(2 * n) / (4 * n))
    V = np.fft.ifft(x) * (2 * n)
    idx = [(r - 1) // 2 for r in _slot_exponents(n)]
    return V[idx] / 2.0 ** logp


# ---------------------------------------------------------------- encrypt / decrypt

def encrypt(pk: PublicKey, m, v, e0, e1, logq: int, logp: int = 0) -> Ciphertext:
    """c0 = [v b + m + e0]_(Q_l), c1 = [v a + e1]_(Q_l) (BGV: t e0, t e1), pk reduced mod Q_l."""
    Q = 1 << logq
    b = [x % Q for x in pk.b]
    a = [x % Q for x in pk.a]
    vb = ring.ring_mul(v, b, Q)
    va = ring.ring_mul(v, a, Q)
    E0 = _err(e0, pk.scheme, pk.t)
    E1 = _err(e1, pk.scheme, pk.t)
    N = len(b)
    c0 = [(vb[i] + int(m[i]) + E0[i]) % Q for i in range(N)]
    c1 = [(va[i] + E1[i]) % Q for i in range(N)]
    return Ciphertext(c0=c0, c1=c1, logN=pk.logN, logq=logq, logp=logp, scheme=pk.scheme,
                      t=pk.t, gamma=1)


def phase(ct: Ciphertext, s) -> list[int]:
    """[c0 + c1 s]_(Q_l)."""
    Q = 1 << ct.logq
    c1s = ring.ring_mul(ct.c1, [int(x) % Q for x in s], Q)
    return [(ct.c0[i] + c1s[i]) % Q for i in range(len(s))]


def decrypt(ct: Ciphertext, s) -> list[int]:
    """mu = [[ c0 + c1 s ]]_(Q_l) (centered, R7)."""
    Q = 1 << ct.logq
    return [center(x, Q) for x in phase(ct, s)]


def bgv_decode(mu, t: int, gamma: int) -> list[int]:
    """m = gamma^-1 [mu]_t mod t."""
    gi = pow(gamma, -1, t)
    return [(x % t) * gi % t for x in mu]


# ---------------------------------------------------------------- the hot path

def _products(pairs, modulus: int, mapper):
    """ring_mul of each (a, b) pair mod ``modulus``; ``mapper`` is ``map`` or a process
    pool's map (the products are independent; the order of results is kept)."""
    return list(mapper(ring.ring_mul, [p[0] for p in pairs], [p[1] for p in pairs],
                       [modulus] * len(pairs)))


def tensor(x: Ciphertext, y: Ciphertext, mapper=map):
    """d0 = c0 c0', d1 = c0 c1' + c1 c0', d2 = c1 c1', all in Z_(Q_l)[X]/(X^N+1)."""
    if (x.logN, x.logq, x.scheme, x.t) != (y.logN, y.logq, y.scheme, y.t):
        raise ValueError("operands must share N, logq, scheme and t")
    Q = 1 << x.logq
    d0, d2, u, w = _products([(x.c0, y.c0), (x.c1, y.c1), (x.c0, y.c1), (x.c1, y.c0)], Q, mapper)
    d1 = [(u[i] + w[i]) % Q for i in range(len(u))]
    return d0, d1, d2


def divide_round(x: int, k: int, scheme: str, t: int) -> int:
    """The rounding division by 2^k of R4 (CKKS) or R5 (BGV), on x >= 0."""
    if scheme == CKKS:
        return (x + (1 << (k - 1))) >> k if k > 0 else x
    r = x & ((1 << k) - 1)
    return (x >> k) + center(r * pow(1 << k, -1, t), t)


def relinearize(d0, d1, d2, evk: EvalKey, logq: int, scheme: str, t: int, mapper=map):
    """k_i = d2 * evk_i mod P Q_l (R3), c_i' = [d_i + R(k_i)]_(Q_l) with R the division of R4/R5."""
    if logq > evk.logQ:
        raise ValueError("ciphertext level above the key level")
    Q = 1 << logq
    PQ = 1 << (evk.logP + logq)
    B = [x % PQ for x in evk.b]
    A = [x % PQ for x in evk.a]
    k0, k1 = _products([(d2, B), (d2, A)], PQ, mapper)
    c0 = [(d0[i] + divide_round(k0[i], evk.logP, scheme, t)) % Q for i in range(len(d0))]
    c1 = [(d1[i] + divide_round(k1[i], evk.logP, scheme, t)) % Q for i in range(len(d1))]
    return c0, c1


def mult(x: Ciphertext, y: Ciphertext, evk: EvalKey, mapper=map) -> Ciphertext:
    """Tensor product then relinearization; logp adds (CKKS), gamma multiplies (BGV)."""
    d0, d1, d2 = tensor(x, y, mapper)
    c0, c1 = relinearize(d0, d1, d2, evk, x.logq, x.scheme, x.t, mapper)
    gamma = x.gamma * y.gamma % x.t if x.scheme == BGV else 1
    return Ciphertext(c0=c0, c1=c1, logN=x.logN, logq=x.logq, logp=x.logp + y.logp,
                      scheme=x.scheme, t=x.t, gamma=gamma)


def rescale(ct: Ciphertext, k: int) -> Ciphertext:
    """rescaleBy k bits: c'' = [R(c)]_(2^(logq - k)) with R of R4/R5; logq -= k, logp -= k
    (CKKS), gamma *= 2^-k mod t (BGV)."""
    if not 0 <= k < ct.logq:
        raise ValueError("bad rescale amount")
    Qn = 1 << (ct.logq - k)
    c0 = [divide_round(x, k, ct.scheme, ct.t) % Qn for x in ct.c0]
    c1 = [divide_round(x, k, ct.scheme, ct.t) % Qn for x in ct.c1]
    if ct.scheme == BGV:
        gamma = ct.gamma * pow(1 << k, -1, ct.t) % ct.t
        logp = ct.logp
    else:
        gamma, logp = 1, ct.logp - k
    return Ciphertext(c0=c0, c1=c1, logN=ct.logN, logq=ct.logq - k, logp=logp,
                      scheme=ct.scheme, t=ct.t, gamma=gamma)


def mult_rescale(x: Ciphertext, y: Ciphertext, evk: EvalKey, k: int, mapper=map) -> Ciphertext:
    """HE-mult: tensor, relinearize, then rescale by k bits (R6)."""
    return rescale(mult(x, y, evk, mapper), k)


def mult_rescale_sampled(x: Ciphertext, y: Ciphertext, evk: EvalKey, k: int, idx):
    """Coefficients ``idx`` of both output polynomials of ``mult_rescale``.

    Computes d2 in full (relinearization needs all of it) and, for each requested
    index only, d0, d1, k0, k1 by ``ring.coefficient``, so a large-N case costs one
    full product plus O(N) work per sampled index."""
    Q = 1 << x.logq
    PQ = 1 << (evk.logP + x.logq)
    d2 = ring.ring_mul(x.c1, y.c1, Q)
    B = [v % PQ for v in evk.b]
    A = [v % PQ for v in evk.a]
    Qn = 1 << (x.logq - k)
    out0, out1 = [], []
    for i in idx:
        d0 = ring.coefficient(x.c0, y.c0, i) % Q
        d1 = (ring.coefficient(x.c0, y.c1, i) + ring.coefficient(x.c1, y.c0, i)) % Q
        k0 = ring.coefficient(d2, B, i) % PQ
        k1 = ring.coefficient(d2, A, i) % PQ
        c0 = (d0 + divide_round(k0, evk.logP, x.scheme, x.t)) % Q
        c1 = (d1 + divide_round(k1, evk.logP, x.scheme, x.t)) % Q
        if k:
            c0 = divide_round(c0, k, x.scheme, x.t) % Qn
            c1 = divide_round(c1, k, x.scheme, x.t) % Qn
        out0.append(c0)
        out1.append(c1)
    return out0, out1
