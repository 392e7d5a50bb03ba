"""The HEAAN-style operation set beside multiplication (test infrastructure).

Section 6.2 ("Homomorphic Operation API") lists, over CipherTensors in pairwise or
broadcast mode (Section 6.1): negate, imult, add, sub, multconstvec, addconst,
rescaleBy, moddownBy, multconst; Table tab:homomorphic_latency times each.  The
paper prints no formulas for them; the definitions below are the HEAAN ones the
paper defers to, written on the same ring Z_(2^logq)[X]/(X^N+1) as ``scheme``:

O1  add / sub:      c_i' = [c_i(x) +- c_i(y)]_(Q_l); operands share N, logq, logp
                    (CKKS scale) and, for BGV, t and gamma.
O2  negate:         c_i' = [-c_i]_(Q_l).
O3  imult:          CKKS multiplication of every slot by the imaginary unit: both
                    components times the monomial X^(N/2) in the ring.  Every slot is
                    an evaluation at a root zeta^r with r = 1 mod 4 (powers of 5), so
                    X^(N/2) evaluates to i there.
O4  moddownBy k:    c_i' = [c_i]_(2^(logq-k)); logq -= k; scale and gamma unchanged.
O5  multconst:      c_i' = [k c_i]_(Q_l) for an integer constant k (a real constant c
                    enters as k = round(c 2^logp_k)); logp += logp_k.  Broadcast mode:
                    one constant for every ciphertext of the tensor.
O6  multconstvec:   c_i' = [c_i * m]_(Q_l), a ring product with a plaintext polynomial
                    m (an encoded vector); logp += logp_m.  Pairwise: one m per
                    ciphertext; broadcast: one m for all.
O7  addconst:       c_0' = [c_0 + m]_(Q_l), c_1' = c_1, with m a plaintext polynomial
                    already at the ciphertext's scale (CKKS) or already multiplied by
                    the ciphertext's gamma mod t (BGV).
"""
from __future__ import annotations

from . import ring
from .scheme import BGV, CKKS, Ciphertext


def _like(x: Ciphertext, c0, c1, **kw) -> Ciphertext:
    d = dict(logN=x.logN, logq=x.logq, logp=x.logp, scheme=x.scheme, t=x.t, gamma=x.gamma)
    d.update(kw)
    return Ciphertext(c0=c0, c1=c1, **d)


def _same_params(x: Ciphertext, y: Ciphertext):
    if (x.logN, x.logq, x.logp, x.scheme, x.t, x.gamma) != (y.logN, y.logq, y.logp, y.scheme, y.t, y.gamma):
        raise ValueError("operands must share N, logq, logp, scheme, t and gamma")


def add(x: Ciphertext, y: Ciphertext) -> Ciphertext:
    """O1: [x + y] per component."""
    _same_params(x, y)
    Q = 1 << x.logq
    return _like(x, [(a + b) % Q for a, b in zip(x.c0, y.c0)], [(a + b) % Q for a, b in zip(x.c1, y.c1)])


def sub(x: Ciphertext, y: Ciphertext) -> Ciphertext:
    """O1: [x - y] per component."""
    _same_params(x, y)
    Q = 1 << x.logq
    return _like(x, [(a - b) % Q for a, b in zip(x.c0, y.c0)], [(a - b) % Q for a, b in zip(x.c1, y.c1)])


def negate(x: Ciphertext) -> Ciphertext:
    """O2: [-x] per component."""
    Q = 1 << x.logq
    return _like(x, [(-a) % Q for a in x.c0], [(-a) % Q for a in x.c1])


def monomial(N: int, k: int) -> list[int]:
    """The polynomial X^k for 0 <= k < N."""
    m = [0] * N
    m[k] = 1
    return m


def imult(x: Ciphertext) -> Ciphertext:
    """O3: both components times X^(N/2) in Z_(Q_l)[X]/(X^N+1) (CKKS only)."""
    if x.scheme != CKKS:
        raise ValueError("imult is a CKKS operation")
    Q = 1 << x.logq
    N = 1 << x.logN
    u = monomial(N, N // 2)
    return _like(x, ring.ring_mul(x.c0, u, Q), ring.ring_mul(x.c1, u, Q))


def moddown(x: Ciphertext, k: int) -> Ciphertext:
    """O4: reduce both components mod 2^(logq - k)."""
    if not 0 <= k < x.logq:
        raise ValueError("bad moddown amount")
    Qn = 1 << (x.logq - k)
    return _like(x, [a % Qn for a in x.c0], [a % Qn for a in x.c1], logq=x.logq - k)


def multconst(x: Ciphertext, k: int, logp_k: int = 0) -> Ciphertext:
    """O5: every coefficient times the integer k, mod Q_l; logp += logp_k (CKKS)."""
    Q = 1 << x.logq
    logp = x.logp + logp_k if x.scheme == CKKS else x.logp
    return _like(x, [a * k % Q for a in x.c0], [a * k % Q for a in x.c1], logp=logp)


def multconstvec(x: Ciphertext, m, logp_m: int = 0) -> Ciphertext:
    """O6: both components times the plaintext polynomial m in the ring mod Q_l."""
    Q = 1 << x.logq
    logp = x.logp + logp_m if x.scheme == CKKS else x.logp
    return _like(x, ring.ring_mul(x.c0, m, Q), ring.ring_mul(x.c1, m, Q), logp=logp)


def addconst(x: Ciphertext, m) -> Ciphertext:
    """O7: the plaintext polynomial m added to c0 mod Q_l."""
    Q = 1 << x.logq
    return _like(x, [(a + int(b)) % Q for a, b in zip(x.c0, m)], list(x.c1))
