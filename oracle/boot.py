"""CKKS bootstrapping (test infrastructure).

Section 6.2 lists ``bootstrap`` (HEAAN's EvalBootstrap) with its keys: rotation keys and
auxiliary polynomials that the bootstrapping circuit needs beside the ciphertext
(Sections 6.1 and 6.2).  Section 7.2 takes the HEAAN setting, whose logT controls the
precision of the circuit.  The paper prints no algorithm; the steps below are the
published bootstrapping for approximate homomorphic encryption (modulus raise,
coefficients to slots, a scaled sine standing in for the reduction modulo q, slots to
coefficients), written with this package's operations (``scheme``, ``ops``,
``galois``) and readings.  n = 2^logslots slots, gap = N / (2n), q0 = 2^logq_in:

B1 ModRaise: the ciphertext at 2^logq_in is read at 2^logQ (the same limbs): its phase
   becomes t = m + e + q0 I, I a small integer polynomial.  Its scale is set to
   2^(logq_in + log2 gap), so that the values below come out as t / q0.
B2 SubSum: add the rotations by 2^i slots, logslots <= i < logN - 1 (the automorphisms
   that fix X^gap): the phase keeps gap times its coefficients at multiples of gap.
B3 CoeffToSlot: with V_jk = zeta^(r_j k) (zeta = exp(2 pi i / 4n), r_j = 5^j mod 4n,
   j, k < n), the slots hold V w / scale where w_k = u_k + i u_(k+n) and u_k is
   coefficient k gap of the phase (zeta^(n r_j) = i).  The slots times V^-1 -- the sum
   over d of rotation by d times the encoded d-th diagonal of V^-1, then a rescale by
   logc -- leave w_k / (q0 gap) = (t_(k gap) + i t_((k+n) gap)) / q0 in slot k.
B4 Split: a = (x + conj x) / 2 and b = i (conj x - x) / 2, each with real slots
   I + m / q0; the halving is a change of scale (logp + 1), the scale being a power
   of two.
B5 EvalMod, on a and b each: y = x 2 pi / 2^logT (a product with the integer
   round(2 pi 2^logc), rescale by logc + logT: the division by 2^logT is part of the
   rescale, so the constant keeps logc bits); E = sum_(k <= degree) (i y)^k / k!
   (real part and imaginary part as two real polynomials in y whose powers come from
   a product tree, each product rescaled by the working scale; coefficients as
   integers round(c 2^logc), rescale by logc; i through imult); then logT squarings,
   E ~ exp(2 pi i x); sin(2 pi x) = i (conj E - E) / 2 ~ 2 pi m / q0 since I is an integer.
B6 Combine: w' = sin(2 pi a) + i sin(2 pi b).
B7 SlotToCoeff: the slots times V / (2 pi) (encoded diagonals, rescale by logc); the
   result decodes to V (m_(k gap) + i m_((k+n) gap)) / q0, which is the input message's
   decoding at scale 2^logp_msg once the scale is lowered by logq_in - logp_msg bits
   (a change of scale only).  The output is at logp = log2 gap + logp_msg.

The encoded diagonals and the integer constants are auxiliary inputs (``boot_aux``),
computed once in double precision and handed to every implementation, so that the
bits of the output depend only on them, the keys and the ciphertext.
Levels: every product and rescale is exact integer arithmetic as in ``scheme``; two
operands of an addition or a product are first brought to the lower one's logq by
moddownBy.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import galois, ops, scheme
from .scheme import CKKS, Ciphertext


@dataclass
class BootParams:
    logN: int
    logslots: int     # n = 2^logslots slots, n < N/2
    logq_in: int      # modulus of the input ciphertext (q0 = 2^logq_in)
    logQ: int         # raised modulus
    logc: int = 40    # scale of the encoded diagonals and constants
    logT: int = 8     # squarings (double angles) after the Taylor step
    degree: int = 11  # Taylor degree of exp(i y)

    @property
    def loggap(self) -> int:
        return self.logN - 1 - self.logslots


@dataclass
class BootAux:
    """Auxiliary inputs: encoded diagonals (signed integer polynomials) and constants."""
    c2s: list = field(default_factory=list)    # n polynomials: diagonals of V^-1 at 2^logc
    s2c: list = field(default_factory=list)    # n polynomials: diagonals of V / (2 pi) at 2^logc
    k_y: int = 0                               # round(2 pi 2^logc)
    taylor: list = field(default_factory=list)  # [k] = round(c_k 2^logc), c_k of the real/imag parts


def slot_matrix(n: int) -> np.ndarray:
    """V_jk = zeta^(r_j k), zeta = exp(2 pi i / 4n), r_j = 5^j mod 4n (B3)."""
    r = [pow(5, j, 4 * n) for j in range(n)]
    return np.array([[np.exp(2j * np.pi * ((rj * k) % (4 * n)) / (4 * n)) for k in range(n)] for rj in r])


def diagonals(A: np.ndarray) -> list:
    """diag_d[j] = A[j][(j + d) mod n]: (A z)_j = sum_d diag_d[j] z_(j+d)."""
    n = A.shape[0]
    return [np.array([A[j][(j + d) % n] for j in range(n)]) for d in range(n)]


def taylor_coefficients(degree: int) -> list:
    """c_k with exp(i y) = sum_k (i y)^k / k!: the real coefficient of y^k in the real
    part (even k: (-1)^(k/2) / k!) or in the imaginary part (odd k: (-1)^((k-1)/2) / k!)."""
    out = []
    for k in range(degree + 1):
        sign = (-1) ** (k // 2)
        out.append(sign / math.factorial(k))
    return out


def boot_aux(P: BootParams) -> BootAux:
    """The auxiliary inputs of ``bootstrap`` for parameters P."""
    N, n = 1 << P.logN, 1 << P.logslots
    V = slot_matrix(n)
    A = np.linalg.inv(V)
    B = V / (2 * np.pi)
    aux = BootAux()
    aux.c2s = [scheme.ckks_encode(d, N, P.logc) for d in diagonals(A)]
    aux.s2c = [scheme.ckks_encode(d, N, P.logc) for d in diagonals(B)]
    aux.k_y = int(round(2 * np.pi * 2.0 ** P.logc))
    aux.taylor = [int(round(c * 2.0 ** P.logc)) for c in taylor_coefficients(P.degree)]
    return aux


def rotation_amounts(P: BootParams) -> list:
    """Left rotations the circuit uses (B2 and the diagonal sums of B3 and B7)."""
    n = 1 << P.logslots
    return sorted(set(range(1, n)) | {1 << i for i in range(P.logslots, P.logN - 1)})


@dataclass
class BootKeys:
    relin: scheme.EvalKey
    rot: dict            # rotation amount -> galois.GaloisKey
    conj: galois.GaloisKey


def _level(x: Ciphertext, logq: int) -> Ciphertext:
    return x if x.logq == logq else ops.moddown(x, x.logq - logq)


def _match(x: Ciphertext, y: Ciphertext):
    q = min(x.logq, y.logq)
    return _level(x, q), _level(y, q)


def _with(x: Ciphertext, **kw) -> Ciphertext:
    d = dict(c0=x.c0, c1=x.c1, logN=x.logN, logq=x.logq, logp=x.logp, scheme=x.scheme, t=x.t, gamma=x.gamma)
    d.update(kw)
    return Ciphertext(**d)


def _add(x, y):
    x, y = _match(x, y)
    return ops.add(x, y)


def _sub(x, y):
    x, y = _match(x, y)
    return ops.sub(x, y)


def _mul(x, y, K: BootKeys, mapper=map):
    """HE-mult at the lower level, then rescale by the working scale (logp of x)."""
    x, y = _match(x, y)
    return scheme.mult_rescale(x, y, K.relin, x.logp, mapper)


def _plain(m, logq: int):
    Q = 1 << logq
    return [int(v) % Q for v in m]


def _linear(x: Ciphertext, diags: list, P: BootParams, K: BootKeys, mapper=map) -> Ciphertext:
    """sum_d rotation_d(x) * diag_d, then rescale by logc (B3, B7)."""
    acc = None
    for d, m in enumerate(diags):
        r = x if d == 0 else galois.leftrotate(x, d, K.rot[d])
        term = ops.multconstvec(r, _plain(m, r.logq), P.logc)
        acc = term if acc is None else ops.add(acc, term)
    return scheme.rescale(acc, P.logc)


def _const(x: Ciphertext, k: int, P: BootParams, extra: int = 0) -> Ciphertext:
    """x times the real constant k / 2^(logc + extra), at x's scale (the product's
    scale 2^(logp + logc) rescaled by logc + extra bits, and logp restored)."""
    y = scheme.rescale(ops.multconst(x, k, P.logc), P.logc + extra)
    return _with(y, logp=x.logp)


def _imag_part_times_2i(E: Ciphertext, K: BootKeys) -> Ciphertext:
    """i (conj E - E) / 2 = Im(E) per slot (the halving as logp + 1)."""
    s = ops.imult(ops.sub(galois.conjugate(E, K.conj), E))
    return _with(s, logp=s.logp + 1)


def eval_mod(x: Ciphertext, P: BootParams, aux: BootAux, K: BootKeys, mapper=map) -> Ciphertext:
    """B5: slots x (real) -> sin(2 pi x)."""
    y = _const(x, aux.k_y, P, P.logT)
    pw = {1: y}
    for k in range(2, P.degree + 1):
        h = 1 << (k.bit_length() - 1)       # largest power of two <= k
        pw[k] = _mul(pw[h], pw[k - h], K, mapper) if h != k else _mul(pw[k // 2], pw[k // 2], K, mapper)
    re, im = None, None
    for k in range(1, P.degree + 1):
        term = _const(pw[k], aux.taylor[k], P)
        if k % 2 == 0:
            re = term if re is None else _add(re, term)
        else:
            im = term if im is None else _add(im, term)
    re, im = _match(re, im)
    one = [0] * len(re.c0)
    one[0] = 1 << re.logp                     # the constant 1 at re's scale
    re = ops.addconst(re, _plain(one, re.logq))
    E = ops.add(re, ops.imult(im))
    for _ in range(P.logT):
        E = _mul(E, E, K, mapper)
    return _imag_part_times_2i(E, K)


def bootstrap(ct: Ciphertext, P: BootParams, aux: BootAux, K: BootKeys, mapper=map) -> Ciphertext:
    """B1-B7: a CKKS ciphertext at logq_in refreshed to a higher level."""
    if ct.scheme != CKKS or ct.logq != P.logq_in or ct.logN != P.logN:
        raise ValueError("bootstrap takes a CKKS ciphertext at logq_in")
    logp_msg = ct.logp
    # B1
    x = _with(ct, logq=P.logQ, logp=P.logq_in + P.loggap)
    # B2
    for i in range(P.logslots, P.logN - 1):
        x = ops.add(x, galois.leftrotate(x, 1 << i, K.rot[1 << i]))
    # B3
    x = _linear(x, aux.c2s, P, K, mapper)
    # B4
    xc = galois.conjugate(x, K.conj)
    a = ops.add(x, xc)
    a = _with(a, logp=a.logp + 1)
    b = ops.imult(ops.sub(xc, x))
    b = _with(b, logp=b.logp + 1)
    # B5, B6
    sa = eval_mod(a, P, aux, K, mapper)
    sb = eval_mod(b, P, aux, K, mapper)
    w = ops.add(sa, ops.imult(sb))
    # B7
    z = _linear(w, aux.s2c, P, K, mapper)
    return _with(z, logp=z.logp - (P.logq_in - logp_msg))
