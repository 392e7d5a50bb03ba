"""Negacyclic polynomial product in Z[X]/(X^N + 1), optionally reduced mod m.

Two implementations of one definition (Section 2.3, Eq. (schoolbook) followed by
Eq. (reduction)):

* ``negacyclic_schoolbook``: the definition written out, O(N^2) big-int products.
* ``negacyclic_kronecker``: the same integer product obtained by Kronecker
  substitution -- pack each polynomial into one huge integer with a decimal slot
  base 10^d larger than any coefficient of the plain product, multiply the two
  integers once with the exact arbitrary-precision multiply of the standard
  ``decimal`` module, unpack the 2N-1 slots and fold with X^N = -1.  It makes no
  blocking or reordering of the sum beyond what the packing implies, and is
  checked against the schoolbook form in the test suite.
"""
from __future__ import annotations

import decimal

_CTX = decimal.Context(prec=decimal.MAX_PREC, Emax=decimal.MAX_EMAX, Emin=decimal.MIN_EMIN)


def negacyclic_schoolbook(a, b, modulus: int | None = None) -> list[int]:
    """c~ = sum_{i,j} a_i b_j X^(i+j) (Eq. schoolbook); c_i = c~_i - c~_(N+i) (Eq. reduction).

    Inputs are integer sequences of equal power-of-two length N.  Returns the N
    integer coefficients, reduced into [0, modulus) when a modulus is given.
    """
    N = len(a)
    if len(b) != N:
        raise ValueError("length mismatch")
    ct = [0] * (2 * N)
    for i in range(N):
        ai = int(a[i])
        if ai == 0:
            continue
        for j in range(N):
            ct[i + j] += ai * int(b[j])
    c = [ct[i] - ct[N + i] for i in range(N)]
    if modulus is not None:
        c = [x % modulus for x in c]
    return c


def _plain_product_nonneg(a: list[int], b: list[int]) -> list[int]:
    """Coefficients of the ordinary (non-reduced) product of two polynomials with
    non-negative integer coefficients, computed by Kronecker substitution."""
    N = len(a)
    amax, bmax = max(a), max(b)
    if amax == 0 or bmax == 0:
        return [0] * (2 * N)
    d = len(str(N * amax * bmax)) + 1          # decimal digits per slot
    A = decimal.Decimal("".join(str(x).zfill(d) for x in reversed(a)))
    B = decimal.Decimal("".join(str(x).zfill(d) for x in reversed(b)))
    C = _CTX.multiply(A, B)
    s = format(C, "f").zfill((2 * N - 1) * d)
    top = 2 * N - 2                             # slot of X^(2N-2) is the leftmost
    out = [int(s[(top - k) * d:(top - k + 1) * d]) for k in range(2 * N - 1)]
    out.append(0)
    return out


def negacyclic_kronecker(a, b, modulus: int | None = None) -> list[int]:
    """Same result as ``negacyclic_schoolbook``; fast for N up to 2^16.

    Without a modulus the inputs must be non-negative.  With a modulus the
    inputs are first taken to their representatives in [0, modulus), which
    leaves the product mod ``modulus`` unchanged.
    """
    N = len(a)
    if len(b) != N:
        raise ValueError("length mismatch")
    if modulus is not None:
        a = [int(x) % modulus for x in a]
        b = [int(x) % modulus for x in b]
    else:
        a = [int(x) for x in a]
        b = [int(x) for x in b]
        if min(a) < 0 or min(b) < 0:
            raise ValueError("negative inputs need a modulus")
    ct = _plain_product_nonneg(a, b)
    c = [ct[i] - ct[N + i] for i in range(N)]
    if modulus is not None:
        c = [x % modulus for x in c]
    return c


def ring_mul(a, b, modulus: int) -> list[int]:
    """Product in Z_modulus[X]/(X^N+1): schoolbook for N <= 64, else Kronecker."""
    if len(a) <= 64:
        return negacyclic_schoolbook(a, b, modulus)
    return negacyclic_kronecker(a, b, modulus)


def coefficient(a, b, k: int) -> int:
    """One coefficient of the exact negacyclic product (no reduction), O(N):
    c_k = sum_{i<=k} a_i b_(k-i) - sum_{i>k} a_i b_(N+k-i)."""
    N = len(a)
    s = 0
    for i in range(N):
        j = k - i
        if j >= 0:
            s += int(a[i]) * int(b[j])
        else:
            s -= int(a[i]) * int(b[j + N])
    return s
