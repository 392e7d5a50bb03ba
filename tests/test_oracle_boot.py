"""Pins of the oracle's CKKS bootstrapping (oracle/boot.py): a fresh encryption at the
bottom modulus, bootstrapped, decrypts to the same slots (within the stated bound) at a
higher level; the pieces are pinned on their own: the slot matrix inverts the
encoding's evaluation, the diagonal sum is a matrix-vector product, the Taylor
coefficients are those of exp(i y), and the circuit's sine step removes the integer
part of the coefficients (what the modulus raise adds)."""
import math

import numpy as np
import pytest

import synth
from oracle import boot, galois, scheme
from tests.gpu_helpers import oracle_pool


def test_slot_matrix_is_the_sparse_decoding():
    """Slots of a sparse plaintext u_k X^(k gap) (k < 2n) are V (u_k + i u_(k+n)) (B3)."""
    rng = np.random.default_rng(1)
    N, n = 64, 4
    gap = N // (2 * n)
    u = rng.integers(-1000, 1000, size=2 * n)
    m = [0] * N
    for k in range(2 * n):
        m[k * gap] = int(u[k])
    z = scheme.ckks_decode(m, n, 0)
    w = u[:n] + 1j * u[n:]
    assert np.allclose(z, boot.slot_matrix(n) @ w, atol=1e-9)


def test_diagonal_sum_is_matrix_product():
    rng = np.random.default_rng(2)
    n = 8
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    z = rng.normal(size=n) + 1j * rng.normal(size=n)
    acc = sum(d * np.roll(z, -k) for k, d in enumerate(boot.diagonals(A)))
    assert np.allclose(acc, A @ z)


def test_taylor_coefficients():
    c = boot.taylor_coefficients(11)
    for y in (0.1, -0.4, 0.49):
        re = sum(c[k] * y ** k for k in range(0, 12, 2))
        im = sum(c[k] * y ** k for k in range(1, 12, 2))
        assert abs(complex(re, im) - complex(math.cos(y), math.sin(y))) < 1e-12


def keys(P, s, rk, logP):
    from oracle import limbs
    N = 1 << P.logN
    uni = lambda bits: limbs.poly_from_limbs(synth.uniform_limbs(rk, bits, N))
    relin = scheme.keygen_relin(s, uni(P.logQ + logP), synth.dg(rk, N, 3.2), P.logQ, logP)
    rot = {r: galois.keygen_galois(s, uni(P.logQ + logP), synth.dg(rk, N, 3.2), galois.rotation_element(r, N),
                                   P.logQ, logP) for r in boot.rotation_amounts(P)}
    conj = galois.keygen_galois(s, uni(P.logQ + logP), synth.dg(rk, N, 3.2), galois.conjugation_element(N),
                                P.logQ, logP)
    return boot.BootKeys(relin, rot, conj)


def test_bootstrap_refreshes_the_message():
    """N = 2^10, 4 slots in the unit disk at scale 2^30, encrypted at logq = 40 with
    h = 64: the bootstrapped ciphertext sits at a higher level and decrypts to the same
    slots within 2^-16."""
    from oracle import limbs
    P = boot.BootParams(logN=10, logslots=2, logq_in=40, logQ=840)
    N, n = 1 << P.logN, 1 << P.logslots
    rk, rm, rn, _ = synth.streams(31)
    s = synth.hwt(rk, N, 64)
    a = limbs.poly_from_limbs(synth.uniform_limbs(rk, P.logQ, N))
    pk = scheme.keygen_public(s, a, synth.dg(rk, N, 3.2), P.logQ)
    K = keys(P, s, rk, P.logQ)
    z = synth.unit_disk(rm, n)
    m = scheme.ckks_encode(z, N, 30)
    ct = scheme.encrypt(pk, m, synth.zo(rn, N), synth.dg(rn, N, 3.2), synth.dg(rn, N, 3.2), P.logq_in, 30)
    aux = boot.boot_aux(P)
    with oracle_pool(8) as pool:
        out = boot.bootstrap(ct, P, aux, K, mapper=pool.map)
    assert out.logq > P.logq_in + 40
    zz = scheme.ckks_decode(scheme.decrypt(out, s), n, out.logp)
    err = float(np.max(np.abs(zz - z)))
    assert err < 2.0 ** -16, err
