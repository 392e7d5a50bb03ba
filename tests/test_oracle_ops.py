"""Pins for the oracle's coefficient-wise operations (oracle.ops) and its Galois
automorphisms and key switching (oracle.galois).  Each check reaches the result by a
route other than the function's own formula: decryption and decoding of the slots,
exact BGV messages, ring homomorphism against the pinned ring product, evaluation at
roots of unity, composition laws."""
import numpy as np
import pytest

import synth
from oracle import galois, limbs, ntt, ops, ring, scheme


def _keys(rk, N, logQ, logP, sch, t, h):
    s = synth.hwt(rk, N, h)
    a = limbs.poly_from_limbs(synth.uniform_limbs(rk, logQ, N))
    pk = scheme.keygen_public(s, a, synth.dg(rk, N, 3.2), logQ, sch, t)
    return s, pk


def _enc(rn, pk, m, logq, logp=0):
    N = len(m)
    return scheme.encrypt(pk, m, synth.zo(rn, N), synth.dg(rn, N, 3.2), synth.dg(rn, N, 3.2), logq, logp)


def _gkey(rk, s, g, logQ, logP, sch, t):
    N = len(s)
    a = limbs.poly_from_limbs(synth.uniform_limbs(rk, logQ + logP, N))
    return galois.keygen_galois(s, a, synth.dg(rk, N, 3.2), g, logQ, logP, sch, t)


def _bgv_msgs(ct, s, t):
    return scheme.bgv_decode(scheme.decrypt(ct, s), t, ct.gamma)


def _slots(ct, s, n):
    return scheme.ckks_decode(scheme.decrypt(ct, s), n, ct.logp)


# ------------------------------------------------------------------ automorphisms

def test_automorphism_is_a_ring_homomorphism():
    """kappa_g(a b) = kappa_g(a) kappa_g(b) in Z_m[X]/(X^N+1) (a dropped sign at the
    wrap X^N = -1 breaks this), and kappa_1 is the identity."""
    rng = np.random.default_rng(1)
    N, m = 32, 1 << 40
    for g in (1, 3, 5, 25, 2 * N - 1, 2 * N - 5):
        for _ in range(3):
            a = [int(v) for v in rng.integers(0, 1 << 40, N)]
            b = [int(v) for v in rng.integers(0, 1 << 40, N)]
            lhs = galois.automorphism(ring.negacyclic_schoolbook(a, b, m), g, m)
            rhs = ring.negacyclic_schoolbook(galois.automorphism(a, g, m), galois.automorphism(b, g, m), m)
            assert lhs == rhs
    a = [int(v) for v in rng.integers(0, m, N)]
    assert galois.automorphism(a, 1, m) == a


def test_automorphism_composition():
    """kappa_g o kappa_h = kappa_(g h mod 2N); kappa_(-1) is an involution."""
    rng = np.random.default_rng(2)
    N = 64
    a = [int(v) for v in rng.integers(-1000, 1000, N)]
    for g, h in ((5, 5), (5, 25), (3, 2 * N - 1), (125, 77)):
        assert galois.automorphism(galois.automorphism(a, h), g) == galois.automorphism(a, g * h % (2 * N))
    c = galois.conjugation_element(N)
    assert galois.automorphism(galois.automorphism(a, c), c) == a


def test_automorphism_evaluation_at_roots():
    """kappa_g(a) evaluated at a primitive 2N-th root psi mod a prime q = 1 (mod 2N)
    equals a evaluated at psi^g (direct sums mod q)."""
    rng = np.random.default_rng(3)
    N = 32
    q = next(p for p in range(2 * N * 1000 + 1, 1 << 31, 2 * N) if ntt.is_prime(p))
    psi = ntt.root_of_unity(q, 2 * N)
    a = [int(v) for v in rng.integers(0, q, N)]
    ev = lambda poly, x: sum(c * pow(x, i, q) for i, c in enumerate(poly)) % q
    for g in (3, 5, 5 ** 3 % (2 * N), 2 * N - 1):
        k = galois.automorphism(a, g, q)
        for r in (psi, pow(psi, 3, q), pow(psi, 2 * N - 1, q)):
            assert ev(k, r) == ev(a, pow(r, g, q))


@pytest.mark.parametrize("n", [128, 16])
def test_rotation_and_conjugation_permute_encoded_slots(n):
    """decode(kappa_(5^r)(encode(z))) = z rotated left by r; kappa_(-1) conjugates every
    slot (full and sparse packing)."""
    rng = np.random.default_rng(4)
    N, logp = 256, 40
    z = synth.unit_disk(rng, n)
    m = scheme.ckks_encode(z, N, logp)
    for r in (1, 3, n - 1):
        got = scheme.ckks_decode(galois.automorphism(m, galois.rotation_element(r, N)), n, logp)
        assert np.max(np.abs(got - np.roll(z, -r))) < 2.0 ** -30
    got = scheme.ckks_decode(galois.automorphism(m, galois.conjugation_element(N)), n, logp)
    assert np.max(np.abs(got - np.conj(z))) < 2.0 ** -30


# ------------------------------------------------------------------ key switching

@pytest.mark.parametrize("r", [1, 5])
def test_leftrotate_and_conjugate_ckks_decrypt(r):
    rk, rm, rn, _ = synth.streams(95)
    N, logq, logP, logp = 512, 200, 200, 40
    n = N // 2
    s, pk = _keys(rk, N, logq, logP, scheme.CKKS, 0, 64)
    z = synth.unit_disk(rm, n)
    ct = _enc(rn, pk, scheme.ckks_encode(z, N, logp), logq, logp)
    rot = galois.leftrotate(ct, r, _gkey(rk, s, galois.rotation_element(r, N), logq, logP, scheme.CKKS, 0))
    assert np.max(np.abs(_slots(rot, s, n) - np.roll(z, -r))) <= 2.0 ** -20
    cj = galois.conjugate(ct, _gkey(rk, s, galois.conjugation_element(N), logq, logP, scheme.CKKS, 0))
    assert np.max(np.abs(_slots(cj, s, n) - np.conj(z))) <= 2.0 ** -20
    # at a lower level, with the key reduced mod P 2^logq
    low = ops.moddown(ct, 60)
    rot = galois.leftrotate(low, r, _gkey(rk, s, galois.rotation_element(r, N), logq, logP, scheme.CKKS, 0))
    assert rot.logq == logq - 60
    assert np.max(np.abs(_slots(rot, s, n) - np.roll(z, -r))) <= 2.0 ** -20


@pytest.mark.parametrize("g", [5, 25, 127, 511])
def test_key_switch_bgv_exact(g):
    """BGV: decrypting kappa_g(ct) gives kappa_g(m) mod t exactly, and the switching
    noise is a multiple of t within N 6 sigma t + (1 + h)(t/2 + 1)."""
    rk, rm, rn, _ = synth.streams(96)
    N, logq, logP, t, h = 256, 200, 200, 65537, 32
    s, pk = _keys(rk, N, logq, logP, scheme.BGV, t, h)
    m = [int(v) for v in synth.uniform_mod(rm, N, t)]
    ct = _enc(rn, pk, m, logq)
    out = galois.key_switch(ct, _gkey(rk, s, g, logq, logP, scheme.BGV, t))
    assert _bgv_msgs(out, s, t) == galois.automorphism(m, g, t)
    Q = 1 << logq
    want = galois.automorphism(scheme.phase(ct, s), g, Q)
    diff = [scheme.center(a - b, Q) for a, b in zip(scheme.phase(out, s), want)]
    assert all(d % t == 0 for d in diff)
    assert max(abs(d) for d in diff) <= N * 6 * 3.2 * t + (1 + h) * (t / 2 + 1) + 2


# ------------------------------------------------------------------ coefficient-wise ops

@pytest.fixture(scope="module")
def bgv():
    rk, rm, rn, _ = synth.streams(97)
    N, logq, t = 256, 160, 65537
    s, pk = _keys(rk, N, logq, logq, scheme.BGV, t, 32)
    m1 = [int(v) for v in synth.uniform_mod(rm, N, t)]
    m2 = [int(v) for v in synth.uniform_mod(rm, N, t)]
    return s, pk, t, m1, m2, _enc(rn, pk, m1, logq), _enc(rn, pk, m2, logq)


def test_bgv_add_sub_negate_exact(bgv):
    s, pk, t, m1, m2, x, y = bgv
    assert _bgv_msgs(ops.add(x, y), s, t) == [(a + b) % t for a, b in zip(m1, m2)]
    assert _bgv_msgs(ops.sub(x, y), s, t) == [(a - b) % t for a, b in zip(m1, m2)]
    assert _bgv_msgs(ops.negate(x), s, t) == [(-a) % t for a in m1]
    with pytest.raises(ValueError):
        ops.add(x, ops.moddown(y, 1))


def test_bgv_moddown_keeps_message(bgv):
    s, pk, t, m1, m2, x, y = bgv
    for k in (1, 31, 64):
        out = ops.moddown(x, k)
        assert out.logq == x.logq - k and _bgv_msgs(out, s, t) == m1


def test_bgv_multconst_multconstvec_addconst_exact(bgv):
    s, pk, t, m1, m2, x, y = bgv
    for k in (3, 65536, 12345):
        assert _bgv_msgs(ops.multconst(x, k), s, t) == [a * k % t for a in m1]
    p = [v % 7 for v in m2]  # a small plaintext keeps the product's noise far below Q
    assert _bgv_msgs(ops.multconstvec(x, p), s, t) == ring.negacyclic_schoolbook(m1, p, t)
    assert _bgv_msgs(ops.addconst(x, m2), s, t) == [(a + b) % t for a, b in zip(m1, m2)]


@pytest.fixture(scope="module")
def ckks():
    rk, rm, rn, _ = synth.streams(98)
    N, logq, logp = 256, 200, 40
    n = N // 2
    s, pk = _keys(rk, N, logq, logq, scheme.CKKS, 0, 32)
    z1, z2 = synth.unit_disk(rm, n), synth.unit_disk(rm, n)
    x = _enc(rn, pk, scheme.ckks_encode(z1, N, logp), logq, logp)
    y = _enc(rn, pk, scheme.ckks_encode(z2, N, logp), logq, logp)
    return s, n, z1, z2, x, y


def test_ckks_linear_ops_and_imult(ckks):
    s, n, z1, z2, x, y = ckks
    tol = 2.0 ** -25
    assert np.max(np.abs(_slots(ops.add(x, y), s, n) - (z1 + z2))) < tol
    assert np.max(np.abs(_slots(ops.sub(x, y), s, n) - (z1 - z2))) < tol
    assert np.max(np.abs(_slots(ops.negate(x), s, n) + z1)) < tol
    assert np.max(np.abs(_slots(ops.imult(x), s, n) - 1j * z1)) < tol
    assert ops.imult(ops.imult(x)).c0 == ops.negate(x).c0     # X^N = -1
    assert np.max(np.abs(_slots(ops.moddown(x, 50), s, n) - z1)) < tol


def test_ckks_constants(ckks):
    s, n, z1, z2, x, y = ckks
    N = 1 << x.logN
    c = -0.6180339887
    out = ops.multconst(x, round(c * 2 ** 30) % (1 << x.logq), 30)
    assert out.logp == x.logp + 30
    assert np.max(np.abs(_slots(out, s, n) - c * z1)) < 2.0 ** -25
    w = synth.unit_disk(np.random.default_rng(6), n)
    out = ops.multconstvec(x, scheme.ckks_encode(w, N, 30), 30)
    assert np.max(np.abs(_slots(out, s, n) - z1 * w)) < 2.0 ** -20
    out = ops.addconst(x, scheme.ckks_encode(w, N, x.logp))
    assert np.max(np.abs(_slots(out, s, n) - (z1 + w))) < 2.0 ** -25
