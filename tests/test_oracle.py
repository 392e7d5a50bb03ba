"""Pins for the CPU oracle: each check ties it to the paper's definitions by a route
other than re-running its own formula (hand-worked values, closed forms, brute force,
invariants, an independent textbook construction)."""
import itertools
import json
import os
import random

import numpy as np
import pytest

from oracle import crt, limbs, ntt, ring, scheme
import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")))


# ------------------------------------------------------------------ ring product

@pytest.mark.parametrize("case", GOLD["ring_mul"])
def test_ring_hand_examples(case):
    for f in (ring.negacyclic_schoolbook, ring.negacyclic_kronecker):
        if case["modulus"] is None and f is ring.negacyclic_kronecker:
            got = f(case["a"], case["b"])
        else:
            got = f(case["a"], case["b"], case["modulus"])
        assert got == case["c"]


def test_ring_n1_n2_exhaustive_closed_form():
    vals = range(-3, 4)
    for a0, b0 in itertools.product(vals, vals):
        assert ring.negacyclic_schoolbook([a0], [b0]) == [a0 * b0]
    for a0, a1, b0, b1 in itertools.product(vals, repeat=4):
        assert ring.negacyclic_schoolbook([a0, a1], [b0, b1]) == [a0 * b0 - a1 * b1, a0 * b1 + a1 * b0]


def test_ring_monomials_xn_is_minus_one():
    N = 8
    for i in range(N):
        for j in range(N):
            a = [0] * N
            b = [0] * N
            a[i] = b[j] = 1
            want = [0] * N
            want[(i + j) % N] = -1 if i + j >= N else 1
            assert ring.negacyclic_schoolbook(a, b) == want


def _skew_circulant_product(a, b):
    """Independent textbook construction: multiplication by b in Z[X]/(X^N+1) is the
    N x N matrix with entry (i, j) = b_(i-j) for i >= j and -b_(N+i-j) for i < j."""
    N = len(a)
    M = np.empty((N, N), dtype=object)
    for i in range(N):
        for j in range(N):
            M[i, j] = b[i - j] if i >= j else -b[N + i - j]
    return [int(x) for x in M.dot(np.array(a, dtype=object))]


@pytest.mark.parametrize("N", [4, 16, 32])
def test_ring_matches_skew_circulant_matrix(N):
    rng = random.Random(N)
    a = [rng.randrange(-2**40, 2**40) for _ in range(N)]
    b = [rng.randrange(-2**40, 2**40) for _ in range(N)]
    assert ring.negacyclic_schoolbook(a, b) == _skew_circulant_product(a, b)


def test_ring_axioms():
    rng = random.Random(7)
    N, m = 16, 2**61 - 1
    a, b, c = ([rng.randrange(m) for _ in range(N)] for _ in range(3))
    ab = ring.negacyclic_schoolbook(a, b, m)
    assert ab == ring.negacyclic_schoolbook(b, a, m)
    assert ring.negacyclic_schoolbook(ab, c, m) == ring.negacyclic_schoolbook(a, ring.negacyclic_schoolbook(b, c, m), m)
    bc = [(x + y) % m for x, y in zip(b, c)]
    lhs = ring.negacyclic_schoolbook(a, bc, m)
    rhs = [(x + y) % m for x, y in zip(ab, ring.negacyclic_schoolbook(a, c, m))]
    assert lhs == rhs


@pytest.mark.parametrize("N,bits", [(64, 120), (256, 200), (1024, 120)])
def test_kronecker_equals_schoolbook(N, bits):
    rng = random.Random(N * bits)
    Q = 1 << bits
    a = [rng.getrandbits(bits) for _ in range(N)]
    b = [rng.getrandbits(bits) for _ in range(N)]
    assert ring.negacyclic_kronecker(a, b, Q) == ring.negacyclic_schoolbook(a, b, Q)
    # unreduced integer products agree as well
    assert ring.negacyclic_kronecker(a, b) == ring.negacyclic_schoolbook(a, b)


def test_truncation_invariant():
    rng = random.Random(3)
    N, logq, k = 128, 300, 77
    a = [rng.getrandbits(logq) for _ in range(N)]
    b = [rng.getrandbits(logq) for _ in range(N)]
    full = ring.ring_mul(a, b, 1 << logq)
    low = ring.ring_mul([x % (1 << k) for x in a], [x % (1 << k) for x in b], 1 << k)
    assert [x % (1 << k) for x in full] == low


def test_single_coefficient():
    rng = random.Random(5)
    N = 64
    a = [rng.getrandbits(90) for _ in range(N)]
    b = [rng.getrandbits(90) for _ in range(N)]
    full = ring.negacyclic_schoolbook(a, b)
    assert [ring.coefficient(a, b, i) for i in range(N)] == full


# ------------------------------------------------------------------ NTT

@pytest.mark.parametrize("case", GOLD["ntt"])
def test_ntt_hand_examples(case):
    q, psi = case["q"], case["psi"]
    assert ntt.ntt_definition(case["a"], q, psi) == case["abar"]
    assert ntt.ntt_fast(case["a"], q, psi) == case["abar"]
    assert ntt.intt_definition(case["abar"], q, psi) == case["a"]
    assert ntt.intt_fast(case["abar"], q, psi) == case["a"]


def _ntt_prime(N, below):
    q = below - (below - 1) % (2 * N)
    while not ntt.is_prime(q):
        q -= 2 * N
    return q


def test_is_prime_small_brute_force():
    for n in range(2, 3000):
        assert ntt.is_prime(n) == all(n % d for d in range(2, int(n ** 0.5) + 1))


@pytest.mark.parametrize("N", [8, 64, 256])
def test_ntt_fast_equals_definition_and_convolution(N):
    q = _ntt_prime(N, 1 << 30)
    psi = ntt.root_of_unity(q, 2 * N)
    assert pow(psi, N, q) == q - 1 and pow(psi, 2 * N, q) == 1
    rng = random.Random(N)
    a = [rng.randrange(q) for _ in range(N)]
    b = [rng.randrange(q) for _ in range(N)]
    A = ntt.ntt_definition(a, q, psi)
    assert ntt.ntt_fast(a, q, psi) == A
    assert ntt.intt_definition(A, q, psi) == a
    B = ntt.ntt_fast(b, q, psi)
    # convolution theorem (Eq. ntt_mul) against the schoolbook product mod q
    C = [x * y % q for x, y in zip(A, B)]
    assert ntt.intt_fast(C, q, psi) == ring.negacyclic_schoolbook(a, b, q)


def test_ntt_fast_roundtrip_large():
    N = 1 << 16
    q = _ntt_prime(N, 1 << 30)
    psi = ntt.root_of_unity(q, 2 * N)
    rng = np.random.default_rng(1)
    a = [int(x) for x in rng.integers(0, q, N)]
    A = ntt.ntt_fast(a, q, psi)
    assert ntt.intt_fast(A, q, psi) == a
    # spot-check three outputs against the definition
    for i in (0, 12345, N - 1):
        e = [(2 * i + 1) * j % (2 * N) for j in range(N)]
        pw = pow(psi, 1, q)
        assert A[i] == sum(a[j] * pow(pw, e[j], q) for j in range(0, N)) % q


# ------------------------------------------------------------------ CRT / Garner

@pytest.mark.parametrize("case", GOLD["crt"])
def test_crt_hand_example(case):
    assert crt.residues(case["X"], case["moduli"]) == case["residues"]
    assert crt.crt_compose(case["residues"], case["moduli"]) == case["X"]
    assert crt.garner_digits(case["residues"], case["moduli"]) == case["digits"]
    assert crt.garner(case["residues"], case["moduli"]) == case["X"]


def test_crt_garner_roundtrip():
    rng = random.Random(11)
    moduli = []
    q = 1 << 30
    while len(moduli) < 40:
        q -= 1
        if ntt.is_prime(q):
            moduli.append(q)
    M = 1
    for m in moduli:
        M *= m
    for _ in range(50):
        X = rng.randrange(M)
        x = crt.residues(X, moduli)
        assert crt.crt_compose(x, moduli) == X
        assert crt.garner(x, moduli) == X
        v = crt.garner_digits(x, moduli)
        assert all(0 <= vk < qk for vk, qk in zip(v, moduli))


# ------------------------------------------------------------------ limbs

def test_limb_codec():
    assert limbs.int_to_limbs((1 << 32) + 5, 2) == [5, 1]
    assert limbs.limbs_to_int([5, 1, 0]) == (1 << 32) + 5
    arr = synth.uniform_limbs(np.random.default_rng(0), 100, 8)
    ints = limbs.poly_from_limbs(arr)
    assert all(0 <= x < 1 << 100 for x in ints)
    assert np.array_equal(limbs.poly_to_limbs(ints, 4), arr)
    assert ints[3] == sum(int(arr[i, 3]) << (32 * i) for i in range(4))


# ------------------------------------------------------------------ scheme

@pytest.mark.parametrize("case", GOLD["rounding"])
def test_rounding_hand_examples(case):
    k = case["k"]
    if "ckks" in case:
        assert [scheme.divide_round(x, k, scheme.CKKS, 0) for x in case["x"]] == case["ckks"]
    if "bgv" in case:
        assert [scheme.divide_round(x, k, scheme.BGV, case["t"]) for x in case["x"]] == case["bgv"]


def test_divide_round_properties():
    rng = random.Random(2)
    t = 65537
    for _ in range(500):
        k = rng.randrange(1, 80)
        x = rng.getrandbits(200)
        r = scheme.divide_round(x, k, scheme.CKKS, 0)
        assert abs(2 * (x - (r << k))) <= (1 << k)          # nearest
        if (x % (1 << k)) == 0:
            assert r == x >> k                              # exact division
        b = scheme.divide_round(x, k, scheme.BGV, t)
        d = x - (b << k)
        assert d % t == 0 and abs(d) <= (1 << k) * (t // 2 + 1)
        assert (b * pow(2, k, t) - x) % t == 0              # message scaled by 2^-k mod t


def _keys(rng_k, N, logQ, logP, scheme_, t, h=None):
    h = h if h is not None else min(192, N // 2)
    s = synth.hwt(rng_k, N, h)
    a = limbs.poly_from_limbs(synth.uniform_limbs(rng_k, logQ, N))
    pk = scheme.keygen_public(s, a, synth.dg(rng_k, N, 3.2), logQ, scheme_, t)
    a2 = limbs.poly_from_limbs(synth.uniform_limbs(rng_k, logQ + logP, N))
    evk = scheme.keygen_relin(s, a2, synth.dg(rng_k, N, 3.2), logQ, logP, scheme_, t)
    return s, pk, evk


def _enc(rng, pk, m, logq, logp=0):
    N = len(m)
    return scheme.encrypt(pk, m, synth.zo(rng, N), synth.dg(rng, N, 3.2), synth.dg(rng, N, 3.2), logq, logp)


def test_tensor_phase_identity():
    """(c0 + c1 s)(c0' + c1' s) = d0 + d1 s + d2 s^2 exactly in Z_Q[X]/(X^N+1)."""
    rk, rm, rn, _ = synth.streams(90)
    N, logq = 64, 160
    s, pk, evk = _keys(rk, N, logq, logq, scheme.CKKS, 0)
    x = _enc(rn, pk, [int(v) for v in rm.integers(0, 1 << 20, N)], logq)
    y = _enc(rn, pk, [int(v) for v in rm.integers(0, 1 << 20, N)], logq)
    Q = 1 << logq
    d0, d1, d2 = scheme.tensor(x, y)
    S = [int(v) % Q for v in s]
    S2 = ring.negacyclic_schoolbook(S, S, Q)
    lhs = ring.negacyclic_schoolbook(scheme.phase(x, s), scheme.phase(y, s), Q)
    d1s = ring.negacyclic_schoolbook(d1, S, Q)
    d2s2 = ring.negacyclic_schoolbook(d2, S2, Q)
    assert lhs == [(a + b + c) % Q for a, b, c in zip(d0, d1s, d2s2)]


@pytest.mark.parametrize("scheme_", [scheme.CKKS, scheme.BGV])
def test_relin_noise_invariant(scheme_):
    """phase(relin(d)) - (d0 + d1 s + d2 s^2) is small: at most N * 6 sigma (* t for BGV) *
    max|d2| / P + (1 + h)/2 (+ t terms for BGV)."""
    rk, rm, rn, _ = synth.streams(91)
    N, logq, logP = 64, 200, 200
    t = 65537 if scheme_ == scheme.BGV else 0
    s, pk, evk = _keys(rk, N, logq, logP, scheme_, t, h=16)
    Q = 1 << logq
    msg = [int(v) for v in rm.integers(0, t if t else 1 << 20, N)]
    x = _enc(rn, pk, msg, logq)
    y = _enc(rn, pk, msg, logq)
    d0, d1, d2 = scheme.tensor(x, y)
    c0, c1 = scheme.relinearize(d0, d1, d2, evk, logq, scheme_, t)
    S = [int(v) % Q for v in s]
    S2 = ring.negacyclic_schoolbook(S, S, Q)
    want = [(a + b + c) % Q for a, b, c in zip(d0, ring.negacyclic_schoolbook(d1, S, Q),
                                                ring.negacyclic_schoolbook(d2, S2, Q))]
    got = scheme.phase(scheme.Ciphertext(c0, c1, 6, logq, scheme=scheme_, t=t), s)
    diff = [scheme.center(g - w, Q) for g, w in zip(got, want)]
    tt = t if t else 1
    bound = N * 6 * 3.2 * tt + (1 + 16) * (tt / 2 + 1) + 2
    assert max(abs(v) for v in diff) <= bound
    if scheme_ == scheme.BGV:
        assert all(v % t == 0 for v in diff)


@pytest.mark.parametrize("k", [32, 20])
def test_bgv_end_to_end_exact(k):
    rk, rm, rn, _ = synth.streams(92)
    N, logq, t = 256, 240, 65537
    s, pk, evk = _keys(rk, N, logq, logq, scheme.BGV, t, h=64)
    m1 = [int(v) for v in synth.uniform_mod(rm, N, t)]
    m2 = [int(v) for v in synth.uniform_mod(rm, N, t)]
    x = _enc(rn, pk, m1, logq)
    y = _enc(rn, pk, m2, logq)
    out = scheme.mult_rescale(x, y, evk, k)
    want = ring.negacyclic_schoolbook(m1, m2, t)
    assert out.logq == logq - k
    assert scheme.bgv_decode(scheme.decrypt(out, s), t, out.gamma) == want
    if k == 32:
        assert out.gamma == 1


def test_ckks_encode_forms_agree_and_roundtrip():
    rng = np.random.default_rng(4)
    N, logp = 256, 40
    for n in (128, 32):
        z = synth.unit_disk(rng, n)
        m1 = scheme.ckks_encode_direct(z, N, logp)
        m2 = scheme.ckks_encode(z, N, logp)
        assert max(abs(a - b) for a, b in zip(m1, m2)) <= 1
        back = scheme.ckks_decode(m2, n, logp)
        assert np.max(np.abs(back - z)) < 2.0 ** -30
        gap = N // (2 * n)
        assert all(m2[i] == 0 for i in range(N) if i % gap)


def test_ckks_end_to_end_precision():
    rk, rm, rn, _ = synth.streams(93)
    N, logq, logp = 1024, 300, 40
    n = N // 2
    s, pk, evk = _keys(rk, N, logq, logq, scheme.CKKS, 0)
    z1 = synth.unit_disk(rm, n)
    z2 = synth.unit_disk(rm, n)
    x = _enc(rn, pk, scheme.ckks_encode(z1, N, logp), logq, logp)
    y = _enc(rn, pk, scheme.ckks_encode(z2, N, logp), logq, logp)
    out = scheme.mult_rescale(x, y, evk, logp)
    assert (out.logq, out.logp) == (logq - logp, logp)
    z = scheme.ckks_decode(scheme.decrypt(out, s), n, out.logp)
    assert np.max(np.abs(z - z1 * z2)) <= 2.0 ** -20


def test_sampled_matches_full():
    rk, rm, rn, _ = synth.streams(94)
    N, logq = 128, 200
    for sch, t, k in ((scheme.CKKS, 0, 40), (scheme.BGV, 65537, 32)):
        s, pk, evk = _keys(rk, N, logq, logq, sch, t, h=32)
        x = _enc(rn, pk, [int(v) for v in rm.integers(0, 1000, N)], logq)
        y = _enc(rn, pk, [int(v) for v in rm.integers(0, 1000, N)], logq)
        full = scheme.mult_rescale(x, y, evk, k)
        idx = [0, 1, 77, N - 1]
        o0, o1 = scheme.mult_rescale_sampled(x, y, evk, k, idx)
        assert o0 == [full.c0[i] for i in idx] and o1 == [full.c1[i] for i in idx]


# ------------------------------------------------------------------ samplers

def test_samplers():
    rng = np.random.default_rng(5)
    s = synth.hwt(rng, 1 << 14, 192)
    assert int(np.count_nonzero(s)) == 192 and set(np.unique(s)) <= {-1, 0, 1}
    e = synth.dg(rng, 1 << 20, 3.2)
    assert abs(np.std(e) - np.sqrt(3.2 ** 2 + 1 / 12)) < 0.02 * 3.2
    v = synth.zo(rng, 1 << 16)
    assert abs(np.mean(v == 0) - 0.5) < 0.01
    z = synth.unit_disk(rng, 1000)
    assert np.all(np.abs(z) <= 1.0)


def test_relinearization_hand_example():
    """R3 pinned: the hand-worked N = 2 relinearization of the golden fixture (d2 taken in
    [0, Q_l)), both schemes; the centered representative of d2 gives another c0."""
    g = GOLD["relin"]
    N = 1 << g["logN"]
    assert len(g["d2"]) == N
    for sch, t, want in ((scheme.CKKS, 0, g["ckks"]), (scheme.BGV, 17, g["bgv_t17"])):
        evk = scheme.EvalKey(g["evk_b"], g["evk_a"], g["logN"], g["logq"], g["logP"], sch, t)
        c0, c1 = scheme.relinearize(g["d0"], g["d1"], g["d2"], evk, g["logq"], sch, t)
        assert c0 == want["c0"] and c1 == want["c1"], (sch, c0, c1)
    # the other representative choice changes the output bits
    Q = 1 << g["logq"]
    centered = [v - Q if v >= Q // 2 else v for v in g["d2"]]
    PQ = 1 << (g["logP"] + g["logq"])
    k0 = ring.ring_mul(centered, [b % PQ for b in g["evk_b"]], PQ)
    c0 = [(g["d0"][i] + scheme.divide_round(k0[i], g["logP"], scheme.CKKS, 0)) % Q for i in range(N)]
    assert c0 == g["ckks_if_d2_centered"]["c0"] != g["ckks"]["c0"]
