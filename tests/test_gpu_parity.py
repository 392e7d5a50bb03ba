"""GPU parity: the HIP library through its C ABI against the CPU oracle.

Integer outputs must match bit for bit.  Small cases are checked on every
coefficient; the N = 2^16, logq = 1555 workload is checked on sampled
coefficients that the oracle computes one by one, plus size-independent properties.
"""
import numpy as np
import pytest

import paper_2607_05920_amd as fhe
import synth
from oracle import ntt as ontt
from oracle import ring, scheme
from tests.gpu_helpers import check, dev, host, ints, keys, limbs_of, oracle_ct, random_ct, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    say("creating context logQ_max=1555 logP_max=1555")
    c = fhe.Context(1555, 1555)
    yield c
    c.close()


def test_prime_table(ctx):
    n = ctx.prime_count()
    assert n >= 150
    prev = 1 << 30
    for i in range(n):
        q, psi = ctx.prime_info(i)
        assert q < prev and q > 1 << 29 and q % (1 << 17) == 1 and ontt.is_prime(q)
        assert pow(psi, 1 << 16, q) == q - 1
        prev = q
    # K rule: smallest K with prod q_i >= 2^(e + 1 + 16) (|X| < 2^e recovered, and the
    # CRT quotient of X + 2^e kept exact by a 16-bit margin)
    for logN, a, b, terms in ((10, 120, 120, 1), (14, 438, 438, 2), (16, 1555, 3110, 1)):
        K = ctx.primes_needed(logN, a, b, terms)
        e = a + b + logN + (terms - 1).bit_length()
        M = 1
        for i in range(K):
            M *= ctx.prime_info(i)[0]
        assert M >= 1 << (e + 17) and M // ctx.prime_info(K - 1)[0] < 1 << (e + 17)


@pytest.mark.parametrize("logN,bits,nprimes", [(10, 120, 9), (12, 1555, 40), (16, 438, 20), (16, 3110, 17)])
def test_lift(ctx, logN, bits, nprimes):
    say(f"lift logN={logN} bits={bits} nprimes={nprimes}")
    rng = np.random.default_rng(logN * 7 + bits)
    N = 1 << logN
    L = synth.nlimbs(bits)
    limbs = synth.uniform_limbs(rng, bits, N, count=2)
    import torch
    res = torch.empty(2 * nprimes * N, dtype=torch.int32, device="cuda")
    ctx.lift(logN, L, nprimes, dev(limbs), res, count=2)
    got = host(res, (2, nprimes, N))
    idx = range(N) if N <= 4096 else np.random.default_rng(1).choice(N, 64, replace=False)
    for c in range(2):
        A = ints(limbs[c])
        for p in range(nprimes):
            q = ctx.prime_info(p)[0]
            assert all(int(got[c, p, j]) == A[j] % q for j in idx)


def _bitrev(i, bits):
    return int(format(i, f"0{bits}b")[::-1], 2)


@pytest.mark.parametrize("logN", [10, 11, 12, 13, 14, 15, 16])
def test_ntt_forward_inverse(ctx, logN):
    say(f"ntt logN={logN}")
    import torch
    N = 1 << logN
    primes = [0, 7] if logN < 16 else [3]
    nprimes = max(primes) + 1
    rng = np.random.default_rng(logN)
    data = np.zeros((nprimes, N), dtype=np.uint32)
    for p in range(nprimes):
        data[p] = rng.integers(0, ctx.prime_info(p)[0], N, dtype=np.uint64)
    t = dev(data)
    ctx.ntt(logN, nprimes, t, count=1, inverse=False, bitrev=True)
    fwd = host(t, (nprimes, N)).copy()
    perm = [_bitrev(i, logN) for i in range(N)]
    for p in primes:
        q, psi_max = ctx.prime_info(p)
        psi = pow(psi_max, (1 << 16) // N, q)
        want = ontt.ntt_fast([int(v) for v in data[p]], q, psi)
        got = [int(fwd[p, perm[i]]) for i in range(N)]
        check(got, want, f"ntt prime {p}")
        if logN == 10 and p == 0:
            check(want, ontt.ntt_definition([int(v) for v in data[p]], q, psi), "ntt definition")
    ctx.ntt(logN, nprimes, t, count=1, inverse=True, bitrev=True)
    assert np.array_equal(host(t, (nprimes, N)), data)


@pytest.mark.parametrize("count,natural", [(4, False), (7, False), (8, True)])
def test_ntt_several_per_prime_logn16(ctx, count, natural):
    """Transforms of `count` polynomials per prime at N = 2^16 (the row pass then takes
    four transforms of a prime per wave; 7 leaves one slot of the last block idle):
    every coefficient against the same transforms one at a time, two against the
    oracle's transform, and the inverse back to the input."""
    say(f"ntt logN=16 count={count} natural={natural}")
    logN, nprimes, prime0 = 16, 2, 5
    N = 1 << logN
    rng = np.random.default_rng(1600 + count)
    data = np.zeros((count, nprimes, N), dtype=np.uint32)
    for c in range(count):
        for p in range(nprimes):
            data[c, p] = rng.integers(0, ctx.prime_info(prime0 + p)[0], N, dtype=np.uint64)
    t = dev(data)
    ctx.ntt(logN, nprimes, t, count=count, bitrev=not natural, prime0=prime0)
    fwd = host(t, (count, nprimes, N)).copy()
    for c in range(count):
        one = dev(data[c])
        ctx.ntt(logN, nprimes, one, count=1, bitrev=not natural, prime0=prime0)
        assert np.array_equal(host(one, (nprimes, N)), fwd[c]), f"transform {c}"
    perm = [_bitrev(i, logN) for i in range(N)]
    for c, p in [(0, 0), (count - 1, 1)]:
        q, psi_max = ctx.prime_info(prime0 + p)
        want = ontt.ntt_fast([int(v) for v in data[c, p]], q, psi_max)
        got = [int(fwd[c, p, i if natural else perm[i]]) for i in range(N)]
        check(got, want, f"ntt transform {c} prime {prime0 + p}")
    ctx.ntt(logN, nprimes, t, count=count, inverse=True, bitrev=not natural, prime0=prime0)
    assert np.array_equal(host(t, (count, nprimes, N)), data)


def test_ring_mul_cfg1_bit_exact(ctx):
    """Bare ring multiply, N = 2^10, Q = 2^120, inputs uniform in [0, Q) from seed 1000."""
    say("ring_mul cfg1")
    import torch
    _, rm, _, _ = synth.streams(1)
    logN, logq = 10, 120
    N = 1 << logN
    a = synth.uniform_limbs(rm, logq, N)
    b = synth.uniform_limbs(rm, logq, N)
    out = torch.empty(4 * N, dtype=torch.int32, device="cuda")
    ctx.ring_mul(logN, logq, dev(a), dev(b), out)
    want = ring.negacyclic_schoolbook(ints(a), ints(b), 1 << logq)
    check(ints(host(out, (4, N))), want, "ring_mul cfg1")


@pytest.mark.parametrize("logN,logq,cnum", [(10, 1, 1), (10, 33, 2), (11, 97, 3), (13, 250, 2)])
def test_ring_mul_ragged_batched_in_place(ctx, logN, logq, cnum):
    say(f"ring_mul logN={logN} logq={logq} cnum={cnum}")
    rng = np.random.default_rng(logq)
    N = 1 << logN
    L = synth.nlimbs(logq)
    a = synth.uniform_limbs(rng, logq, N, count=cnum)
    b = synth.uniform_limbs(rng, logq, N, count=cnum)
    ta = dev(a)
    ctx.ring_mul(logN, logq, ta, dev(b), ta, cnum=cnum)   # output over the first operand
    got = host(ta, (cnum, L, N))
    for c in range(cnum):
        want = ring.ring_mul(ints(a[c]), ints(b[c]), 1 << logq)
        check(ints(got[c]), want, f"ring_mul {c}")


@pytest.mark.parametrize("logq", [2600, 3000, 3500])
def test_ring_mul_many_primes(logq):
    """Products that need 175-235 primes: the reconstruction's 6, 7 and 8 k-block
    forms and the lift's table in global memory, against the oracle on every
    coefficient (N = 2^10)."""
    say(f"ring_mul many primes logq={logq}")
    import torch
    c = fhe.Context(2400, 2400)
    try:
        logN = 10
        N = 1 << logN
        need = c.primes_needed(logN, logq, logq, 1)
        assert 160 < need <= 256 and need <= c.prime_count()
        rng = np.random.default_rng(logq + 7)
        a = synth.uniform_limbs(rng, logq, N)
        b = synth.uniform_limbs(rng, logq, N)
        out = torch.empty(synth.nlimbs(logq) * N, dtype=torch.int32, device="cuda")
        c.ring_mul(logN, logq, dev(a), dev(b), out)
        want = ring.ring_mul(ints(a), ints(b), 1 << logq)
        check(ints(host(out, (synth.nlimbs(logq), N))), want, f"ring_mul logq={logq}")
    finally:
        c.close()


def _gpu_he_mult(ctx, evk_limbs, sch, t, logN, logq, logP, x, y, bits, fused=True):
    import torch
    N = 1 << logN
    L = synth.nlimbs(logq)
    lsch = fhe.BGV if sch == scheme.BGV else fhe.CKKS
    ek = fhe.EvalKey(ctx, lsch, t, logN, logq, logP, evk_limbs[0], evk_limbs[1])
    Lo = synth.nlimbs(logq - bits)
    o0 = torch.empty(Lo * N, dtype=torch.int32, device="cuda")
    o1 = torch.empty(Lo * N, dtype=torch.int32, device="cuda")
    if fused:
        ctx.mul_relin_rescale(ek, logq, bits, dev(x[0]), dev(x[1]), dev(y[0]), dev(y[1]), o0, o1)
    else:
        m0 = torch.empty(L * N, dtype=torch.int32, device="cuda")
        m1 = torch.empty(L * N, dtype=torch.int32, device="cuda")
        ctx.mul_relin(ek, logq, dev(x[0]), dev(x[1]), dev(y[0]), dev(y[1]), m0, m1)
        ctx.rescale(lsch, t, logN, logq, bits, m0, m1, o0, o1)
    torch.cuda.synchronize()
    ek.close()
    return host(o0, (Lo, N)), host(o1, (Lo, N))


@pytest.mark.parametrize("sch,t,bits", [(scheme.CKKS, 0, 40), (scheme.BGV, 65537, 32), (scheme.BGV, 65537, 20),
                                        (scheme.BGV, 1001, 20)])
def test_he_mult_small_encrypted(ctx, sch, t, bits):
    """N = 2^10, logq = logP = 200, real keys and encryptions: bit-exact and decrypts."""
    say(f"he_mult small {sch} bits={bits}")
    rk, rm, rn, _ = synth.streams(50)
    logN, logq, logP = 10, 200, 200
    N = 1 << logN
    s, pk, evk, eb, ea = keys(rk, logN, logq, logP, sch, t, h=64)
    if sch == scheme.CKKS:
        z1, z2 = synth.unit_disk(rm, N // 2), synth.unit_disk(rm, N // 2)
        m1, m2 = scheme.ckks_encode(z1, N, 40), scheme.ckks_encode(z2, N, 40)
    else:
        m1 = [int(v) for v in synth.uniform_mod(rm, N, t)]
        m2 = [int(v) for v in synth.uniform_mod(rm, N, t)]
    enc = lambda m: scheme.encrypt(pk, m, synth.zo(rn, N), synth.dg(rn, N, 3.2), synth.dg(rn, N, 3.2), logq, 40)
    cx, cy = enc(m1), enc(m2)
    x = (limbs_of(cx.c0, logq), limbs_of(cx.c1, logq))
    y = (limbs_of(cy.c0, logq), limbs_of(cy.c1, logq))
    g0, g1 = _gpu_he_mult(ctx, (eb, ea), sch, t, logN, logq, logP, x, y, bits)
    want = scheme.mult_rescale(cx, cy, evk, bits)
    check(ints(g0), want.c0, "c0")
    check(ints(g1), want.c1, "c1")
    out = scheme.Ciphertext(ints(g0), ints(g1), logN, logq - bits, want.logp, sch, t, want.gamma)
    if sch == scheme.BGV:
        check(scheme.bgv_decode(scheme.decrypt(out, s), t, out.gamma), ring.negacyclic_schoolbook(m1, m2, t), "m1 m2")
    else:
        z = scheme.ckks_decode(scheme.decrypt(out, s), N // 2, out.logp)
        assert np.max(np.abs(z - z1 * z2)) <= 2.0 ** -20


@pytest.mark.parametrize("sch,t,bits", [(scheme.CKKS, 0, 40), (scheme.BGV, 65537, 32)])
def test_he_mult_cfg2_encrypted(ctx, sch, t, bits):
    """N = 2^14, logq = logP = 438, h = 192, sigma = 3.2; CKKS 2^13 slots in the unit disk at
    scale 2^40, BGV t = 65537 uniform plaintexts.  Every coefficient bit-exact; decrypts."""
    say(f"he_mult cfg2 {sch}")
    rk, rm, rn, _ = synth.streams(2)
    logN, logq, logP = 14, 438, 438
    N = 1 << logN
    s, pk, evk, eb, ea = keys(rk, logN, logq, logP, sch, t, h=192)
    if sch == scheme.CKKS:
        z1, z2 = synth.unit_disk(rm, N // 2), synth.unit_disk(rm, N // 2)
        m1, m2 = scheme.ckks_encode(z1, N, 40), scheme.ckks_encode(z2, N, 40)
    else:
        m1 = [int(v) for v in synth.uniform_mod(rm, N, t)]
        m2 = [int(v) for v in synth.uniform_mod(rm, N, t)]
    enc = lambda m: scheme.encrypt(pk, m, synth.zo(rn, N), synth.dg(rn, N, 3.2), synth.dg(rn, N, 3.2), logq, 40)
    cx, cy = enc(m1), enc(m2)
    x = (limbs_of(cx.c0, logq), limbs_of(cx.c1, logq))
    y = (limbs_of(cy.c0, logq), limbs_of(cy.c1, logq))
    g0, g1 = _gpu_he_mult(ctx, (eb, ea), sch, t, logN, logq, logP, x, y, bits)
    want = scheme.mult_rescale(cx, cy, evk, bits)
    check(ints(g0), want.c0, "c0")
    check(ints(g1), want.c1, "c1")
    out = scheme.Ciphertext(ints(g0), ints(g1), logN, logq - bits, want.logp, sch, t, want.gamma)
    if sch == scheme.BGV:
        check(scheme.bgv_decode(scheme.decrypt(out, s), t, out.gamma), ring.negacyclic_kronecker(m1, m2, t), "m1 m2")
    else:
        z = scheme.ckks_decode(scheme.decrypt(out, s), N // 2, out.logp)
        assert np.max(np.abs(z - z1 * z2)) <= 2.0 ** -20


@pytest.mark.parametrize("sch,t,bits", [(scheme.CKKS, 0, 1), (scheme.CKKS, 0, 31), (scheme.CKKS, 0, 32),
                                        (scheme.CKKS, 0, 33), (scheme.CKKS, 0, 64), (scheme.CKKS, 0, 73),
                                        (scheme.CKKS, 0, 150), (scheme.BGV, 65537, 1), (scheme.BGV, 65537, 64),
                                        (scheme.BGV, 1001, 73), (scheme.BGV, 65537, 150)])
def test_fused_rescale_equals_separate(ctx, sch, t, bits):
    """The one-pass relinearization + rescale gives the same bits as fhe_mul_relin then
    fhe_rescale (uniform inputs, N = 2^10, logq = 181, logP = 200; rescale widths below,
    at and above limb boundaries, up to logq - 31), and matches the oracle."""
    say(f"fused vs separate rescale {sch} bits={bits}")
    rk, rm, _, _ = synth.streams(80 + bits)
    logN, logq, logP = 10, 181, 200
    N = 1 << logN
    x, y = random_ct(rm, logN, logq), random_ct(rm, logN, logq)
    eb, ea = synth.uniform_limbs(rk, logq + logP, N), synth.uniform_limbs(rk, logq + logP, N)
    f0, f1 = _gpu_he_mult(ctx, (eb, ea), sch, t, logN, logq, logP, x, y, bits, fused=True)
    s0, s1 = _gpu_he_mult(ctx, (eb, ea), sch, t, logN, logq, logP, x, y, bits, fused=False)
    assert np.array_equal(f0, s0) and np.array_equal(f1, s1)
    want = scheme.mult_rescale(oracle_ct(*x, logN, logq, sch, t), oracle_ct(*y, logN, logq, sch, t),
                               scheme.EvalKey(ints(eb), ints(ea), logN, logq, logP, sch, t), bits)
    check(ints(f0), want.c0, "c0")
    check(ints(f1), want.c1, "c1")


@pytest.mark.parametrize("sch,t,bits", [(scheme.CKKS, 0, 40), (scheme.BGV, 65537, 32)])
def test_he_mult_cfg3_sampled(ctx, sch, t, bits):
    """N = 2^16, logq = logP = 1555 (49 limbs; key 98 limbs): uniformly random
    ciphertexts and key; 12 sampled output coefficients of both polynomials against the
    oracle, and the fused call bit-identical to mul_relin followed by rescale."""
    say(f"he_mult cfg3 sampled {sch}")
    rk, rm, _, _ = synth.streams(3)
    logN, logq, logP = 16, 1555, 1555
    N = 1 << logN
    x = random_ct(rm, logN, logq)
    y = random_ct(rm, logN, logq)
    eb = synth.uniform_limbs(rk, logq + logP, N)
    ea = synth.uniform_limbs(rk, logq + logP, N)
    g0, g1 = _gpu_he_mult(ctx, (eb, ea), sch, t, logN, logq, logP, x, y, bits, fused=True)
    s0, s1 = _gpu_he_mult(ctx, (eb, ea), sch, t, logN, logq, logP, x, y, bits, fused=False)
    assert np.array_equal(g0, s0) and np.array_equal(g1, s1)
    idx = [0, 1, 2, N // 2, N - 2, N - 1] + [int(v) for v in np.random.default_rng(9).choice(N, 6, replace=False)]
    ox, oy = oracle_ct(*x, logN, logq, sch, t), oracle_ct(*y, logN, logq, sch, t)
    evk = scheme.EvalKey(ints(eb), ints(ea), logN, logq, logP, sch, t)
    say("oracle sampled coefficients")
    w0, w1 = scheme.mult_rescale_sampled(ox, oy, evk, bits, idx)
    Lo = synth.nlimbs(logq - bits)
    got0 = [sum(int(g0[l, i]) << (32 * l) for l in range(Lo)) for i in idx]
    got1 = [sum(int(g1[l, i]) << (32 * l) for l in range(Lo)) for i in idx]
    check(got0, w0, "sampled c0")
    check(got1, w1, "sampled c1")


@pytest.mark.parametrize("sch,t,bits", [(scheme.CKKS, 0, 1), (scheme.CKKS, 0, 32), (scheme.CKKS, 0, 73),
                                        (scheme.BGV, 65537, 32), (scheme.BGV, 65537, 45), (scheme.BGV, 257, 7)])
def test_rescale(ctx, sch, t, bits):
    say(f"rescale {sch} bits={bits}")
    import torch
    rng = np.random.default_rng(bits)
    logN, logq, cnum = 11, 300, 2
    N = 1 << logN
    c0 = synth.uniform_limbs(rng, logq, N, count=cnum)
    c1 = synth.uniform_limbs(rng, logq, N, count=cnum)
    Lo = synth.nlimbs(logq - bits)
    o0 = torch.empty(cnum * Lo * N, dtype=torch.int32, device="cuda")
    o1 = torch.empty(cnum * Lo * N, dtype=torch.int32, device="cuda")
    lsch = fhe.BGV if sch == scheme.BGV else fhe.CKKS
    ctx.rescale(lsch, t, logN, logq, bits, dev(c0), dev(c1), o0, o1, cnum=cnum)
    g0, g1 = host(o0, (cnum, Lo, N)), host(o1, (cnum, Lo, N))
    for c in range(cnum):
        ct = scheme.Ciphertext(ints(c0[c]), ints(c1[c]), logN, logq, 60, sch, t, 1)
        want = scheme.rescale(ct, bits)
        check(ints(g0[c]), want.c0, f"c0 [{c}]")
        check(ints(g1[c]), want.c1, f"c1 [{c}]")
    # in place, one ciphertext
    t0, t1 = dev(c0[0]), dev(c1[0])
    ctx.rescale(lsch, t, logN, logq, bits, t0, t1, t0, t1)
    ct = scheme.Ciphertext(ints(c0[0]), ints(c1[0]), logN, logq, 60, sch, t, 1)
    check(ints(host(t0, (-1, N))[:Lo]), scheme.rescale(ct, bits).c0, "in-place rescale")


def test_zero_and_batched_he_mult(ctx):
    """Zero ciphertexts map to zero; a batch of 3 equals three single calls."""
    say("he_mult zero + batch")
    import torch
    rk, rm, _, _ = synth.streams(51)
    logN, logq, logP = 12, 300, 300
    N = 1 << logN
    eb = synth.uniform_limbs(rk, logq + logP, N)
    ea = synth.uniform_limbs(rk, logq + logP, N)
    z = np.zeros((synth.nlimbs(logq), N), dtype=np.uint32)
    g0, g1 = _gpu_he_mult(ctx, (eb, ea), scheme.CKKS, 0, logN, logq, logP, (z, z), (z, z), 40)
    assert not g0.any() and not g1.any()
    cnum = 3
    L = synth.nlimbs(logq)
    xs = [random_ct(rm, logN, logq) for _ in range(cnum)]
    ys = [random_ct(rm, logN, logq) for _ in range(cnum)]
    ek = fhe.EvalKey(ctx, fhe.CKKS, 0, logN, logq, logP, eb, ea)
    cat = lambda lst, i: dev(np.stack([v[i] for v in lst]))
    o0 = torch.empty(cnum * L * N, dtype=torch.int32, device="cuda")
    o1 = torch.empty(cnum * L * N, dtype=torch.int32, device="cuda")
    ctx.mul_relin(ek, logq, cat(xs, 0), cat(xs, 1), cat(ys, 0), cat(ys, 1), o0, o1, cnum=cnum)
    b0, b1 = host(o0, (cnum, L, N)), host(o1, (cnum, L, N))
    for c in range(cnum):
        s0 = torch.empty(L * N, dtype=torch.int32, device="cuda")
        s1 = torch.empty(L * N, dtype=torch.int32, device="cuda")
        ctx.mul_relin(ek, logq, dev(xs[c][0]), dev(xs[c][1]), dev(ys[c][0]), dev(ys[c][1]), s0, s1)
        assert np.array_equal(host(s0, (L, N)), b0[c]) and np.array_equal(host(s1, (L, N)), b1[c])
    # against the oracle for the first one
    ox, oy = oracle_ct(*xs[0], logN, logq, scheme.CKKS, 0), oracle_ct(*ys[0], logN, logq, scheme.CKKS, 0)
    want = scheme.mult(ox, oy, scheme.EvalKey(ints(eb), ints(ea), logN, logq, logP))
    check(ints(b0[0]), want.c0, "c0")
    check(ints(b1[0]), want.c1, "c1")
    ek.close()


def test_error_paths(ctx):
    say("error paths")
    import torch
    N = 1 << 10
    eb = np.zeros((synth.nlimbs(400), N), dtype=np.uint32)
    ek = fhe.EvalKey(ctx, fhe.CKKS, 0, 10, 200, 200, eb, eb)
    buf = torch.zeros(8 * (1 << 11), dtype=torch.int32, device="cuda")
    with pytest.raises(fhe.FheError) as e:
        fhe.load_library()
        import ctypes
        st = fhe.load_library().fhe_mul_relin(ctx.handle, ek.handle, 11, 100, *(ctypes.c_void_p(buf.data_ptr()),) * 6,
                                              1, None)
        fhe._check("fhe_mul_relin", st)
    assert e.value.status == -2
    with pytest.raises(fhe.FheError) as e:
        ctx.mul_relin(ek, 201, *(torch.zeros(7 * N, dtype=torch.int32, device="cuda") for _ in range(6)))
    assert e.value.status == -3
    with pytest.raises(fhe.FheError) as e:
        fhe.EvalKey(ctx, fhe.BGV, 4, 10, 200, 200, eb, eb)
    assert e.value.status == -1
    ek.close()
    assert ctx.reset_error() == 0
