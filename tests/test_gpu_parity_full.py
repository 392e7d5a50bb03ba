"""GPU parity on every coefficient at the full workload sizes and on the paths that
the smaller cases do not reach:

- N = 2^16, logq = logP = 1555 (49 limbs, key 98 limbs), CKKS rescale by 40, in the
  launch configuration the benchmark times (a CipherTensor of 4): all 4 x 2 x 65536
  output coefficients against the oracle;
- the same size with oracle keys and encryptions, decrypted within 2^-20;
- BGV and CKKS with the ciphertext below the key's level (the key reduced mod P Q_l);
- N = 2^15 (the 2^8 x 2^7 transform split), per-op and through an autotuned batch plan
  (which may pick the other split and the key's second layout);
- N = 2^16 CipherTensors of 7 and 8 pairs (the fused row pass then takes four
  ciphertexts per sub-row, the last group of 7 with one slot idle) against the same pairs
  one at a time, and one ciphertext of the idle-slot group against the oracle;
- a relinearization product whose reconstruction table exceeds the LDS (the
  reconstruction's global-memory form).

The oracle's independent ring products run in a process pool."""
import numpy as np
import pytest

import paper_2607_05920_amd as fhe
import synth
from oracle import scheme
from tests.gpu_helpers import check, dev, host, ints, keys, limbs_of, oracle_ct, oracle_pool, random_ct, say

pytestmark = pytest.mark.gpu


def _run(ctx, evk, logN, logq, bits, x, y, cnum):
    """fhe_mul_relin_rescale on a CipherTensor; x, y: (c0, c1) uint32[cnum][L][N]."""
    import torch
    N = 1 << logN
    Lo = synth.nlimbs(logq - bits)
    o0 = torch.empty(cnum * Lo * N, dtype=torch.int32, device="cuda")
    o1 = torch.empty_like(o0)
    if bits:
        ctx.mul_relin_rescale(evk, logq, bits, dev(x[0]), dev(x[1]), dev(y[0]), dev(y[1]), o0, o1, cnum=cnum)
    else:
        ctx.mul_relin(evk, logq, dev(x[0]), dev(x[1]), dev(y[0]), dev(y[1]), o0, o1, cnum=cnum)
    torch.cuda.synchronize()
    return host(o0, (cnum, Lo, N)), host(o1, (cnum, Lo, N))


@pytest.mark.timeout(900)
def test_he_mult_cfg3_every_coefficient():
    """N = 2^16, logq = logP = 1555, CKKS, rescale 40, CipherTensor of 4 uniform
    ciphertext pairs (the benchmark's inputs and launch): every output coefficient of
    every ciphertext equals the oracle's."""
    logN, logq, logP, bits, cnum = 16, 1555, 1555, 40, 4
    N = 1 << logN
    say("cfg3 full: context and inputs")
    ctx = fhe.Context(logq, logP)
    try:
        rk, rm, _, _ = synth.streams(3)
        eb = synth.uniform_limbs(rk, logq + logP, N)
        ea = synth.uniform_limbs(rk, logq + logP, N)
        x = (synth.uniform_limbs(rm, logq, N, count=cnum), synth.uniform_limbs(rm, logq, N, count=cnum))
        y = (synth.uniform_limbs(rm, logq, N, count=cnum), synth.uniform_limbs(rm, logq, N, count=cnum))
        evk = fhe.EvalKey(ctx, fhe.CKKS, 0, logN, logq, logP, eb, ea)
        say("cfg3 full: GPU CipherTensor of 4")
        g0, g1 = _run(ctx, evk, logN, logq, bits, x, y, cnum)
        evk.close()
    finally:
        ctx.close()
    ok = scheme.EvalKey(ints(eb), ints(ea), logN, logq, logP)
    say("cfg3 full: oracle, 4 HE-mults (24 ring products in a process pool)")
    from concurrent.futures import ThreadPoolExecutor
    with oracle_pool(16) as pool, ThreadPoolExecutor(cnum) as th:
        wants = list(th.map(lambda c: scheme.mult_rescale(oracle_ct(x[0][c], x[1][c], logN, logq, scheme.CKKS, 0),
                                                          oracle_ct(y[0][c], y[1][c], logN, logq, scheme.CKKS, 0),
                                                          ok, bits, mapper=pool.map), range(cnum)))
    for c, want in enumerate(wants):
        check(ints(g0[c]), want.c0, f"ciphertext {c} c0")
        check(ints(g1[c]), want.c1, f"ciphertext {c} c1")


@pytest.mark.timeout(900)
def test_he_mult_cfg3_encrypted_decrypts():
    """N = 2^16, logq = logP = 1555, h = 192, sigma = 3.2, CKKS 2^15 slots in the unit disk
    at scale 2^40: oracle keys and encryptions, GPU HE-mult + relin + rescale 40 bit-exact
    against the oracle, and the product decrypts within 2^-20 of z1 z2."""
    logN, logq, logP, bits = 16, 1555, 1555, 40
    N = 1 << logN
    rk, rm, rn, _ = synth.streams(3)
    say("cfg3 encrypted: oracle keys")
    s, pk, evk, eb, ea = keys(rk, logN, logq, logP, scheme.CKKS, 0, h=192)
    z1, z2 = synth.unit_disk(rm, N // 2), synth.unit_disk(rm, N // 2)
    m1, m2 = scheme.ckks_encode(z1, N, 40), scheme.ckks_encode(z2, N, 40)
    say("cfg3 encrypted: oracle encryptions")
    cx = scheme.encrypt(pk, m1, synth.zo(rn, N), synth.dg(rn, N, 3.2), synth.dg(rn, N, 3.2), logq, 40)
    cy = scheme.encrypt(pk, m2, synth.zo(rn, N), synth.dg(rn, N, 3.2), synth.dg(rn, N, 3.2), logq, 40)
    x = (limbs_of(cx.c0, logq)[None], limbs_of(cx.c1, logq)[None])
    y = (limbs_of(cy.c0, logq)[None], limbs_of(cy.c1, logq)[None])
    ctx = fhe.Context(logq, logP)
    try:
        k = fhe.EvalKey(ctx, fhe.CKKS, 0, logN, logq, logP, eb, ea)
        say("cfg3 encrypted: GPU")
        g0, g1 = _run(ctx, k, logN, logq, bits, x, y, 1)
        k.close()
    finally:
        ctx.close()
    with oracle_pool() as pool:
        say("cfg3 encrypted: oracle HE-mult")
        want = scheme.mult_rescale(cx, cy, evk, bits, mapper=pool.map)
    check(ints(g0[0]), want.c0, "c0")
    check(ints(g1[0]), want.c1, "c1")
    say("cfg3 encrypted: decrypt")
    z = scheme.ckks_decode(scheme.decrypt(want, s), N // 2, want.logp)
    err = float(np.max(np.abs(z - z1 * z2)))
    assert err <= 2.0 ** -20, err


@pytest.mark.parametrize("sch,t,logN,logQ,logq,logP,bits", [
    (scheme.BGV, 65537, 12, 400, 250, 300, 32),
    (scheme.BGV, 257, 11, 438, 97, 438, 5),
    (scheme.CKKS, 0, 12, 400, 218, 300, 40),
])
def test_he_mult_below_key_level(sch, t, logN, logQ, logq, logP, bits):
    """A key at logQ above the ciphertexts' logq: the library reduces it mod P 2^logq
    (R2); every coefficient against the oracle, fused and separate rescale."""
    say(f"below key level {sch} logN={logN} logQ={logQ} logq={logq}")
    N = 1 << logN
    rk, rm, _, _ = synth.streams(90 + logN)
    eb = synth.uniform_limbs(rk, logQ + logP, N)
    ea = synth.uniform_limbs(rk, logQ + logP, N)
    cnum = 2
    x = (synth.uniform_limbs(rm, logq, N, count=cnum), synth.uniform_limbs(rm, logq, N, count=cnum))
    y = (synth.uniform_limbs(rm, logq, N, count=cnum), synth.uniform_limbs(rm, logq, N, count=cnum))
    ctx = fhe.Context(logQ, logP)
    try:
        lsch = fhe.BGV if sch == scheme.BGV else fhe.CKKS
        k = fhe.EvalKey(ctx, lsch, t, logN, logQ, logP, eb, ea)
        g0, g1 = _run(ctx, k, logN, logq, bits, x, y, cnum)
        m0, m1 = _run(ctx, k, logN, logq, 0, x, y, cnum)
        k.close()
    finally:
        ctx.close()
    ok = scheme.EvalKey(ints(eb), ints(ea), logN, logQ, logP, sch, t)
    for c in range(cnum):
        ox = oracle_ct(x[0][c], x[1][c], logN, logq, sch, t)
        oy = oracle_ct(y[0][c], y[1][c], logN, logq, sch, t)
        m = scheme.mult(ox, oy, ok)
        check(ints(m0[c]), m.c0, f"relin c0[{c}]")
        check(ints(m1[c]), m.c1, f"relin c1[{c}]")
        r = scheme.rescale(m, bits)
        check(ints(g0[c]), r.c0, f"rescaled c0[{c}]")
        check(ints(g1[c]), r.c1, f"rescaled c1[{c}]")


def test_he_mult_logn15_per_op_and_autotuned_plan():
    """N = 2^15 (columns 2^8 x rows 2^7, or the other split when the autotuner picks it,
    with the key in its second layout): per-op and an autotuned graph plan of both
    schemes' jobs, every coefficient against the oracle."""
    import torch
    logN, logQ, logP = 15, 438, 438
    N = 1 << logN
    rk, rm, _, _ = synth.streams(15)
    ctx = fhe.Context(logQ, logP)
    try:
        cases = [(fhe.CKKS, 0, 218, 40), (fhe.BGV, 65537, 218, 32), (fhe.CKKS, 0, 438, 40)]
        jobs, data, klist = [], [], []
        for sch, t, logq, bits in cases:
            eb = synth.uniform_limbs(rk, logQ + logP, N)
            ea = synth.uniform_limbs(rk, logQ + logP, N)
            k = fhe.EvalKey(ctx, sch, t, logN, logQ, logP, eb, ea)
            klist.append(k)
            x = random_ct(rm, logN, logq)
            y = random_ct(rm, logN, logq)
            Lo = synth.nlimbs(logq - bits)
            outs = [torch.zeros(Lo * N, dtype=torch.int32, device="cuda") for _ in range(2)]
            jobs.append((k, logq, bits, *[dev(v) for v in x + y], *outs))
            data.append((sch, t, logq, bits, x, y, eb, ea))
        say("logN=15 per-op")
        per = []
        for (k, logq, bits, x0, x1, y0, y1, o0, o1) in jobs:
            a, b = torch.empty_like(o0), torch.empty_like(o1)
            ctx.mul_relin_rescale(k, logq, bits, x0, x1, y0, y1, a, b)
            per.append((a, b))
        say("logN=15 autotuned plan")
        plan = fhe.BatchPlan(ctx, jobs, flags=fhe.PLAN_GRAPH | fhe.PLAN_AUTOTUNE)
        for j in jobs:
            j[7].zero_()
            j[8].zero_()
        plan.run()
        torch.cuda.synchronize()
        plan.close()
        for (sch, t, logq, bits, x, y, eb, ea), j, (a, b) in zip(data, jobs, per):
            osch = scheme.BGV if sch == fhe.BGV else scheme.CKKS
            say(f"logN=15 oracle scheme={osch} logq={logq}")
            want = scheme.mult_rescale(oracle_ct(*x, logN, logq, osch, t), oracle_ct(*y, logN, logq, osch, t),
                                       scheme.EvalKey(ints(eb), ints(ea), logN, logQ, logP, osch, t), bits)
            Lo = synth.nlimbs(logq - bits)
            for got, what in ((a, "per-op c0"), (j[7], "plan c0")):
                check(ints(host(got, (Lo, N))), want.c0, what)
            for got, what in ((b, "per-op c1"), (j[8], "plan c1")):
                check(ints(host(got, (Lo, N))), want.c1, what)
        for k in klist:
            k.close()
    finally:
        ctx.close()


@pytest.mark.parametrize("cnum", [7, 8])
def test_he_mult_logn16_ciphertext_groups(cnum):
    """N = 2^16, logq = logP = 218: a CipherTensor of cnum pairs equals the same pairs
    run one at a time (one ciphertext per sub-row), and ciphertext 6 equals the oracle on
    every coefficient."""
    logN, logq, logP, bits = 16, 218, 218, 40
    N = 1 << logN
    rk, rm, _, _ = synth.streams(16 + cnum)
    eb = synth.uniform_limbs(rk, logq + logP, N)
    ea = synth.uniform_limbs(rk, logq + logP, N)
    x = (synth.uniform_limbs(rm, logq, N, count=cnum), synth.uniform_limbs(rm, logq, N, count=cnum))
    y = (synth.uniform_limbs(rm, logq, N, count=cnum), synth.uniform_limbs(rm, logq, N, count=cnum))
    ctx = fhe.Context(logq, logP)
    try:
        k = fhe.EvalKey(ctx, fhe.CKKS, 0, logN, logq, logP, eb, ea)
        say(f"logN=16 CipherTensor of {cnum}")
        g0, g1 = _run(ctx, k, logN, logq, bits, x, y, cnum)
        for c in range(cnum):
            say(f"logN=16 single ciphertext {c}")
            s0, s1 = _run(ctx, k, logN, logq, bits, tuple(v[c:c + 1] for v in x), tuple(v[c:c + 1] for v in y), 1)
            assert np.array_equal(g0[c], s0[0]) and np.array_equal(g1[c], s1[0]), f"ciphertext {c}"
        k.close()
    finally:
        ctx.close()
    say("logN=16 oracle, ciphertext 6")
    evk = scheme.EvalKey(ints(eb), ints(ea), logN, logq, logP, scheme.CKKS, 0)
    with oracle_pool(6) as pool:
        want = scheme.mult_rescale(oracle_ct(x[0][6], x[1][6], logN, logq, scheme.CKKS, 0),
                                   oracle_ct(y[0][6], y[1][6], logN, logq, scheme.CKKS, 0), evk, bits,
                                   mapper=pool.map)
    check(ints(g0[6]), want.c0, "c0[6]")
    check(ints(g1[6]), want.c1, "c1[6]")


def test_relin_reconstruction_table_in_global_memory():
    """logq = 1555 with logP = 4000: the relinearization product needs 238 primes and 174
    output limbs, whose reconstruction table (22 tiles x 8 k-blocks of 1 KiB) exceeds the
    LDS, so the reconstruction reads it from global memory.  N = 2^10, every coefficient
    against the oracle."""
    logN, logq, logP, bits = 10, 1555, 4000, 40
    N = 1 << logN
    rk, rm, _, _ = synth.streams(91)
    ctx = fhe.Context(logq, logP)
    try:
        assert ctx.primes_needed(logN, logq, logq + logP, 1) > 224
        eb = synth.uniform_limbs(rk, logq + logP, N)
        ea = synth.uniform_limbs(rk, logq + logP, N)
        x = random_ct(rm, logN, logq)
        y = random_ct(rm, logN, logq)
        k = fhe.EvalKey(ctx, fhe.CKKS, 0, logN, logq, logP, eb, ea)
        say("relin with the table in global memory")
        g0, g1 = _run(ctx, k, logN, logq, bits, (x[0][None], x[1][None]), (y[0][None], y[1][None]), 1)
        k.close()
    finally:
        ctx.close()
    want = scheme.mult_rescale(oracle_ct(*x, logN, logq, scheme.CKKS, 0), oracle_ct(*y, logN, logq, scheme.CKKS, 0),
                               scheme.EvalKey(ints(eb), ints(ea), logN, logq, logP), bits)
    check(ints(g0[0]), want.c0, "c0")
    check(ints(g1[0]), want.c1, "c1")
