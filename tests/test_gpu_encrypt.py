"""GPU: the encryption / decryption helpers of the C ABI against the oracle (bit
exact), the standalone NTT in natural order over a prime offset, and whole
round trips that run every device step through the library: encode (host) ->
encrypt -> HE-mult + relin + rescale -> decrypt -> decode (host)."""
import numpy as np
import pytest

import paper_2607_05920_amd as fhe
import synth
from oracle import ntt as ontt
from oracle import ring, scheme
from tests.gpu_helpers import check, dev, host, ints, keys, limbs_of, say

pytestmark = pytest.mark.gpu

LSCH = {scheme.CKKS: fhe.CKKS, scheme.BGV: fhe.BGV}


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = fhe.Context(438, 438)
    yield c
    c.close()


def _small(arr, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(arr, dtype=dtype))).cuda()


def _message(rng, sch, t, N, logq):
    if sch == scheme.CKKS:
        return scheme.ckks_encode(synth.unit_disk(rng, N // 2), N, 40)
    return [int(v) for v in synth.uniform_mod(rng, N, t)]


@pytest.mark.parametrize("sch,t,logN,logQ,logq", [(scheme.CKKS, 0, 10, 300, 200), (scheme.BGV, 65537, 10, 200, 200),
                                                  (scheme.BGV, 1001, 11, 160, 64), (scheme.CKKS, 0, 12, 97, 33)])
def test_encrypt_decrypt_bit_exact(ctx, sch, t, logN, logQ, logq):
    """pk at logQ >= logq (its low rows are the key mod Q_l); c0, c1 and the phase
    equal the oracle's on every coefficient; BGV messages decode exactly."""
    import torch
    say(f"encrypt {sch} t={t} logN={logN} logq={logq}")
    rk, rm, rn, _ = synth.streams(60 + logN)
    N = 1 << logN
    s, pk, _, _, _ = keys(rk, logN, logQ, 20, sch, t, h=64)
    m = _message(rm, sch, t, N, logq)
    v, e0, e1 = synth.zo(rn, N), synth.dg(rn, N, 3.2), synth.dg(rn, N, 3.2)
    want = scheme.encrypt(pk, m, v, e0, e1, logq)
    L = synth.nlimbs(logq)
    Q = 1 << logq
    c0 = torch.empty(L * N, dtype=torch.int32, device="cuda")
    c1 = torch.empty_like(c0)
    ctx.encrypt(LSCH[sch], t, logN, logq, dev(limbs_of(pk.b, logQ)), dev(limbs_of(pk.a, logQ)),
                dev(limbs_of([x % Q for x in m], logq)), _small(v, np.int8), _small(e0, np.int32),
                _small(e1, np.int32), c0, c1)
    torch.cuda.synchronize()
    check(ints(host(c0, (L, N))), want.c0, "c0")
    check(ints(host(c1, (L, N))), want.c1, "c1")
    if sch == scheme.CKKS:
        ph = torch.empty(L * N, dtype=torch.int32, device="cuda")
        ctx.decrypt(fhe.CKKS, 0, 1, logN, logq, c0, c1, _small(s, np.int8), ph)
        torch.cuda.synchronize()
        check(ints(host(ph, (L, N))), scheme.phase(want, s), "phase")
    else:
        gamma = pow(2, -20, t)   # any invertible factor: decoding multiplies by its inverse
        out = torch.empty(N, dtype=torch.int32, device="cuda")
        ctx.decrypt(fhe.BGV, t, gamma, logN, logq, c0, c1, _small(s, np.int8), out)
        torch.cuda.synchronize()
        check(fhe.to_host(out).tolist(), scheme.bgv_decode(scheme.decrypt(want, s), t, gamma), "message")
        ctx.decrypt(fhe.BGV, t, 1, logN, logq, c0, c1, _small(s, np.int8), out)
        torch.cuda.synchronize()
        check(fhe.to_host(out).tolist(), m, "message (gamma 1)")


@pytest.mark.parametrize("sch,t,bits", [(scheme.CKKS, 0, 40), (scheme.BGV, 65537, 32)])
def test_round_trip_through_the_library(ctx, sch, t, bits):
    """N = 2^13, logq = logP = 438: every device step in the library, decrypting to
    z1 z2 within 2^-20 (CKKS, scale 2^40) or to m1 m2 mod t exactly (BGV)."""
    import torch
    say(f"round trip {sch}")
    rk, rm, rn, _ = synth.streams(70)
    logN, logq, logP = 13, 438, 438
    N = 1 << logN
    L = synth.nlimbs(logq)
    s, pk, _, eb, ea = keys(rk, logN, logq, logP, sch, t, h=192)
    evk = fhe.EvalKey(ctx, LSCH[sch], t, logN, logq, logP, eb, ea)
    if sch == scheme.CKKS:
        z = [synth.unit_disk(rm, N // 2) for _ in range(2)]
        ms = [fhe.ckks_encode(zz, logN, 40, logq) for zz in z]
    else:
        mi = [[int(v) for v in synth.uniform_mod(rm, N, t)] for _ in range(2)]
        ms = [limbs_of(mm, logq) for mm in mi]
    cts = []
    for mm in ms:
        c0 = torch.empty(L * N, dtype=torch.int32, device="cuda")
        c1 = torch.empty_like(c0)
        ctx.encrypt(LSCH[sch], t, logN, logq, dev(limbs_of(pk.b, logq)), dev(limbs_of(pk.a, logq)), dev(mm),
                    _small(synth.zo(rn, N), np.int8), _small(synth.dg(rn, N, 3.2), np.int32),
                    _small(synth.dg(rn, N, 3.2), np.int32), c0, c1)
        cts.append((c0, c1))
    Lo = synth.nlimbs(logq - bits)
    o0 = torch.empty(Lo * N, dtype=torch.int32, device="cuda")
    o1 = torch.empty_like(o0)
    ctx.mul_relin_rescale(evk, logq, bits, cts[0][0], cts[0][1], cts[1][0], cts[1][1], o0, o1)
    sd = _small(s, np.int8)
    if sch == scheme.CKKS:
        ph = torch.empty(Lo * N, dtype=torch.int32, device="cuda")
        ctx.decrypt(fhe.CKKS, 0, 1, logN, logq - bits, o0, o1, sd, ph)
        torch.cuda.synchronize()
        got = fhe.ckks_decode(host(ph, (Lo, N)), logN, logN - 1, 80 - bits, logq - bits)
        assert np.max(np.abs(got - z[0] * z[1])) <= 2.0 ** -20
    else:
        out = torch.empty(N, dtype=torch.int32, device="cuda")
        ctx.decrypt(fhe.BGV, t, pow(2, -bits, t), logN, logq - bits, o0, o1, sd, out)
        torch.cuda.synchronize()
        check(fhe.to_host(out).tolist(), ring.ring_mul(mi[0], mi[1], t), "m1 m2")
    evk.close()


@pytest.mark.parametrize("logN,prime0,nprimes,count", [(10, 5, 3, 2), (13, 0, 2, 1), (16, 40, 2, 1)])
def test_ntt_natural_order_prime_offset(ctx, logN, prime0, nprimes, count):
    """Natural-order forward = Eq. negacyclic_ntt position by position over primes
    prime0.. (the oracle's transform with that prime's root); inverse restores."""
    import torch
    say(f"ntt natural logN={logN} prime0={prime0}")
    N = 1 << logN
    rng = np.random.default_rng(logN + prime0)
    data = np.zeros((count, nprimes, N), dtype=np.uint32)
    for p in range(nprimes):
        data[:, p] = rng.integers(0, ctx.prime_info(prime0 + p)[0], (count, N), dtype=np.uint64)
    t = dev(data)
    ctx.ntt(logN, nprimes, t, count=count, prime0=prime0)
    fwd = host(t, (count, nprimes, N))
    for c in range(count):
        for p in range(nprimes):
            q, psi_max = ctx.prime_info(prime0 + p)
            psi = pow(psi_max, (1 << 16) // N, q)
            check([int(x) for x in fwd[c, p]], ontt.ntt_fast([int(x) for x in data[c, p]], q, psi), f"ntt {c} {p}")
    ctx.ntt(logN, nprimes, t, count=count, inverse=True, prime0=prime0)
    torch.cuda.synchronize()
    assert np.array_equal(host(t, (count, nprimes, N)), data)
    with pytest.raises(fhe.FheError):
        ctx.ntt(logN, 1, t, prime0=ctx.prime_count())
