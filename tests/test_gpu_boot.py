"""GPU: CKKS bootstrapping (fhe_ct_bootstrap) against the oracle's (oracle/boot.py).
The circuit is a fixed sequence of exact operations on the ciphertext, the keys and
the auxiliary inputs (encoded diagonals, integer constants), so the output must equal
the oracle's on every coefficient and metadata field; it must also decrypt to the input
slots within 2^-16 (N = 2^10, 4 slots at scale 2^30 encrypted at logq = 40, h = 64)."""
import numpy as np
import pytest

import paper_2607_05920_amd as fhe
import synth
from oracle import boot, galois, limbs, scheme
from tests.gpu_helpers import check, dev, host, ints, limbs_of, oracle_pool, say
from tests.test_oracle_boot import keys as oracle_keys

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(600)
def test_bootstrap_matches_oracle_and_decrypts():
    import torch
    assert torch.cuda.is_available()
    P = boot.BootParams(logN=10, logslots=2, logq_in=40, logQ=840)
    N, n = 1 << P.logN, 1 << P.logslots
    LQ = synth.nlimbs(P.logQ)
    say("bootstrap: oracle keys and encryption")
    rk, rm, rn, _ = synth.streams(31)
    s = synth.hwt(rk, N, 64)
    a = limbs.poly_from_limbs(synth.uniform_limbs(rk, P.logQ, N))
    pk = scheme.keygen_public(s, a, synth.dg(rk, N, 3.2), P.logQ)
    K = oracle_keys(P, s, rk, P.logQ)
    z = synth.unit_disk(rm, n)
    m = scheme.ckks_encode(z, N, 30)
    ct = scheme.encrypt(pk, m, synth.zo(rn, N), synth.dg(rn, N, 3.2), synth.dg(rn, N, 3.2), P.logq_in, 30)
    aux = boot.boot_aux(P)
    ctx = fhe.Context(P.logQ, P.logQ)
    try:
        kl = lambda k: (limbs_of(k.b, P.logQ + P.logQ), limbs_of(k.a, P.logQ + P.logQ))
        relin = fhe.EvalKey(ctx, fhe.CKKS, 0, P.logN, P.logQ, P.logQ, *kl(K.relin))
        rot = {r: fhe.EvalKey(ctx, fhe.CKKS, 0, P.logN, P.logQ, P.logQ, *kl(k), g=k.g) for r, k in K.rot.items()}
        conj = fhe.EvalKey(ctx, fhe.CKKS, 0, P.logN, P.logQ, P.logQ, *kl(K.conj), g=K.conj.g)
        Q = 1 << P.logQ
        diag = lambda ds: dev(np.stack([limbs_of([v % Q for v in d], P.logQ) for d in ds])).reshape(-1)
        c2s, s2c = diag(aux.c2s), diag(aux.s2c)
        x = fhe.Ciphertext(dev(limbs_of(ct.c0, P.logq_in)).reshape(-1), dev(limbs_of(ct.c1, P.logq_in)).reshape(-1),
                           P.logN, P.logq_in, 30, fhe.CKKS, 0, 1, 1)
        out = (torch.zeros(LQ * N, dtype=torch.int32, device="cuda"),
               torch.zeros(LQ * N, dtype=torch.int32, device="cuda"))
        params = dict(logN=P.logN, logslots=P.logslots, logq_in=P.logq_in, logQ=P.logQ, logc=P.logc, logT=P.logT,
                      degree=P.degree)
        say("bootstrap: GPU")
        got = ctx.ct_bootstrap(params, relin, rot, conj, c2s, s2c, aux.k_y, aux.taylor, x, out)
        torch.cuda.synchronize()
        for k in [relin, conj, *rot.values()]:
            k.close()
    finally:
        ctx.close()
    say("bootstrap: oracle")
    with oracle_pool(8) as pool:
        want = boot.bootstrap(ct, P, aux, K, mapper=pool.map)
    assert (got.logN, got.logq, got.logp, got.cnum) == (want.logN, want.logq, want.logp, 1)
    L = synth.nlimbs(got.logq)
    check(ints(host(got.c0, (-1, N))[:L]), want.c0, "c0")
    check(ints(host(got.c1, (-1, N))[:L]), want.c1, "c1")
    zz = scheme.ckks_decode(scheme.decrypt(want, s), n, want.logp)
    assert float(np.max(np.abs(zz - z))) < 2.0 ** -16
