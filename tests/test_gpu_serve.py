"""GPU: the continuous-batching request loop (fhe_server_*).  Every served result must
equal the same request computed alone (tolerance 0: exact arithmetic), under
Poisson arrivals over mixed CKKS/BGV cells; admission by HBM footprint rejects what
cannot fit and throttles what can."""
import numpy as np
import pytest

import paper_2607_05920_amd as fhe
import synth
from oracle import scheme
from tests.gpu_helpers import check, dev, host, ints, oracle_ct, oracle_pool, say

pytestmark = pytest.mark.gpu

LOGQ, LOGP = 438, 438


@pytest.fixture(scope="module")
def world():
    import torch
    assert torch.cuda.is_available()
    say("serve setup")
    ctx = fhe.Context(LOGQ, LOGP)
    rk, rm, _, rs = synth.streams(5)
    keys, khost = {}, {}
    for sch, t in ((fhe.CKKS, 0), (fhe.BGV, 65537)):
        for logN in (13, 14):
            N = 1 << logN
            kb, ka = synth.uniform_limbs(rk, LOGQ + LOGP, N), synth.uniform_limbs(rk, LOGQ + LOGP, N)
            keys[(sch, logN)] = fhe.EvalKey(ctx, sch, t, logN, LOGQ, LOGP, kb, ka)
            khost[(sch, logN)] = (kb, ka)
    reqs, inputs = [], []
    for i in range(96):
        sch = fhe.CKKS if rs.random() < 0.7 else fhe.BGV
        logN = int(rs.integers(13, 15))
        logq = int(rs.choice([218, 438]))
        bits = 40 if sch == fhe.CKKS else 32
        N = 1 << logN
        hin = [synth.uniform_limbs(rm, logq, N) for _ in range(4)]
        ins = [dev(v) for v in hin]
        Lo = synth.nlimbs(logq - bits)
        outs = [torch.zeros(Lo * N, dtype=torch.int32, device="cuda") for _ in range(2)]
        reqs.append((keys[(sch, logN)], logq, bits, *ins, *outs))
        inputs.append((sch, logN, logq, bits, hin))
    # every key level used, prepared outside the loop
    for (evk, logq, *_rest) in reqs:
        evk.prepare(logq)
    # results alone
    alone = []
    for (evk, logq, bits, x0, x1, y0, y1, o0, o1) in reqs:
        a, b = torch.empty_like(o0), torch.empty_like(o1)
        ctx.mul_relin_rescale(evk, logq, bits, x0, x1, y0, y1, a, b)
        alone.append((a, b))
    torch.cuda.synchronize()
    yield ctx, reqs, alone, (khost, inputs)
    for k in keys.values():
        k.close()
    ctx.close()


def serve(ctx, reqs, budget, nstreams, max_batch, rate=None, seed=1):
    """Queues `reqs` with scheduled arrival times (a burst, or Poisson at `rate`/s)
    and returns the completion records once all are done."""
    srv = fhe.Server(ctx, budget, nstreams=nstreams, max_batch=max_batch)
    rng = np.random.default_rng(seed)
    t0 = fhe.clock_ns() + 20_000_000
    gaps = np.zeros(len(reqs)) if rate is None else rng.exponential(1e9 / rate, len(reqs))
    for r, ta in zip(reqs, t0 + np.cumsum(gaps).astype(np.int64)):
        srv.submit(r, int(ta))
    srv.drain()
    done = srv.poll(4096)
    srv.close()
    return done


def _clear(reqs):
    import torch
    for (*_, o0, o1) in reqs:
        o0.zero_()
        o1.zero_()
    torch.cuda.synchronize()   # the server's streams do not wait for torch's stream


def _same(reqs, alone):
    import torch
    return all(torch.equal(o0, a) and torch.equal(o1, b) for (*_, o0, o1), (a, b) in zip(reqs, alone))


def test_served_equals_alone_under_poisson_arrivals(world):
    ctx, reqs, alone, _ = world
    say("serve poisson")
    _clear(reqs)
    done = serve(ctx, reqs, budget=8 << 30, nstreams=4, max_batch=8, rate=20000.0)
    assert len(done) == len(reqs) and all(d.status == 0 for d in done)
    assert sorted(d.ticket for d in done) == list(range(1, len(reqs) + 1))
    assert all(d.t_done >= d.t_start >= d.t_arrive for d in done)
    assert _same(reqs, alone)


def test_burst_is_batched_by_cell(world):
    ctx, reqs, alone, _ = world
    say("serve burst")
    _clear(reqs)
    done = serve(ctx, reqs, budget=8 << 30, nstreams=4, max_batch=8)
    assert all(d.status == 0 for d in done)
    assert max(d.batch for d in done) > 1            # requests queued behind running batches were merged
    assert max(d.batch for d in done) <= 8
    assert _same(reqs, alone)


def test_admission_tight_budget_and_rejection(world):
    ctx, reqs, alone, _ = world
    say("serve budget")
    _clear(reqs)
    # a logN=14, logq=438 request holds about 25 MB of scratch: at most two fit in 60 MB
    done = serve(ctx, reqs, budget=60 << 20, nstreams=4, max_batch=8)
    assert len(done) == len(reqs) and all(d.status == 0 for d in done)
    big = {i + 1 for i, r in enumerate(reqs) if r[0].logN == 14 and r[1] == 438}
    assert big and max(d.batch for d in done if d.ticket in big) <= 2
    assert _same(reqs, alone)
    done = serve(ctx, reqs[:8], budget=1 << 20, nstreams=2, max_batch=4)
    assert len(done) == 8 and all(d.status == -4 for d in done)


def test_served_sample_matches_oracle(world):
    """A seeded sample of served requests against the oracle on every coefficient: both
    schemes, both ring degrees, both levels (logq = 218 runs with the key above its
    level), served under Poisson arrivals with batching."""
    import torch
    ctx, reqs, alone, (khost, inputs) = world
    say("serve vs oracle")
    _clear(reqs)
    done = serve(ctx, reqs, budget=8 << 30, nstreams=4, max_batch=8, rate=20000.0, seed=7)
    assert len(done) == len(reqs) and all(d.status == 0 for d in done)
    # one request of every (scheme, logN, logq) cell present, plus a few more by seed
    pick, seen = [], set()
    for i, (sch, logN, logq, bits, _) in enumerate(inputs):
        if (sch, logN, logq) not in seen:
            seen.add((sch, logN, logq))
            pick.append(i)
    rest = [i for i in range(len(reqs)) if i not in pick]
    pick += [int(i) for i in np.random.default_rng(11).choice(rest, 4, replace=False)]
    assert {(inputs[i][0], inputs[i][1]) for i in pick} == {(s, n) for s in (fhe.CKKS, fhe.BGV) for n in (13, 14)}
    with oracle_pool() as pool:
        for i in pick:
            sch, logN, logq, bits, hin = inputs[i]
            osch, t = (scheme.BGV, 65537) if sch == fhe.BGV else (scheme.CKKS, 0)
            say(f"serve vs oracle: request {i} scheme={osch} logN={logN} logq={logq}")
            kb, ka = khost[(sch, logN)]
            want = scheme.mult_rescale(oracle_ct(hin[0], hin[1], logN, logq, osch, t),
                                       oracle_ct(hin[2], hin[3], logN, logq, osch, t),
                                       scheme.EvalKey(ints(kb), ints(ka), logN, LOGQ, LOGP, osch, t), bits,
                                       mapper=pool.map)
            N = 1 << logN
            Lo = synth.nlimbs(logq - bits)
            check(ints(host(reqs[i][7], (Lo, N))), want.c0, f"request {i} c0")
            check(ints(host(reqs[i][8], (Lo, N))), want.c1, f"request {i} c1")
