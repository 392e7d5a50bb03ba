"""GPU: the continuous-batching request loop (fhe_server_*).  Every served result must
equal the same request computed alone (tolerance 0: exact arithmetic), under
Poisson arrivals over mixed CKKS/BGV cells; admission by HBM footprint rejects what
cannot fit and throttles what can."""
import numpy as np
import pytest

import paper_2607_05920_amd as fhe
import synth
from tests.gpu_helpers import dev, say

pytestmark = pytest.mark.gpu

LOGQ, LOGP = 438, 438


@pytest.fixture(scope="module")
def world():
    import torch
    assert torch.cuda.is_available()
    say("serve setup")
    ctx = fhe.Context(LOGQ, LOGP)
    rk, rm, _, rs = synth.streams(5)
    keys = {}
    for sch, t in ((fhe.CKKS, 0), (fhe.BGV, 65537)):
        for logN in (13, 14):
            N = 1 << logN
            keys[(sch, logN)] = fhe.EvalKey(ctx, sch, t, logN, LOGQ, LOGP, synth.uniform_limbs(rk, LOGQ + LOGP, N),
                                            synth.uniform_limbs(rk, LOGQ + LOGP, N))
    reqs = []
    for i in range(96):
        sch = fhe.CKKS if rs.random() < 0.7 else fhe.BGV
        logN = int(rs.integers(13, 15))
        logq = int(rs.choice([218, 438]))
        bits = 40 if sch == fhe.CKKS else 32
        N = 1 << logN
        ins = [dev(synth.uniform_limbs(rm, logq, N)) for _ in range(4)]
        Lo = synth.nlimbs(logq - bits)
        outs = [torch.zeros(Lo * N, dtype=torch.int32, device="cuda") for _ in range(2)]
        reqs.append((keys[(sch, logN)], logq, bits, *ins, *outs))
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
    yield ctx, reqs, alone
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
    ctx, reqs, alone = world
    say("serve poisson")
    _clear(reqs)
    done = serve(ctx, reqs, budget=8 << 30, nstreams=4, max_batch=8, rate=20000.0)
    assert len(done) == len(reqs) and all(d.status == 0 for d in done)
    assert sorted(d.ticket for d in done) == list(range(1, len(reqs) + 1))
    assert all(d.t_done >= d.t_start >= d.t_arrive for d in done)
    assert _same(reqs, alone)


def test_burst_is_batched_by_cell(world):
    ctx, reqs, alone = world
    say("serve burst")
    _clear(reqs)
    done = serve(ctx, reqs, budget=8 << 30, nstreams=4, max_batch=8)
    assert all(d.status == 0 for d in done)
    assert max(d.batch for d in done) > 1            # requests queued behind running batches were merged
    assert max(d.batch for d in done) <= 8
    assert _same(reqs, alone)


def test_admission_tight_budget_and_rejection(world):
    ctx, reqs, alone = world
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
