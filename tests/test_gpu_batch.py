"""GPU: batched uneven HE-mults (fhe_batch_plan / fhe_batch_run) against per-op calls
and the oracle: cell pipelines and stage-batched launches (FHE_PLAN_QUEUE), eager and
graph-captured, with the autotuner on and off."""
import numpy as np
import pytest

import paper_2607_05920_amd as fhe
import synth
from oracle import scheme
from tests.gpu_helpers import check, dev, host, ints, oracle_ct, say

pytestmark = pytest.mark.gpu

LOGQ_TOP = LOGP = 438


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available()
    say("batch setup")
    ctx = fhe.Context(LOGQ_TOP, LOGP)
    rk, rm, _, rs = synth.streams(4)
    keys, khost = {}, {}
    for logN in (13, 14, 15, 16):
        N = 1 << logN
        eb = synth.uniform_limbs(rk, LOGQ_TOP + LOGP, N)
        ea = synth.uniform_limbs(rk, LOGQ_TOP + LOGP, N)
        keys[logN] = fhe.EvalKey(ctx, fhe.CKKS, 0, logN, LOGQ_TOP, LOGP, eb, ea)
        khost[logN] = (eb, ea)
    # 14 jobs over 8 cells: every logN with logq 218 and 438, some cells repeated
    shapes = [(13, 218), (14, 438), (15, 218), (16, 438), (13, 438), (14, 218), (15, 438), (16, 218),
              (13, 218), (16, 438), (14, 438), (13, 218), (15, 218), (16, 218)]
    jobs, data = [], []
    for logN, logq in shapes:
        N = 1 << logN
        x = [synth.uniform_limbs(rm, logq, N) for _ in range(2)]
        y = [synth.uniform_limbs(rm, logq, N) for _ in range(2)]
        Lo = synth.nlimbs(logq - 40)
        outs = [torch.zeros(Lo * N, dtype=torch.int32, device="cuda") for _ in range(2)]
        ins = [dev(v) for v in x + y]
        jobs.append((keys[logN], logq, 40, *ins, *outs))
        data.append((logN, logq, x, y))
    yield ctx, keys, khost, jobs, data
    for k in keys.values():
        k.close()
    ctx.close()


def per_op(ctx, jobs):
    import torch
    res = []
    for (evk, logq, bits, x0, x1, y0, y1, o0, o1) in jobs:
        a, b = torch.empty_like(o0), torch.empty_like(o1)
        ctx.mul_relin_rescale(evk, logq, bits, x0, x1, y0, y1, a, b)
        res.append((a, b))
    torch.cuda.synchronize()
    return res


@pytest.mark.parametrize("flags", [0, fhe.PLAN_GRAPH, fhe.PLAN_GRAPH | fhe.PLAN_AUTOTUNE, fhe.PLAN_QUEUE,
                                   fhe.PLAN_QUEUE | fhe.PLAN_GRAPH,
                                   fhe.PLAN_QUEUE | fhe.PLAN_GRAPH | fhe.PLAN_AUTOTUNE])
def test_batch_equals_per_op(setup, flags):
    import torch
    ctx, keys, khost, jobs, data = setup
    say(f"batch flags={flags}")
    ref = per_op(ctx, jobs)
    for j in jobs:
        j[7].zero_()
        j[8].zero_()
    plan = fhe.BatchPlan(ctx, jobs, flags=flags)
    info = plan.info()
    assert info["cells"] == 8 and info["graphed"] == bool(flags & fhe.PLAN_GRAPH)
    if flags & fhe.PLAN_QUEUE:
        # 11 pipeline steps, each one launch per kernel variant in use: far fewer than
        # the 8 cells' 88 launches
        assert 11 <= info["kernels"] < 8 * 11, info
    for rep in range(3):
        for j in jobs:           # eager work between replays
            j[7].fill_(rep + 1)
            j[8].fill_(-rep)
        plan.run()
        torch.cuda.synchronize()
        for (j, (a, b)) in zip(jobs, ref):
            assert torch.equal(j[7], a) and torch.equal(j[8], b)
    plan.close()


@pytest.mark.parametrize("flags", [fhe.PLAN_GRAPH, fhe.PLAN_QUEUE | fhe.PLAN_GRAPH])
def test_batch_sampled_jobs_match_oracle(setup, flags):
    import torch
    ctx, keys, khost, jobs, data = setup
    say(f"batch vs oracle flags={flags}")
    for j in jobs:
        j[7].zero_()
        j[8].zero_()
    plan = fhe.BatchPlan(ctx, jobs, flags=flags)
    plan.run()
    torch.cuda.synchronize()
    for i in (0, 5):   # (13, 218) and (14, 218): full oracle products are cheap
        logN, logq, x, y = data[i]
        N = 1 << logN
        eb, ea = khost[logN]
        evk = scheme.EvalKey(ints(eb), ints(ea), logN, LOGQ_TOP, LOGP)
        want = scheme.mult_rescale(oracle_ct(*x, logN, logq, scheme.CKKS, 0), oracle_ct(*y, logN, logq, scheme.CKKS, 0),
                                   evk, 40)
        Lo = synth.nlimbs(logq - 40)
        check(ints(host(jobs[i][7], (Lo, N))), want.c0, f"job {i} c0")
        check(ints(host(jobs[i][8], (Lo, N))), want.c1, f"job {i} c1")
    plan.close()


def test_stage_batched_both_schemes_and_levels():
    """Stage-batched plans (eager and graph) over CKKS and BGV cells at logN 13 and 14,
    levels 218 and 438 under a key at 438, rescale 0, 7 and 40 bits: bit-identical to
    per-op calls; one BGV job against the oracle on every coefficient."""
    import torch
    logQ = logP = 438
    rk, rm, _, _ = synth.streams(21)
    ctx = fhe.Context(logQ, logP)
    try:
        keys, khost = {}, {}
        for sch, t in ((fhe.CKKS, 0), (fhe.BGV, 65537)):
            for logN in (13, 14):
                N = 1 << logN
                eb = synth.uniform_limbs(rk, logQ + logP, N)
                ea = synth.uniform_limbs(rk, logQ + logP, N)
                keys[(sch, logN)] = fhe.EvalKey(ctx, sch, t, logN, logQ, logP, eb, ea)
                khost[(sch, logN)] = (eb, ea)
        shapes = [(fhe.CKKS, 13, 218, 40), (fhe.BGV, 14, 438, 7), (fhe.BGV, 13, 218, 0), (fhe.CKKS, 14, 438, 40),
                  (fhe.BGV, 14, 438, 7), (fhe.CKKS, 13, 438, 0), (fhe.BGV, 13, 218, 0)]
        jobs, data = [], []
        for sch, logN, logq, bits in shapes:
            N = 1 << logN
            x = [synth.uniform_limbs(rm, logq, N) for _ in range(2)]
            y = [synth.uniform_limbs(rm, logq, N) for _ in range(2)]
            Lo = synth.nlimbs(logq - bits)
            outs = [torch.zeros(Lo * N, dtype=torch.int32, device="cuda") for _ in range(2)]
            jobs.append((keys[(sch, logN)], logq, bits, *[dev(v) for v in x + y], *outs))
            data.append((sch, logN, logq, bits, x, y))
        say("stage-batched both schemes: per-op reference")
        ref = []
        for (evk, logq, bits, x0, x1, y0, y1, o0, o1) in jobs:
            a, b = torch.empty_like(o0), torch.empty_like(o1)
            if bits:
                ctx.mul_relin_rescale(evk, logq, bits, x0, x1, y0, y1, a, b)
            else:
                ctx.mul_relin(evk, logq, x0, x1, y0, y1, a, b)
            ref.append((a, b))
        torch.cuda.synchronize()
        for flags in (fhe.PLAN_QUEUE, fhe.PLAN_QUEUE | fhe.PLAN_GRAPH):
            say(f"stage-batched both schemes flags={flags}")
            for j in jobs:
                j[7].zero_()
                j[8].zero_()
            plan = fhe.BatchPlan(ctx, jobs, flags=flags)
            assert plan.info()["cells"] == 5
            for _ in range(2):
                plan.run()
                torch.cuda.synchronize()
                for (j, (a, b)) in zip(jobs, ref):
                    assert torch.equal(j[7], a) and torch.equal(j[8], b)
            plan.close()
        sch, logN, logq, bits, x, y = data[1]
        N = 1 << logN
        eb, ea = khost[(sch, logN)]
        say("stage-batched both schemes: oracle, BGV job 1")
        evk = scheme.EvalKey(ints(eb), ints(ea), logN, logQ, logP, scheme.BGV, 65537)
        want = scheme.mult_rescale(oracle_ct(*x, logN, logq, scheme.BGV, 65537),
                                   oracle_ct(*y, logN, logq, scheme.BGV, 65537), evk, bits)
        Lo = synth.nlimbs(logq - bits)
        check(ints(host(jobs[1][7], (Lo, N))), want.c0, "BGV job 1 c0")
        check(ints(host(jobs[1][8], (Lo, N))), want.c1, "BGV job 1 c1")
        for k in keys.values():
            k.close()
    finally:
        ctx.close()
