"""GPU: the allocation-free ring multiply (fhe_ring_mul_noalloc), through the C ABI,
against the allocating entry point (fhe_ring_mul) bit for bit: two calls in a row, the
second with a smaller input, then a call beyond the fixed scratch (refused) and a shape
whose tables were never built (refused).  Runs alone in a fresh process and after the
other tests (it creates its own context)."""
import numpy as np
import pytest

import paper_2607_05920_amd as fhe
import synth
from tests.gpu_helpers import dev, say

pytestmark = pytest.mark.gpu


def _pair(rng, logN, logq, cnum):
    N = 1 << logN
    a = dev(synth.uniform_limbs(rng, logq, N, count=cnum)).reshape(-1)
    b = dev(synth.uniform_limbs(rng, logq, N, count=cnum)).reshape(-1)
    return a, b


def test_ring_mul_noalloc_equals_ring_mul():
    import torch
    assert torch.cuda.is_available()
    ctx = fhe.Context(1555, 1555)
    try:
        rng = np.random.default_rng(2024)
        shapes = [(16, 1555, 1), (12, 300, 3)]   # the second call is smaller
        for logN, logq, cnum in shapes:
            say(f"no-alloc ring multiply logN={logN} logq={logq} cnum={cnum}")
            a, b = _pair(rng, logN, logq, cnum)
            want = torch.empty_like(a)
            ctx.ring_mul(logN, logq, a, b, want, cnum=cnum)       # also builds the tables of this shape
            got = torch.full_like(a, -1)
            ctx.ring_mul_noalloc(logN, logq, a, b, got, cnum=cnum)
            torch.cuda.synchronize()
            assert torch.equal(got, want), f"logN={logN} logq={logq}"
        # beyond the 16 Mi-word scratch: 2 cnum K N words with K = 106 at N = 2^16
        a, b = _pair(rng, 16, 1555, 2)
        out = torch.empty_like(a)
        with pytest.raises(fhe.FheError) as ei:
            ctx.ring_mul_noalloc(16, 1555, a, b, out, cnum=2)
        assert ei.value.status == -3
        # a shape whose tables were never built is refused rather than built
        a, b = _pair(rng, 11, 97, 1)
        out = torch.empty_like(a)
        with pytest.raises(fhe.FheError) as ei:
            ctx.ring_mul_noalloc(11, 97, a, b, out)
        assert ei.value.status == -6
    finally:
        ctx.close()
