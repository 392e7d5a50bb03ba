"""Shared helpers for the GPU parity tests (oracle side + device marshalling)."""
import sys

import numpy as np

import paper_2607_05920_amd as fhe
import synth
from oracle import limbs as olimbs
from oracle import scheme


def say(msg: str):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def dev(arr):
    return fhe.to_device(arr)


def host(t, shape):
    return fhe.to_host(t).reshape(shape)


def ints(arr):
    return olimbs.poly_from_limbs(arr)


def limbs_of(coeffs, bits):
    return olimbs.poly_to_limbs(coeffs, synth.nlimbs(bits))


def random_ct(rng, logN, logq):
    """A uniformly random ciphertext (c0, c1) as limb arrays uint32[L][N]."""
    N = 1 << logN
    return synth.uniform_limbs(rng, logq, N), synth.uniform_limbs(rng, logq, N)


def oracle_ct(c0, c1, logN, logq, sch, t):
    return scheme.Ciphertext(ints(c0), ints(c1), logN, logq, scheme=sch, t=t)


def keys(rk, logN, logQ, logP, sch, t, h):
    """Oracle keygen with explicit randomness; returns s, pk, evk and evk limbs."""
    N = 1 << logN
    s = synth.hwt(rk, N, h)
    a = ints(synth.uniform_limbs(rk, logQ, N))
    pk = scheme.keygen_public(s, a, synth.dg(rk, N, 3.2), logQ, sch, t)
    a2 = ints(synth.uniform_limbs(rk, logQ + logP, N))
    evk = scheme.keygen_relin(s, a2, synth.dg(rk, N, 3.2), logQ, logP, sch, t)
    return s, pk, evk, limbs_of(evk.b, logQ + logP), limbs_of(evk.a, logQ + logP)


def check(got, want, what: str = "values"):
    """Element-by-element equality of two sequences, failing with the count and the
    first mismatching positions (a plain `assert list == list` on 10^4 big integers
    makes pytest build a quadratic diff that runs for minutes)."""
    got, want = list(got), list(want)
    if got == want:
        return
    if len(got) != len(want):
        raise AssertionError(f"{what}: length {len(got)} != {len(want)}")
    bad = [i for i, (a, b) in enumerate(zip(got, want)) if a != b]
    first = ", ".join(f"[{i}] {str(got[i])[:24]} != {str(want[i])[:24]}" for i in bad[:4])
    raise AssertionError(f"{what}: {len(bad)} of {len(want)} differ; first: {first}")


def oracle_pool(workers: int = 12):
    """A process pool for the oracle's independent ring products (its ``map`` is the
    ``mapper`` argument of oracle.scheme).  Workers are fresh interpreters (spawn):
    they run only the pure-Python oracle and never touch the GPU."""
    import multiprocessing
    import os
    from concurrent.futures import ProcessPoolExecutor
    n = max(1, min(workers, os.cpu_count() or 1))
    return ProcessPoolExecutor(max_workers=n, mp_context=multiprocessing.get_context("spawn"))
