#!/usr/bin/env python3
"""Throughput of homomorphic multiplication (tensor + relinearization + rescale) on one
MI355X, at N = 2^16, logq = 1555, logP = 1555 (CKKS, rescale by 40 bits).

One step = one HE-mult + relin + rescale of a CipherTensor of ``--cnum`` ciphertext
pairs (default 4, the paper's CipherTensor size) through the C ABI.  Inputs are
seeded synthetic ciphertexts and key, uniform in [0, 2^logq) / [0, 2^(logP+logq))
(the distribution of real RLWE ciphertexts), resident in HBM before timing starts.

Prints one JSON line: the metric, the per-op comparison (cnum = 1 per launch), the
roofline of the dominant kernel from HIP events recorded on the launch stream over
the timed region, standalone NTT throughput, and the CPU oracle's rate on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

LOGN, LOGQ, LOGP, BITS = 16, 1555, 1555, 40
PEAK_PRODUCTS = 256 * 64 * 2.4e9  # 32x32-bit products per second: 256 CUs x 64 lanes x 2.4 GHz
PEAK_HBM = 8.0e12                  # bytes per second
PEAK_MFMA_I8 = 5.0e15              # dense int8 matrix-core operations per second
# The library reports each kernel's algorithmic work as HBM bytes (what it must read
# and write at least once); every kernel class is reported against the HBM peak.
ALU_KERNELS = set()
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_n16_q1555_cnum4.json")


def device_code_hash() -> str:
    """SHA-256 of the device code the library carries (its `.hip_fatbin` ELF section,
    the gfx950 code objects).  The build is deterministic: edits that change no kernel
    (comments, host code) keep it; any kernel change alters it."""
    import hashlib
    import struct
    try:
        with open(os.path.join(ROOT, "paper_2607_05920_amd", "libfhe_mi355x.so"), "rb") as f:
            b = f.read()
    except OSError:
        return ""
    if b[:4] != b"\x7fELF" or b[4] != 2:
        return ""
    shoff, = struct.unpack_from("<Q", b, 0x28)
    shentsize, shnum, shstrndx = struct.unpack_from("<HHH", b, 0x3A)

    def header(i):  # (name offset, type, flags, addr, file offset, size, ...)
        return struct.unpack_from("<IIQQQQIIQQ", b, shoff + i * shentsize)

    names = header(shstrndx)[4]
    for i in range(shnum):
        h = header(i)
        name = b[names + h[0]:b.index(b"\0", names + h[0])]
        if name == b".hip_fatbin":
            return hashlib.sha256(b[h[4]:h[4] + h[5]]).hexdigest()
    return ""


def measured_traffic(kernel: str):
    """HBM bytes per dispatch of `kernel` from the committed rocprofv3 counter summary,
    or None when there is none or the device code changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if not t.get("device_code_sha256") or t.get("device_code_sha256") != device_code_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return k.get("traffic_bytes_per_dispatch") if k else None


def bound_of(kernel: str):
    if kernel in ALU_KERNELS:
        return "alu", PEAK_PRODUCTS, "T word-products/s (32x32-bit)", 1e12
    return "hbm", PEAK_HBM, "GB/s", 1e9


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _oracle_product(args):
    """Worker: one exact negacyclic product (the oracle's ring_mul) of seeded uniform
    polynomials with bits_a- and bits_b-bit coefficients at N = 2^logN, mod 2^(bits_a +
    bits_b - bits_a) (the modulus of the HE-mult product it stands for).  Returns seconds."""
    seed, logN, bits_a, bits_b, mod_bits = args
    import numpy as np
    from oracle import limbs, ring
    import synth
    rng = np.random.default_rng(seed)
    N = 1 << logN
    a = limbs.poly_from_limbs(synth.uniform_limbs(rng, bits_a, N))
    b = limbs.poly_from_limbs(synth.uniform_limbs(rng, bits_b, N))
    t0 = time.perf_counter()
    ring.ring_mul(a, b, 1 << mod_bits)
    return time.perf_counter() - t0


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline():
    """The oracle (never tuned) timed on the host's cores, on a bounded sample of the
    workload: W worker processes (W = host cores, at most 16) each compute one
    tensor-size exact product (1555 x 1555 bits, N = 2^16), then each one
    relinearization-size product (1555 x 3110 bits); one HE-mult is 4 + 2 such
    products, so the all-core rate is W / (4 t_tensor + 2 t_relin) with the per-worker
    times measured under that load.  Also single-core per-op times: the workload's
    bare ring multiply (literal schoolbook, N = 2^10, Q = 2^120), one HE-mult + relin +
    rescale at N = 2^14 / logq = 438, and one textbook 2^16-point NTT."""
    import multiprocessing
    import platform
    from concurrent.futures import ProcessPoolExecutor
    import numpy as np
    from oracle import limbs, ntt, ring, scheme
    import synth
    W = max(1, min(16, os.cpu_count() or 1))
    out = {"unit": "HE-mults/s", "cores": W, "kind": "oracle", "nproc": os.cpu_count(), "cpu_model": _cpu_model(),
           "python": platform.python_version()}
    t_all = time.perf_counter()
    with ProcessPoolExecutor(W, mp_context=multiprocessing.get_context("spawn")) as pool:
        tt = list(pool.map(_oracle_product, [(100 + i, LOGN, LOGQ, LOGQ, LOGQ) for i in range(W)]))
        tr = list(pool.map(_oracle_product, [(200 + i, LOGN, LOGQ, LOGQ + LOGP, LOGQ + LOGP) for i in range(W)]))
    t1, t2 = float(np.mean(tt)), float(np.mean(tr))
    out["value"] = W / (4 * t1 + 2 * t2)
    out["sample"] = (f"{W} workers x (1 tensor-size + 1 relin-size exact product, N=2^16, logq=logP=1555); "
                     f"mean {t1:.1f} s and {t2:.1f} s per product under load; HE-mult = 4 + 2 products "
                     f"(rescale and compose are O(N L), not counted); Python ints + decimal, one process per core")
    out["sample_wall_s"] = time.perf_counter() - t_all
    # single-core per-op times
    rng = np.random.default_rng(1)
    N = 1 << 10
    a = limbs.poly_from_limbs(synth.uniform_limbs(rng, 120, N))
    b = limbs.poly_from_limbs(synth.uniform_limbs(rng, 120, N))
    t0 = time.perf_counter()
    ring.negacyclic_schoolbook(a, b, 1 << 120)
    out["ring_mul_n10_q120_schoolbook_ms"] = 1e3 * (time.perf_counter() - t0)
    N = 1 << 14
    ct = lambda: scheme.Ciphertext(limbs.poly_from_limbs(synth.uniform_limbs(rng, 438, N)),
                                   limbs.poly_from_limbs(synth.uniform_limbs(rng, 438, N)), 14, 438, 40)
    x, y = ct(), ct()
    evk = scheme.EvalKey(limbs.poly_from_limbs(synth.uniform_limbs(rng, 876, N)),
                         limbs.poly_from_limbs(synth.uniform_limbs(rng, 876, N)), 14, 438, 438)
    t0 = time.perf_counter()
    scheme.mult_rescale(x, y, evk, 40)
    out["he_mult_n14_q438_s"] = time.perf_counter() - t0
    q = (1 << 30) - (1 << 17) + 1
    while not ntt.is_prime(q):
        q -= 1 << 17
    psi = ntt.root_of_unity(q, 1 << 17)
    v = [int(u) for u in rng.integers(0, q, size=1 << 16)]
    t0 = time.perf_counter()
    ntt.ntt_fast(v, q, psi)
    out["ntt_n16_textbook_s"] = time.perf_counter() - t0
    out["he_mult_n16_q1555_s_per_core"] = 4 * t1 + 2 * t2
    return out


def batched_uneven(fhe, torch, synth, dev, stream, njobs):
    """`njobs` CKKS HE-mults + relin + rescale(40) with logN ~ U{13..16} and logq ~
    U{218, 438, 874, 1555} drawn independently from the workload-4 schedule stream;
    one key per N at logQ = logP = 1555.  One autotuned, graph-captured plan run
    against the same jobs as separate per-op calls; outputs compared bit for bit."""
    import numpy as np

    rk, rm, _, rs = synth.streams(4)
    ctx = fhe.Context(LOGQ, LOGP)
    keys = {n: fhe.EvalKey(ctx, fhe.CKKS, 0, n, LOGQ, LOGP, synth.uniform_limbs(rk, LOGQ + LOGP, 1 << n),
                           synth.uniform_limbs(rk, LOGQ + LOGP, 1 << n)) for n in (13, 14, 15, 16)}
    logNs = rs.integers(13, 17, size=njobs)
    logqs = np.array([218, 438, 874, 1555])[rs.integers(0, 4, size=njobs)]
    jobs, ref = [], []
    for n, q in zip(logNs.tolist(), logqs.tolist()):
        N = 1 << n
        ins = [fhe.to_device(synth.uniform_limbs(rm, q, N)).reshape(-1) for _ in range(4)]
        Lo = synth.nlimbs(q - BITS)
        outs = [torch.zeros(Lo * N, dtype=torch.int32, device=dev) for _ in range(2)]
        ref.append([torch.zeros(Lo * N, dtype=torch.int32, device=dev) for _ in range(2)])
        jobs.append((keys[n], q, BITS, *ins, *outs))
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def per_op():
        for j, r in zip(jobs, ref):
            ctx.mul_relin_rescale(j[0], j[1], j[2], j[3], j[4], j[5], j[6], r[0], r[1])

    per_op()  # prepares every key level; warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = fhe.BatchPlan(ctx, jobs, flags=fhe.PLAN_GRAPH | fhe.PLAN_AUTOTUNE)
    plan_s = time.perf_counter() - t0
    info = plan.info()
    plan.run()
    torch.cuda.synchronize()
    reps = 3
    ev0.record(stream)
    for _ in range(reps):
        plan.run()
    ev1.record(stream)
    torch.cuda.synchronize()
    batched = reps * njobs / (ev0.elapsed_time(ev1) / 1e3)
    ev0.record(stream)
    for _ in range(reps):
        per_op()
    ev1.record(stream)
    torch.cuda.synchronize()
    perop = reps * njobs / (ev0.elapsed_time(ev1) / 1e3)
    exact = all(torch.equal(j[7], r[0]) and torch.equal(j[8], r[1]) for j, r in zip(jobs, ref))
    plan.close()
    # the same jobs stage by stage: one launch per pipeline step and kernel variant over
    # every cell (a device table of cell segments), captured in one graph
    for j in jobs:
        j[7].zero_()
        j[8].zero_()
    t0 = time.perf_counter()
    qplan = fhe.BatchPlan(ctx, jobs, flags=fhe.PLAN_QUEUE | fhe.PLAN_GRAPH | fhe.PLAN_AUTOTUNE)
    qplan_s = time.perf_counter() - t0
    qinfo = qplan.info()
    qplan.run()
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(reps):
        qplan.run()
    ev1.record(stream)
    torch.cuda.synchronize()
    queued = reps * njobs / (ev0.elapsed_time(ev1) / 1e3)
    qexact = all(torch.equal(j[7], r[0]) and torch.equal(j[8], r[1]) for j, r in zip(jobs, ref))
    qplan.close()
    # one stream, no graph: every stage one launch per kernel variant over all cells
    for j in jobs:
        j[7].zero_()
        j[8].zero_()
    eplan = fhe.BatchPlan(ctx, jobs, flags=fhe.PLAN_QUEUE | fhe.PLAN_AUTOTUNE)
    einfo = eplan.info()
    ev0.record(stream)
    for _ in range(reps):
        eplan.run()
    ev1.record(stream)
    torch.cuda.synchronize()
    eager_q = reps * njobs / (ev0.elapsed_time(ev1) / 1e3)
    eexact = all(torch.equal(j[7], r[0]) and torch.equal(j[8], r[1]) for j, r in zip(jobs, ref))
    eplan.close()
    out = {"jobs": njobs, "cells": info["cells"], "kernels_per_run": info["kernels"], "graphed": info["graphed"],
           "plan_seconds": plan_s, "he_mults_per_s": batched, "per_op_he_mults_per_s": perop,
           "speedup_vs_per_op": batched / perop, "bit_exact_vs_per_op": bool(exact),
           "stage_batched_graph": {"he_mults_per_s": queued, "kernels_per_run": qinfo["kernels"],
                                   "plan_seconds": qplan_s, "speedup_vs_per_op": queued / perop,
                                   "bit_exact_vs_per_op": bool(qexact),
                                   "layout": "cells on up to 4 graph branches, each branch stage-batched"},
           "stage_batched_one_stream": {"he_mults_per_s": eager_q, "kernels_per_run": einfo["kernels"],
                                        "speedup_vs_per_op": eager_q / perop, "bit_exact_vs_per_op": bool(eexact),
                                        "layout": "every stage one launch per kernel variant over all cells, "
                                                  "no graph"},
           "workload": "CKKS, logN ~ U{13..16}, logq ~ U{218,438,874,1555}, rescale 40, one key per N at "
                       "logQ = logP = 1555 (seed 4000)"}
    for k in keys.values():
        k.close()
    ctx.close()
    return out


def op_latency_leg(fhe, torch, synth, dev, stream, reps=10):
    """Latency of each homomorphic operation of the paper's operation table at its
    parameters (a CipherTensor of cnum = 4 ciphertexts, logN = 16, logQ = 1024, scale
    2^60; CKKS), through the fhe_ct entry points: the CipherTensor latency and the
    amortized latency per ciphertext, with the paper's Tesla T4 figures beside them as
    context (another machine, another implementation).  Inputs and keys are uniform
    synthetic limbs; moddownBy and rescaleBy take 60 bits, leftrotate one slot,
    multconstvec one plaintext per ciphertext, the broadcast forms one shared operand.
    Bootstrapping is the separate leg (its own parameters)."""
    logN, logQ, logP, logp, cnum = 16, 1024, 1024, 60, 4
    N, L = 1 << logN, synth.nlimbs(logQ)
    rk, rm, _, _ = synth.streams(8)
    ctx = fhe.Context(logQ, logP)

    def key(g=0):
        return fhe.EvalKey(ctx, fhe.CKKS, 0, logN, logQ, logP, synth.uniform_limbs(rk, logQ + logP, N),
                           synth.uniform_limbs(rk, logQ + logP, N), g=g)

    relin, rot1, conj = key(), key(pow(5, 1, 2 * N)), key(2 * N - 1)

    def ct():
        c0 = fhe.to_device(synth.uniform_limbs(rm, logQ, N, count=cnum)).reshape(-1)
        c1 = fhe.to_device(synth.uniform_limbs(rm, logQ, N, count=cnum)).reshape(-1)
        return fhe.Ciphertext(c0, c1, logN, logQ, logp, fhe.CKKS, 0, 1, cnum)

    x, y = ct(), ct()
    pv = fhe.to_device(synth.uniform_limbs(rm, logQ, N, count=cnum)).reshape(-1)   # one plaintext per ciphertext
    p1 = fhe.to_device(synth.uniform_limbs(rm, logQ, N, count=1)).reshape(-1)      # one shared plaintext
    out = (torch.empty(cnum * L * N, dtype=torch.int32, device=dev), torch.empty(cnum * L * N, dtype=torch.int32,
                                                                                  device=dev))
    kconst = (1 << 59) + 12345
    ops = {
        "negate_pairwise_into": lambda: ctx.ct_negate(x, out),
        "moddownBy_pairwise_into": lambda: ctx.ct_moddown(x, 60, out),
        "rescaleBy_pairwise_into": lambda: ctx.ct_rescale(x, 60, out),
        "conjugate_pairwise_into": lambda: ctx.ct_conjugate(conj, x, out),
        "mult_pairwise_into": lambda: ctx.ct_mul_relin(relin, x, y, out),
        "leftrotate_broadcast_into": lambda: ctx.ct_leftrotate(rot1, 1, x, out),
        "add_pairwise_into": lambda: ctx.ct_add(x, y, out),
        "sub_pairwise_into": lambda: ctx.ct_sub(x, y, out),
        "addconst_broadcast_into": lambda: ctx.ct_addconst(x, p1, 1, out),
        "addconst_pairwise_into": lambda: ctx.ct_addconst(x, pv, cnum, out),
        "imult_pairwise_into": lambda: ctx.ct_imult(x, out),
        "multconst_broadcast_into": lambda: ctx.ct_multconst(x, kconst, out, logp_k=logp),
        "multconstvec_pairwise_into": lambda: ctx.ct_multconstvec(x, pv, cnum, out, logp_m=logp),
    }
    paper_t4 = {"negate_pairwise_into": 0.0191, "moddownBy_pairwise_into": 0.0131, "rescaleBy_pairwise_into": 0.0770,
                "conjugate_pairwise_into": 5.5614, "mult_pairwise_into": 8.1862,
                "leftrotate_broadcast_into": 5.6852, "add_pairwise_into": 0.0286, "sub_pairwise_into": 0.0260,
                "addconst_broadcast_into": 0.0007, "addconst_pairwise_into": 0.0170,
                "imult_pairwise_into": 0.0170, "multconst_broadcast_into": 0.6219,
                "multconstvec_pairwise_into": 1.9930}
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    res = {}
    for name, f in ops.items():
        f()  # prepares key levels and tables
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(reps):
            f()
        ev1.record(stream)
        torch.cuda.synchronize()
        s_ = ev0.elapsed_time(ev1) / 1e3 / reps
        res[name] = {"ciphertensor_s": s_, "per_ciphertext_s": s_ / cnum, "paper_t4_ciphertensor_s": paper_t4[name]}
    for k in (relin, rot1, conj):
        k.close()
    ctx.close()
    return {"ops": res, "workload": "CKKS CipherTensor of 4, logN = 16, logQ = logP = 1024, scale 2^60; "
                                    "uniform synthetic ciphertexts and keys (seed 8000); mean of 10 calls after one"}


def bootstrap_leg(fhe, torch, synth, dev, reps=3):
    """CKKS bootstrapping of one ciphertext at N = 2^16 with 4 slots (logs = 2), input at
    logq = 40 and scale 2^30 (the paper's bootstrapping setting), raised to logQ = 1024;
    logT = 8 squarings, a degree-11 Taylor step, constants at 2^40.  Keys and ciphertext
    are uniform synthetic limbs (the circuit's cost does not depend on their values); the
    diagonals of V^-1 and V / (2 pi) are encoded by the library's host encoder.  The
    first call prepares every key level it meets; the next `reps` calls are timed."""
    import math
    import numpy as np
    logN, logslots, logq_in, logQ, logc, logT, degree = 16, 2, 40, 1024, 40, 8, 11
    N, n = 1 << logN, 1 << logslots
    rk, rm, _, _ = synth.streams(6)
    ctx = fhe.Context(logQ, logQ)

    def key(g=0):
        return fhe.EvalKey(ctx, fhe.CKKS, 0, logN, logQ, logQ, synth.uniform_limbs(rk, 2 * logQ, N),
                           synth.uniform_limbs(rk, 2 * logQ, N), g=g)

    relin = key()
    amounts = sorted(set(range(1, n)) | {1 << i for i in range(logslots, logN - 1)})
    rot = {r: key(pow(5, r, 2 * N)) for r in amounts}
    conj = key(2 * N - 1)
    r_ = [pow(5, j, 4 * n) for j in range(n)]
    V = np.array([[np.exp(2j * np.pi * ((rj * k) % (4 * n)) / (4 * n)) for k in range(n)] for rj in r_])

    def diags(A):
        return [np.array([A[j][(j + d) % n] for j in range(n)]) for d in range(n)]

    enc = lambda ds: fhe.to_device(np.stack([fhe.ckks_encode(d, logN, logc, logQ) for d in ds])).reshape(-1)
    c2s, s2c = enc(diags(np.linalg.inv(V))), enc(diags(V / (2 * np.pi)))
    k_y = int(round(2 * np.pi * 2.0 ** logc))
    taylor = [int(round((-1) ** (k // 2) / math.factorial(k) * 2.0 ** logc)) for k in range(degree + 1)]
    x = fhe.Ciphertext(fhe.to_device(synth.uniform_limbs(rm, logq_in, N)).reshape(-1),
                       fhe.to_device(synth.uniform_limbs(rm, logq_in, N)).reshape(-1), logN, logq_in, 30, fhe.CKKS,
                       0, 1, 1)
    LQ = synth.nlimbs(logQ)
    out = (torch.empty(LQ * N, dtype=torch.int32, device=dev), torch.empty(LQ * N, dtype=torch.int32, device=dev))
    params = dict(logN=logN, logslots=logslots, logq_in=logq_in, logQ=logQ, logc=logc, logT=logT, degree=degree)
    t0 = time.perf_counter()
    o = ctx.ct_bootstrap(params, relin, rot, conj, c2s, s2c, k_y, taylor, x, out)
    first = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.ct_bootstrap(params, relin, rot, conj, c2s, s2c, k_y, taylor, x, out)
    per = (time.perf_counter() - t0) / reps
    for k in [relin, conj, *rot.values()]:
        k.close()
    ctx.close()
    return {"seconds_per_bootstrap": per, "first_call_seconds": first, "out_logq": o.logq, "out_logp": o.logp,
            "workload": "CKKS bootstrapping, N=2^16, 4 slots, input logq=40 logp=30, logQ=1024, logT=8, "
                        "Taylor degree 11, logc=40; uniform synthetic keys and ciphertext; wall clock per call "
                        "(each call synchronizes)",
            "paper_context": "57.9 s per ciphertext (amortized, CipherTensor of 4) on a Tesla T4, HEAAN setting"}


def serving(fhe, torch, synth, dev, nreq, loads=(0.5, 0.8, 0.95), nstreams=4, max_batch=16,
            budget=24 << 30):
    """The request loop under open-loop Poisson arrivals.  Requests: CKKS with
    probability 0.7 (rescale 40) else BGV (t = 65537, rescale 32); logN ~ U{15, 16};
    logq ~ U{218, 438, 874, 1555}; four resident keys (scheme x N) at logQ = logP = 1555.
    Operands come from a pool of 8 sets per (scheme, N, logq) cell; a request writes
    the output pair of its pool index, so overlapping writers hold the same values.
    mu_sat = completed / makespan of the whole stream queued at once; then Poisson
    streams at load x mu_sat, served by the batching loop and by per-op FIFO launches
    (one stream, batch of one).  Latency = completion seen by the scheduler - scheduled
    arrival."""
    import numpy as np

    rk, rm, _, rs = synth.streams(5)
    ctx = fhe.Context(LOGQ, LOGP)
    keys = {}
    for sch, t in ((fhe.CKKS, 0), (fhe.BGV, 65537)):
        for n in (15, 16):
            keys[(sch, n)] = fhe.EvalKey(ctx, sch, t, n, LOGQ, LOGP, synth.uniform_limbs(rk, LOGQ + LOGP, 1 << n),
                                         synth.uniform_limbs(rk, LOGQ + LOGP, 1 << n))
    sch_draw = np.where(rs.random(nreq) < 0.7, fhe.CKKS, fhe.BGV)
    n_draw = rs.integers(15, 17, size=nreq)
    q_draw = np.array([218, 438, 874, 1555])[rs.integers(0, 4, size=nreq)]
    pool, reqs, used = {}, [], {}
    for sch, n, q in zip(sch_draw.tolist(), n_draw.tolist(), q_draw.tolist()):
        cell = (sch, n, q)
        if cell not in pool:
            N = 1 << n
            bits = BITS if sch == fhe.CKKS else 32
            Lo = synth.nlimbs(q - bits)
            sets = []
            for _ in range(8):
                ins = [fhe.to_device(synth.uniform_limbs(rm, q, N)).reshape(-1) for _ in range(4)]
                outs = [torch.zeros(Lo * N, dtype=torch.int32, device=dev) for _ in range(2)]
                ref = [torch.zeros(Lo * N, dtype=torch.int32, device=dev) for _ in range(2)]
                ctx.mul_relin_rescale(keys[(sch, n)], q, bits, *ins, *ref)
                sets.append((ins, outs, ref))
            pool[cell] = (bits, sets)
        bits, sets = pool[cell]
        k = used.get(cell, 0)
        used[cell] = k + 1
        ins, outs, _ = sets[k % 8]
        reqs.append((keys[(sch, n)], q, bits, *ins, *outs))
    torch.cuda.synchronize()

    def run(rate, streams, batch, seed):
        for _, sets in pool.values():
            for _, outs, _ in sets:
                for o in outs:
                    o.zero_()
        torch.cuda.synchronize()
        srv = fhe.Server(ctx, budget, nstreams=streams, max_batch=batch)
        rng = np.random.default_rng(seed)
        t0 = fhe.clock_ns() + 200_000_000
        gaps = np.zeros(nreq) if rate is None else rng.exponential(1e9 / rate, nreq)
        for r, ta in zip(reqs, t0 + np.cumsum(gaps).astype(np.int64)):
            srv.submit(r, int(ta))
        srv.drain()
        done = srv.poll(nreq + 16)
        srv.close()
        ok = len(done) == nreq and all(d.status == 0 for d in done)
        lat = np.array([d.t_done - d.t_arrive for d in done], dtype=np.float64) / 1e6
        span = (max(d.t_done for d in done) - t0) / 1e9
        exact = all(torch.equal(o, r) for _, sets in pool.values() for _, outs, ref in sets
                    for o, r in zip(outs, ref))
        return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "throughput_per_s": nreq / span, "mean_batch": float(np.mean([d.batch for d in done])),
                "all_ok": bool(ok), "bit_exact_vs_alone": bool(exact)}

    log(f"serving: saturation ({nreq} requests at once)")
    sat = run(None, nstreams, max_batch, 0)
    mu = sat["throughput_per_s"]
    log("serving: per-op FIFO saturation")
    sat_p = run(None, 1, 1, 0)
    mu_p = sat_p["throughput_per_s"]
    runs = []
    # loads relative to the batched saturation rate, then to the per-op one (where the
    # per-op FIFO is itself stable, so its latency is not backlog growth)
    for i, (f, ref, which) in enumerate([(f, mu, "batched") for f in loads] +
                                        [(f, mu_p, "per_op") for f in (0.5, 0.8)]):
        log(f"serving: load {f} of the {which} saturation rate {ref:.0f}/s")
        b = run(f * ref, nstreams, max_batch, 10 + i)
        p = run(f * ref, 1, 1, 10 + i)
        runs.append({"load": f, "of": f"{which} saturation", "rate_per_s": f * ref, "batched": b,
                     "per_op_fifo": p, "p99_speedup_vs_per_op": p["p99_ms"] / b["p99_ms"]})
    for k in keys.values():
        k.close()
    ctx.close()
    return {"requests": nreq, "mu_sat_per_s": mu, "saturation_run": sat, "per_op_mu_sat_per_s": mu_p,
            "per_op_saturation_run": sat_p, "nstreams": nstreams,
            "max_batch": max_batch, "hbm_budget_bytes": budget, "runs": runs,
            "workload": "70% CKKS (rescale 40) / 30% BGV t=65537 (rescale 32), logN ~ U{15,16}, "
                        "logq ~ U{218,438,874,1555}, 4 resident keys at logQ = logP = 1555, 8 operand sets "
                        "per cell, open-loop Poisson arrivals (seed 5000)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cnum", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip per-op and NTT legs")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched uneven leg")
    ap.add_argument("--batch-jobs", type=int, default=256)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-boot", action="store_true", help="skip the bootstrapping leg")
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="also run one plain device copy of this size (HBM counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: HE-mult requests shard across GPUs with no exchange, "
              "and this benchmark runs on a single MI355X; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2607_05920_amd as fhe
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    N = 1 << LOGN
    L = synth.nlimbs(LOGQ)
    Lo = synth.nlimbs(LOGQ - BITS)
    LK = synth.nlimbs(LOGQ + LOGP)
    cnum = args.cnum

    log("context + inputs")
    ctx = fhe.Context(LOGQ, LOGP)
    Kt = ctx.primes_needed(LOGN, LOGQ, LOGQ, 2)          # tensor: |d1| < 2^(2 logq + logN + 1)
    Kr = ctx.primes_needed(LOGN, LOGQ, LOGQ + LOGP, 1)   # relinearization: d2 times the key
    rk, rm, _, _ = synth.streams(3)
    eb = synth.uniform_limbs(rk, LOGQ + LOGP, N)
    ea = synth.uniform_limbs(rk, LOGQ + LOGP, N)
    evk = fhe.EvalKey(ctx, fhe.CKKS, 0, LOGN, LOGQ, LOGP, eb, ea)
    evk.prepare(LOGQ)
    xs = [fhe.to_device(synth.uniform_limbs(rm, LOGQ, N, count=cnum)).reshape(-1) for _ in range(4)]
    o0 = torch.empty(cnum * Lo * N, dtype=torch.int32, device=dev)
    o1 = torch.empty(cnum * Lo * N, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    def step(c=cnum, ins=xs, outs=(o0, o1)):
        ctx.mul_relin_rescale(evk, LOGQ, BITS, ins[0], ins[1], ins[2], ins[3], outs[0], outs[1], cnum=c)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # ---- timed region: K steps bracketed by two HIP events on the launch stream
    log(f"timed: {args.steps} steps of cnum={cnum}")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    value = cnum * args.steps / (ms / 1e3)

    # ---- the same K steps again with a HIP event pair around every kernel launch (on
    # the launch stream): per-kernel times for the roofline.  The event pairs keep
    # consecutive kernels from overlapping, so this pass is a little slower and is not
    # the one `value` comes from.
    log(f"instrumented: {args.steps} steps of cnum={cnum}")
    ctx.profile(True)
    ev2, ev3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev2.record(stream)
    for _ in range(args.steps):
        step()
    ev3.record(stream)
    torch.cuda.synchronize()
    ms_instr = ev2.elapsed_time(ev3)
    prof = ctx.profile_read()
    ctx.profile(False)

    dom = max(prof, key=lambda k: prof[k]["ms"])
    d = prof[dom]
    bound, peak, unit, scale = bound_of(dom)
    achieved = d["work"] / (d["ms"] / 1e3)
    total_kernel_ms = sum(v["ms"] for v in prof.values())
    roofline = {
        "bound": bound, "kernel": dom, "achieved": achieved / scale, "peak": peak / scale, "unit": unit,
        "frac": achieved / peak, "traffic": measured_traffic(dom),
        "work_per_launch": d["work"] / max(1, d["launches"]),
        "avg_launch_ms": d["ms"] / max(1, d["launches"]), "launches": d["launches"],
        "share_of_kernel_time": d["ms"] / total_kernel_ms if total_kernel_ms else None,
        "instrumented_ms_per_step": ms_instr / args.steps,
    }
    kernels = {}
    for k, v in prof.items():
        b, pk, u, sc = bound_of(k)
        rate = v["work"] / (v["ms"] / 1e3) if v["ms"] and v["work"] else None
        kernels[k] = {"ms_per_step": v["ms"] / args.steps, "launches_per_step": v["launches"] / args.steps,
                      "bound": b, "achieved": rate / sc if rate else None, "unit": u,
                      "frac": rate / pk if rate else None}
    # The lift and the reconstruction run their column sums on the i8 matrix cores:
    # their algorithmic int8 operations (2 per multiply-add of the digit-plane contraction,
    # unpadded) against the dense i8 peak, beside the HBM figure above.
    N4 = 2.0 * N * 16  # 2 ops x 4 digit bytes x 4 planes per (coefficient, limb, prime)
    mfma_ops = {"lift": N4 * L * (4 * cnum * Kt + cnum * Kr),
                "crt": N4 * (3 * cnum * Kt * L + 2 * cnum * Kr * LK)}
    for k, ops in mfma_ops.items():
        if prof.get(k, {}).get("ms"):
            r = ops * args.steps / (prof[k]["ms"] / 1e3)
            kernels[k]["mfma_i8"] = {"achieved": r / 1e15, "peak": PEAK_MFMA_I8 / 1e15, "unit": "POP/s",
                                     "frac": r / PEAK_MFMA_I8, "ops_per_step": ops}

    extras = {}
    if not args.no_extras:
        # per-op: the same work as cnum separate launches of one pair each
        log("per-op leg")
        singles = [[x[i * L * N:(i + 1) * L * N] for x in xs] for i in range(cnum)]
        so = [(o0[i * Lo * N:(i + 1) * Lo * N], o1[i * Lo * N:(i + 1) * Lo * N]) for i in range(cnum)]
        for i in range(cnum):
            step(1, singles[i], so[i])
        torch.cuda.synchronize()
        steps1 = max(2, args.steps // 2)
        ev0.record(stream)
        for _ in range(steps1):
            for i in range(cnum):
                step(1, singles[i], so[i])
        ev1.record(stream)
        torch.cuda.synchronize()
        extras["per_op_he_mults_per_s"] = cnum * steps1 / (ev0.elapsed_time(ev1) / 1e3)
        extras["batched_over_per_op"] = value / extras["per_op_he_mults_per_s"]
        # the same step as a graph: a plan of the cnum pairs (one cell, the same kernels
        # through pointer arrays) captured once and replayed
        log("graph replay leg")
        gjobs = [(evk, LOGQ, BITS, *singles[i], *so[i]) for i in range(cnum)]
        gplan = fhe.BatchPlan(ctx, gjobs, flags=fhe.PLAN_GRAPH)
        gplan.run()
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            gplan.run()
        ev1.record(stream)
        torch.cuda.synchronize()
        gms = ev0.elapsed_time(ev1) / args.steps
        extras["graph_replay"] = {"he_mults_per_s": cnum / (gms / 1e3), "ms_per_step": gms,
                                  "kernels_per_step": gplan.info()["kernels"]}
        gplan.close()
        # standalone NTT throughput: 64 polynomials of this size lifted to the tensor primes
        log("NTT leg")
        del xs, o0, o1, singles, so
        torch.cuda.empty_cache()
        polys = fhe.to_device(synth.uniform_limbs(rm, LOGQ, N, count=64)).reshape(-1)
        res = torch.empty(64 * Kt * N, dtype=torch.int32, device=dev)
        ctx.lift(LOGN, L, Kt, polys, res, count=64)
        ctx.ntt(LOGN, Kt, res, count=64, bitrev=True)
        ctx.ntt(LOGN, Kt, res, count=64, inverse=True, bitrev=True)
        torch.cuda.synchronize()
        for inv in (False, True):
            reps = 3
            ev0.record(stream)
            for _ in range(reps):
                ctx.ntt(LOGN, Kt, res, count=64, inverse=inv, bitrev=True)
            ev1.record(stream)
            torch.cuda.synchronize()
            extras["ntt_inv_per_s" if inv else "ntt_fwd_per_s"] = reps * 64 * Kt / (ev0.elapsed_time(ev1) / 1e3)
        extras["ntt_transforms_per_call"] = 64 * Kt
        del polys, res
        torch.cuda.empty_cache()

    if not args.no_extras and not args.no_batch:
        log("batched uneven leg")
        extras["batched_uneven"] = batched_uneven(fhe, torch, synth, dev, stream, args.batch_jobs)

    if not args.no_extras and not args.no_boot:
        log("operation latency leg")
        extras["op_latency"] = op_latency_leg(fhe, torch, synth, dev, stream)
        log("bootstrapping leg")
        extras["bootstrap"] = bootstrap_leg(fhe, torch, synth, dev)

    if not args.no_extras and not args.no_serve:
        log("serving leg")
        extras["serving"] = serving(fhe, torch, synth, dev, args.serve_requests)

    if args.copy_calib_mb:
        nb = args.copy_calib_mb << 20
        src = torch.empty(nb // 4, dtype=torch.int32, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        extras["copy_calib_bytes"] = nb

    out = {
        "metric": "HE-mults/s (N=2^16, logQ~1555) batched vs per-op; p50/p99 serve latency",
        "value": value, "unit": "HE-mults/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"CKKS HE-mult + relinearization + rescale by {BITS} bits, N=2^16, logq=1555, "
                               f"logP=1555, CipherTensor of {cnum} ciphertext pairs per step",
                   "logN": LOGN, "logq": LOGQ, "logP": LOGP, "rescale_bits": BITS, "cnum": cnum,
                   "primes_tensor": Kt, "primes_relin": Kr,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "kernels": kernels,
        "wall_s": wall,
        **extras,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle sample)")
        out["cpu_baseline"] = cpu_baseline()
    evk.close()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
