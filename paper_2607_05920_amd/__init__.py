"""MI355X (gfx950) homomorphic multiplication for non-RNS CKKS/BGV.

Thin ctypes binding over the C ABI of ``libfhe_mi355x.so`` (declared in
``include/fhe_mi355x.h``).  Every step of the computation runs in the library's
HIP kernels; this module only marshals arguments: torch CUDA tensors for device
buffers (int32 tensors holding the uint32 limb bits) and the current torch stream.
Importing the module does not need a GPU; calling a compute function without the
built library raises ``LibraryMissing``.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfhe_mi355x.so")

CKKS = 0
BGV = 1

STATUS = {
    0: "ok", -1: "invalid argument", -2: "shape mismatch", -3: "out of range",
    -4: "out of memory", -5: "device error", -6: "bad state",
}

# Every exported symbol and its ctypes signature (restype, argtypes).
_P = ctypes.c_void_p
_I = ctypes.c_int
_U = ctypes.c_uint32
EXPORTS = {
    "fhe_strerror": (ctypes.c_char_p, [_I]),
    "fhe_error_detail": (ctypes.c_char_p, []),
    "fhe_ctx_create": (_I, [_I, _I, _I, ctypes.POINTER(_P)]),
    "fhe_ctx_destroy": (None, [_P]),
    "fhe_ctx_reset_error": (_I, [_P]),
    "fhe_ctx_profile": (_I, [_P, _I]),
    "fhe_ctx_profile_read": (_I, [_P, _I, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_longlong)]),
    "fhe_prime_count": (_I, [_P, ctypes.POINTER(_I)]),
    "fhe_prime_info": (_I, [_P, _I, ctypes.POINTER(_U), ctypes.POINTER(_U)]),
    "fhe_primes_needed": (_I, [_P, _I, _I, _I, _I, ctypes.POINTER(_I)]),
    "fhe_lift": (_I, [_P, _I, _I, _I, _P, _P, _I, _P]),
    "fhe_ntt": (_I, [_P, _I, _I, _I, _I, _P, _I, _P]),
    "fhe_ring_mul": (_I, [_P, _I, _I, _P, _P, _P, _I, _P]),
    "fhe_ring_mul_noalloc": (_I, [_P, _I, _I, _P, _P, _P, _I, _P]),
    "fhe_evk_create": (_I, [_P, _I, _U, _I, _I, _I, _P, _P, ctypes.POINTER(_P)]),
    "fhe_evk_prepare": (_I, [_P, _I, _P]),
    "fhe_evk_destroy": (None, [_P]),
    "fhe_mul_relin": (_I, [_P, _P, _I, _I, _P, _P, _P, _P, _P, _P, _I, _P]),
    "fhe_rescale": (_I, [_P, _I, _U, _I, _I, _I, _P, _P, _P, _P, _I, _P]),
    "fhe_mul_relin_rescale": (_I, [_P, _P, _I, _I, _I, _P, _P, _P, _P, _P, _P, _I, _P]),
    "fhe_batch_plan": (_I, [_P, _P, _I, _I, _P, ctypes.POINTER(_P)]),
    "fhe_batch_run": (_I, [_P, _P]),
    "fhe_batch_info": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "fhe_batch_destroy": (None, [_P]),
    "fhe_ckks_encode": (_I, [_I, _I, _I, _I, _P, _P, _P]),
    "fhe_ckks_decode": (_I, [_I, _I, _I, _I, _P, _P, _P]),
    "fhe_encrypt": (_I, [_P, _I, _U, _I, _I, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "fhe_decrypt": (_I, [_P, _I, _U, _U, _I, _I, _P, _P, _P, _P, _P]),
    "fhe_clock_ns": (ctypes.c_uint64, []),
    "fhe_server_create": (_I, [_P, ctypes.c_size_t, _I, _I, ctypes.POINTER(_P)]),
    "fhe_server_submit": (_I, [_P, _P, ctypes.c_uint64, _P, ctypes.POINTER(ctypes.c_uint64)]),
    "fhe_server_cancel": (_I, [_P]),
    "fhe_server_poll": (_I, [_P, _P, _I, ctypes.POINTER(_I)]),
    "fhe_server_drain": (_I, [_P]),
    "fhe_server_destroy": (None, [_P]),
    "fhe_automorphism": (_I, [_P, _I, _I, _U, _P, _P, _I, _P]),
    "fhe_galois_key_create": (_I, [_P, _I, _U, _I, _I, _I, _U, _P, _P, ctypes.POINTER(_P)]),
    "fhe_key_switch": (_I, [_P, _P, _I, _I, _P, _P, _P, _P, _I, _P]),
    "fhe_ct_mul_relin": (_I, [_P, _P, _P, _P, _P, _P]),
    "fhe_ct_mul_relin_rescale": (_I, [_P, _P, _P, _P, _I, _P, _P]),
    "fhe_ct_rescale": (_I, [_P, _P, _I, _P, _P]),
    "fhe_ct_moddown": (_I, [_P, _P, _I, _P, _P]),
    "fhe_ct_add": (_I, [_P, _P, _P, _P, _P]),
    "fhe_ct_sub": (_I, [_P, _P, _P, _P, _P]),
    "fhe_ct_negate": (_I, [_P, _P, _P, _P]),
    "fhe_ct_imult": (_I, [_P, _P, _P, _P]),
    "fhe_ct_multconst": (_I, [_P, _P, _P, _I, _I, _I, _P, _P]),
    "fhe_ct_multconstvec": (_I, [_P, _P, _P, _I, _I, _P, _P]),
    "fhe_ct_addconst": (_I, [_P, _P, _P, _I, _P, _P]),
    "fhe_ct_key_switch": (_I, [_P, _P, _P, _P, _P]),
    "fhe_ct_leftrotate": (_I, [_P, _P, _I, _P, _P, _P]),
    "fhe_ct_conjugate": (_I, [_P, _P, _P, _P, _P]),
    "fhe_ct_bootstrap": (_I, [_P, _P, _P, _P, _P, _P]),
}

PLAN_GRAPH = 1
PLAN_AUTOTUNE = 2
PLAN_QUEUE = 4
NTT_INVERSE = 1
NTT_BITREV = 2


class Job(ctypes.Structure):
    """fhe_job: one HE-mult (+ optional rescale) of a batch; pointers are device addresses."""
    _fields_ = [("evk", _P), ("logq", _I), ("bits", _I), ("x0", _P), ("x1", _P), ("y0", _P), ("y1", _P),
                ("out0", _P), ("out1", _P)]


class CT(ctypes.Structure):
    """fhe_ct: a CipherTensor's device buffers and metadata."""
    _fields_ = [("c0", _P), ("c1", _P), ("cnum", ctypes.c_int32), ("logN", ctypes.c_int32),
                ("logq", ctypes.c_int32), ("logp", ctypes.c_int32), ("scheme", ctypes.c_int32),
                ("t", ctypes.c_uint32), ("gamma", ctypes.c_uint32)]


class BootParams(ctypes.Structure):
    """fhe_boot_params."""
    _fields_ = [("logN", _I), ("logslots", _I), ("logq_in", _I), ("logQ", _I), ("logc", _I), ("logT", _I),
                ("degree", _I)]


class BootKeys(ctypes.Structure):
    """fhe_boot_keys (pointers: keys, a host array of rotation keys, device diagonals,
    a host array of Taylor constants)."""
    _fields_ = [("relin", _P), ("rot", _P), ("nrot", _I), ("conj", _P), ("c2s", _P), ("s2c", _P),
                ("k_y", ctypes.c_int64), ("taylor", _P)]


class LibraryMissing(RuntimeError):
    pass


class FheError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn} failed: {STATUS.get(status, status)} ({status})")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP library (no GPU needed to load it).

    torch is imported first so that the library binds to the HIP runtime torch
    already carries (same soname): device pointers and stream handles from torch
    are then valid in the library.  Loading the library first would bring a second
    runtime into the process, which does not see torch's device state."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise LibraryMissing(f"{path} is not built; run paper_2607_05920_amd/build.py")
    lib = ctypes.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(fn: str, status: int):
    if status != 0:
        err = FheError(fn, status)
        detail = _lib.fhe_error_detail() if _lib is not None else b""
        if detail:
            err.args = (f"{err.args[0]} [{detail.decode(errors='replace')}]",)
        raise err


def _ptr(t) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("device buffers must be torch CUDA tensors")
    if t.dtype not in (torch.int32, torch.uint32):
        raise TypeError("limb buffers must be 32-bit integer tensors")
    if not t.is_contiguous():
        raise ValueError("buffers must be contiguous")
    return t.data_ptr()


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def nlimbs(bits: int) -> int:
    return (bits + 31) // 32


def _need(t, words: int, name: str):
    if t.numel() < words:
        raise ValueError(f"{name}: {t.numel()} words, {words} needed")


class Context:
    """A library context on one device: prime, twiddle, lift and CRT tables."""

    def __init__(self, logQ_max: int, logP_max: int, device: int = 0):
        lib = load_library()
        h = ctypes.c_void_p()
        _check("fhe_ctx_create", lib.fhe_ctx_create(device, logQ_max, logP_max, ctypes.byref(h)))
        self._h = h
        self.logQ_max, self.logP_max, self.device = logQ_max, logP_max, device

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load_library().fhe_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    KERNELS = ["lift", "ntt_fwd_cols", "ntt_fwd_rows", "ntt_inv_rows", "ntt_inv_cols", "pointwise", "crt",
               "compose", "rescale", "ntt_rows_fused", "compose_rescale", "coeffwise"]

    def profile(self, enable: bool):
        _check("fhe_ctx_profile", load_library().fhe_ctx_profile(self._h, int(enable)))

    def profile_read(self) -> dict:
        out = {}
        for i, name in enumerate(self.KERNELS):
            ms, work, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_longlong()
            _check("fhe_ctx_profile_read", load_library().fhe_ctx_profile_read(
                self._h, i, ctypes.byref(ms), ctypes.byref(work), ctypes.byref(n)))
            out[name] = {"ms": ms.value, "work": work.value, "launches": n.value}
        return out

    def prime_count(self) -> int:
        n = ctypes.c_int()
        _check("fhe_prime_count", load_library().fhe_prime_count(self._h, ctypes.byref(n)))
        return n.value

    def prime_info(self, idx: int):
        q, psi = ctypes.c_uint32(), ctypes.c_uint32()
        _check("fhe_prime_info", load_library().fhe_prime_info(self._h, idx, ctypes.byref(q), ctypes.byref(psi)))
        return q.value, psi.value

    def primes_needed(self, logN: int, bits_a: int, bits_b: int, terms: int = 1) -> int:
        k = ctypes.c_int()
        _check("fhe_primes_needed",
               load_library().fhe_primes_needed(self._h, logN, bits_a, bits_b, terms, ctypes.byref(k)))
        return k.value

    def reset_error(self) -> int:
        return load_library().fhe_ctx_reset_error(self._h)

    # -------------------------------------------------------------- compute
    def lift(self, logN: int, L: int, nprimes: int, limbs, res, count: int = 1, stream=None):
        N = 1 << logN
        _need(limbs, count * L * N, "limbs")
        _need(res, count * nprimes * N, "res")
        _check("fhe_lift", load_library().fhe_lift(self._h, logN, L, nprimes, _ptr(limbs), _ptr(res), count,
                                                   _stream(stream)))

    def ntt(self, logN: int, nprimes: int, data, count: int = 1, inverse: bool = False, bitrev: bool = False,
            prime0: int = 0, stream=None):
        """In-place negacyclic NTT of uint32[count][nprimes][N] over primes prime0.. ;
        natural order unless bitrev (the transform's own order, no permutation)."""
        _need(data, count * nprimes << logN, "data")
        flags = (NTT_INVERSE if inverse else 0) | (NTT_BITREV if bitrev else 0)
        _check("fhe_ntt", load_library().fhe_ntt(self._h, logN, prime0, nprimes, flags, _ptr(data), count,
                                                 _stream(stream)))

    def encrypt(self, scheme: int, t: int, logN: int, logq: int, pk_b, pk_a, m, v, e0, e1, c0, c1, stream=None):
        """c0 = [v pk_b + m + e0']_(2^logq), c1 = [v pk_a + e1']; v int8, e0/e1 int32 device tensors."""
        import torch
        N = 1 << logN
        L = nlimbs(logq)
        for t_, n in ((pk_b, "pk_b"), (pk_a, "pk_a"), (m, "m"), (c0, "c0"), (c1, "c1")):
            _need(t_, L * N, n)
        _small(v, torch.int8, N, "v")
        _small(e0, torch.int32, N, "e0")
        _small(e1, torch.int32, N, "e1")
        _check("fhe_encrypt", load_library().fhe_encrypt(
            self._h, scheme, t, logN, logq, _ptr(pk_b), _ptr(pk_a), _ptr(m), v.data_ptr(), e0.data_ptr(),
            e1.data_ptr(), _ptr(c0), _ptr(c1), _stream(stream)))

    def decrypt(self, scheme: int, t: int, gamma: int, logN: int, logq: int, c0, c1, s, out, stream=None):
        """CKKS: out = phase [c0 + c1 s] (uint32[L][N]); BGV: out = message uint32[N]."""
        import torch
        N = 1 << logN
        L = nlimbs(logq)
        _need(c0, L * N, "c0")
        _need(c1, L * N, "c1")
        _need(out, L * N if scheme == CKKS else N, "out")
        _small(s, torch.int8, N, "s")
        _check("fhe_decrypt", load_library().fhe_decrypt(
            self._h, scheme, t, gamma, logN, logq, _ptr(c0), _ptr(c1), s.data_ptr(), _ptr(out), _stream(stream)))

    def ring_mul(self, logN: int, logq: int, a, b, out, cnum: int = 1, stream=None):
        w = cnum * nlimbs(logq) << logN
        for t, n in ((a, "a"), (b, "b"), (out, "out")):
            _need(t, w, n)
        _check("fhe_ring_mul", load_library().fhe_ring_mul(self._h, logN, logq, _ptr(a), _ptr(b), _ptr(out), cnum,
                                                           _stream(stream)))

    def ring_mul_noalloc(self, logN: int, logq: int, a, b, out, cnum: int = 1, stream=None):
        """fhe_ring_mul_noalloc: the same product with the library's static scratch."""
        w = cnum * nlimbs(logq) << logN
        for t, n in ((a, "a"), (b, "b"), (out, "out")):
            _need(t, w, n)
        _check("fhe_ring_mul_noalloc", load_library().fhe_ring_mul_noalloc(
            self._h, logN, logq, _ptr(a), _ptr(b), _ptr(out), cnum, _stream(stream)))

    def rescale(self, scheme: int, t: int, logN: int, logq: int, bits: int, in0, in1, out0, out1,
                cnum: int = 1, stream=None):
        _need(in0, cnum * nlimbs(logq) << logN, "in0")
        _need(in1, cnum * nlimbs(logq) << logN, "in1")
        _need(out0, cnum * nlimbs(logq - bits) << logN, "out0")
        _need(out1, cnum * nlimbs(logq - bits) << logN, "out1")
        _check("fhe_rescale", load_library().fhe_rescale(self._h, scheme, t, logN, logq, bits, _ptr(in0), _ptr(in1),
                                                         _ptr(out0), _ptr(out1), cnum, _stream(stream)))

    def mul_relin(self, evk: "EvalKey", logq: int, x0, x1, y0, y1, out0, out1, cnum: int = 1, stream=None):
        w = cnum * nlimbs(logq) << evk.logN
        for t, n in ((x0, "x0"), (x1, "x1"), (y0, "y0"), (y1, "y1"), (out0, "out0"), (out1, "out1")):
            _need(t, w, n)
        _check("fhe_mul_relin", load_library().fhe_mul_relin(
            self._h, evk.handle, evk.logN, logq, _ptr(x0), _ptr(x1), _ptr(y0), _ptr(y1), _ptr(out0), _ptr(out1),
            cnum, _stream(stream)))

    def mul_relin_rescale(self, evk: "EvalKey", logq: int, bits: int, x0, x1, y0, y1, out0, out1, cnum: int = 1,
                          stream=None):
        w = cnum * nlimbs(logq) << evk.logN
        for t, n in ((x0, "x0"), (x1, "x1"), (y0, "y0"), (y1, "y1")):
            _need(t, w, n)
        wo = cnum * nlimbs(logq - bits) << evk.logN
        _need(out0, wo, "out0")
        _need(out1, wo, "out1")
        _check("fhe_mul_relin_rescale", load_library().fhe_mul_relin_rescale(
            self._h, evk.handle, evk.logN, logq, bits, _ptr(x0), _ptr(x1), _ptr(y0), _ptr(y1), _ptr(out0),
            _ptr(out1), cnum, _stream(stream)))


def _ct_in(x: "Ciphertext") -> CT:
    w = x.cnum * nlimbs(x.logq) << x.logN
    _need(x.c0, w, "c0")
    _need(x.c1, w, "c1")
    return CT(_ptr(x.c0), _ptr(x.c1), x.cnum, x.logN, x.logq, x.logp, x.scheme, x.t, x.gamma)


def _ct_call(ctx: Context, fn: str, args, out, cnum: int, logN: int, logq_out: int, stream):
    """Calls an fhe_ct entry point whose last two arguments are (out, stream) and
    returns the output Ciphertext with the metadata the library wrote."""
    o0, o1 = out
    w = cnum * nlimbs(logq_out) << logN
    _need(o0, w, "out c0")
    _need(o1, w, "out c1")
    o = CT(_ptr(o0), _ptr(o1), 0, 0, 0, 0, 0, 0, 0)
    _check(fn, getattr(load_library(), fn)(ctx.handle, *args, ctypes.byref(o), _stream(stream)))
    return Ciphertext(o0, o1, o.logN, o.logq, o.logp, o.scheme, o.t, o.gamma, o.cnum)


def _ctx_ct_methods():
    """Context methods over Ciphertext (fhe_ct) values: each takes the output buffers
    ``out = (c0, c1)`` and returns the output Ciphertext with its metadata."""

    def ct_mul_relin(self, evk, x, y, out, bits: int = 0, stream=None):
        return _ct_call(self, "fhe_ct_mul_relin_rescale",
                        (evk.handle, ctypes.byref(_ct_in(x)), ctypes.byref(_ct_in(y)), bits), out, x.cnum,
                        x.logN, x.logq - bits, stream)

    def ct_rescale(self, x, bits: int, out, stream=None):
        return _ct_call(self, "fhe_ct_rescale", (ctypes.byref(_ct_in(x)), bits), out, x.cnum, x.logN,
                        x.logq - bits, stream)

    def ct_moddown(self, x, bits: int, out, stream=None):
        return _ct_call(self, "fhe_ct_moddown", (ctypes.byref(_ct_in(x)), bits), out, x.cnum, x.logN,
                        x.logq - bits, stream)

    def ct_add(self, x, y, out, stream=None):
        return _ct_call(self, "fhe_ct_add", (ctypes.byref(_ct_in(x)), ctypes.byref(_ct_in(y))), out, x.cnum,
                        x.logN, x.logq, stream)

    def ct_sub(self, x, y, out, stream=None):
        return _ct_call(self, "fhe_ct_sub", (ctypes.byref(_ct_in(x)), ctypes.byref(_ct_in(y))), out, x.cnum,
                        x.logN, x.logq, stream)

    def ct_negate(self, x, out, stream=None):
        return _ct_call(self, "fhe_ct_negate", (ctypes.byref(_ct_in(x)),), out, x.cnum, x.logN, x.logq, stream)

    def ct_imult(self, x, out, stream=None):
        return _ct_call(self, "fhe_ct_imult", (ctypes.byref(_ct_in(x)),), out, x.cnum, x.logN, x.logq, stream)

    def ct_multconst(self, x, k: int, out, logp_k: int = 0, stream=None):
        """k: a Python int, |k| < 2^256."""
        import numpy as np
        mag = abs(int(k))
        kl = max(1, (mag.bit_length() + 31) // 32)
        if kl > 8:
            raise ValueError("constant beyond 256 bits")
        arr = np.array([(mag >> (32 * i)) & 0xFFFFFFFF for i in range(kl)], dtype=np.uint32)
        return _ct_call(self, "fhe_ct_multconst",
                        (ctypes.byref(_ct_in(x)), arr.ctypes.data_as(_P), kl, int(k < 0), logp_k), out, x.cnum,
                        x.logN, x.logq, stream)

    def ct_multconstvec(self, x, m, mcount: int, out, logp_m: int = 0, stream=None):
        _need(m, mcount * nlimbs(x.logq) << x.logN, "m")
        return _ct_call(self, "fhe_ct_multconstvec", (ctypes.byref(_ct_in(x)), _ptr(m), mcount, logp_m), out,
                        x.cnum, x.logN, x.logq, stream)

    def ct_addconst(self, x, m, mcount: int, out, stream=None):
        _need(m, mcount * nlimbs(x.logq) << x.logN, "m")
        return _ct_call(self, "fhe_ct_addconst", (ctypes.byref(_ct_in(x)), _ptr(m), mcount), out, x.cnum,
                        x.logN, x.logq, stream)

    def ct_key_switch(self, key, x, out, stream=None):
        return _ct_call(self, "fhe_ct_key_switch", (key.handle, ctypes.byref(_ct_in(x))), out, x.cnum, x.logN,
                        x.logq, stream)

    def ct_leftrotate(self, key, r: int, x, out, stream=None):
        return _ct_call(self, "fhe_ct_leftrotate", (key.handle, r, ctypes.byref(_ct_in(x))), out, x.cnum,
                        x.logN, x.logq, stream)

    def ct_conjugate(self, key, x, out, stream=None):
        return _ct_call(self, "fhe_ct_conjugate", (key.handle, ctypes.byref(_ct_in(x))), out, x.cnum, x.logN,
                        x.logq, stream)

    def automorphism(self, logN: int, logq: int, g: int, inp, out, count: int = 1, stream=None):
        w = count * nlimbs(logq) << logN
        _need(inp, w, "in")
        _need(out, w, "out")
        _check("fhe_automorphism", load_library().fhe_automorphism(self._h, logN, logq, g, _ptr(inp), _ptr(out),
                                                                   count, _stream(stream)))

    def key_switch(self, key, logq: int, in0, in1, out0, out1, cnum: int = 1, stream=None):
        w = cnum * nlimbs(logq) << key.logN
        for t, n in ((in0, "in0"), (in1, "in1"), (out0, "out0"), (out1, "out1")):
            _need(t, w, n)
        _check("fhe_key_switch", load_library().fhe_key_switch(self._h, key.handle, key.logN, logq, _ptr(in0),
                                                               _ptr(in1), _ptr(out0), _ptr(out1), cnum,
                                                               _stream(stream)))

    def ct_bootstrap(self, params: dict, relin, rot: dict, conj, c2s, s2c, k_y: int, taylor, x, out, stream=None):
        """fhe_ct_bootstrap.  params: the fhe_boot_params fields; rot: rotation amount ->
        EvalKey (Galois); c2s, s2c: device uint32[n][L_Q][N]; taylor: ints (degree + 1).
        out = (c0, c1), each L_Q N words; returns the output Ciphertext."""
        P = BootParams(**params)
        n, LQ, N = 1 << P.logslots, nlimbs(P.logQ), 1 << P.logN
        _need(c2s, n * LQ * N, "c2s")
        _need(s2c, n * LQ * N, "s2c")
        for t, nm in ((out[0], "out c0"), (out[1], "out c1")):
            _need(t, LQ * N, nm)
        nrot = max(rot) + 1
        arr = (_P * nrot)()
        for r, k in rot.items():
            arr[r] = k.handle.value
        tay = (ctypes.c_int64 * len(taylor))(*[int(v) for v in taylor])
        K = BootKeys(relin.handle.value, ctypes.cast(arr, _P), nrot, conj.handle.value, _ptr(c2s), _ptr(s2c),
                     int(k_y), ctypes.cast(tay, _P))
        o = CT(_ptr(out[0]), _ptr(out[1]), 0, 0, 0, 0, 0, 0, 0)
        _check("fhe_ct_bootstrap", load_library().fhe_ct_bootstrap(self._h, ctypes.byref(P), ctypes.byref(K),
                                                                   ctypes.byref(_ct_in(x)), ctypes.byref(o),
                                                                   _stream(stream)))
        return Ciphertext(out[0], out[1], o.logN, o.logq, o.logp, o.scheme, o.t, o.gamma, o.cnum)

    for f in (ct_mul_relin, ct_rescale, ct_moddown, ct_add, ct_sub, ct_negate, ct_imult, ct_multconst,
              ct_multconstvec, ct_addconst, ct_key_switch, ct_leftrotate, ct_conjugate, automorphism, key_switch,
              ct_bootstrap):
        setattr(Context, f.__name__, f)


_ctx_ct_methods()


class EvalKey:
    """Relinearization key (b', a') at modulus P 2^logQ; host limb arrays uint32[L][N].
    With ``g`` (odd), a Galois switching key for X -> X^g (fhe_galois_key_create)."""

    def __init__(self, ctx: Context, scheme: int, t: int, logN: int, logQ: int, logP: int, b_limbs, a_limbs,
                 g: int = 0):
        import numpy as np
        lib = load_library()
        L = nlimbs(logP + logQ)
        b = np.ascontiguousarray(b_limbs, dtype=np.uint32)
        a = np.ascontiguousarray(a_limbs, dtype=np.uint32)
        if b.shape != (L, 1 << logN) or a.shape != (L, 1 << logN):
            raise ValueError(f"key limbs must be uint32[{L}][{1 << logN}]")
        h = ctypes.c_void_p()
        bp, ap = b.ctypes.data_as(ctypes.c_void_p), a.ctypes.data_as(ctypes.c_void_p)
        if g:
            _check("fhe_galois_key_create", lib.fhe_galois_key_create(ctx.handle, scheme, t, logN, logQ, logP, g,
                                                                      bp, ap, ctypes.byref(h)))
        else:
            _check("fhe_evk_create", lib.fhe_evk_create(ctx.handle, scheme, t, logN, logQ, logP, bp, ap,
                                                        ctypes.byref(h)))
        self._h = h
        self.ctx, self.scheme, self.t, self.g = ctx, scheme, t, g
        self.logN, self.logQ, self.logP = logN, logQ, logP

    @property
    def handle(self):
        return self._h

    def prepare(self, logq: int, stream=None):
        _check("fhe_evk_prepare", load_library().fhe_evk_prepare(self._h, logq, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load_library().fhe_evk_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPlan:
    """A planned batch of uneven HE-mults (fhe_batch_plan).  `jobs` is a list of
    (evk, logq, bits, x0, x1, y0, y1, out0, out1) with torch CUDA tensors; the tensors
    must stay alive while the plan exists."""

    def __init__(self, ctx: Context, jobs, flags: int = PLAN_GRAPH, stream=None):
        lib = load_library()
        arr = (Job * len(jobs))()
        self._keep = []
        for i, (evk, logq, bits, x0, x1, y0, y1, o0, o1) in enumerate(jobs):
            w = nlimbs(logq) << evk.logN
            wo = nlimbs(logq - bits) << evk.logN
            for t, n in ((x0, w), (x1, w), (y0, w), (y1, w), (o0, wo), (o1, wo)):
                _need(t, n, "job buffer")
            arr[i] = Job(evk.handle.value, logq, bits, _ptr(x0), _ptr(x1), _ptr(y0), _ptr(y1), _ptr(o0), _ptr(o1))
            self._keep.append((evk, x0, x1, y0, y1, o0, o1))
        h = ctypes.c_void_p()
        _check("fhe_batch_plan", lib.fhe_batch_plan(ctx.handle, arr, len(jobs), flags, _stream(stream),
                                                    ctypes.byref(h)))
        self._h = h
        self.ctx = ctx

    def run(self, stream=None):
        _check("fhe_batch_run", load_library().fhe_batch_run(self._h, _stream(stream)))

    def info(self) -> dict:
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check("fhe_batch_info", load_library().fhe_batch_info(self._h, ctypes.byref(a), ctypes.byref(b),
                                                               ctypes.byref(c)))
        return {"cells": a.value, "kernels": b.value, "graphed": bool(c.value)}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load_library().fhe_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Done(ctypes.Structure):
    """fhe_done: completion record of one served request."""
    _fields_ = [("ticket", ctypes.c_uint64), ("status", _I), ("batch", _I), ("t_arrive", ctypes.c_uint64),
                ("t_start", ctypes.c_uint64), ("t_done", ctypes.c_uint64)]


def clock_ns() -> int:
    return int(load_library().fhe_clock_ns())


class Server:
    """Continuous-batching request loop (fhe_server_*).  Jobs are tuples
    (evk, logq, bits, x0, x1, y0, y1, out0, out1) of torch CUDA tensors, which must stay
    alive until reported done."""

    def __init__(self, ctx: Context, hbm_budget: int, nstreams: int = 4, max_batch: int = 16):
        h = ctypes.c_void_p()
        _check("fhe_server_create", load_library().fhe_server_create(ctx.handle, hbm_budget, nstreams, max_batch,
                                                                     ctypes.byref(h)))
        self._h = h
        self.ctx = ctx

    def submit(self, job, arrival_ns: int = 0, stream=None) -> int:
        """Queue a request; its inputs are read after the work queued so far on `stream`
        (default: torch's current stream)."""
        evk, logq, bits, x0, x1, y0, y1, o0, o1 = job
        j = Job(evk.handle.value, logq, bits, _ptr(x0), _ptr(x1), _ptr(y0), _ptr(y1), _ptr(o0), _ptr(o1))
        t = ctypes.c_uint64()
        _check("fhe_server_submit", load_library().fhe_server_submit(self._h, ctypes.byref(j), arrival_ns,
                                                                     _stream(stream), ctypes.byref(t)))
        return t.value

    def cancel(self):
        _check("fhe_server_cancel", load_library().fhe_server_cancel(self._h))

    def poll(self, max_n: int = 1024):
        buf = (Done * max_n)()
        n = ctypes.c_int()
        _check("fhe_server_poll", load_library().fhe_server_poll(self._h, buf, max_n, ctypes.byref(n)))
        return [buf[i] for i in range(n.value)]

    def drain(self):
        _check("fhe_server_drain", load_library().fhe_server_drain(self._h))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load_library().fhe_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _small(t, dtype, n: int, name: str):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name}: contiguous CUDA {dtype} tensor expected")
    _need(t, n, name)


def ckks_encode(z, logN: int, logp: int, logq: int):
    """Host CKKS encoding of complex slots z (length n = 2^logslots <= N/2) into
    [m]_(2^logq) limbs uint32[L][N] (numpy)."""
    import numpy as np
    z = np.ascontiguousarray(z, dtype=np.complex128)
    n = z.shape[0]
    logs = n.bit_length() - 1
    if n < 1 or n != 1 << logs:
        raise ValueError("slot count must be a power of two")
    re = np.ascontiguousarray(z.real)
    im = np.ascontiguousarray(z.imag)
    m = np.zeros((nlimbs(logq), 1 << logN), dtype=np.uint32)
    _check("fhe_ckks_encode", load_library().fhe_ckks_encode(
        logN, logs, logp, logq, re.ctypes.data_as(_P), im.ctypes.data_as(_P), m.ctypes.data_as(_P)))
    return m


def ckks_decode(phase, logN: int, logslots: int, logp: int, logq: int):
    """Host CKKS decoding of a phase uint32[L][N] (numpy) into n = 2^logslots complex slots."""
    import numpy as np
    ph = np.ascontiguousarray(phase, dtype=np.uint32)
    if ph.shape != (nlimbs(logq), 1 << logN):
        raise ValueError("phase must be uint32[L][N]")
    n = 1 << logslots
    re = np.zeros(n)
    im = np.zeros(n)
    _check("fhe_ckks_decode", load_library().fhe_ckks_decode(
        logN, logslots, logp, logq, ph.ctypes.data_as(_P), re.ctypes.data_as(_P), im.ctypes.data_as(_P)))
    return re + 1j * im


def to_device(arr, device: int = 0):
    """numpy uint32 array -> contiguous torch int32 CUDA tensor with the same bits."""
    import numpy as np
    import torch
    a = np.ascontiguousarray(arr, dtype=np.uint32)
    return torch.from_numpy(a.view(np.int32)).to(f"cuda:{device}")


def to_host(t):
    """torch int32 CUDA tensor -> numpy uint32 array with the same bits."""
    import numpy as np
    return t.detach().cpu().numpy().view(np.uint32)


@dataclass
class Ciphertext:
    """Device CipherTensor: c0, c1 int32 CUDA tensors holding uint32[cnum][L][N], plus
    the metadata of fhe_ct."""
    c0: object
    c1: object
    logN: int
    logq: int
    logp: int = 0
    scheme: int = CKKS
    t: int = 0
    gamma: int = 1
    cnum: int = 1
