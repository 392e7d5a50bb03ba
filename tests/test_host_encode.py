"""Host CKKS encoding helpers of the C ABI (fhe_ckks_encode / fhe_ckks_decode; no
device needed) against the oracle's encoding (R9).  Both sides evaluate the same
map in double precision through different FFTs, so an encoded coefficient may
differ by one where 2^logp u_k + 1/2 falls within rounding of an integer; the
decoded slots agree to double-precision rounding of the transform."""
import numpy as np
import pytest

import paper_2607_05920_amd as fhe
import synth
from oracle import limbs as olimbs
from oracle import scheme

try:
    fhe.load_library()
    HAVE_LIB = True
except fhe.LibraryMissing:
    HAVE_LIB = False

pytestmark = pytest.mark.skipif(not HAVE_LIB, reason="library not built")


def _coeffs(m, logq):
    """Centered integer coefficients of limbs uint32[L][N] modulo 2^logq."""
    Q = 1 << logq
    return [scheme.center(v, Q) for v in olimbs.poly_from_limbs(m)]


@pytest.mark.parametrize("logN,logslots,logp,logq", [(10, 9, 40, 200), (10, 0, 30, 64), (11, 4, 40, 96),
                                                    (12, 11, 50, 438), (13, 7, 20, 33),
                                                    (13, 12, 50, 438)])
def test_encode_matches_oracle(logN, logslots, logp, logq):
    rng = np.random.default_rng(logN * 100 + logslots)
    N, n = 1 << logN, 1 << logslots
    z = synth.unit_disk(rng, n)
    m = fhe.ckks_encode(z, logN, logp, logq)
    assert m.shape == (synth.nlimbs(logq), N)
    got = _coeffs(m, logq)
    want = scheme.ckks_encode(z, N, logp)
    Q = 1 << logq
    want_c = [scheme.center(v, Q) for v in want]
    diff = [abs(a - b) for a, b in zip(got, want_c)]
    assert max(diff) <= 1
    # where the two double-precision transforms round differently, the value being
    # rounded must lie at a rounding boundary: checked with the direct sum in
    # extended precision
    gap = N // (2 * n)
    r = np.array([pow(5, j, 4 * n) for j in range(n)], dtype=np.int64)
    zl = z.astype(np.clongdouble)
    for i in np.nonzero(diff)[0]:
        k = i // gap
        ang = np.longdouble(2) * np.pi * ((r * k) % (4 * n)).astype(np.longdouble) / np.longdouble(4 * n)
        u = np.sum(zl.real * np.cos(ang) + zl.imag * np.sin(ang)) / n
        v = u * np.longdouble(2) ** logp + np.longdouble(0.5)
        assert abs(v - np.round(v)) < 2.0 ** (logp - 52)   # two ulps at magnitude 2^logp
    assert all(got[k] == 0 for k in range(N) if k % gap)          # sparse packing
    assert int(m[-1].max()) < (1 << (logq - 32 * (m.shape[0] - 1)))  # top limb masked


@pytest.mark.parametrize("logN,logslots,logp,logq", [(10, 9, 40, 200), (12, 5, 45, 128), (13, 12, 40, 438)])
def test_decode_roundtrip_and_oracle(logN, logslots, logp, logq):
    rng = np.random.default_rng(7 + logN)
    N, n = 1 << logN, 1 << logslots
    z = synth.unit_disk(rng, n)
    m = fhe.ckks_encode(z, logN, logp, logq)
    back = fhe.ckks_decode(m, logN, logslots, logp, logq)
    # rounding the scaled coefficients to integers: error <= 2n * 2^-logp / 2 per slot
    assert np.max(np.abs(back - z)) <= n * 2.0 ** -logp + 1e-12
    want = scheme.ckks_decode(_coeffs(m, logq), n, logp)
    assert np.max(np.abs(back - want)) <= 1e-9


def test_decode_large_and_negative_phase():
    """A phase with coefficients spread over the whole centered range mod 2^logq
    (negative ones included): decoded slots agree with the oracle's to double
    rounding, relative to their size."""
    logN, logslots, logp, logq = 10, 9, 40, 150
    rng = np.random.default_rng(3)
    ph = synth.uniform_limbs(rng, logq, 1 << logN)
    got = fhe.ckks_decode(ph, logN, logslots, logp, logq)
    want = scheme.ckks_decode(_coeffs(ph, logq), 1 << logslots, logp)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


def test_encode_rejects_bad_ranges():
    lib = fhe.load_library()
    z = np.zeros(4)
    m = np.zeros(64 * 1024, dtype=np.uint32)
    P = fhe._P
    args = lambda: (z.ctypes.data_as(P), z.ctypes.data_as(P), m.ctypes.data_as(P))
    assert lib.fhe_ckks_encode(10, 10, 40, 64, *args()) == -3     # logslots > logN - 1
    assert lib.fhe_ckks_encode(9, 2, 40, 64, *args()) == -3       # logN below the range
    assert lib.fhe_ckks_encode(10, 2, 63, 64, *args()) == -3      # scale too large
    assert lib.fhe_ckks_encode(10, 2, 40, 64, None, None, None) == -1
    with pytest.raises(fhe.FheError):
        fhe.ckks_encode(np.full(4, 2.0 ** 30), 10, 40, 64)      # |2^logp u_k| >= 2^62
