// Word-level modular arithmetic for 30-bit primes q < 2^30 on gfx950.
//
// On gfx950 the 32-bit multiplies (v_mul_lo_u32, v_mul_hi_u32) and the 32x32+64
// multiply-add (v_mad_u64_u32) issue at the full VALU rate, the same as an add.
// Every helper is therefore written to minimise the total instruction count, not
// only the multiplies: lazy ranges ([0, 2q), [0, 4q)) and the unsigned
// min(x, x - m) trick replace compare-and-branch reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fhe {

// Per-prime constants, read wave-uniformly (scalar loads).
struct PrimeC {
  uint32_t q;      // the prime, 2^29 < q < 2^30, q = 1 mod 2^17
  uint32_t qneg;   // -q^-1 mod 2^32 (Montgomery)
  uint32_t c32;    // 2^32 mod q (folds a 64-bit accumulator)
  uint32_t two_q;  // 2q
};

// x mod m for x < 2m: if x < m, x - m wraps above x and min keeps x.
__device__ __forceinline__ uint32_t csub(uint32_t x, uint32_t m) {
  uint32_t y = x - m;
  return y < x ? y : x;
}

__device__ __forceinline__ uint32_t add_mod(uint32_t a, uint32_t b, uint32_t q) {
  return csub(a + b, q);
}

__device__ __forceinline__ uint32_t sub_mod(uint32_t a, uint32_t b, uint32_t q) {
  return csub(a + q - b, q);
}

// 32x32 -> 64 product plus a 64-bit addend: one v_mad_u64_u32.
__device__ __forceinline__ uint64_t mad64(uint32_t a, uint32_t b, uint64_t c) {
  return (uint64_t)a * (uint64_t)b + c;
}

// Shoup multiplication by a constant w < q with wp = floor(w 2^32 / q):
// for any a < 2^32 returns a w mod q in [0, 2q).
__device__ __forceinline__ uint32_t shoup_lazy(uint32_t a, uint32_t w, uint32_t wp, uint32_t q) {
  uint32_t qh = __umulhi(a, wp);
  return a * w - qh * q;
}

// Montgomery reduction: for T < q 2^32 returns T 2^-32 mod q in [0, 2q).
__device__ __forceinline__ uint32_t redc_lazy(uint64_t T, uint32_t q, uint32_t qneg) {
  uint32_t m = (uint32_t)T * qneg;
  uint64_t s = mad64(m, q, T);  // T + m q < 2^63, divisible by 2^32
  return (uint32_t)(s >> 32);
}

// Montgomery product a b 2^-32 mod q for a, b < q, canonical.
__device__ __forceinline__ uint32_t mont_mul(uint32_t a, uint32_t b, uint32_t q, uint32_t qneg) {
  return csub(redc_lazy(mad64(a, b, 0), q, qneg), q);
}

// acc = hi 2^32 + lo  ->  hi (2^32 mod q) + lo, same value mod q, below 2^62 + 2^32.
__device__ __forceinline__ uint64_t fold64(uint64_t acc, uint32_t c32) {
  return mad64((uint32_t)(acc >> 32), c32, (uint64_t)(uint32_t)acc);
}

// Any 64-bit accumulator -> acc 2^-32 mod q, canonical.  Two folds bring it below
// 2^60 + 2^32 < q 2^32, the Montgomery input range.
__device__ __forceinline__ uint32_t reduce64_mont(uint64_t acc, const PrimeC& p) {
  acc = fold64(acc, p.c32);
  acc = fold64(acc, p.c32);
  return csub(redc_lazy(acc, p.q, p.qneg), p.q);
}

}  // namespace fhe
