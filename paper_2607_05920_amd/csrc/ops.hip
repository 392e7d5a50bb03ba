// gfx950 kernels of the operations beside multiplication (Section 6.2 operation list;
// Section 6.1 pairwise and broadcast modes; Section 2.5 Galois automorphisms):
// coefficient-wise sums and negation, reduction to a lower level, products with an
// integer constant, and the signed permutations X^k -> X^(k g) and X^k -> X^(k + s).
//
// Every kernel runs one thread per coefficient over a polynomial's limbs (limb-major
// layout: a wave's loads and stores of one limb row are 256 contiguous bytes), with
// the carry chain of the multiprecision value in registers.  A thread reads limb l of
// its own coefficient before it writes limb l, so the coefficient-wise kernels may run
// in place; the permutations read other coefficients and may not.
#include "fhe_internal.h"

namespace fhe {

// out_z = [(-1)^negx x_z + (-1)^negy y_z]_(2^logq) for polynomial z = 2 c + i
// (ciphertext c, component i); y_z is zero where its component pointer is null.
// Negation is two's complement over the limbs (~v + 1), so both signs fold into one
// add-with-carry chain whose carry starts at negx + negy.
__global__ __launch_bounds__(256) void limb_sum_kernel(LimbSumArgs a) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= a.N) return;
  const int z = blockIdx.y, c = z >> 1, i = z & 1;
  const uint32_t* x = (i ? a.x1 : a.x0) + (long long)c * a.xstride + j;
  const uint32_t* yb = i ? a.y1 : a.y0;
  const uint32_t* y = yb ? yb + (long long)c * a.ystride + j : nullptr;
  uint32_t* o = (i ? a.out1 : a.out0) + (long long)c * a.ostride + j;
  const uint32_t mx = a.negx ? 0xFFFFFFFFu : 0u, my = a.negy ? 0xFFFFFFFFu : 0u;
  uint64_t carry = (uint64_t)(a.negx != 0) + (uint64_t)(y && a.negy);
  for (int l = 0; l < a.L; ++l) {
    const long long off = (long long)l * a.N;
    const uint64_t s = (uint64_t)(x[off] ^ mx) + (y ? (uint64_t)(y[off] ^ my) : 0ull) + carry;
    uint32_t w = (uint32_t)s;
    carry = s >> 32;
    if (l == a.L - 1) w &= a.topmask;
    o[off] = w;
  }
}

// Signed permutation of coefficients: output position k < N takes the input at
// i = (k mul + add) mod 2N, negated when i >= N (then from position i - N), since
// X^N = -1.  With mul = g^-1 mod 2N, add = 0 this is the automorphism X -> X^g
// (input coefficient i lands at i g mod 2N); with mul = 1, add = 2N - s it is the
// product with the monomial X^s.
__global__ __launch_bounds__(256) void signed_perm_kernel(PermArgs a) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  const int N = 1 << a.logN;
  if (k >= N) return;
  const int z = blockIdx.y, c = z / a.comps, i = z % a.comps;
  const uint32_t twoN_mask = (2u << a.logN) - 1u;
  const uint32_t src = ((uint32_t)k * a.mul + a.add) & twoN_mask;
  const bool neg = src >= (uint32_t)N;
  const uint32_t* x = (i ? a.in1 : a.in0) + (long long)c * a.istride + (src & (uint32_t)(N - 1));
  uint32_t* o = (i ? a.out1 : a.out0) + (long long)c * a.ostride + k;
  const uint32_t m = neg ? 0xFFFFFFFFu : 0u;
  uint64_t carry = neg ? 1u : 0u;
  for (int l = 0; l < a.L; ++l) {
    const long long off = (long long)l * N;
    const uint64_t s = (uint64_t)(x[off] ^ m) + carry;
    uint32_t w = (uint32_t)s;
    carry = s >> 32;
    if (l == a.L - 1) w &= a.topmask;
    o[off] = w;
  }
}

// out_z = [(-1)^neg x_z k]_(2^logq) for an integer constant k of klimbs <= 8 limbs.
// Product limb l is sum_(j < klimbs) x_(l-j) k_j plus the carry from limb l - 1: the
// thread keeps the last 8 limbs of x in a register window.  The products' low and
// high halves are summed apart so that no sum overflows 64 bits.
__global__ __launch_bounds__(256) void const_mul_kernel(ConstMulArgs a) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= a.N) return;
  const int z = blockIdx.y, c = z >> 1, i = z & 1;
  const uint32_t* x = (i ? a.in1 : a.in0) + (long long)c * a.istride + j;
  uint32_t* o = (i ? a.out1 : a.out0) + (long long)c * a.ostride + j;
  uint32_t win[kConstMaxLimbs];
#pragma unroll
  for (int t = 0; t < kConstMaxLimbs; ++t) win[t] = 0u;
  const uint32_t nm = a.neg ? 0xFFFFFFFFu : 0u;
  uint64_t carry = 0, ncarry = a.neg ? 1u : 0u;
  for (int l = 0; l < a.L; ++l) {
#pragma unroll
    for (int t = kConstMaxLimbs - 1; t > 0; --t) win[t] = win[t - 1];
    win[0] = x[(long long)l * a.N];
    uint64_t lo = carry & 0xFFFFFFFFull, hi = carry >> 32;
#pragma unroll
    for (int t = 0; t < kConstMaxLimbs; ++t) {
      if (t < a.klimbs) {
        const uint64_t p = (uint64_t)win[t] * a.k[t];
        lo += (uint32_t)p;
        hi += p >> 32;
      }
    }
    carry = (lo >> 32) + hi;
    const uint64_t s = (uint64_t)((uint32_t)lo ^ nm) + ncarry;
    uint32_t w = (uint32_t)s;
    ncarry = s >> 32;
    if (l == a.L - 1) w &= a.topmask;
    o[(long long)l * a.N] = w;
  }
}

hipError_t launch_limb_sum(const LimbSumArgs& a, int cnum, hipStream_t st) {
  if (cnum <= 0) return hipSuccess;
  if (a.N <= 0 || a.L <= 0) return hipErrorInvalidValue;
  // bytes: x read, y read where present, out written
  const double ypolys = (a.y0 ? 1.0 : 0.0) + (a.y1 ? 1.0 : 0.0);
  Bracket br(KID_COEFFWISE, st, 4.0 * cnum * a.N * (double)a.L * (4.0 + ypolys));
  hipLaunchKernelGGL(limb_sum_kernel, dim3((a.N + 255) / 256, 2 * cnum), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_signed_perm(const PermArgs& a, int cnum, hipStream_t st) {
  if (cnum <= 0) return hipSuccess;
  if (a.logN < 1 || a.logN > kLogNMax || a.L <= 0) return hipErrorInvalidValue;
  const int N = 1 << a.logN;
  Bracket br(KID_COEFFWISE, st, 8.0 * a.comps * cnum * N * (double)a.L);
  if (a.comps != 1 && a.comps != 2) return hipErrorInvalidValue;
  hipLaunchKernelGGL(signed_perm_kernel, dim3((N + 255) / 256, a.comps * cnum), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_const_mul(const ConstMulArgs& a, int cnum, hipStream_t st) {
  if (cnum <= 0) return hipSuccess;
  if (a.N <= 0 || a.L <= 0 || a.klimbs < 1 || a.klimbs > kConstMaxLimbs) return hipErrorInvalidValue;
  Bracket br(KID_COEFFWISE, st, 16.0 * cnum * a.N * (double)a.L);
  hipLaunchKernelGGL(const_mul_kernel, dim3((a.N + 255) / 256, 2 * cnum), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace fhe
