// CKKS encoding and decoding with sparse packing (host code, double precision).
//
// The canonical embedding evaluates a real polynomial at the primitive 4n-th roots
// zeta^(r_j), r_j = 5^j mod 4n, j < n (the slot order of the paper's HEAAN-based
// scheme, Section 6: logs slots, scale 2^logp).  Both directions reduce to one
// length-2n complex DFT: the values at the odd powers zeta^(2s+1) are the DFT of
// u_k zeta^k with root omega = zeta^2, and the slots fill half of them (the other
// half are their conjugates).  This file holds its own radix-2 FFT.
#include <cmath>
#include <complex>
#include <cstdint>
#include <vector>

#include "fhe_mi355x.h"

namespace {

using cd = std::complex<double>;

// In place X_k = sum_j x_j exp(sign 2 pi i j k / n), n a power of two.
void fft(std::vector<cd>& x, int sign) {
  const size_t n = x.size();
  for (size_t i = 1, j = 0; i < n; ++i) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(x[i], x[j]);
  }
  std::vector<cd> w(n / 2 > 0 ? n / 2 : 1);
  for (size_t k = 0; k < n / 2; ++k) {
    const double a = sign * 2.0 * M_PI * (double)k / (double)n;
    w[k] = cd(std::cos(a), std::sin(a));
  }
  for (size_t len = 2; len <= n; len <<= 1) {
    const size_t step = n / len;
    for (size_t i = 0; i < n; i += len)
      for (size_t k = 0; k < len / 2; ++k) {
        const cd u = x[i + k], v = x[i + k + len / 2] * w[k * step];
        x[i + k] = u + v;
        x[i + k + len / 2] = u - v;
      }
  }
}

int check(int logN, int logslots, int logp, int logq) {
  if (logN < FHE_LOGN_MIN || logN > FHE_LOGN_MAX) return FHE_E_RANGE;
  if (logslots < 0 || logslots > logN - 1) return FHE_E_RANGE;
  if (logp < 1 || logp > 62 || logq < 1 || logq > 4096) return FHE_E_RANGE;
  return FHE_OK;
}

// Index into the 2n odd-power values of slot j (r_j = 5^j mod 4n) and of its conjugate.
void slot_index(int n, std::vector<size_t>& idx, std::vector<size_t>& cidx) {
  const uint64_t M = 4ull * (uint64_t)n;
  uint64_t r = 1;
  idx.resize(n);
  cidx.resize(n);
  for (int j = 0; j < n; ++j) {
    idx[j] = (size_t)((r - 1) / 2);
    cidx[j] = (size_t)((M - r - 1) / 2);
    r = r * 5 % M;
  }
}

}  // namespace

extern "C" {

int fhe_ckks_encode(int logN, int logslots, int logp, int logq, const double* re, const double* im, uint32_t* m) {
  if (!re || !im || !m) return FHE_E_INVAL;
  int rc = check(logN, logslots, logp, logq);
  if (rc != FHE_OK) return rc;
  const int N = 1 << logN, n = 1 << logslots, L = (logq + 31) / 32;
  const int gap = N / (2 * n);
  std::vector<size_t> idx, cidx;
  slot_index(n, idx, cidx);
  std::vector<cd> W(2 * (size_t)n, cd(0, 0));
  for (int j = 0; j < n; ++j) {
    W[idx[j]] = cd(re[j], im[j]);
    W[cidx[j]] = cd(re[j], -im[j]);
  }
  fft(W, -1);
  std::vector<int64_t> val(2 * (size_t)n);
  const double scale = std::ldexp(1.0, logp);
  for (int k = 0; k < 2 * n; ++k) {
    const double a = -2.0 * M_PI * (double)k / (4.0 * n);
    const double u = (W[k] * cd(std::cos(a), std::sin(a))).real() / (2.0 * n);
    const double v = std::floor(u * scale + 0.5);
    if (!(std::fabs(v) < std::ldexp(1.0, 62))) return FHE_E_RANGE;
    val[k] = (int64_t)v;
  }
  const uint32_t top = (logq & 31) ? (1u << (logq & 31)) - 1u : 0xFFFFFFFFu;
  for (long long i = 0; i < (long long)L * N; ++i) m[i] = 0;
  for (int k = 0; k < 2 * n; ++k) {
    const int64_t x = val[k];
    const uint32_t ext = x < 0 ? 0xFFFFFFFFu : 0u;
    for (int l = 0; l < L; ++l) {
      uint32_t w = l == 0 ? (uint32_t)x : (l == 1 ? (uint32_t)((uint64_t)x >> 32) : ext);
      if (l == L - 1) w &= top;
      m[(long long)l * N + (long long)k * gap] = w;
    }
  }
  return FHE_OK;
}

int fhe_ckks_decode(int logN, int logslots, int logp, int logq, const uint32_t* phase, double* re, double* im) {
  if (!phase || !re || !im) return FHE_E_INVAL;
  int rc = check(logN, logslots, logp, logq);
  if (rc != FHE_OK) return rc;
  const int N = 1 << logN, n = 1 << logslots, L = (logq + 31) / 32;
  const int gap = N / (2 * n);
  const int hb = (logq - 1) & 31, hl = (logq - 1) >> 5;
  const uint32_t top = (logq & 31) ? (1u << (logq & 31)) - 1u : 0xFFFFFFFFu;
  std::vector<cd> x(2 * (size_t)n);
  std::vector<uint32_t> w(L);
  for (int k = 0; k < 2 * n; ++k) {
    bool hi = false, low = false;
    for (int l = 0; l < L; ++l) {
      w[l] = phase[(long long)l * N + (long long)k * gap];
      if (l == L - 1) w[l] &= top;
      if (l == hl) {
        hi = (w[l] >> hb) & 1u;
        low = low || (w[l] & ((1u << hb) - 1u)) != 0;
      } else if (l < hl) {
        low = low || w[l] != 0;
      }
    }
    const bool neg = hi && low;  // x > 2^(logq-1): the centered value is x - 2^logq
    if (neg) {                   // magnitude 2^logq - x = (~x + 1) within logq bits
      uint64_t carry = 1;
      for (int l = 0; l < L; ++l) {
        const uint64_t t = (uint64_t)(uint32_t)~w[l] + carry;
        w[l] = (uint32_t)t;
        carry = t >> 32;
      }
      w[L - 1] &= top;
    }
    double mag = 0.0;
    for (int l = L - 1; l >= 0; --l) mag = mag * 4294967296.0 + (double)w[l];
    const double mu = neg ? -mag : mag;
    const double a = 2.0 * M_PI * (double)k / (4.0 * n);
    x[k] = mu * cd(std::cos(a), std::sin(a));
  }
  fft(x, +1);
  std::vector<size_t> idx, cidx;
  slot_index(n, idx, cidx);
  const double inv = std::ldexp(1.0, -logp);
  for (int j = 0; j < n; ++j) {
    re[j] = x[idx[j]].real() * inv;
    im[j] = x[idx[j]].imag() * inv;
  }
  return FHE_OK;
}

}  // extern "C"
