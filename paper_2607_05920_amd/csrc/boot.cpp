// CKKS bootstrapping (Section 6.2 `bootstrap`; Section 7.2 logT) composed from the
// library's own fhe_ct operations on one stream: modulus raise, SubSum (rotations),
// CoeffToSlot (rotations times encoded diagonals), the real/imaginary split
// (conjugation, imult), EvalMod (a product with 2 pi / 2^logT, a Taylor polynomial of
// exp(i y) from a product tree, logT squarings, the imaginary part), and SlotToCoeff.
// Every step is exact integer arithmetic through the C ABI; the encoded diagonals and
// the integer constants are inputs, so the output bits follow from the inputs alone.
// Steps and level matching (moddown of the higher operand before an addition or a
// product) are the reading written out in the header.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <vector>

#include "fhe_mi355x.h"

namespace {

// Device buffers of ciphertexts at the top level (2 L_Q N words each), reused.
class CtPool {
 public:
  CtPool(size_t words) : words_(words) {}
  ~CtPool() {
    for (uint32_t* p : all_) hipFree(p);
  }
  uint32_t* get() {
    if (!free_.empty()) {
      uint32_t* p = free_.back();
      free_.pop_back();
      return p;
    }
    uint32_t* p = nullptr;
    if (hipMalloc((void**)&p, words_ * 4) != hipSuccess) return nullptr;
    all_.push_back(p);
    return p;
  }
  void put(uint32_t* p) {
    if (p) free_.push_back(p);
  }

 private:
  size_t words_;
  std::vector<uint32_t*> all_, free_;
};

class Boot {
 public:
  Boot(fhe_ctx* c, const fhe_boot_params& P, const fhe_boot_keys& K, void* st)
      : c_(c), P_(P), K_(K), st_(st), half_((size_t)((P.logQ + 31) / 32) << P.logN), pool_(4 * half_) {}

  int rc = FHE_OK;

  // A ciphertext value owning one pool buffer, room for a CipherTensor of up to two at
  // the top level: c0 at its start, c1 at 2 half_ (a CipherTensor's ciphertexts follow
  // each other at its level's stride inside each).
  struct V {
    fhe_ct ct{};
    uint32_t* buf = nullptr;
  };

  V fresh() {
    V v;
    v.buf = pool_.get();
    if (!v.buf && rc == FHE_OK) rc = FHE_E_NOMEM;
    v.ct.c0 = v.buf;
    v.ct.c1 = v.buf ? v.buf + 2 * half_ : nullptr;
    return v;
  }
  // ciphertext i of a CipherTensor value, as a one-ciphertext view (not owned)
  fhe_ct part(const V& x, int i) const {
    fhe_ct p = x.ct;
    const size_t stride = (size_t)((x.ct.logq + 31) / 32) << P_.logN;
    p.c0 = x.ct.c0 + i * stride;
    p.c1 = x.ct.c1 + i * stride;
    p.cnum = 1;
    return p;
  }
  void drop(V& v) {
    pool_.put(v.buf);
    v.buf = nullptr;
  }
  bool ok() const { return rc == FHE_OK; }
  void check(int r) {
    if (rc == FHE_OK && r != FHE_OK) rc = r;
  }

  // a copy at level logq (moddown, or a plain copy at the same level)
  V level(const V& x, int logq) {
    V y = fresh();
    if (ok()) check(fhe_ct_moddown(c_, &x.ct, x.ct.logq - logq, &y.ct, st_));
    return y;
  }
  // the pair brought to the lower of the two levels (new values)
  void match(const V& x, const V& y, V& xo, V& yo) {
    const int q = std::min(x.ct.logq, y.ct.logq);
    xo = level(x, q);
    yo = level(y, q);
  }
  V add(const V& x, const V& y, bool sub = false) {
    V a, b;
    match(x, y, a, b);
    V o = fresh();
    if (ok()) check(sub ? fhe_ct_sub(c_, &a.ct, &b.ct, &o.ct, st_) : fhe_ct_add(c_, &a.ct, &b.ct, &o.ct, st_));
    drop(a);
    drop(b);
    return o;
  }
  V mul(const V& x, const V& y) {  // product at the lower level, rescaled by the working scale
    V a, b;
    match(x, y, a, b);
    V o = fresh();
    if (ok()) check(fhe_ct_mul_relin_rescale(c_, K_.relin, &a.ct, &b.ct, a.ct.logp, &o.ct, st_));
    drop(a);
    drop(b);
    return o;
  }
  V imult(const V& x) {
    V o = fresh();
    if (ok()) check(fhe_ct_imult(c_, &x.ct, &o.ct, st_));
    return o;
  }
  V rotate(const V& x, int r) {
    V o = fresh();
    fhe_evk* k = (r > 0 && r < K_.nrot) ? K_.rot[r] : nullptr;
    if (!k && rc == FHE_OK) rc = FHE_E_INVAL;
    if (ok()) check(fhe_ct_leftrotate(c_, k, r, &x.ct, &o.ct, st_));
    return o;
  }
  V conj(const V& x) {
    V o = fresh();
    if (ok()) check(fhe_ct_conjugate(c_, K_.conj, &x.ct, &o.ct, st_));
    return o;
  }
  V rescale(const V& x, int bits) {
    V o = fresh();
    if (ok()) check(fhe_ct_rescale(c_, &x.ct, bits, &o.ct, st_));
    return o;
  }
  // x times k / 2^(logc + extra), kept at x's scale
  V constant(const V& x, int64_t k, int extra) {
    uint32_t limbs[2];
    const uint64_t mag = k < 0 ? (uint64_t)0 - (uint64_t)k : (uint64_t)k;
    limbs[0] = (uint32_t)mag;
    limbs[1] = (uint32_t)(mag >> 32);
    V t = fresh();
    if (ok()) check(fhe_ct_multconst(c_, &x.ct, limbs, 2, k < 0, P_.logc, &t.ct, st_));
    V o = rescale(t, P_.logc + extra);
    drop(t);
    o.ct.logp = x.ct.logp;
    return o;
  }
  // sum_d rotation_d(x) * diag_d, rescaled by logc; diags: device [n][L_Q][N] mod 2^logQ
  V linear(const V& x, const uint32_t* diags) {
    const int n = 1 << P_.logslots;
    V acc;
    bool have = false;
    for (int d = 0; d < n && ok(); ++d) {
      V r = d == 0 ? level(x, x.ct.logq) : rotate(x, d);
      // the diagonal mod 2^logq: its low limbs, the top one masked (a moddown of a
      // one-ciphertext view whose two components are the diagonal)
      fhe_ct dg{};
      dg.c0 = dg.c1 = const_cast<uint32_t*>(diags) + (size_t)d * half_;
      dg.cnum = 1;
      dg.logN = P_.logN;
      dg.logq = P_.logQ;
      dg.scheme = FHE_CKKS;
      dg.gamma = 1;
      V m = fresh();
      if (ok()) check(fhe_ct_moddown(c_, &dg, P_.logQ - r.ct.logq, &m.ct, st_));
      V term = fresh();
      if (ok()) check(fhe_ct_multconstvec(c_, &r.ct, m.ct.c0, 1, P_.logc, &term.ct, st_));
      drop(m);
      drop(r);
      if (!have) {
        acc = term;
        have = true;
      } else {
        V s = add(acc, term);
        drop(acc);
        drop(term);
        acc = s;
      }
    }
    V o = rescale(acc, P_.logc);
    drop(acc);
    return o;
  }
  // i (conj E - E) / 2: the imaginary part of every slot (the halving as logp + 1)
  V imag_part(const V& E) {
    V ec = conj(E);
    V d = add(ec, E, true);
    drop(ec);
    V o = imult(d);
    drop(d);
    o.ct.logp += 1;
    return o;
  }
  // EvalMod: real slots x -> sin(2 pi x)
  V eval_mod(const V& x) {
    std::map<int, V> pw;
    pw[1] = constant(x, K_.k_y, P_.logT);
    for (int k = 2; k <= P_.degree && ok(); ++k) {
      int h = 1;
      while (2 * h <= k) h *= 2;
      pw[k] = h != k ? mul(pw[h], pw[k - h]) : mul(pw[k / 2], pw[k / 2]);
    }
    V re, im;
    bool hre = false, him = false;
    for (int k = 1; k <= P_.degree && ok(); ++k) {
      V term = constant(pw[k], K_.taylor[k], 0);
      V& tgt = (k % 2 == 0) ? re : im;
      bool& have = (k % 2 == 0) ? hre : him;
      if (!have) {
        tgt = term;
        have = true;
      } else {
        V s = add(tgt, term);
        drop(tgt);
        drop(term);
        tgt = s;
      }
    }
    for (auto& kv : pw) drop(kv.second);
    if (!ok()) return V{};
    V a, b;
    match(re, im, a, b);
    drop(re);
    drop(im);
    // the constant 1 at a's scale: 2^logp at coefficient 0
    V one = fresh();
    if (ok()) {
      const size_t words = (size_t)((a.ct.logq + 31) / 32) << P_.logN;
      check(hipMemsetAsync(one.ct.c0, 0, words * 4, (hipStream_t)st_) == hipSuccess ? FHE_OK : FHE_E_DEVICE);
      const int lp = a.ct.logp;
      if (ok() && lp < a.ct.logq)
        check(hipMemsetD32Async((hipDeviceptr_t)(one.ct.c0 + ((size_t)(lp >> 5) << P_.logN)), 1u << (lp & 31), 1,
                                (hipStream_t)st_) == hipSuccess
                  ? FHE_OK
                  : FHE_E_DEVICE);
    }
    V c = fresh();
    if (ok()) check(fhe_ct_addconst(c_, &a.ct, one.ct.c0, 1, &c.ct, st_));
    drop(one);
    drop(a);
    V is = imult(b);
    drop(b);
    V E = add(c, is);
    drop(c);
    drop(is);
    for (int i = 0; i < P_.logT && ok(); ++i) {
      V e2 = mul(E, E);
      drop(E);
      E = e2;
    }
    V o = imag_part(E);
    drop(E);
    return o;
  }

  int run(const fhe_ct* in, fhe_ct* out) {
    const int loggap = P_.logN - 1 - P_.logslots;
    const int logp_msg = in->logp;
    // B1: the same limbs read at 2^logQ (higher limbs zero)
    V x = fresh();
    if (!ok()) return rc;
    {
      const size_t inw = (size_t)((P_.logq_in + 31) / 32) << P_.logN;
      hipStream_t s = (hipStream_t)st_;
      hipError_t e = hipMemsetAsync(x.buf, 0, 2 * half_ * 4, s);
      if (e == hipSuccess) e = hipMemcpyAsync(x.ct.c0, in->c0, inw * 4, hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess) e = hipMemcpyAsync(x.ct.c1, in->c1, inw * 4, hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return FHE_E_DEVICE;
      x.ct.cnum = 1;
      x.ct.logN = P_.logN;
      x.ct.logq = P_.logQ;
      x.ct.logp = P_.logq_in + loggap;
      x.ct.scheme = FHE_CKKS;
      x.ct.gamma = 1;
    }
    // B2
    for (int i = P_.logslots; i < P_.logN - 1 && ok(); ++i) {
      V r = rotate(x, 1 << i);
      V s = add(x, r);
      drop(r);
      drop(x);
      x = s;
    }
    // B3
    V y = linear(x, K_.c2s);
    drop(x);
    // B4: a and b written as the two ciphertexts of one CipherTensor, so that B5 runs
    // once on both (every operation of EvalMod is pairwise or broadcast)
    V yc = conj(y);
    V ab = fresh();
    if (ok()) {
      fhe_ct a = part(ab, 0);
      a.logq = y.ct.logq;  // the output level sets the stride of ciphertext 1 below
      check(fhe_ct_add(c_, &y.ct, &yc.ct, &a, st_));
      V d = add(yc, y, true);
      fhe_ct b = a;
      const size_t stride = (size_t)((a.logq + 31) / 32) << P_.logN;
      b.c0 = ab.ct.c0 + stride;
      b.c1 = ab.ct.c1 + stride;
      if (ok()) check(fhe_ct_imult(c_, &d.ct, &b, st_));
      drop(d);
      ab.ct = a;
      ab.ct.c0 = ab.buf;
      ab.ct.c1 = ab.buf + 2 * half_;
      ab.ct.cnum = 2;
      ab.ct.logp += 1;  // the halving of both
    }
    drop(y);
    drop(yc);
    // B5, B6
    V sab = eval_mod(ab);
    drop(ab);
    V w;
    if (ok()) {
      const fhe_ct sa = part(sab, 0), sb = part(sab, 1);
      V isb = fresh();
      if (ok()) check(fhe_ct_imult(c_, &sb, &isb.ct, st_));
      w = fresh();
      if (ok()) check(fhe_ct_add(c_, &sa, &isb.ct, &w.ct, st_));
      drop(isb);
    }
    drop(sab);
    // B7
    V z = linear(w, K_.s2c);
    drop(w);
    if (!ok()) return rc;
    // the output: z's limbs and metadata, the scale lowered by logq_in - logp_msg bits
    const size_t zw = (size_t)((z.ct.logq + 31) / 32) << P_.logN;
    hipStream_t s = (hipStream_t)st_;
    if (hipMemcpyAsync(out->c0, z.ct.c0, zw * 4, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(out->c1, z.ct.c1, zw * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return FHE_E_DEVICE;
    out->cnum = 1;
    out->logN = z.ct.logN;
    out->logq = z.ct.logq;
    out->logp = z.ct.logp - (P_.logq_in - logp_msg);
    out->scheme = FHE_CKKS;
    out->t = 0;
    out->gamma = 1;
    drop(z);
    // the pool's buffers are freed when this object goes: wait for the queued work
    return hipStreamSynchronize(s) == hipSuccess ? FHE_OK : FHE_E_DEVICE;
  }

 private:
  fhe_ctx* c_;
  const fhe_boot_params& P_;
  const fhe_boot_keys& K_;
  void* st_;
  size_t half_;
  CtPool pool_;
};

}  // namespace

extern "C" int fhe_ct_bootstrap(fhe_ctx* ctx, const fhe_boot_params* P, const fhe_boot_keys* K, const fhe_ct* in,
                                fhe_ct* out, void* stream) {
  if (!ctx || !P || !K || !in || !out || !out->c0 || !out->c1 || !in->c0 || !in->c1) return FHE_E_INVAL;
  if (!K->relin || !K->conj || !K->rot || !K->c2s || !K->s2c || !K->taylor) return FHE_E_INVAL;
  if (P->logN < FHE_LOGN_MIN || P->logN > FHE_LOGN_MAX) return FHE_E_RANGE;
  if (P->logslots < 0 || P->logslots >= P->logN - 1 || P->logc < 1 || P->logc > 60 || P->logT < 0 ||
      P->degree < 1 || P->degree > 31 || P->logq_in < 1 || P->logQ <= P->logq_in)
    return FHE_E_INVAL;
  if (in->cnum != 1 || in->scheme != FHE_CKKS || in->logN != P->logN || in->logq != P->logq_in ||
      in->logp > P->logq_in)
    return FHE_E_SHAPE;
  int maxr = (1 << P->logslots) - 1;  // the largest rotation the circuit uses
  for (int i = P->logslots; i < P->logN - 1; ++i) maxr = std::max(maxr, 1 << i);
  if (K->nrot <= maxr) return FHE_E_INVAL;
  Boot b(ctx, *P, *K, stream);
  const int rc = b.run(in, out);
  return rc != FHE_OK ? rc : b.rc;
}
