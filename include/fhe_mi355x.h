/*
 * fhe_mi355x.h -- C ABI of the MI355X (gfx950) library for homomorphic
 * multiplication in non-RNS CKKS / BGV (HEAAN-style parameterization).
 *
 * Representation (Section 4.1 "The Radix Representation", Section 5.1
 * "Representation Overview"): a polynomial of Z_Q[X]/(X^N+1) with Q = 2^logq is
 * stored limb-major as uint32[L][N], L = ceil(logq / 32).  Entry [i][j] is the
 * 32-bit limb i (limb 0 least significant) of coefficient j.  Bits at positions
 * >= logq must be zero on input and are zero on output.  A ciphertext is two such
 * polynomials (c0, c1).  A batch of cnum ciphertexts with equal parameters (the
 * CipherTensor of Section 6.1) is uint32[cnum][L][N] per component, contiguous.
 *
 * Ring products (Section 5.1, pipeline summary) lift limbs onto 30-bit
 * NTT-friendly primes q = 1 (mod 2^17), run negacyclic NTTs (Eq. negacyclic_ntt,
 * Eq. negacyclic_intt), multiply pointwise (Eq. ntt_mul), and rebuild limbs from
 * the residues (the reconstruction of Section 5.1 and Eq. garner_mrc, computed as
 * a direct CRT sum with its exact quotient).  All arithmetic is exact.
 *
 * Conventions where the paper is silent (the same readings as the CPU oracle):
 *   - Q_l = 2^logq and the special modulus P = 2^logP; "mod Q_l" keeps logq bits.
 *   - Relinearization multiplies the representative of d2 in [0, Q_l).
 *   - CKKS divisions by 2^k round half up: floor((x + 2^(k-1)) / 2^k).
 *   - BGV divisions by 2^k are t-corrected:
 *       floor(x / 2^k) + [[ (x mod 2^k) * (2^-k mod t) ]]_t, centered in (-t/2, t/2].
 *   - Relinearization rounding, then the addition, then the rescale rounding.
 *
 * Pointers: "device" pointers are HIP device memory owned by the caller, which must
 * keep them alive until the work queued on `stream` has completed; "host" pointers
 * are read before the call returns.  `stream` is a hipStream_t (NULL = default
 * stream).  Work is queued asynchronously; argument errors are reported
 * synchronously; a HIP launch or runtime error is returned as FHE_E_DEVICE and kept
 * as the context's sticky error until fhe_ctx_reset_error.  Inputs must be
 * canonical; the library does not check the values of device data.
 *
 * Thread safety: a context may be used from several host threads, but calls that
 * share a context serialize on an internal lock; scratch memory is held per
 * (context, stream), so work on different streams does not alias.
 */
#ifndef FHE_MI355X_H
#define FHE_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status codes */
#define FHE_OK 0
#define FHE_E_INVAL (-1)  /* null pointer or argument out of its documented range  */
#define FHE_E_SHAPE (-2)  /* operands of different N, logq, scheme or t            */
#define FHE_E_RANGE (-3)  /* beyond the context limits or the key's level          */
#define FHE_E_NOMEM (-4)  /* device or host allocation failed                      */
#define FHE_E_DEVICE (-5) /* HIP runtime or launch error (sticky, see above)       */
#define FHE_E_STATE (-6)  /* object in the wrong state (e.g. destroyed, mismatched) */

#define FHE_CKKS 0
#define FHE_BGV 1

/* Supported ring degrees: 2^10 <= N <= 2^16 (the prime table has q = 1 mod 2^17). */
#define FHE_LOGN_MIN 10
#define FHE_LOGN_MAX 16

typedef struct fhe_ctx fhe_ctx;
typedef struct fhe_evk fhe_evk;
typedef struct fhe_plan fhe_plan;

/* Text for a status code (static storage). */
const char* fhe_strerror(int status);

/* Text naming the last failing HIP call made by the library on the calling host
 * thread, with the runtime's message (thread-local storage; empty if none). */
const char* fhe_error_detail(void);

/* Create a context on HIP device `device` able to hold ciphertexts with
 * logq <= logQ_max and keys with logP <= logP_max.  Builds on the device the
 * tables of Section 5.2 (twiddles psi^j and their inverses, n^-1, the limb
 * weights 2^(32i) mod q_j, 1/q_j), for as many primes as the largest
 * relinearization product at these limits needs; the reconstruction constants of
 * each prime count (the CRT factors (M/q_i)^-1 mod q_i and the limbs of M/q_i) are
 * built on first use.  *out receives the context (library-owned;
 * release with fhe_ctx_destroy).  Errors: FHE_E_INVAL (bad limits or null out),
 * FHE_E_RANGE (limits need more primes than the table holds), FHE_E_NOMEM,
 * FHE_E_DEVICE. */
int fhe_ctx_create(int device, int logQ_max, int logP_max, fhe_ctx** out);

/* Destroy a context and every table and scratch buffer it owns (waits for the
 * device first).  Keys created on it must be destroyed before.  NULL is a no-op. */
void fhe_ctx_destroy(fhe_ctx* ctx);

/* Return and clear the sticky device error of the context. */
int fhe_ctx_reset_error(fhe_ctx* ctx);

/* Instrumentation.  fhe_ctx_profile(ctx, 1) starts recording a pair of HIP events
 * on the launch stream around every kernel the context launches (and clears the
 * totals); fhe_ctx_profile(ctx, 0) stops.  fhe_ctx_profile_read waits for the
 * recorded events and returns, for one kernel class, the summed event time (ms),
 * the summed algorithmic work and the number of launches (host outputs).  The
 * work is the kernel's algorithmic HBM bytes: every input element it must read and
 * every output element it must write, once (limbs and residues of the lift and the
 * reconstruction, transform rows of the NTT passes, ...).  Kernel classes:
 * 0 lift, 1 forward NTT column pass, 2 forward NTT row pass, 3 inverse NTT row
 * pass, 4 inverse NTT column pass, 5 pointwise (no longer launched: the fused row
 * pass does the products), 6 reconstruction (CRT),
 * 7 relinearization compose, 8 rescale, 9 fused row pass (last forward NTT row
 * pass + pointwise products + first inverse row pass, used by the HE-mult and the
 * ring multiply), 10 compose and rescale in one pass (HE-mult with rescale),
 * 11 coefficient-wise operations (add, sub, negate, moddown, addconst, multconst,
 * the signed permutations of imult and the automorphisms).  Errors: FHE_E_INVAL,
 * FHE_E_STATE (not recording). */
int fhe_ctx_profile(fhe_ctx* ctx, int enable);
int fhe_ctx_profile_read(fhe_ctx* ctx, int kernel, double* ms, double* work, long long* launches);

/* Number of primes in the context's table. */
int fhe_prime_count(const fhe_ctx* ctx, int* count);

/* Prime `idx` of the table and its primitive 2^17-th root of unity psi (host
 * outputs).  The transform of size N uses psi^(2^16 / N) (Section 2.3: q = 1 mod
 * 2N, psi a primitive 2N-th root).  Primes are the largest q < 2^30 with
 * q = 1 (mod 2^17), in decreasing order; psi = g^((q-1)/2^17) for the smallest
 * g >= 2 giving an element of order 2^17. */
int fhe_prime_info(const fhe_ctx* ctx, int idx, uint32_t* q, uint32_t* psi);

/* Number of primes K the library uses for the exact product of two polynomials
 * of degree < N with coefficients in [0, 2^bits_a) and [0, 2^bits_b), summed over
 * `terms` products: the smallest K with prod_(i<K) q_i >= 2^(e+17), where
 * e = bits_a + bits_b + logN + ceil(log2(terms)) bounds the signed exact result,
 * |X| < 2^e.  The 16 bits beyond 2^(e+1) keep the CRT quotient of X + 2^e exact
 * when it is evaluated in double precision.  (Host output.) */
int fhe_primes_needed(const fhe_ctx* ctx, int logN, int bits_a, int bits_b, int terms, int* K);

/* Limb -> RNS projection (Section 5.1 "Limb-to-RNS Conversion"): for each of
 * `count` polynomials, res[c][p][j] = A_j mod q_p for primes p < nprimes, where A_j
 * is coefficient j of limbs[c] (uint32[count][L][N], device) and res is
 * uint32[count][nprimes][N] (device).  Errors: FHE_E_INVAL, FHE_E_RANGE. */
int fhe_lift(fhe_ctx* ctx, int logN, int L, int nprimes, const uint32_t* limbs,
             uint32_t* res, int count, void* stream);

/* Standalone negacyclic NTT (Section 2.3, Eq. negacyclic_ntt / negacyclic_intt, with
 * the twist by powers of psi merged into the butterflies as Section 5.1 describes)
 * over primes prime0 .. prime0+nprimes-1 of the context's table, in place on
 * data = uint32[count][nprimes][N] (device), values in [0, q_p).  For N < 2^16 the
 * root is psi_N = psi^(2^16 / N), psi from fhe_prime_info.
 * flags = 0:                    forward, abar_i at position i (natural order).
 * flags = FHE_NTT_BITREV:       forward, abar_i at position bitrev_(logN)(i), the
 *                               order the transform produces (no permutation pass).
 * flags = FHE_NTT_INVERSE:      inverse of the natural-order forward.
 * flags = INVERSE | BITREV:     inverse taking the bit-reversed order.
 * Errors: FHE_E_INVAL (flags, null, negative sizes), FHE_E_RANGE (logN outside
 * [10, 16], prime0 + nprimes beyond the table). */
#define FHE_NTT_INVERSE 1
#define FHE_NTT_BITREV 2
int fhe_ntt(fhe_ctx* ctx, int logN, int prime0, int nprimes, int flags, uint32_t* data, int count,
            void* stream);

/* Ring multiply (Section 2.3, Eq. schoolbook then Eq. reduction, mod Q = 2^logq):
 * c[i] = a[i] * b[i] in Z_(2^logq)[X]/(X^N+1) for i < cnum.  a, b, c are device
 * uint32[cnum][L][N]; c may alias a or b.  Errors: FHE_E_INVAL, FHE_E_RANGE,
 * FHE_E_NOMEM, FHE_E_DEVICE. */
int fhe_ring_mul(fhe_ctx* ctx, int logN, int logq, const uint32_t* a, const uint32_t* b,
                 uint32_t* c, int cnum, void* stream);

/* fhe_ring_mul without any allocation, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid it): the same
 * product and bits, with the residues of the operands (2 cnum K N words, K the primes of
 * the product, fhe_primes_needed(logN, logq, logq, 1)) held in a static device array of
 * 64 MiB (16 Mi words) that each device the library runs on keeps until the process
 * ends.  Calls no allocating routine: the context's tables for this (logN, logq) must
 * exist already, i.e. one fhe_ring_mul of the same shape has run on the context.
 * Every call on a device shares that device's array, so calls that overlap on one
 * device (concurrent streams, contexts or threads) race and must be serialized by the
 * caller.  Errors: FHE_E_INVAL, FHE_E_RANGE (shape beyond the context, or 2 cnum K N
 * above 16 Mi words), FHE_E_STATE (tables not built yet, or profiling enabled),
 * FHE_E_DEVICE. */
int fhe_ring_mul_noalloc(fhe_ctx* ctx, int logN, int logq, const uint32_t* a, const uint32_t* b, uint32_t* c,
                         int cnum, void* stream);

/* Upload a relinearization key (b', a') (Section 6.2 "Cryptographic Key
 * Management": relinearization keys) given at modulus P * 2^logQ_key:
 * b_host, a_host are host uint32[L_PQ][N], L_PQ = ceil((logP + logQ_key) / 32).
 * The library keeps a host copy of the limbs and, per ciphertext level logq used
 * with it, the NTT form of the key reduced mod P * 2^logq resident on the device
 * (built on first use or by fhe_evk_prepare; 2 K_r N words, plus a second layout
 * for odd logN).  *out is library-owned; release with fhe_evk_destroy.
 * scheme is FHE_CKKS or FHE_BGV; t (odd, 3 <= t < 2^24, so that the t-corrected
 * divisions' sums stay within 64 bits) is read for BGV only.
 * Errors: FHE_E_INVAL, FHE_E_RANGE (logQ_key > logQ_max or logP > logP_max),
 * FHE_E_NOMEM, FHE_E_DEVICE. */
int fhe_evk_create(fhe_ctx* ctx, int scheme, uint32_t t, int logN, int logQ_key, int logP,
                   const uint32_t* b_host, const uint32_t* a_host, fhe_evk** out);

/* Build (if not yet built) the resident NTT form of the key for level logq. */
int fhe_evk_prepare(fhe_evk* evk, int logq, void* stream);

/* Release a key and its device memory (waits for the device).  NULL is a no-op. */
void fhe_evk_destroy(fhe_evk* evk);

/* Homomorphic multiplication with relinearization (the HE-mult of Section 6.2,
 * "multiplication followed by relinearization"; Karatsuba-equivalent tensor of
 * Section 5.4): for each i < cnum,
 *   d0 = x0 y0, d1 = x0 y1 + x1 y0, d2 = x1 y1            (mod Q_l = 2^logq)
 *   k0 = d2 b', k1 = d2 a'                                (mod P Q_l)
 *   out0 = [d0 + R(k0)]_(Q_l), out1 = [d1 + R(k1)]_(Q_l)
 * with R the CKKS or BGV division by P of the header notes.  x0, x1, y0, y1,
 * out0, out1 are device uint32[cnum][L][N]; outputs must not alias inputs.
 * Metadata (logp adds, BGV gamma multiplies) is the caller's.
 * Errors: FHE_E_INVAL, FHE_E_SHAPE (logN differs from the key's),
 * FHE_E_RANGE (logq > key level), FHE_E_NOMEM, FHE_E_DEVICE. */
int fhe_mul_relin(fhe_ctx* ctx, fhe_evk* evk, int logN, int logq, const uint32_t* x0,
                  const uint32_t* x1, const uint32_t* y0, const uint32_t* y1, uint32_t* out0,
                  uint32_t* out1, int cnum, void* stream);

/* Rescale by `bits` (rescaleBy of Section 6.2; arbitrary bit counts as in Section
 * 3.2): out = [R(in)]_(2^(logq - bits)) per component, R the CKKS or BGV division
 * by 2^bits.  in0/in1 device uint32[cnum][L][N], out0/out1 device
 * uint32[cnum][L'][N] with L' = ceil((logq - bits) / 32); in place is allowed.
 * 1 <= bits < logq.  Errors: FHE_E_INVAL, FHE_E_DEVICE. */
int fhe_rescale(fhe_ctx* ctx, int scheme, uint32_t t, int logN, int logq, int bits,
                const uint32_t* in0, const uint32_t* in1, uint32_t* out0, uint32_t* out1,
                int cnum, void* stream);

/* fhe_mul_relin followed by fhe_rescale(bits), fused; bit-identical to the two
 * calls.  out0/out1 are uint32[cnum][L'][N], L' = ceil((logq - bits) / 32). */
int fhe_mul_relin_rescale(fhe_ctx* ctx, fhe_evk* evk, int logN, int logq, int bits,
                          const uint32_t* x0, const uint32_t* x1, const uint32_t* y0,
                          const uint32_t* y1, uint32_t* out0, uint32_t* out1, int cnum,
                          void* stream);

/* ---------------------------------------------------------------- Galois automorphisms
 * Section 2.5 permutes the slots with the automorphisms kappa_g: X -> X^g (g odd), and
 * Section 6.2 ("Cryptographic Key Management", rotation and conjugation keys; the
 * operation list's leftrotate and conjugate) switches the result back to the secret s
 * with a key per g.  Readings (the paper gives no formulas; the CPU oracle's):
 *   - kappa_g(a): coefficient i of a moves to position i g mod 2N, negated when that
 *     position is >= N (X^N = -1), then taken mod 2^logq.
 *   - A left rotation of the slots by r uses g = 5^r mod 2N; conjugation g = 2N - 1.
 *   - The switching key for kappa_g is (b', a') over P 2^logQ_key,
 *     b' = [-a' s + e' + P kappa_g(s)] (BGV: t e'), used mod P 2^logq at level logq.
 *   - Key switch of (c0, c1): u = kappa_g(c1) in [0, 2^logq),
 *       c0' = [kappa_g(c0) + R(u b')]_(2^logq),  c1' = [R(u a')]_(2^logq),
 *     R the CKKS or BGV division by P of the notes at the top of this header. */

/* Signed permutation kappa_g of `count` polynomials: out[c] = kappa_g(in[c]) mod 2^logq,
 * in/out device uint32[count][L][N], L = ceil(logq / 32); out must not overlap in.
 * Errors: FHE_E_INVAL (g even or g >= 2N, null, overlap), FHE_E_RANGE (logN, logq). */
int fhe_automorphism(fhe_ctx* ctx, int logN, int logq, uint32_t g, const uint32_t* in, uint32_t* out, int count,
                     void* stream);

/* Upload a switching key for kappa_g (host uint32[L_PQ][N] limbs, as fhe_evk_create).
 * The returned key works with fhe_key_switch and the fhe_ct rotation / conjugation
 * calls only (the HE-mult entry points reject it with FHE_E_STATE); its limbs stay in
 * host memory and the NTT form per level is built on the device on first use (or by
 * fhe_evk_prepare).  Release with fhe_evk_destroy.  Errors: as fhe_evk_create, and
 * FHE_E_INVAL for g even or g >= 2N. */
int fhe_galois_key_create(fhe_ctx* ctx, int scheme, uint32_t t, int logN, int logQ_key, int logP, uint32_t g,
                          const uint32_t* b_host, const uint32_t* a_host, fhe_evk** out);

/* Key switch of cnum ciphertexts by the key's automorphism (see above): in0, in1,
 * out0, out1 device uint32[cnum][L][N]; outputs must not overlap inputs.  Runs the
 * signed permutation, then the relinearization half of the HE-mult pipeline (lift of
 * u onto the relinearization primes, NTT, products with the resident key, inverse NTT,
 * reconstruction, rounding division by P and addition).  Metadata is unchanged.
 * Errors: FHE_E_INVAL, FHE_E_STATE (not a Galois key of this context), FHE_E_SHAPE
 * (logN), FHE_E_RANGE (logq above the key level), FHE_E_NOMEM, FHE_E_DEVICE. */
int fhe_key_switch(fhe_ctx* ctx, fhe_evk* key, int logN, int logq, const uint32_t* in0, const uint32_t* in1,
                   uint32_t* out0, uint32_t* out1, int cnum, void* stream);

/* ---------------------------------------------------------------- ciphertexts with metadata
 * A CipherTensor (Section 6.1) of cnum ciphertexts with equal parameters, with the
 * metadata of Section 6: logN, logq (the modulus 2^logq), logp (CKKS scale 2^logp),
 * the scheme, and for BGV the plaintext modulus t and the message factor gamma (the
 * ciphertext decrypts to gamma m mod t; 1 after encryption).  c0, c1 are caller-owned
 * device buffers uint32[cnum][L][N], L = ceil(logq / 32).
 * Every fhe_ct entry point reads all fields of its inputs; of its output it reads only
 * c0 and c1 (the buffers it writes) and, on success, sets every other field.  For
 * CKKS gamma is ignored and set to 1 on outputs.
 * Pairwise mode: a second operand with the same cnum; broadcast mode (Section 6.1): a
 * second operand (ciphertext or plaintext) with cnum = 1, applied to every ciphertext.
 * Errors of every call: FHE_E_INVAL (null, bad field, bad argument, forbidden
 * overlap of output and input), FHE_E_RANGE (logN outside [10, 16], logq beyond the
 * context's logQ_max + logP_max or the key's level), FHE_E_SHAPE (operands that
 * differ), plus the errors of the underlying computation. */
typedef struct {
  uint32_t* c0;
  uint32_t* c1;
  int32_t cnum;
  int32_t logN, logq, logp, scheme;
  uint32_t t, gamma;
} fhe_ct;

/* HE-mult (fhe_mul_relin) with metadata: x, y must share cnum, logN, logq, scheme and
 * t, and match the key's logN, scheme and t.  out: logq = x.logq,
 * logp = x.logp + y.logp, gamma = x.gamma y.gamma mod t (BGV).  Output buffers must not
 * overlap the inputs. */
int fhe_ct_mul_relin(fhe_ctx* ctx, fhe_evk* evk, const fhe_ct* x, const fhe_ct* y, fhe_ct* out, void* stream);

/* fhe_ct_mul_relin then rescale by `bits` (0: none), fused as fhe_mul_relin_rescale:
 * out.logq = x.logq - bits; CKKS logp = x.logp + y.logp - bits; BGV
 * gamma = x.gamma y.gamma 2^-bits mod t. */
int fhe_ct_mul_relin_rescale(fhe_ctx* ctx, fhe_evk* evk, const fhe_ct* x, const fhe_ct* y, int bits, fhe_ct* out,
                             void* stream);

/* rescaleBy (Section 6.2; Section 3.2 arbitrary bit counts): out = [R(x)]_(2^(logq-bits)),
 * 1 <= bits < logq; out.logq = logq - bits; CKKS logp -= bits; BGV gamma *= 2^-bits mod
 * t.  In place allowed (out buffers = x buffers). */
int fhe_ct_rescale(fhe_ctx* ctx, const fhe_ct* x, int bits, fhe_ct* out, void* stream);

/* moddownBy (Section 6.2): out = [x]_(2^(logq - bits)), 0 <= bits < logq, logq -= bits,
 * logp and gamma kept (levels are matched this way before a multiplication).  In place
 * allowed for cnum = 1 or an unchanged limb count. */
int fhe_ct_moddown(fhe_ctx* ctx, const fhe_ct* x, int bits, fhe_ct* out, void* stream);

/* add / sub (Section 6.2): out_i = [x_i +- y_(i or 0)]_(2^logq) per component, pairwise
 * or broadcast.  x and y must agree in logN, logq, logp, scheme, t and gamma.  In place
 * allowed (out = x or out = y). */
int fhe_ct_add(fhe_ctx* ctx, const fhe_ct* x, const fhe_ct* y, fhe_ct* out, void* stream);
int fhe_ct_sub(fhe_ctx* ctx, const fhe_ct* x, const fhe_ct* y, fhe_ct* out, void* stream);

/* negate (Section 6.2): out = [-x]_(2^logq).  In place allowed. */
int fhe_ct_negate(fhe_ctx* ctx, const fhe_ct* x, fhe_ct* out, void* stream);

/* imult (Section 6.2, CKKS only): every slot times the imaginary unit, i.e. both
 * components times the monomial X^(N/2) (every slot is an evaluation at a root
 * zeta^r with r = 1 mod 4, where X^(N/2) is i).  out must not overlap x. */
int fhe_ct_imult(fhe_ctx* ctx, const fhe_ct* x, fhe_ct* out, void* stream);

/* multconst (Section 6.2, broadcast): out = [(-1)^negative k x]_(2^logq) for the integer
 * constant k = sum_i k_host[i] 2^(32 i), 1 <= klimbs <= 8 (host array).  A real
 * constant enters as k = round(c 2^logp_k): CKKS logp += logp_k (BGV keeps logp).  In
 * place allowed. */
int fhe_ct_multconst(fhe_ctx* ctx, const fhe_ct* x, const uint32_t* k_host, int klimbs, int negative, int logp_k,
                     fhe_ct* out, void* stream);

/* multconstvec (Section 6.2): out_i = [x_i m_(i or 0)]_(2^logq), a ring product with a
 * plaintext polynomial per ciphertext (mcount = cnum, pairwise) or one for all
 * (mcount = 1, broadcast); m: device uint32[mcount][L][N] in [0, 2^logq) (an encoded
 * vector at scale 2^logp_m: CKKS logp += logp_m).  Exact, through the ring-product
 * pipeline.  In place allowed. */
int fhe_ct_multconstvec(fhe_ctx* ctx, const fhe_ct* x, const uint32_t* m, int mcount, int logp_m, fhe_ct* out,
                        void* stream);

/* addconst (Section 6.2): out_0 = [x_0 + m_(i or 0)]_(2^logq), out_1 = x_1, with m a
 * plaintext polynomial already at the ciphertext's scale (CKKS) or already times gamma
 * (BGV); m: device uint32[mcount][L][N], mcount = cnum or 1.  In place allowed. */
int fhe_ct_addconst(fhe_ctx* ctx, const fhe_ct* x, const uint32_t* m, int mcount, fhe_ct* out, void* stream);

/* Key switch by a Galois key (fhe_key_switch) with metadata (unchanged); leftrotate
 * checks that the key's element is 5^r mod 2N, conjugate that it is 2N - 1
 * (FHE_E_STATE otherwise).  out must not overlap x. */
int fhe_ct_key_switch(fhe_ctx* ctx, fhe_evk* key, const fhe_ct* x, fhe_ct* out, void* stream);
int fhe_ct_leftrotate(fhe_ctx* ctx, fhe_evk* key, int r, const fhe_ct* x, fhe_ct* out, void* stream);
int fhe_ct_conjugate(fhe_ctx* ctx, fhe_evk* key, const fhe_ct* x, fhe_ct* out, void* stream);

/* ---------------------------------------------------------------- bootstrapping
 * CKKS bootstrapping (Section 6.2 `bootstrap`, HEAAN's EvalBootstrap; Section 7.2: logT
 * sets the precision of the circuit).  The paper gives no algorithm; the reading is the
 * published bootstrapping for approximate HE, composed from this library's fhe_ct
 * operations (n = 2^logslots slots, gap = N / 2n, q0 = 2^logq_in, V_jk = zeta^(r_j k)
 * with zeta = exp(2 pi i / 4n), r_j = 5^j mod 4n):
 *   1. modulus raise: the input's limbs read at 2^logQ, scale 2^(logq_in + log2 gap);
 *   2. SubSum: x += leftrotate(x, 2^i) for logslots <= i < logN - 1;
 *   3. CoeffToSlot: sum_d leftrotate(x, d) * c2s[d], rescale by logc;
 *   4. a = (x + conj x) / 2, b = i (conj x - x) / 2 (the halving as logp + 1);
 *   5. on a and b: y = x * k_y / 2^(logc + logT) (rescale by logc + logT, scale kept);
 *      powers y^k (k <= degree) by y^k = y^h y^(k-h), h the largest power of two below
 *      k (y^(k/2) squared when k is a power of two), each product rescaled by the
 *      working scale; re = sum over even k, im = sum over odd k of y^k * taylor[k] /
 *      2^logc; E = (re + 1) + i im; logT squarings; sin = i (conj E - E) / 2;
 *   6. w = sin(a) + i sin(b);
 *   7. SlotToCoeff: sum_d leftrotate(w, d) * s2c[d], rescale by logc; the output's
 *      scale is lowered by logq_in - logp bits (a change of scale only).
 * Operands of an addition or a product are first brought to the lower one's logq
 * (moddownBy); products are HE-mults with the relinearization key.  c2s and s2c are
 * the encodings at 2^logc of the diagonals d of V^-1 and V / (2 pi) (diag_d[j] =
 * A[j][(j + d) mod n]), k_y = round(2 pi 2^logc), taylor[k] = round(c_k 2^logc) with c_k
 * the coefficients of exp(i y)'s real part (even k) or imaginary part (odd k). */
typedef struct {
  int logN, logslots, logq_in, logQ, logc, logT, degree;
} fhe_boot_params;

typedef struct {
  fhe_evk* relin;         /* relinearization key at logQ_key >= logQ */
  fhe_evk* const* rot;    /* host array: rot[r] = switching key of 5^r (NULL where unused) */
  int nrot;               /* entries of rot: above every rotation the circuit uses */
  fhe_evk* conj;          /* switching key of 2N - 1 */
  const uint32_t* c2s;    /* device uint32[n][L_Q][N]: [c2s_d]_(2^logQ), L_Q = ceil(logQ / 32) */
  const uint32_t* s2c;    /* device uint32[n][L_Q][N] */
  int64_t k_y;
  const int64_t* taylor;  /* host, degree + 1 entries (entry 0 unused) */
} fhe_boot_keys;

/* Bootstrap one CKKS ciphertext (cnum = 1) at logq = logq_in (its logp <= logq_in):
 * out receives the refreshed ciphertext; out->c0, out->c1 must each hold L_Q N words
 * (the output's level is below logQ; the call writes out's metadata).  Allocates its
 * temporaries and synchronizes `stream` before returning.  Errors: FHE_E_INVAL (null,
 * parameters, a missing key), FHE_E_SHAPE (the input is not a one-ciphertext CKKS tensor
 * at logq_in of ring degree 2^logN), FHE_E_RANGE (levels exhausted: logQ too small for
 * the circuit), plus the errors of the operations. */
int fhe_ct_bootstrap(fhe_ctx* ctx, const fhe_boot_params* params, const fhe_boot_keys* keys, const fhe_ct* in,
                     fhe_ct* out, void* stream);

/* ---------------------------------------------------------------- batches
 * A batch of HE-mults of uneven ring degree and level (the CipherTensor of Section
 * 6.1 generalised: ciphertexts of one cell share parameters, cells differ).
 * One job = fhe_mul_relin on one ciphertext pair, then rescale by `bits` (0: none).
 * All pointers are caller-owned device buffers: x0..y1 uint32[L][N], outputs
 * uint32[L'][N] with L = ceil(logq / 32), L' = ceil((logq - bits) / 32), N = 2^logN
 * of the job's key.  Outputs must not alias inputs or other jobs' outputs. */
typedef struct {
  fhe_evk* evk;  /* relinearization key; its logN, scheme and t apply */
  int logq;      /* level of both operands, <= the key's logQ */
  int bits;      /* rescale after relinearization: 0 or 1 <= bits < logq */
  const uint32_t *x0, *x1, *y0, *y1;
  uint32_t *out0, *out1;
} fhe_job;

#define FHE_PLAN_GRAPH 1    /* capture the whole batch in one hipGraph */
#define FHE_PLAN_AUTOTUNE 2 /* time launch-parameter candidates per cell at plan time */
#define FHE_PLAN_QUEUE 4    /* stage-batched: each pipeline stage as one launch over all cells */

/* Build a plan for `njobs` jobs (host array, read during the call).  Jobs are grouped
 * into cells of equal (key, logq, bits); each cell runs as one CipherTensor pipeline
 * reading and writing the jobs' buffers through device pointer arrays.  The plan
 * owns its scratch memory, the prepared key levels it needs, and (FHE_PLAN_GRAPH)
 * an instantiated hipGraph in which the cells run on up to 4 concurrent branches,
 * each with its own scratch (so a graphed plan holds up to 4 cells' scratch at once,
 * against 1 for an eager plan).  With FHE_PLAN_QUEUE the cells instead run stage by
 * stage: each stage of the pipeline (lift, transforms, products, reconstruction,
 * composition) is one launch per kernel variant whose workgroups are drawn from a
 * device table of (cell, workgroup) units over every cell using that variant, so a
 * batch takes about as many launches as one cell; every cell then holds scratch of its
 * own.  With FHE_PLAN_GRAPH as well, the cells are spread over the same branches as
 * above and each branch's cells run stage-batched on it.  Planning prepares keys
 * and, with FHE_PLAN_AUTOTUNE, runs
 * every cell a few times on `stream` (writing the outputs); it synchronizes.  The
 * job buffers must stay valid for the plan's lifetime.  Errors: FHE_E_INVAL,
 * FHE_E_SHAPE, FHE_E_RANGE, FHE_E_NOMEM, FHE_E_DEVICE. */
int fhe_batch_plan(fhe_ctx* ctx, const fhe_job* jobs, int njobs, int flags, void* stream, fhe_plan** out);

/* Queue one execution of the plan on `stream` (graph launch, or the cells' kernels
 * in order).  Errors: FHE_E_INVAL, FHE_E_DEVICE. */
int fhe_batch_run(fhe_plan* plan, void* stream);

/* Cells, kernel launches per run, and whether the plan is a graph (host outputs). */
int fhe_batch_info(const fhe_plan* plan, int* cells, int* kernels, int* graphed);

/* Release a plan (waits for the device).  NULL is a no-op. */
void fhe_batch_destroy(fhe_plan* plan);

/* ---------------------------------------------------------------- test helpers
 * Encoding, encryption and decryption (Section 6.2 operation list; the readings of
 * the scheme are those of the CPU oracle).  All randomness is passed in, so the
 * results can be compared bit for bit with the oracle.  Keys are not generated here.
 * Sign conventions: "[x]_m" is the representative in [0, m); the centered one lies
 * in (-m/2, m/2]. */

/* CKKS encoding with sparse packing (host arrays; no device needed).
 * z_j = re[j] + i im[j], j < n = 2^logslots <= N/2.  With zeta = exp(2 pi i / 4n),
 * r_j = 5^j mod 4n and gap = N / 2n:
 *   u_k = (1/n) Re(sum_j z_j zeta^(-r_j k)),   k < 2n,
 *   m_(k gap) = floor(2^logp u_k + 1/2), other coefficients 0,
 * written as [m]_(2^logq) into m = uint32[L][N], L = ceil(logq / 32).  Computed in
 * double precision through a length-2n FFT, so a coefficient can differ by one from
 * an exact evaluation where 2^logp u_k + 1/2 lies within rounding of an integer.
 * Errors: FHE_E_INVAL (null), FHE_E_RANGE (logN outside [10, 16], logslots outside
 * [0, logN-1], logp outside [1, 62], |2^logp u_k| >= 2^62, logq outside [1, 4096]). */
int fhe_ckks_encode(int logN, int logslots, int logp, int logq, const double* re, const double* im,
                    uint32_t* m);

/* CKKS decoding (host arrays): mu = centered representative of the phase
 * uint32[L][N] (mod 2^logq), z_j = 2^-logp sum_(k<2n) mu_(k gap) zeta^(r_j k),
 * in double precision.  Errors as for fhe_ckks_encode. */
int fhe_ckks_decode(int logN, int logslots, int logp, int logq, const uint32_t* phase, double* re,
                    double* im);

/* Public-key encryption at level logq (device arrays, on `stream`):
 *   c0 = [v pk_b + m + e0']_(Q_l),  c1 = [v pk_a + e1']_(Q_l),  Q_l = 2^logq,
 * e' = e (CKKS) or t e (BGV).  pk_b, pk_a: uint32[L'][N] with L' >= L, a public key
 * at a modulus 2^logQ >= Q_l (its low L limb rows, top row masked, are the key
 * mod Q_l).  m: uint32[L][N] in [0, Q_l).  v: int8[N] (ternary), e0, e1: int32[N].
 * c0, c1: uint32[L][N], caller-owned.  t is ignored for CKKS; BGV needs odd t in
 * [3, 2^24).  Errors: FHE_E_INVAL, FHE_E_RANGE (logN, logq beyond the context). */
int fhe_encrypt(fhe_ctx* ctx, int scheme, uint32_t t, int logN, int logq, const uint32_t* pk_b,
                const uint32_t* pk_a, const uint32_t* m, const int8_t* v, const int32_t* e0,
                const int32_t* e1, uint32_t* c0, uint32_t* c1, void* stream);

/* Decryption (device arrays): the phase [c0 + c1 s]_(Q_l), s: int8[N] the ternary
 * secret.  CKKS: out = the phase, uint32[L][N] (decode it with fhe_ckks_decode).
 * BGV: out = uint32[N], m_j = gamma^-1 [[phase_j]] mod t (centered phase, then mod t),
 * where gamma is the ciphertext's factor (1 after encryption; a multiplication
 * multiplies the factors, a rescale by k bits multiplies by 2^-k mod t).
 * Errors: FHE_E_INVAL (gamma not invertible mod t, bad t), FHE_E_RANGE. */
int fhe_decrypt(fhe_ctx* ctx, int scheme, uint32_t t, uint32_t gamma, int logN, int logq,
                const uint32_t* c0, const uint32_t* c1, const int8_t* s, uint32_t* out, void* stream);

/* ---------------------------------------------------------------- serving
 * A request loop for HE-mult requests (one fhe_job each) that arrive over time.
 * A scheduler thread keeps `nstreams` device streams busy: whenever one is free it
 * forms a batch from the oldest pending request and the other pending requests of
 * the same cell (key, logq, bits), up to `max_batch`, and launches it as one
 * CipherTensor pipeline (continuous batching; batches on different streams overlap
 * on the device).  Admission is by HBM footprint: fhe_server_create reserves one
 * device arena of `hbm_budget` bytes, and every running batch takes its scratch from
 * it (the pipeline's scratch, linear in the batch size); a batch is cut to what the
 * budget allows, waits while the arena has no room, and a request that cannot fit
 * even alone completes with status FHE_E_NOMEM.  The scheduler allocates no device
 * memory.  The caller's operand and output buffers and the evaluation keys are not
 * part of the budget: the key level a request uses must already be resident
 * (fhe_evk_prepare).  Times are fhe_clock_ns() values. */
typedef struct fhe_server fhe_server;

typedef struct {
  uint64_t ticket;   /* as returned by fhe_server_submit */
  int status;        /* FHE_OK or an error code (FHE_E_STATE: cancelled) */
  int batch;         /* size of the batch the request ran in (0: never launched) */
  uint64_t t_arrive; /* arrival time given at submit */
  uint64_t t_start;  /* launch of its batch */
  uint64_t t_done;   /* completion of its batch as seen by the scheduler */
} fhe_done;

/* Monotonic clock in nanoseconds (the server's time base). */
uint64_t fhe_clock_ns(void);

/* Start a server on a context.  nstreams in [1, 16], max_batch in [1, 256].  Reserves
 * the arena (hbm_budget rounded down to 256 bytes; 0 reserves nothing and every
 * request is rejected).  Errors: FHE_E_INVAL, FHE_E_NOMEM (the arena), FHE_E_DEVICE. */
int fhe_server_create(fhe_ctx* ctx, size_t hbm_budget, int nstreams, int max_batch, fhe_server** out);

/* Queue one request (job fields as in fhe_batch_plan; the buffers must stay valid
 * until the request is reported done).  The request's inputs are read only after the
 * work queued on `stream` (the caller's stream, NULL = default stream) before this
 * call has completed: an event recorded there is waited for by the batch's stream.
 * arrival_ns = 0 means "now"; a time in the future (fhe_clock_ns base) makes the request
 * eligible only from then on, so an arrival schedule can be queued ahead.  Latency is
 * reported from arrival_ns.  Builds the context's tables for the job's shape if this
 * is the first request of that shape.  Errors: FHE_E_INVAL, FHE_E_RANGE, FHE_E_STATE
 * (a Galois key, a key of another context, the key level not prepared, or the server
 * stopping), FHE_E_DEVICE. */
int fhe_server_submit(fhe_server* srv, const fhe_job* job, uint64_t arrival_ns, void* stream, uint64_t* ticket);

/* Move up to `max` completed requests to `out` (host array); *n receives the count. */
int fhe_server_poll(fhe_server* srv, fhe_done* out, int max, int* n);

/* Block until every submitted request has completed. */
int fhe_server_drain(fhe_server* srv);

/* Requests not yet launched (queued or scheduled for later) complete at once with
 * status FHE_E_STATE; batches already on the device run to completion. */
int fhe_server_cancel(fhe_server* srv);

/* Stop the scheduler after the pending work completes and release the server. */
void fhe_server_destroy(fhe_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* FHE_MI355X_H */
