// gfx950 kernels for the non-RNS HE-mult pipeline:
//   lift (limbs -> residues), negacyclic NTT / iNTT, pointwise products,
//   Garner reconstruction (residues -> limbs), relinearization compose, rescale.
#include <algorithm>
#include <utility>

#include "fhe_internal.h"

namespace fhe {

static thread_local EventRecorder* g_rec = nullptr;
static thread_local long long g_launches = 0;
void set_recorder(EventRecorder* r) { g_rec = r; }
long long kernel_launch_count() { return g_launches; }

// Brackets one kernel launch with the recorder's events; `work` is the kernel's
// algorithmic 32x32-bit word-product count (0 when not tracked).
struct Bracket {
  int kid;
  hipStream_t s;
  double work;
  Bracket(int k, hipStream_t st, double w) : kid(k), s(st), work(w) {
    ++g_launches;
    if (g_rec) g_rec->begin(kid, s);
  }
  ~Bracket() {
    if (g_rec) g_rec->end(kid, s, work);
  }
};

// ============================================================================ NTT
//
// Negacyclic transforms (Section 2.3, Eq. negacyclic_ntt / negacyclic_intt) with
// the psi-twist merged into the twiddles (Section 5.1): the forward transform is
// the Cooley-Tukey network whose stage with m groups uses psi^bitrev(m + i) for
// group i and leaves the output in bit-reversed order; the inverse is the mirrored
// Gentleman-Sande network with psi^-bitrev(h + i), then the factor N^-1.
//
// N = 2^logN is split as N = n1 * n2 (the two-pass / four-step scheme of Section
// 5.3).  The n1-point stages run over columns {c + n2 u}; the n2-point stages run
// over contiguous blocks.  Both passes use one kernel shape: a sub-transform of
// n = 2^S points is held by T = n / 16 threads with 16 values each.  The first
// register phase works on elements {u T + j} ("strided"), the other on
// {16 j + u} ("contiguous"); one LDS exchange connects them.  Forward passes run
// strided then contiguous; inverse passes the reverse.

__device__ __forceinline__ void ct_bfly(uint32_t& X, uint32_t& Y, uint2 w, uint32_t q,
                                        uint32_t two_q) {
  // Lazy Cooley-Tukey butterfly: X, Y in [0, 4q) -> [0, 4q).
  uint32_t x = csub(X, two_q);
  uint32_t t = shoup_lazy(Y, w.x, w.y, q);
  X = x + t;
  Y = x - t + two_q;
}

__device__ __forceinline__ void gs_bfly(uint32_t& X, uint32_t& Y, uint2 w, uint32_t q,
                                        uint32_t two_q) {
  // Lazy Gentleman-Sande butterfly: X, Y in [0, 2q) -> [0, 2q).
  uint32_t x = X, y = Y;
  X = csub(x + y, two_q);
  Y = shoup_lazy(x - y + two_q, w.x, w.y, q);
}

template <int S, bool INV, bool ROWS>
__global__ __launch_bounds__(256) void ntt_pass_kernel(NttArgs a) {
  constexpr int n = 1 << S;
  constexpr int T = n / 16;
  constexpr int NSUB = 256 / T;
  // Row stride in LDS, chosen so that both access patterns are free of bank
  // conflicts (element e sits at s * SS + e + e / 16).
  constexpr int SS = ((n + n / 16 + 1 + 31) / 32) * 32 + (ROWS ? T : (NSUB >= 32 ? 1 : 2));
  __shared__ uint32_t lds[NSUB * SS];

  const int tid = threadIdx.x;
  const int s = ROWS ? tid / T : tid % NSUB;
  const int j = ROWS ? tid % T : tid / NSUB;

  const int N = 1 << a.logN;
  const int nsub_total = N / n;  // blocks (ROWS) or columns (COLS)
  // Workgroup w runs on XCD w % 8 (round-robin dispatch).  XCD x takes the primes
  // p = x (mod 8), one at a time, and every transform of that prime in turn, so a
  // prime's twiddle table is read into one L2 once.
  const int nwg = (nsub_total + NSUB - 1) / NSUB;  // workgroups per transform
  const int npp = a.ntr / a.K;                     // transforms per prime
  const int w = blockIdx.x, xcd = w & 7, l = w >> 3;
  const int per_prime = npp * nwg;
  const int p = (l / per_prime) * 8 + xcd;
  if (p >= a.K) return;  // whole workgroup exits (primes not a multiple of 8)
  const int rem = l % per_prime;
  const int jp = rem / nwg;  // transform index among those of prime p
  const int sg = (rem % nwg) * NSUB + s;
  const bool valid = sg < nsub_total;
  // transform jp of prime p: polynomial i of group grp, row r = i K + p
  const int pk = a.per_group / a.K;  // polynomials per group
  const int grp = jp / pk, r = (jp % pk) * a.K + p;
  uint32_t* base = a.data + (long long)grp * a.group_stride + (long long)r * N;
  const PrimeC pc = a.pc[p];
  const uint32_t q = pc.q, two_q = pc.two_q;
  const uint2* tw = a.tw + (long long)p * kNMax;

  // ROWS: element e of block sg at sg * n + e.  COLS: element e of column sg at
  // sg + (N / n) e.
  const long long gstride = ROWS ? 1 : (long long)nsub_total;
  uint32_t* gp = base + (ROWS ? (long long)sg * n : (long long)sg);
  // Twiddle index of local stage m (groups) and local group i:
  // COLS -> m + i; ROWS -> (N / n + sg) m + i.
  const int tw_mul = ROWS ? (nsub_total + sg) : 1;

  uint32_t x[16];
  uint32_t* lrow = lds + s * SS;

  if (!INV) {
    if (valid) {
#pragma unroll
      for (int u = 0; u < 16; ++u) x[u] = gp[(long long)(u * T + j) * gstride];
    }
    // strided stages: m = 1, 2, 4, 8 groups, register distance 8 / m
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int m = 1 << st, h = 8 >> st;
#pragma unroll
      for (int g = 0; g < m; ++g) {
        const uint2 w = tw[tw_mul * m + g];
#pragma unroll
        for (int u = 2 * h * g; u < 2 * h * g + h; ++u) ct_bfly(x[u], x[u + h], w, q, two_q);
      }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = u * T + j;
      lrow[e + (e >> 4)] = x[u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = 16 * j + u;
      x[u] = lrow[e + (e >> 4)];
    }
    // contiguous stages: half-distance t = T/2 .. 1, m = n / (2t) groups
#pragma unroll
    for (int t = T / 2; t >= 1; t >>= 1) {
      const int m = n / (2 * t);
#pragma unroll
      for (int b0 = 0; b0 < 16; b0 += 2 * t) {
        const uint2 w = tw[tw_mul * m + j * (8 / t) + b0 / (2 * t)];
#pragma unroll
        for (int u = b0; u < b0 + t; ++u) ct_bfly(x[u], x[u + t], w, q, two_q);
      }
    }
    if (ROWS) {  // last forward pass: canonical output
#pragma unroll
      for (int u = 0; u < 16; ++u) x[u] = csub(csub(x[u], two_q), q);
    }
    if (valid) {
#pragma unroll
      for (int u = 0; u < 16; ++u) gp[(long long)(16 * j + u) * gstride] = x[u];
    }
  } else {
    if (valid) {
#pragma unroll
      for (int u = 0; u < 16; ++u) x[u] = gp[(long long)(16 * j + u) * gstride];
    }
    // contiguous stages: t = 1 .. T/2, h = n / (2t) groups
#pragma unroll
    for (int t = 1; t < T; t <<= 1) {
      const int h = n / (2 * t);
#pragma unroll
      for (int b0 = 0; b0 < 16; b0 += 2 * t) {
        const uint2 w = tw[tw_mul * h + j * (8 / t) + b0 / (2 * t)];
#pragma unroll
        for (int u = b0; u < b0 + t; ++u) gs_bfly(x[u], x[u + t], w, q, two_q);
      }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = 16 * j + u;
      lrow[e + (e >> 4)] = x[u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = u * T + j;
      x[u] = lrow[e + (e >> 4)];
    }
    // strided stages: register distance hd = 1, 2, 4, 8; h = 8 / hd groups
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int hd = 1 << st, h = 8 >> st;
#pragma unroll
      for (int g = 0; g < h; ++g) {
        const uint2 w = tw[tw_mul * h + g];
#pragma unroll
        for (int u = 2 * hd * g; u < 2 * hd * g + hd; ++u) gs_bfly(x[u], x[u + hd], w, q, two_q);
      }
    }
    if (!ROWS) {  // last inverse pass: final factor, canonical output
      const uint2 sc = a.scale[p];
#pragma unroll
      for (int u = 0; u < 16; ++u) x[u] = csub(shoup_lazy(x[u], sc.x, sc.y, q), q);
    }
    if (valid) {
#pragma unroll
      for (int u = 0; u < 16; ++u) gp[(long long)(u * T + j) * gstride] = x[u];
    }
  }
}

template <int S, bool INV, bool ROWS>
static hipError_t ntt_pass(const NttArgs& a, int ntr, hipStream_t st) {
  constexpr int n = 1 << S;
  constexpr int NSUB = 256 / (n / 16);
  const int nsub_total = (1 << a.logN) / n;
  const int nwg = (nsub_total + NSUB - 1) / NSUB;
  const int kx = (a.K + 7) / 8;  // primes per XCD (the largest share)
  dim3 grid(8 * kx * (ntr / a.K) * nwg);
  // algorithmic work: (N / 2) S butterflies per transform, one constant product each
  Bracket br(INV ? (ROWS ? KID_NTT_INV_ROWS : KID_NTT_INV_COLS) : (ROWS ? KID_NTT_FWD_ROWS : KID_NTT_FWD_COLS), st,
             (double)ntr * (double)((1 << a.logN) / 2) * S);
  hipLaunchKernelGGL((ntt_pass_kernel<S, INV, ROWS>), grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

template <bool INV, bool ROWS>
static hipError_t ntt_pass_s(int S, const NttArgs& a, int ntr, hipStream_t st) {
  switch (S) {
    case 5: return ntt_pass<5, INV, ROWS>(a, ntr, st);
    case 6: return ntt_pass<6, INV, ROWS>(a, ntr, st);
    case 7: return ntt_pass<7, INV, ROWS>(a, ntr, st);
    case 8: return ntt_pass<8, INV, ROWS>(a, ntr, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ntt(const NttArgs& a0, int ntr, bool inverse, hipStream_t st, const Tuning& tu) {
  if (ntr <= 0) return hipSuccess;
  if (ntr % a0.K != 0 || a0.per_group % a0.K != 0) return hipErrorInvalidValue;
  NttArgs a = a0;
  a.ntr = ntr;
  // the split groups the same stages differently and does not change the result
  const int s_cols = tu.ntt_cols_first ? a.logN - a.logN / 2 : a.logN / 2;
  const int s_rows = a.logN - s_cols;
  hipError_t e;
  if (!inverse) {
    if ((e = ntt_pass_s<false, false>(s_cols, a, ntr, st)) != hipSuccess) return e;
    return ntt_pass_s<false, true>(s_rows, a, ntr, st);
  }
  if ((e = ntt_pass_s<true, true>(s_rows, a, ntr, st)) != hipSuccess) return e;
  return ntt_pass_s<true, false>(s_cols, a, ntr, st);
}

// ============================================================================ lift
//
// Limb -> RNS projection (Section 5.1, "Limb-to-RNS Conversion"): residue of
// A = sum_i limb_i 2^(32 i) modulo each prime.  The limbs are re-cut into 28-bit
// digits (8 digits per 7 limbs), so every digit-constant product is below 2^58 and
// 40 of them fit a 64-bit accumulator between folds.  The constants are
// 2^(28 i) 2^32 mod q, and the final Montgomery reduction removes the 2^32.

template <int PB>
__global__ __launch_bounds__(256) void lift_kernel(LiftArgs a) {
  // Workgroup w runs on XCD w % 8.  The prime groups of one (polynomial,
  // coefficient block) unit are consecutive workgroups of one XCD, so the unit's
  // limbs are read from HBM once and then from that XCD's L2.
  const int G = (a.K + PB - 1) / PB;
  const int nb = (a.N + 255) / 256;
  const int w = blockIdx.x, xcd = w & 7, l = w >> 3;
  const int unit = (l / G) * 8 + xcd;
  if (unit >= nb * a.npoly) return;
  const int p0 = (l % G) * PB;
  const int z = unit / nb;
  const int jc = (unit % nb) * 256 + threadIdx.x;  // coefficient
  if (jc >= a.N) return;
  const uint32_t* src = (a.in_ptrs ? a.in_ptrs[z] : a.limbs + (long long)z * a.in_stride) + jc;
  uint64_t acc[PB];
#pragma unroll
  for (int pp = 0; pp < PB; ++pp) acc[pp] = 0;
  const int nchunk = (a.L + 6) / 7;
  for (int ch = 0; ch < nchunk; ++ch) {
    uint32_t w[8];
#pragma unroll
    for (int v = 0; v < 7; ++v) {
      const int li = 7 * ch + v;
      w[v] = li < a.L ? src[(long long)li * a.N] : 0u;
    }
    w[7] = 0;
    uint32_t d[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int bit = 28 * u, wi = bit >> 5, sh = bit & 31;
      uint32_t lo = w[wi] >> sh;
      if (sh > 4) lo |= w[wi + 1] << (32 - sh);
      d[u] = lo & 0x0FFFFFFFu;
    }
    const uint32_t* Tp = a.T + (long long)p0 * a.TS + 8 * ch;
#pragma unroll
    for (int pp = 0; pp < PB; ++pp) {
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[pp] = mad64(d[u], Tp[(long long)pp * a.TS + u], acc[pp]);
    }
    if (ch % 5 == 4) {
#pragma unroll
      for (int pp = 0; pp < PB; ++pp) acc[pp] = fold64(acc[pp], a.pc[p0 + pp].c32);
    }
  }
  uint32_t* dst = a.res + (long long)z * a.out_stride + jc;
#pragma unroll
  for (int pp = 0; pp < PB; ++pp) {
    const int p = p0 + pp;
    if (p < a.K) dst[(long long)p * a.N] = reduce64_mont(acc[pp], a.pc[p]);
  }
}

template <int PB>
static void lift_launch(const LiftArgs& b, int npoly, hipStream_t st) {
  const int G = (b.K + PB - 1) / PB;
  const int units = ((b.N + 255) / 256) * npoly;
  dim3 grid(8 * ((units + 7) / 8) * G);
  hipLaunchKernelGGL((lift_kernel<PB>), grid, dim3(256), 0, st, b);
}

hipError_t launch_lift(const LiftArgs& a, int npoly, hipStream_t st, const Tuning& t) {
  if (npoly <= 0) return hipSuccess;
  LiftArgs b = a;
  b.npoly = npoly;
  // algorithmic work: L limb-constant products per (coefficient, prime)
  Bracket br(KID_LIFT, st, (double)npoly * a.N * a.K * a.L);
  switch (t.lift_primes) {
    case 8: lift_launch<8>(b, npoly, st); break;
    case 32: lift_launch<32>(b, npoly, st); break;
    default: lift_launch<16>(b, npoly, st); break;
  }
  return hipGetLastError();
}

// ============================================================================ pointwise
//
// Hadamard products in the NTT domain (Section 2.3, Eq. ntt_mul).  Montgomery
// products carry a factor 2^-32, compensated in the inverse transform's final
// factor.  Tensor: d0 = x0 y0, d1 = x0 y1 + x1 y0, d2 = x1 y1 (the Karatsuba
// identity of Section 5.4 gives the same d1; with full-rate multiplies the direct
// form issues fewer instructions).

__global__ __launch_bounds__(256) void tensor_pointwise_kernel(PointwiseArgs a) {
  const int jc = blockIdx.x * 256 + threadIdx.x;
  const int p = blockIdx.y;
  const int c = blockIdx.z;
  if (jc >= a.N) return;
  const long long KN = (long long)a.K * a.N;
  uint32_t* g = a.a + (long long)c * a.group_stride + (long long)p * a.N + jc;
  const PrimeC pc = a.pc[p];
  const uint32_t x0 = g[0], x1 = g[KN], y0 = g[2 * KN], y1 = g[3 * KN];
  const uint32_t d0 = mont_mul(x0, y0, pc.q, pc.qneg);
  const uint32_t d2 = mont_mul(x1, y1, pc.q, pc.qneg);
  const uint32_t d1 = add_mod(mont_mul(x0, y1, pc.q, pc.qneg), mont_mul(x1, y0, pc.q, pc.qneg), pc.q);
  g[0] = d0;
  g[KN] = d1;
  g[2 * KN] = d2;
}

__global__ __launch_bounds__(256) void relin_pointwise_kernel(PointwiseArgs a) {
  const int jc = blockIdx.x * 256 + threadIdx.x;
  const int p = blockIdx.y;
  const int c = blockIdx.z;
  if (jc >= a.N) return;
  const long long KN = (long long)a.K * a.N;
  const long long off = (long long)p * a.N + jc;
  const PrimeC pc = a.pc[p];
  const uint32_t d = a.a[(long long)c * a.group_stride + off];
  uint32_t* o = a.out + (long long)c * a.out_stride + off;
  o[0] = mont_mul(d, a.b[off], pc.q, pc.qneg);
  o[KN] = mont_mul(d, a.b[KN + off], pc.q, pc.qneg);
}

__global__ __launch_bounds__(256) void ring_pointwise_kernel(PointwiseArgs a) {
  const int jc = blockIdx.x * 256 + threadIdx.x;
  const int p = blockIdx.y;
  const int c = blockIdx.z;
  if (jc >= a.N) return;
  const long long off = (long long)p * a.N + jc;
  const PrimeC pc = a.pc[p];
  uint32_t* x = a.a + (long long)c * a.group_stride + off;
  const uint32_t y = a.b[(long long)c * a.group_stride + off];
  *x = mont_mul(*x, y, pc.q, pc.qneg);
}

hipError_t launch_tensor_pointwise(const PointwiseArgs& a, int cnum, hipStream_t st) {
  dim3 grid((a.N + 255) / 256, a.K, cnum);
  Bracket br(KID_POINTWISE, st, 4.0 * cnum * a.K * a.N);
  hipLaunchKernelGGL(tensor_pointwise_kernel, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_relin_pointwise(const PointwiseArgs& a, int cnum, hipStream_t st) {
  dim3 grid((a.N + 255) / 256, a.K, cnum);
  Bracket br(KID_POINTWISE, st, 2.0 * cnum * a.K * a.N);
  hipLaunchKernelGGL(relin_pointwise_kernel, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_ring_pointwise(const PointwiseArgs& a, int cnum, hipStream_t st) {
  dim3 grid((a.N + 255) / 256, a.K, cnum);
  Bracket br(KID_POINTWISE, st, 1.0 * cnum * a.K * a.N);
  hipLaunchKernelGGL(ring_pointwise_kernel, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

// ============================================================================ Garner
//
// RNS -> limbs (Section 5.1, "RNS-to-Limb Reconstruction"; Section 2.5,
// Eq. garner_mrc).  The integer recovered is Y = X + 2^e, where X is the signed
// exact coefficient and 2^e exceeds |X|; Y lies in [0, M), so no sign test is
// needed, and Y = X mod 2^outbits because e >= outbits.
//
// Mixed-radix digits: with M_k = prod_(i<k) q_i and I_k = [M_k^-1]_(q_k),
//   v_k = [ x_k I_k + [2^e I_k] - sum_(j<k) v_j [M_j I_k] ]_(q_k),
// the same digits as Garner's nested recurrence.  The factor I_k of x_k is
// applied by the inverse NTT's final multiply.  The sum is a dot product of
// 30-bit values: lazily accumulated in 64 bits (folded every 11 terms) against
// constants in Montgomery form, reduced once per digit.
//
// One wave handles 64 coefficients (one per lane).  Digits are kept in LDS
// ([k][lane]); digits are finalized in blocks of 16: the block's 16 sums first
// take every earlier digit (one LDS read feeds 16 multiply-adds), then the block
// is finished sequentially in registers.
//
// Limbs: Y = sum_k v_k M_k, taken mod 2^(26 D) as column sums over radix-2^26
// digits of M_k (each product < 2^56, so a column of up to 255 terms fits 64 bits),
// then carried and re-packed into 32-bit limbs.

// Tables are read through the constant address space so the compiler may treat
// them as invariant and keep wave-uniform loads scalar.
typedef __attribute__((address_space(4))) const uint32_t cu32;
typedef __attribute__((address_space(4))) const PrimeC cprime;

#define FHE_FENCE() __builtin_amdgcn_sched_barrier(0)

__device__ __forceinline__ PrimeC load_prime(cprime* p) {
  PrimeC r;
  r.q = p->q;
  r.qneg = p->qneg;
  r.c32 = p->c32;
  r.two_q = p->two_q;
  return r;
}

struct Row16 {
  uint32_t c[16];
};

__device__ __forceinline__ Row16 load_row(cu32* p) {
  Row16 r;
#pragma unroll
  for (int u = 0; u < 16; ++u) r.c[u] = p[u];
  return r;
}

// Digits of the wave's 64 coefficients, two per lane word pair: digit k of lane l
// at vd[(k / 2) * 128 + 2 l + (k % 2)], so one ds_read_b64 returns digits 2p, 2p+1.
__device__ __forceinline__ uint2 load_pair(const uint32_t* vd, int pair, int lane) {
  return *(const uint2*)(vd + pair * 128 + 2 * lane);
}

// Copies a wave-uniform value into a vector register (keeps it out of the scalar
// register budget, which the pipelined constant rows need).
__device__ __forceinline__ uint32_t to_vgpr(uint32_t x) {
  uint32_t r;
  asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
  return r;
}

// acc[u] += sum over digits k in [2 p0, 2 p1) of v_k T[k][u], T's 16-word rows stored
// contiguously from `t`.  Rows are consumed in turn from two scalar buffers: the
// first product of a row waits for it, the next row (the following 64 bytes) is
// requested right after, and the row's other 15 products cover that latency.
// (Scalar loads complete out of order, so a wait placed after the request would
// also wait for it.)  Digit pairs come from LDS one pair per two rows.  With FOLD every
// accumulator is folded (hi 2^32 + lo -> hi c32[u] + lo) after every 10 products,
// so it stays below 2^64; the last action is then a fold.
template <bool FOLD>
__device__ __forceinline__ void mac_rows(uint64_t (&acc)[16], const uint32_t* vd, int lane, cu32* t, int p0,
                                         int p1, const uint32_t (&c32)[16]) {
  if (p1 <= p0) return;
  const int k1 = 2 * p1;
  int k = 2 * p0;
  cu32* tp = t + 16 * k;
  const uint32_t* vp = vd + p0 * 128 + 2 * lane;
  Row16 ra = load_row(tp), rb;
  uint2 d = *(const uint2*)vp;
  for (; k + 10 <= k1; k += 10, tp += 160, vp += 640) {
    // pair read after the last row of this iteration: the next one, or (at the end)
    // the last pair again, so that no pair beyond p1 is read
    const int last = (k + 10 < k1) ? 5 : 4;
#pragma unroll
    for (int q = 0; q < 10; ++q) {
      const uint32_t x = (q % 2 == 0) ? d.x : d.y;
      Row16& cur = (q % 2 == 0) ? ra : rb;
      Row16& nxt = (q % 2 == 0) ? rb : ra;
      acc[0] = mad64(x, cur.c[0], acc[0]);
      FHE_FENCE();
      nxt = load_row(tp + 16 * (q + 1));  // the row after the last one reads padding
      FHE_FENCE();
#pragma unroll
      for (int u = 1; u < 16; ++u) acc[u] = mad64(x, cur.c[u], acc[u]);
      if (q % 2 == 1) d = *(const uint2*)(vp + ((q < 9 ? (q + 1) / 2 : last)) * 128);
      FHE_FENCE();
    }
    if (FOLD) {
#pragma unroll
      for (int u = 0; u < 16; ++u) acc[u] = fold64(acc[u], c32[u]);
    }
  }
  // remainder: fewer than 10 rows (an even number)
  for (; k < k1; k += 2, tp += 32, vp += 128) {
    const uint2 dd = *(const uint2*)vp;
    const Row16 r0 = load_row(tp), r1 = load_row(tp + 16);
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = mad64(dd.x, r0.c[u], acc[u]);
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = mad64(dd.y, r1.c[u], acc[u]);
  }
  if (FOLD) {
#pragma unroll
    for (int u = 0; u < 16; ++u) acc[u] = fold64(acc[u], c32[u]);
  }
}

__global__ __launch_bounds__(64) void garner_kernel(GarnerArgs a) {
  // This wave's digits, in a private scratch region (pair layout of load_pair).  Each
  // digit is written once, after which this wave alone reads it; stores complete
  // (s_waitcnt) before any read of the same block, and no line of a block is read
  // before the block is written, so no stale line can sit in the vector L1.
  uint32_t* vd = a.dig + (long long)(blockIdx.y * gridDim.x + blockIdx.x) * garner_wave_words(a.K);
  constexpr int B = kGarnerBlock;   // 16: digits finalized per block
  const int lane = threadIdx.x;
  const int jc = blockIdx.x * 64 + lane;
  const int z = blockIdx.y;
  const bool active = jc < a.N;
  const int jcc = active ? jc : 0;
  const uint32_t* in = a.res + (long long)(z / a.per_group) * a.gstride +
                       (long long)(z % a.per_group) * a.pstride + jcc;
  const int K = a.K;
  cu32* Gt = (cu32*)a.Gt;
  cu32* Ow = (cu32*)a.Ow;
  cprime* pcs = (cprime*)a.pc;

  for (int kb = 0; kb < K; kb += B) {
    // residues of this block (rows past K are valid memory; those digits are zeroed)
    uint32_t xin[B];
#pragma unroll
    for (int u = 0; u < B; ++u) xin[u] = in[(long long)min(kb + u, K - 1) * a.N];
    uint32_t c32[B];
#pragma unroll
    for (int u = 0; u < B; ++u) c32[u] = to_vgpr(pcs[kb + u].c32);
    uint64_t acc[B];
#pragma unroll
    for (int u = 0; u < B; ++u) acc[u] = 0;
    // all earlier digits, pairs 0 .. kb/2 - 1 (accumulators folded at least every 10 products)
    cu32* gb = Gt + 256 * (kb / B) * (kb / B + 1) / 2;  // this digit block's rows
    mac_rows<true>(acc, vd, lane, gb, 0, kb >> 1, c32);
    // this block's digits in order (branch-free; digits k >= K are zero)
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int k = kb + u;
      const PrimeC pk = load_prime(pcs + k);
      const uint32_t sred = reduce64_mont(acc[u], pk);
      const uint32_t xk = add_mod(xin[u], Ow[k], pk.q);
      const uint32_t vk = k < K ? sub_mod(xk, sred, pk.q) : 0u;
      vd[(k >> 1) * 128 + 2 * lane + (k & 1)] = vk;
      cu32* g = gb + 16 * k;
#pragma unroll
      for (int w = u + 1; w < B; ++w) acc[w] = mad64(vk, g[w], acc[w]);
      if (u == 10) {  // the in-block sums hold at most 11 products before this fold
#pragma unroll
        for (int w = 11; w < B; ++w) acc[w] = fold64(acc[w], c32[w]);
      }
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this block's digit stores are done
  }

  // Column sums over radix-2^26 digits of M_k, carried and packed into limbs.
  const int D = (a.outbits + kHornerDigitBits - 1) / kHornerDigitBits;
  const int npair = (K + 1) >> 1;  // a digit K (K odd) is stored as zero
  uint32_t* out = a.out + (long long)z * a.ostride + jcc;
  cu32* Ct = (cu32*)a.Ct;
  uint64_t carry = 0, bitbuf = 0;
  int nbits = 0, li = 0;
  const int topbits = a.outbits - 32 * (a.Lout - 1);
  const uint32_t topmask = topbits >= 32 ? 0xFFFFFFFFu : ((1u << topbits) - 1u);
  constexpr int BC = kHornerBlock;
  static_assert(BC == 16, "a column block is one constant row");
  const uint32_t nofold[16] = {};
  for (int m0 = 0; m0 < D; m0 += BC) {
    uint64_t col[BC];
#pragma unroll
    for (int m = 0; m < BC; ++m) col[m] = 0;
    // digits k < kstart[m0] have no radix-2^26 digit at or above m0
    const int ps = ((__attribute__((address_space(4))) const int*)a.kstart)[m0] >> 1;
    mac_rows<false>(col, vd, lane, Ct + (long long)(m0 / BC) * a.CS, ps, npair, nofold);
#pragma unroll
    for (int m = 0; m < BC; ++m) {
      if (m0 + m < D) {
        const uint64_t t = col[m] + carry;
        carry = t >> kHornerDigitBits;
        bitbuf |= (t & ((1u << kHornerDigitBits) - 1u)) << nbits;
        nbits += kHornerDigitBits;
        if (nbits >= 32) {
          if (li < a.Lout && active) {
            uint32_t wv = (uint32_t)bitbuf;
            if (li == a.Lout - 1) wv &= topmask;
            out[(long long)li * a.N] = wv;
          }
          ++li;
          bitbuf >>= 32;
          nbits -= 32;
        }
      }
    }
  }
  if (li < a.Lout && active) {
    uint32_t wv = (uint32_t)bitbuf;
    if (li == a.Lout - 1) wv &= topmask;
    out[(long long)li * a.N] = wv;
  }
}

// Word products Garner's method needs per coefficient: K(K-1)/2 for the
// mixed-radix digits, plus one per limb of each M_k (up to Lout limbs) for the
// limb-form sum.  mbits[k] is the bit length of M_k.
static double garner_products(int K, int Lout, const int* mbits) {
  double w = 0.5 * K * (K - 1);
  for (int k = 0; k < K; ++k) w += std::min(Lout, (mbits[k] + 31) / 32);
  return w;
}

hipError_t launch_garner(const GarnerArgs& a, int npoly, hipStream_t st) {
  if (npoly <= 0) return hipSuccess;
  dim3 grid((a.N + 63) / 64, npoly);
  // digits padded to the 16-digit block (the last block writes through k < K + 16),
  // plus one pair read ahead by the last prefetch
  const size_t lds = (size_t)((a.K + kGarnerBlock - 1) / kGarnerBlock * kGarnerBlock + 2) * 64 * sizeof(uint32_t);
  Bracket br(KID_GARNER, st, (double)npoly * a.N * garner_products(a.K, a.Lout, a.mbits));
  (void)lds;
  hipLaunchKernelGGL(garner_kernel, grid, dim3(64), 0, st, a);
  return hipGetLastError();
}

// ============================================================================ compose / rescale
//
// Limb-serial finishing steps, one thread per coefficient.
//   compose:  c_i = [d_i + R(k_i)]_(2^logq), R the rounding division by P = 2^logP
//   rescale:  c'' = [R(c)]_(2^(logq - bits)), R the rounding division by 2^bits
// CKKS rounds half up: floor(x / 2^s) + bit_(s-1)(x).  BGV adds the centered
// [[ (x mod 2^s) 2^-s ]]_t instead (the t-corrected division).

__device__ __forceinline__ int64_t round_correction(const uint32_t* x, long long stride, int nl,
                                                    int sbits, int scheme, uint32_t t,
                                                    uint32_t inv, const uint32_t* pw) {
  // Correction added to floor(x / 2^sbits), x = sum_l x[l stride] 2^(32 l), nl limbs.
  if (sbits <= 0) return 0;
  if (scheme == 0) {
    const int bi = sbits - 1;
    if ((bi >> 5) >= nl) return 0;
    return (x[(long long)(bi >> 5) * stride] >> (bi & 31)) & 1u;
  }
  // BGV: r = (x mod 2^sbits) mod t, then j = [[ r 2^-s ]]_t.
  const int full = sbits >> 5, part = sbits & 31;
  uint64_t acc = 0;
  for (int l = 0; l < full && l < nl; ++l) acc += (uint64_t)x[(long long)l * stride] * pw[l];
  if (part && full < nl) acc += (uint64_t)(x[(long long)full * stride] & ((1u << part) - 1u)) * pw[full];
  const uint64_t rr = (acc % t) * inv % t;
  return (2 * rr > t) ? (int64_t)rr - (int64_t)t : (int64_t)rr;
}

__global__ __launch_bounds__(256) void compose_kernel(ComposeArgs a) {
  const int jc = blockIdx.x * 256 + threadIdx.x;
  const int z = blockIdx.y;  // 2 c + i
  if (jc >= a.N) return;
  const int c = z >> 1, i = z & 1;
  const uint32_t* k = a.k + (long long)z * a.kstride + jc;
  const uint32_t* d = a.d + (long long)(3 * c + i) * a.dstride + jc;
  uint32_t* o = (a.out0s ? (i ? a.out1s[c] : a.out0s[c]) : (i ? a.out1 : a.out0) + (long long)c * a.ostride) + jc;
  const int64_t corr = round_correction(k, a.N, a.LK, a.logP, a.scheme, a.t, a.invP, a.pw);
  const int sl = a.logP >> 5, rs = a.logP & 31;
  const uint32_t ext = corr < 0 ? 0xFFFFFFFFu : 0u;
  uint64_t carry = 0;
  uint32_t klo = sl < a.LK ? k[(long long)sl * a.N] : 0u;
  const int topbits = a.logq - 32 * (a.L - 1);
  for (int l = 0; l < a.L; ++l) {
    const uint32_t khi = (sl + l + 1 < a.LK) ? k[(long long)(sl + l + 1) * a.N] : 0u;
    const uint32_t ks = rs ? ((klo >> rs) | (khi << (32 - rs))) : klo;
    klo = khi;
    const uint32_t cl = l == 0 ? (uint32_t)corr : ext;
    const uint64_t sum = (uint64_t)d[(long long)l * a.N] + ks + cl + carry;
    uint32_t wv = (uint32_t)sum;
    carry = sum >> 32;
    if (l == a.L - 1 && topbits < 32) wv &= (1u << topbits) - 1u;
    o[(long long)l * a.N] = wv;
  }
}

__global__ __launch_bounds__(256) void rescale_kernel(RescaleArgs a) {
  const int jc = blockIdx.x * 256 + threadIdx.x;
  const int z = blockIdx.y;
  if (jc >= a.N) return;
  const int c = z >> 1, i = z & 1;
  const int Lin = (a.logq + 31) >> 5;
  const int newq = a.logq - a.bits;
  const int Lout = (newq + 31) >> 5;
  const uint32_t* x = (i ? a.in1 : a.in0) + (long long)c * a.istride + jc;
  uint32_t* o = (a.out0s ? (i ? a.out1s[c] : a.out0s[c]) : (i ? a.out1 : a.out0) + (long long)c * a.ostride) + jc;
  const int64_t corr = round_correction(x, a.N, Lin, a.bits, a.scheme, a.t, a.invB, a.pw);
  const int sl = a.bits >> 5, rs = a.bits & 31;
  const uint32_t ext = corr < 0 ? 0xFFFFFFFFu : 0u;
  uint64_t carry = 0;
  uint32_t xlo = sl < Lin ? x[(long long)sl * a.N] : 0u;
  const int topbits = newq - 32 * (Lout - 1);
  for (int l = 0; l < Lout; ++l) {
    // reads of limbs >= sl + l precede the write of limb l (in place is safe)
    const uint32_t xhi = (sl + l + 1 < Lin) ? x[(long long)(sl + l + 1) * a.N] : 0u;
    const uint32_t xs = rs ? ((xlo >> rs) | (xhi << (32 - rs))) : xlo;
    xlo = xhi;
    const uint32_t cl = l == 0 ? (uint32_t)corr : ext;
    const uint64_t sum = (uint64_t)xs + cl + carry;
    uint32_t wv = (uint32_t)sum;
    carry = sum >> 32;
    if (l == Lout - 1 && topbits < 32) wv &= (1u << topbits) - 1u;
    o[(long long)l * a.N] = wv;
  }
}

hipError_t launch_compose(const ComposeArgs& a, int cnum, hipStream_t st) {
  dim3 grid((a.N + 255) / 256, 2 * cnum);
  Bracket br(KID_COMPOSE, st, 0.0);
  hipLaunchKernelGGL(compose_kernel, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_rescale(const RescaleArgs& a, int cnum, hipStream_t st) {
  dim3 grid((a.N + 255) / 256, 2 * cnum);
  Bracket br(KID_RESCALE, st, 0.0);
  hipLaunchKernelGGL(rescale_kernel, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

// ============================================================================ encryption helpers
// Limb kernels for encryption and decryption (Section 6.2 encrypt / decrypt): the
// ring products go through the exact ring multiply above; these do the rest.
// One thread per (coefficient, limb) or per coefficient; limb-major layout keeps
// every access of a wave on consecutive words of one limb row.

// [v]_(2^logq) of small signed coefficients: limb 0 holds v mod 2^32, higher limbs
// the sign extension, the top limb masked to logq bits.
__global__ __launch_bounds__(256) void small_to_limbs_kernel(const int8_t* __restrict__ v, uint32_t* __restrict__ out,
                                                             int N, int L, uint32_t topmask) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int l = blockIdx.y;
  if (j >= N) return;
  const int32_t x = v[j];
  uint32_t w = l == 0 ? (uint32_t)x : (x < 0 ? 0xFFFFFFFFu : 0u);
  if (l == L - 1) w &= topmask;
  out[(long long)l * N + j] = w;
}

// The low L limb rows of a polynomial, the top one masked: [x]_(2^logq).
__global__ __launch_bounds__(256) void mask_rows_kernel(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                        int N, int L, uint32_t topmask) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int l = blockIdx.y;
  if (j >= N) return;
  uint32_t w = in[(long long)l * N + j];
  if (l == L - 1) w &= topmask;
  out[(long long)l * N + j] = w;
}

// out = [x + y + mult * e]_(2^logq); y and e may be null.  The signed addend is
// taken in two's complement over all limbs; one carry chain per coefficient.
__global__ __launch_bounds__(256) void add_small_kernel(const uint32_t* __restrict__ x, const uint32_t* __restrict__ y,
                                                        const int32_t* __restrict__ e, long long mult,
                                                        uint32_t* __restrict__ out, int N, int L, uint32_t topmask) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= N) return;
  const long long s = e ? mult * (long long)e[j] : 0;
  const uint32_t ext = s < 0 ? 0xFFFFFFFFu : 0u;
  uint64_t carry = 0;
  for (int l = 0; l < L; ++l) {
    const long long o = (long long)l * N + j;
    const uint32_t a = l == 0 ? (uint32_t)s : (l == 1 ? (uint32_t)((unsigned long long)s >> 32) : ext);
    const uint64_t t = (uint64_t)x[o] + (y ? y[o] : 0u) + a + carry;
    uint32_t w = (uint32_t)t;
    carry = t >> 32;
    if (l == L - 1) w &= topmask;
    out[o] = w;
  }
}

// BGV decoding of a phase x in [0, 2^logq): m = gamma^-1 [[x]]_(2^logq) mod t, with
// the centered representative (x > 2^(logq-1) maps to x - 2^logq).
__global__ __launch_bounds__(256) void bgv_decode_kernel(const uint32_t* __restrict__ ph, uint32_t* __restrict__ m,
                                                         int N, int L, int logq, uint32_t t, uint32_t qmodt,
                                                         uint32_t ginv) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= N) return;
  const int hb = (logq - 1) & 31, hl = (logq - 1) >> 5;
  uint64_t r = 0;
  bool top = false, low = false;
  for (int l = L - 1; l >= 0; --l) {
    const uint32_t w = ph[(long long)l * N + j];
    r = ((r << 32) | w) % t;
    if (l == hl) {
      top = (w >> hb) & 1u;
      low = low || (w & ((1u << hb) - 1u)) != 0;
    } else if (l < hl) {
      low = low || w != 0;
    }
  }
  if (top && low) r = (r + t - qmodt) % t;
  m[j] = (uint32_t)(r * ginv % t);
}

// In-place bit-reversal permutation of each length-2^logN row.  The thread at i
// swaps with bitrev(i) when i < bitrev(i), so every pair has one owner.
__global__ __launch_bounds__(256) void bitrev_kernel(uint32_t* __restrict__ data, int logN, long long total) {
  for (long long idx = (long long)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (long long)gridDim.x * 256) {
    const long long row = idx >> logN;
    const uint32_t i = (uint32_t)(idx & ((1LL << logN) - 1));
    const uint32_t r = __builtin_bitreverse32(i) >> (32 - logN);
    if (i < r) {
      uint32_t* d = data + (row << logN);
      const uint32_t a = d[i], b = d[r];
      d[i] = b;
      d[r] = a;
    }
  }
}

hipError_t launch_small_to_limbs(const int8_t* v, uint32_t* out, int N, int L, uint32_t topmask, hipStream_t st) {
  hipLaunchKernelGGL(small_to_limbs_kernel, dim3((N + 255) / 256, L), dim3(256), 0, st, v, out, N, L, topmask);
  return hipGetLastError();
}

hipError_t launch_mask_rows(const uint32_t* in, uint32_t* out, int N, int L, uint32_t topmask, hipStream_t st) {
  hipLaunchKernelGGL(mask_rows_kernel, dim3((N + 255) / 256, L), dim3(256), 0, st, in, out, N, L, topmask);
  return hipGetLastError();
}

hipError_t launch_add_small(const uint32_t* x, const uint32_t* y, const int32_t* e, long long mult, uint32_t* out,
                            int N, int L, uint32_t topmask, hipStream_t st) {
  hipLaunchKernelGGL(add_small_kernel, dim3((N + 255) / 256), dim3(256), 0, st, x, y, e, mult, out, N, L, topmask);
  return hipGetLastError();
}

hipError_t launch_bgv_decode(const uint32_t* ph, uint32_t* m, int N, int L, int logq, uint32_t t, uint32_t qmodt,
                             uint32_t ginv, hipStream_t st) {
  hipLaunchKernelGGL(bgv_decode_kernel, dim3((N + 255) / 256), dim3(256), 0, st, ph, m, N, L, logq, t, qmodt, ginv);
  return hipGetLastError();
}

hipError_t launch_bitrev(uint32_t* data, int logN, long long rows, hipStream_t st) {
  const long long total = rows << logN;
  const long long blocks = std::min<long long>((total + 255) / 256, 1LL << 16);
  hipLaunchKernelGGL(bitrev_kernel, dim3((unsigned)blocks), dim3(256), 0, st, data, logN, total);
  return hipGetLastError();
}

}  // namespace fhe
