// gfx950 kernels for the non-RNS HE-mult pipeline:
//   lift (limbs -> residues), negacyclic NTT / iNTT, pointwise products,
//   CRT reconstruction (residues -> limbs, on the i8 matrix cores), relinearization
//   compose, rescale.
#include <algorithm>
#include <utility>

#include "fhe_internal.h"

namespace fhe {

typedef v4i_t v4i;
typedef int v16i __attribute__((ext_vector_type(16)));

// Makes a register value opaque to the optimizer.  Uses here: multipliers that must
// stay 64-bit multiply-adds (not shifts and adds), values that must be computed where
// written (not re-derived later), and per-iteration offsets of persistent loops (not
// hoisted out of the loop, where each would hold a register).
__device__ __forceinline__ void opaque(uint32_t& v) { asm volatile("" : "+v"(v)); }

// A pointer the caller knows to be equal on every lane of the wave, moved to scalar
// registers: buffer resources need it there, and stores through it take the scalar
// base + 32-bit lane offset form (no 64-bit address arithmetic per lane).
template <typename T>
__device__ __forceinline__ T* wave_uniform(T* p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (T*)(((uint64_t)hi << 32) | lo);
}

// Raw buffer over `bytes` bytes from the wave-uniform `base`.  Loads at lane offsets at
// or beyond `bytes` return zero (the buffer range check), which stands in for clamping
// and masking rows past the end of a polynomial.
// `bytes` is uniform too: it is moved to a scalar register, so that a value the compiler
// happened to compute in vector registers does not make the descriptor divergent (which
// would wrap every access in a loop over lanes).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_buffer(const uint32_t* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)__builtin_amdgcn_readfirstlane(bytes),
                                           0x00020000);
}

__device__ __forceinline__ uint32_t buffer_word(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, 0, 0);
}

// Global store at a byte offset from a wave-uniform base (the global address space is
// stated: the pointer's provenance is lost through the scalar move).
__device__ __forceinline__ void store_at(uint32_t* base, uint32_t byte_off, uint32_t v) {
  typedef __attribute__((address_space(1))) char gchar;
  typedef __attribute__((address_space(1))) uint32_t gu32;
  *(gu32*)((gchar*)base + byte_off) = v;
}

// a * b + c as one v_mad_i64_i32.  b must be opaque (a register the compiler cannot
// see the value of), or the product is strength-reduced into shifts and adds; and two
// terms of one sum must not share a multiplier register, or the compiler merges them
// into a 64 x 64-bit product.  (Not inline asm: a compiler-visible instruction gets
// the wait states after the matrix-core op that produced its operand.)
__device__ __forceinline__ int64_t mad_i64(int32_t a, uint32_t b, int64_t c) { return (int64_t)a * (int32_t)b + c; }

// Exchanges between the wave's lane halves with v_permlane32_swap (a vector op, no LDS
// round trip).  swap(x, x) returns {r0, r1}: r0 holds, in lanes 32..63, x of the lane 32
// below (lanes 0..31 keep theirs); r1 holds, in lanes 0..31, x of the lane 32 above.
__device__ __forceinline__ int64_t from_lane_below(int64_t x) {  // valid in lanes 32..63
  const uint32_t lo = (uint32_t)x, hi = (uint32_t)((uint64_t)x >> 32);
  const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto u = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return (int64_t)(((uint64_t)u[0] << 32) | l[0]);
}
__device__ __forceinline__ int64_t from_lane_above(int64_t x) {  // valid in lanes 0..31
  const uint32_t lo = (uint32_t)x, hi = (uint32_t)((uint64_t)x >> 32);
  const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto u = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return (int64_t)(((uint64_t)u[1] << 32) | l[1]);
}
// x plus x of the lane 32 apart, in every lane
__device__ __forceinline__ uint64_t sum_lane_halves(uint64_t x) {
  const uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
  const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto u = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return ((((uint64_t)u[0] << 32) | l[0])) + ((((uint64_t)u[1] << 32) | l[1]));
}

// o += cin over 4 limbs (unsigned words, least significant first), cin signed 64-bit:
// one add-with-carry chain over (cin_lo, cin_hi, ext, ext), ext the sign extension.
// Returns the signed carry out of the top limb, in {-1, 0, 1}.
__device__ __forceinline__ int32_t add_carry4(uint32_t (&o)[4], int64_t cin) {
  const uint32_t lo = (uint32_t)cin, hi = (uint32_t)((uint64_t)cin >> 32);
  const uint32_t ext = (uint32_t)((int32_t)hi >> 31);
  uint32_t co;
  asm("v_add_co_u32 %0, vcc, %0, %5\n\t"
      "v_addc_co_u32 %1, vcc, %1, %6, vcc\n\t"
      "v_addc_co_u32 %2, vcc, %2, %7, vcc\n\t"
      "v_addc_co_u32 %3, vcc, %3, %7, vcc\n\t"
      "v_addc_co_u32 %4, vcc, 0, %7, vcc"
      : "+v"(o[0]), "+v"(o[1]), "+v"(o[2]), "+v"(o[3]), "=&v"(co)
      : "v"(lo), "v"(hi), "v"(ext)
      : "vcc");
  return (int32_t)co;
}

static thread_local EventRecorder* g_rec = nullptr;
static thread_local long long g_launches = 0;
void set_recorder(EventRecorder* r) { g_rec = r; }
long long kernel_launch_count() { return g_launches; }

static thread_local LaunchSink* g_sink = nullptr;
void set_launch_sink(LaunchSink* s) { g_sink = s; }

// Issues a launch of `single` (one struct argument), or records it with its
// stage-batched entry point `multi` while a sink is installed.
template <typename A>
static hipError_t emit(const void* single, const void* multi, dim3 grid, dim3 block, size_t lds, hipStream_t st,
                       const A& a) {
  if (g_sink) {
    LaunchRec r;
    r.multi = multi;
    r.grid = grid;
    r.block = block;
    r.lds = lds;
    r.args.assign((const char*)&a, (const char*)&a + sizeof(A));
    g_sink->recs.push_back(std::move(r));
    return hipSuccess;
  }
  void* args[] = {(void*)&a};
  return hipLaunchKernel(single, grid, block, args, lds, st);
}

void bracket_begin(int kid, hipStream_t s) {
  ++g_launches;
  if (g_rec) g_rec->begin(kid, s);
}
void bracket_end(int kid, hipStream_t s, double work) {
  if (g_rec) g_rec->end(kid, s, work);
}

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

// Workgroup coordinates within one launch's grid.  A kernel body takes them as an
// argument, so that it runs either as its own launch (own_blk) or as one cell's
// segment of a stage-batched launch over many cells (cell_of).
struct Blk {
  uint32_t x, y, nx;  // block index (x, y) and the grid's width in x
};

__device__ __forceinline__ Blk own_blk() { return Blk{blockIdx.x, blockIdx.y, gridDim.x}; }

// The cell that workgroup blockIdx.x of a stage-batched launch belongs to: seg[c].off
// (ascending, multiples of 8, so that a workgroup's XCD, blockIdx.x mod 8, is the one
// its own launch would give it) is the first workgroup of cell c, whose own grid is
// gx x gy.  Workgroups past a cell's grid (the rounding to 8) take -1 and exit.
__device__ __forceinline__ int cell_of(const CellSeg* seg, int ncells, Blk& bk) {
  const uint32_t w = blockIdx.x;
  int lo = 0, hi = ncells;  // the last cell with off <= w
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (seg[mid].off <= w) lo = mid;
    else hi = mid;
  }
  const CellSeg sg = seg[lo];
  const uint32_t l = w - sg.off;
  if (l >= sg.gx * sg.gy) return -1;
  bk = Blk{l % sg.gx, l / sg.gx, sg.gx};
  return lo;
}

// A pointer read from memory (a stage-batched launch's table of cell arguments) is
// generic to the compiler, and its loads become flat loads into vector registers even
// where the address is wave-uniform.  Held as a global-memory pointer, its loads are
// global ones, or scalar ones where uniform, as in a single launch.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;

// One prime's twiddle table (Shoup pairs) through such a pointer.
struct TwTab {
  gptr<uint64_t> p;
  __device__ __forceinline__ uint2 operator[](int i) const {
    const uint64_t v = p[i];
    return make_uint2((uint32_t)v, (uint32_t)(v >> 32));
  }
  // entries i and i + 1 in one 16-byte load (i even)
  __device__ __forceinline__ v4i_t pair(int i) const { return *(gptr<v4i_t>)(p + i); }
};
__device__ __forceinline__ TwTab tw_table(const uint2* t, int p) {
  return TwTab{(gptr<uint64_t>)t + (long long)p * kNMax};
}

// Low 32 bits of a b + c in one v_mad_u64_u32 (the compiler would otherwise narrow
// the expression to a 32-bit multiply and an add).
__device__ __forceinline__ uint32_t mad_lo(uint32_t a, uint32_t b, uint32_t c) {
  uint64_t r;
  asm("v_mad_u64_u32 %0, vcc, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"((uint64_t)c) : "vcc");
  return (uint32_t)r;
}

__device__ __forceinline__ void ct_bfly(uint32_t& X, uint32_t& Y, uint2 w, uint32_t q,
                                        uint32_t two_q) {
  // Lazy Cooley-Tukey butterfly: X, Y in [0, 4q) -> [0, 4q).  With the Shoup product
  // t = Y w - qh q in [0, 2q), nt = qh q - Y w = -t (mod 2^32); then X + t = X - nt
  // and X - t + 2q = X + nt + 2q (one three-input add).  The forward table holds
  // (-w mod 2^32, floor(w 2^32 / q)), so nt = qh q + Y (-w) is one multiply and one
  // multiply-add: 7 operations per butterfly.
  const uint32_t x = csub(X, two_q);
  const uint32_t qh = __umulhi(Y, w.y);
  const uint32_t nt = mad_lo(qh, q, Y * w.x);
  X = x - nt;
  Y = x + nt + two_q;
}

__device__ __forceinline__ void gs_bfly(uint32_t& X, uint32_t& Y, uint2 w, uint32_t q,
                                        uint32_t two_q) {
  // Lazy Gentleman-Sande butterfly: X, Y in [0, 2q) -> [0, 2q); the Shoup product of
  // d = X - Y + 2q is d w - qh q = d w + qh (-q), one multiply-add.
  const uint32_t x = X, y = Y;
  X = csub(x + y, two_q);
  const uint32_t d = x - y + two_q;
  const uint32_t qh = __umulhi(d, w.y);
  Y = mad_lo(qh, 0u - q, d * w.x);
}

// Inverse twiddles from the forward table.  The bit-reversed index (over the table's
// 16 bits) of 2H - 1 - i is 2^16 minus that of H + i (H a power of two, i < H), and
// psi^(2^16) = -1, so psi^-bitrev(H + i) = -v for v = psi^bitrev(2H - 1 - i): for a
// stage of H groups starting at table index mi H - H (mi the caller's mirrored
// multiplier), group g's inverse twiddle is minus forward entry mi H - 1 - g.  That
// entry holds (-v mod 2^32, floor(v 2^32 / q)); mirror_tw makes it the Shoup pair of v
// (the negation opaque, else the compiler moves it into every butterfly), which
// gs_bfly_neg takes.
__device__ __forceinline__ uint2 mirror_tw(uint2 f) {
  uint32_t v = 0u - f.x;
  opaque(v);
  return make_uint2(v, f.y);
}
// The same for a wave-uniform twiddle: the negation stays in scalar registers (the
// compiler rejects the constraint for a value it cannot keep there).
__device__ __forceinline__ uint2 mirror_tw_s(uint2 f) {
  uint32_t v = 0u - f.x;
  asm volatile("" : "+s"(v));
  return make_uint2(v, f.y);
}

// gs_bfly with the twiddle given as -v (the Shoup pair of v): (X - Y)(-v) = (Y - X) v,
// the Shoup product of d = Y - X + 2q.
__device__ __forceinline__ void gs_bfly_neg(uint32_t& X, uint32_t& Y, uint2 v, uint32_t q,
                                            uint32_t two_q) {
  const uint32_t x = X, y = Y;
  X = csub(x + y, two_q);
  const uint32_t d = y - x + two_q;
  const uint32_t qh = __umulhi(d, v.y);
  Y = mad_lo(qh, 0u - q, d * v.x);
}

// Threads per workgroup: column passes of 2^8 and 2^7 points take 64 columns of 1024
// threads and 64 of 512 (256- and 128-byte runs per row); row passes, and column passes
// of shorter transforms (fewer columns exist), take 256.
template <int S, bool ROWS>
constexpr int ntt_pass_threads() { return ROWS ? 256 : (S >= 8 ? 1024 : (S == 7 ? 512 : 256)); }

// BLK: threads per workgroup (the autotuner may take fewer columns per workgroup than
// ntt_pass_threads gives).  CG (row passes of 256 points over transforms one group
// apart): the four 16-lane slots of a wave take one block of four consecutive
// transforms of a prime, so that its twiddles are wave-uniform (scalar loads) and
// read once for four transforms.
template <int S, bool INV, bool ROWS, int BLK, int CG = 1>
__device__ __forceinline__ void ntt_pass_kernel_body(const NttArgs& a, const Blk bk) {
  constexpr int n = 1 << S;
  constexpr int T = n / 16;
  constexpr int NSUB = BLK / T;  // slots (LDS rows) per workgroup
  static_assert(CG == 1 || (ROWS && CG * T == 64), "four transforms fill one wave");
  constexpr int RPW = NSUB / CG;  // blocks or columns per workgroup
  // Row stride in LDS, chosen so that both access patterns are free of bank
  // conflicts (element e sits at s * SS + e + e / 16).
  constexpr int SS = ((n + n / 16 + 1 + 31) / 32) * 32 + (ROWS ? T : (NSUB >= 32 ? 1 : 2));
  __shared__ uint32_t lds[NSUB * SS];

  const int tid = threadIdx.x;
  const int s = ROWS ? tid / T : tid % NSUB;
  const int j = ROWS ? tid % T : tid / NSUB;
  const int cs = CG > 1 ? s % CG : 0;  // transform within the block of CG
  const int sl = CG > 1 ? s / CG : s;  // block or column within the workgroup

  const int N = 1 << a.logN;
  const int nsub_total = N / n;  // blocks (ROWS) or columns (COLS)
  // Workgroup w runs on XCD w % 8 (round-robin dispatch).  XCD x takes the primes
  // p = x (mod 8).  A row pass takes them one at a time, and every transform of that
  // prime in turn, so a prime's twiddle table is read into one L2 once.  A column
  // pass reads only the first n entries of each table; the forward one goes through
  // the transforms in descending order instead, all its primes for each, so that it
  // starts on the residues the lift wrote last (the last-level cache still holds them).
  const int nwg = (nsub_total + RPW - 1) / RPW;  // workgroups per transform (block)
  const int npp = a.ntr / a.K;                    // transforms per prime
  const int ncg = (npp + CG - 1) / CG;            // blocks of CG transforms per prime
  const int kx = (a.K + 7) >> 3;                  // primes per XCD (the largest share)
  const int w = bk.x, xcd = w & 7, l = w >> 3;
  constexpr bool BY_TRANSFORM = !INV && !ROWS;
  const int p = (BY_TRANSFORM ? (l / nwg) % kx : l / (ncg * nwg)) * 8 + xcd;
  if (p >= a.K) return;  // whole workgroup exits (primes not a multiple of 8)
  // transform (block) index among those of prime p
  const int jg = BY_TRANSFORM ? ncg - 1 - l / (kx * nwg) : (l / nwg) % ncg;
  const int sg = (l % nwg) * RPW + sl;
  const bool valid = sg < nsub_total && (CG == 1 || jg * CG + cs < npp);
  // transform jg CG of prime p (the first of the block): polynomial i of group grp,
  // row r = i K + p; with CG > 1 the block's transforms are one group apart
  const int pk = a.per_group / a.K;  // polynomials per group
  const int jb = jg * CG;
  const int grp = jb / pk, r = (jb % pk) * a.K + p;
  uint32_t* base = a.data + (long long)grp * a.group_stride + (long long)r * N;
  const PrimeC pc = a.pc[p];
  const uint32_t q = pc.q, two_q = pc.two_q;
  const uint2* tw = a.tw + (long long)p * kNMax;

  // ROWS: element e of block sg at sg * n + e.  COLS: element e of column sg at
  // sg + (N / n) e.  Elements are addressed through a buffer resource over the transform
  // (N words from its first): a lane's 32-bit offset holds its block or column and its
  // thread index, the element index's part that is the same on every lane goes into the
  // scalar offset, and lanes past the last block or column take an offset beyond the
  // buffer (their loads return zero and their stores are dropped).
  const uint32_t es = ROWS ? 4u : 4u * (uint32_t)nsub_total;  // bytes from element e to e + 1
  const __amdgpu_buffer_rsrc_t rb =
      row_buffer(wave_uniform(base), 4u * (uint32_t)((CG - 1) * a.group_stride + N));
  const uint32_t sub = 4u * (uint32_t)(ROWS ? sg * n + cs * a.group_stride : sg);
  const uint32_t o_str = valid ? sub + (uint32_t)j * es : 0x7FFFFF00u;        // e = u T + j
  const uint32_t o_con = valid ? sub + 16u * (uint32_t)j * es : 0x7FFFFF00u;  // e = 16 j + u
  // Twiddle index of local stage m (groups) and local group i:
  // COLS -> m + i; ROWS -> (N / n + sg) m + i.
  const int tw_mul = CG > 1 ? __builtin_amdgcn_readfirstlane(nsub_total + sg) : (ROWS ? (nsub_total + sg) : 1);
  // a column pass of 64 columns or more per workgroup has one j per wave: its contiguous
  // stages' twiddles are then wave-uniform (scalar loads)
  const int jt = (!ROWS && NSUB % 64 == 0) ? __builtin_amdgcn_readfirstlane(j) : j;

  uint32_t x[16];
  uint32_t* lrow = lds + s * SS;

  if (!INV) {
#pragma unroll
    for (int u = 0; u < 16; ++u) x[u] = __builtin_amdgcn_raw_buffer_load_b32(rb, (int)o_str, (int)(u * T * es), 0);
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
        const uint2 w = tw[tw_mul * m + jt * (8 / t) + b0 / (2 * t)];
#pragma unroll
        for (int u = b0; u < b0 + t; ++u) ct_bfly(x[u], x[u + t], w, q, two_q);
      }
    }
    if (ROWS) {  // last forward pass: canonical output
#pragma unroll
      for (int u = 0; u < 16; ++u) x[u] = csub(csub(x[u], two_q), q);
    }
    if (ROWS) {  // a lane's 16 consecutive words: four 16-byte stores
#pragma unroll
      for (int v = 0; v < 4; ++v)
        __builtin_amdgcn_raw_buffer_store_b128(
            v4i_t{(int)x[4 * v], (int)x[4 * v + 1], (int)x[4 * v + 2], (int)x[4 * v + 3]}, rb, (int)o_con, 16 * v, 0);
    } else {
#pragma unroll
      for (int u = 0; u < 16; ++u) __builtin_amdgcn_raw_buffer_store_b32(x[u], rb, (int)o_con, (int)(u * es), 0);
    }
  } else {
    if (ROWS) {  // a lane's 16 consecutive words: four 16-byte loads
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const v4i_t w = __builtin_amdgcn_raw_buffer_load_b128(rb, (int)o_con, 16 * v, 0);
        x[4 * v] = (uint32_t)w[0];
        x[4 * v + 1] = (uint32_t)w[1];
        x[4 * v + 2] = (uint32_t)w[2];
        x[4 * v + 3] = (uint32_t)w[3];
      }
    } else {
#pragma unroll
      for (int u = 0; u < 16; ++u) x[u] = __builtin_amdgcn_raw_buffer_load_b32(rb, (int)o_con, (int)(u * es), 0);
    }
    // contiguous stages: t = 1 .. T/2, h = n / (2t) groups
#pragma unroll
    for (int t = 1; t < T; t <<= 1) {
      const int h = n / (2 * t);
#pragma unroll
      for (int b0 = 0; b0 < 16; b0 += 2 * t) {
        const uint2 w = tw[tw_mul * h + jt * (8 / t) + b0 / (2 * t)];
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
    // strided stages: register distance hd = 1, 2, 4, 8; h = 8 / hd groups.  The last
    // inverse pass with a final factor takes its last stage below.
    const bool fold = !ROWS && a.scale != nullptr;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int hd = 1 << st, h = 8 >> st;
      if (st == 3 && fold) break;
#pragma unroll
      for (int g = 0; g < h; ++g) {
        const uint2 w = tw[tw_mul * h + g];
#pragma unroll
        for (int u = 2 * hd * g; u < 2 * hd * g + hd; ++u) gs_bfly(x[u], x[u + hd], w, q, two_q);
      }
    }
    if (!ROWS) {  // last inverse pass: final factor (unless the inputs carry it), canonical output
      if (fold) {
        // the last stage (one group, twiddle w = entry 1) with the factor c folded in:
        // X + Y times c and (X - Y) times w c (scale_w), both below 4q, then canonical
        const uint2 sc = a.scale[p], sw = a.scale_w[p];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const uint32_t xs = x[u], ys = x[u + 8];
          x[u] = csub(shoup_lazy(xs + ys, sc.x, sc.y, q), q);
          x[u + 8] = csub(shoup_lazy(xs - ys + two_q, sw.x, sw.y, q), q);
        }
      } else {
#pragma unroll
        for (int u = 0; u < 16; ++u) x[u] = csub(x[u], q);
      }
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) __builtin_amdgcn_raw_buffer_store_b32(x[u], rb, (int)o_str, (int)(u * T * es), 0);
  }
}

template <int S, bool INV, bool ROWS, int BLK = ntt_pass_threads<S, ROWS>(), int CG = 1>
__global__ __launch_bounds__(BLK) void ntt_pass_kernel(NttArgs a) {
  ntt_pass_kernel_body<S, INV, ROWS, BLK, CG>(a, own_blk());
}

// The same over the cells of a stage-batched plan: one launch, each workgroup in its
// cell's segment (cell_of) with that cell's arguments.
template <int S, bool INV, bool ROWS, int BLK, int CG = 1>
__global__ __launch_bounds__(BLK) void ntt_pass_kernel_multi(
    const NttArgs* __restrict__ cells, const CellSeg* __restrict__ seg, int ncells) {
  Blk bk;
  const int c = cell_of(seg, ncells, bk);
  if (c < 0) return;
  ntt_pass_kernel_body<S, INV, ROWS, BLK, CG>(cells[c], bk);
}

// ---------------------------------------------------------------------------- fused row pass
// Every LDS exchange of the row passes stays inside one T-thread slot, and a slot
// (T <= 16 threads) never straddles two waves: a wave-level ordering point is enough
// between the writes and the reads (a wave's LDS accesses are performed in order), so
// the two waves of a workgroup never wait for each other.
__device__ __forceinline__ void slot_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The last forward pass, the pointwise products and the first inverse pass touch
// the same n-point rows: one kernel loads each input row once, finishes its forward
// transform in registers, multiplies (Eq. ntt_mul), runs the first inverse stages
// and stores the outputs, instead of three kernels each reading and writing them.
// After the forward row pass a thread holds elements e = 16 j + u of its row, which
// is where the pointwise step and the inverse row pass work, so no exchange is
// needed between them.  The transposes go through kRowsBuffers LDS buffers, one
// barrier per exchange of that many rows.
//   tensor: rows x0, x1, y0, y1 -> d0 = x0 y0, d1 = x0 y1 + x1 y0, d2 = x1 y1 (slots 0..2)
//   relin:  row d2 and the key's rows b', a' -> k0 = d2 b', k1 = d2 a' (to out)
//   ring:   rows a, b -> a b (in place of a)

// A row's twiddles for one direction, loaded ahead of the stages that use them: the
// exchange's ordering points keep the compiler from moving loads across them, so the
// loads are issued before (the strided stages' 15, wave-uniform when a wave holds one
// sub-row, land in scalar registers; the contiguous stages' up to 15 per thread).
// MIR: the inverse direction's come from the forward table (mirror_tw, applied where
// they are used, so that the loads stay in flight until then).
template <int S>
struct RowTw {
  uint2 s[15];  // strided stages: stage st, group g at (1 << st) - 1 + g
  uint2 c[15];  // contiguous stages, in the order the stages run
};

// MIR (inverse only): tw is the forward table and tw_mul the mirrored multiplier.
template <int S, bool INV, bool MIR = false>
__device__ __forceinline__ void load_strided_tw(RowTw<S>& w, TwTab tw, int tw_mul) {
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int m = INV ? (8 >> st) : (1 << st);
#pragma unroll
    for (int g = 0; g < m; ++g) w.s[m - 1 + g] = tw[MIR ? tw_mul * m - 1 - g : tw_mul * m + g];
  }
}

// Index in RowTw::c of the contiguous stage with half-distance t, block b0: the forward
// stages run t = T/2 .. 1 (8/t twiddles each), the inverse ones t = 1 .. T/2.
template <int S>
__device__ constexpr int fwd_ci(int t, int b0) { return 8 / t - 256 / (1 << S) + b0 / (2 * t); }
__device__ constexpr int inv_ci(int t, int b0) { return 16 - 16 / t + b0 / (2 * t); }

template <int S, bool INV, bool MIR = false>
__device__ __forceinline__ void load_contig_tw(RowTw<S>& w, TwTab tw, int tw_mul, int j) {
  constexpr int n = 1 << S, T = n / 16;
#pragma unroll
  for (int t = 1; t < T; t <<= 1) {
    const int cnt = 8 / t;  // this thread's twiddles of the stage: groups j cnt + k, k < cnt
    if (!MIR) {
#pragma unroll
      for (int b0 = 0; b0 < 16; b0 += 2 * t)
        w.c[INV ? inv_ci(t, b0) : fwd_ci<S>(t, b0)] = tw[tw_mul * (n / (2 * t)) + j * cnt + b0 / (2 * t)];
    } else if (cnt == 1) {
      w.c[inv_ci(t, 0)] = tw[tw_mul * (n / (2 * t)) - 1 - j];
    } else {
      // group j cnt + k is entry tw_mul h - 1 - j cnt - k: element cnt - 1 - k of the
      // ascending block from tw_mul h - (j + 1) cnt, two entries per 16-byte load (h and
      // cnt are even, so the block starts on a 16-byte boundary)
      const int b = tw_mul * (n / (2 * t)) - (j + 1) * cnt;
#pragma unroll
      for (int e = 0; e < cnt; e += 2) {
        const v4i_t v = tw.pair(b + e);
        w.c[inv_ci(t, 2 * t * (cnt - 1 - e))] = make_uint2((uint32_t)v[0], (uint32_t)v[1]);
        w.c[inv_ci(t, 2 * t * (cnt - 2 - e))] = make_uint2((uint32_t)v[2], (uint32_t)v[3]);
      }
    }
  }
}

// The inverse direction's twiddles, issued at once (before the products that precede
// their first use): from the inverse table, or with MIR from the forward table at the
// mirrored multiplier.
template <int S, bool MIR = false>
__device__ __forceinline__ void load_inv_tw(RowTw<S>& w, TwTab tab, int tw_mul, int j) {
  load_contig_tw<S, true, MIR>(w, tab, tw_mul, j);
  load_strided_tw<S, true, MIR>(w, tab, tw_mul);
  __builtin_amdgcn_sched_barrier(0);
}

// Forward n-point row transforms of NP rows at once (the values x[r][u] at
// e = u T + j, loaded by the caller): each twiddle is loaded once for all rows and
// the NP exchanges share one ordering point.  Leaves values in [0, 2q) at e = 16 j + u.
// HOIST: twiddles loaded ahead of their stages (RowTw).
template <int S, int NP, int NB, bool HOIST = false>
__device__ __forceinline__ void fwd_rows(uint32_t (&x)[NP][16], uint32_t* const (&l)[NB], int j, TwTab tw,
                                         int tw_mul, uint32_t q, uint32_t two_q) {
  constexpr int n = 1 << S, T = n / 16;
  RowTw<S> w;
  if (HOIST) {  // all of this direction's twiddles issued before the first stage
    load_strided_tw<S, false>(w, tw, tw_mul);
    load_contig_tw<S, false>(w, tw, tw_mul, j);
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int m = 1 << st, h = 8 >> st;
#pragma unroll
    for (int g = 0; g < m; ++g) {
      const uint2 wg = HOIST ? w.s[m - 1 + g] : tw[tw_mul * m + g];
#pragma unroll
      for (int r = 0; r < NP; ++r)
#pragma unroll
        for (int u = 2 * h * g; u < 2 * h * g + h; ++u) ct_bfly(x[r][u], x[r][u + h], wg, q, two_q);
    }
  }
  // the transpose through LDS, NB rows at a time (fewer buffers, more workgroups per CU)
#pragma unroll
  for (int r0 = 0; r0 < NP; r0 += NB) {
    if (r0 > 0) slot_sync();  // every lane of the slot has read the previous round
#pragma unroll
    for (int r = r0; r < NP && r < r0 + NB; ++r)
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = u * T + j;
        l[r - r0][e + (e >> 4)] = x[r][u];
      }
    slot_sync();
#pragma unroll
    for (int r = r0; r < NP && r < r0 + NB; ++r)
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = 16 * j + u;
        x[r][u] = l[r - r0][e + (e >> 4)];
      }
  }
#pragma unroll
  for (int t = T / 2; t >= 1; t >>= 1) {
    const int m = n / (2 * t);
#pragma unroll
    for (int b0 = 0; b0 < 16; b0 += 2 * t) {
      const uint2 wg = HOIST ? w.c[fwd_ci<S>(t, b0)] : tw[tw_mul * m + j * (8 / t) + b0 / (2 * t)];
#pragma unroll
      for (int r = 0; r < NP; ++r)
#pragma unroll
        for (int u = b0; u < b0 + t; ++u) ct_bfly(x[r][u], x[r][u + t], wg, q, two_q);
    }
  }
  // [0, 4q) -> [0, 2q): the products below take lazy inputs
#pragma unroll
  for (int r = 0; r < NP; ++r)
#pragma unroll
    for (int u = 0; u < 16; ++u) x[r][u] = csub(x[r][u], two_q);
}

// First inverse n-point row stages of NP rows at once, values at e = 16 j + u in
// [0, 2q); leaves values in [0, 2q) at e = u T + j for the caller to store.  HOIST: the
// caller has loaded the twiddles into pre (load_inv_tw, before the products).  MIR: tw
// is the forward table and tw_mul the mirrored multiplier (mirror_tw).  SU: the strided
// stages' twiddles are wave-uniform (mirror_tw_s).
template <int S, int NP, int NB, bool HOIST = false, bool MIR = false, bool SU = false>
__device__ __forceinline__ void inv_rows(uint32_t (&x)[NP][16], uint32_t* const (&l)[NB], int j, TwTab tw,
                                         int tw_mul, uint32_t q, uint32_t two_q, RowTw<S>& pre) {
  constexpr int n = 1 << S, T = n / 16;
#pragma unroll
  for (int t = 1; t < T; t <<= 1) {
    const int h = n / (2 * t);
#pragma unroll
    for (int b0 = 0; b0 < 16; b0 += 2 * t) {
      const int g = j * (8 / t) + b0 / (2 * t);
      const uint2 wf = HOIST ? pre.c[inv_ci(t, b0)] : tw[MIR ? tw_mul * h - 1 - g : tw_mul * h + g];
      const uint2 wg = MIR ? mirror_tw(wf) : wf;
#pragma unroll
      for (int r = 0; r < NP; ++r)
#pragma unroll
        for (int u = b0; u < b0 + t; ++u) {
          if (MIR) gs_bfly_neg(x[r][u], x[r][u + t], wg, q, two_q);
          else gs_bfly(x[r][u], x[r][u + t], wg, q, two_q);
        }
    }
  }
#pragma unroll
  for (int r0 = 0; r0 < NP; r0 += NB) {
    if (r0 > 0) slot_sync();  // every lane of the slot has read the previous round
#pragma unroll
    for (int r = r0; r < NP && r < r0 + NB; ++r)
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = 16 * j + u;
        l[r - r0][e + (e >> 4)] = x[r][u];
      }
    slot_sync();
#pragma unroll
    for (int r = r0; r < NP && r < r0 + NB; ++r)
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int e = u * T + j;
        x[r][u] = l[r - r0][e + (e >> 4)];
      }
  }
#pragma unroll
  for (int st = 0; st < 4; ++st) {
    const int hd = 1 << st, h = 8 >> st;
#pragma unroll
    for (int g = 0; g < h; ++g) {
      const uint2 wf = HOIST ? pre.s[h - 1 + g] : tw[MIR ? tw_mul * h - 1 - g : tw_mul * h + g];
      const uint2 wg = MIR ? (SU ? mirror_tw_s(wf) : mirror_tw(wf)) : wf;
#pragma unroll
      for (int r = 0; r < NP; ++r)
#pragma unroll
        for (int u = 2 * hd * g; u < 2 * hd * g + hd; ++u) {
          if (MIR) gs_bfly_neg(x[r][u], x[r][u + hd], wg, q, two_q);
          else gs_bfly(x[r][u], x[r][u + hd], wg, q, two_q);
        }
    }
  }
}

// Rows per workgroup of the fused pass: 8 rows of 256 points (128 threads).  The LDS
// transposes of the tensor and ring forms go through kRowsBuffers buffers of 8 rows, as
// many rows at a time: with the registers of 3 waves per SIMD (168), 6 workgroups of 2
// buffers fit in the LDS.  The relinearization form (under 96 registers) takes one
// buffer, so that 10 of its workgroups (5 waves per SIMD) fit.
constexpr int kRowsBuffers = 2;
template <int S>
struct RowsShape {
  static constexpr int n = 1 << S, T = n / 16;
  static constexpr int NSUB = 128 / T;
  static constexpr int SS = ((n + n / 16 + 1 + 31) / 32) * 32 + T;
};

// At least 3 waves per SIMD where the LDS allows it (rows of 64 points and more); the
// relinearization form's registers give it 5.
// CG ciphertexts per sub-row: with CG = 4 (rows of 256 points, 16 threads each), the
// four 16-lane slots of a wave take one sub-row of four ciphertexts, so that its
// twiddles are wave-uniform (scalar loads) and, in the relinearization form, one wave
// instruction reads a key row once for four ciphertexts.
template <int S, int MODE, int CG>
__device__ __forceinline__ void rows_fused_kernel_body(const RowsArgs& a, const Blk bk) {
  constexpr int n = RowsShape<S>::n, T = RowsShape<S>::T, NSUB = RowsShape<S>::NSUB, SS = RowsShape<S>::SS;
  // the relinearization form exchanges one row at a time through one buffer: half the
  // LDS, so that its registers and not the LDS bound its waves per SIMD
  constexpr int NB = MODE == 1 ? 1 : kRowsBuffers;
  static_assert(kRowsBuffers == 2, "the tensor and ring forms below pair their exchanges with 2 buffers");
  static_assert(CG == 1 || (CG == 4 && T * CG == 64 && MODE != 2), "four ciphertexts fill one wave");
  constexpr int RPW = NSUB / CG;  // sub-rows per workgroup
  // twiddles loaded ahead (scalar registers for the strided stages when CG > 1); the
  // one-ciphertext relinearization form has the registers for them too
  constexpr bool HOIST = CG > 1 || MODE == 1;
  __shared__ uint32_t lds[NB][NSUB * SS];

  const int tid = threadIdx.x;
  const int s = tid / T, j = tid % T;
  const int cs = CG > 1 ? s % CG : 0;  // ciphertext within the group
  const int sl = CG > 1 ? s / CG : s;  // sub-row within the workgroup
  const int N = 1 << a.logN;
  const int nsub_total = N / n;
  // XCD-aware: workgroup w runs on XCD w % 8, which takes primes p = w % 8 (mod 8).
  // The primes run in descending order, the reverse of the column passes, so that
  // this pass starts on the rows the forward column pass wrote last and the inverse
  // column pass on the rows this pass wrote last: those still sit in the device's
  // last-level cache.
  const int nwg = (nsub_total + RPW - 1) / RPW;
  const int ncg = (a.cnum + CG - 1) / CG;
  const int per_prime = ncg * nwg;
  const int w = bk.x, xcd = w & 7, l = w >> 3;
  const int p = (((a.K + 7) >> 3) - 1 - l / per_prime) * 8 + xcd;
  if (p >= a.K) return;  // whole workgroup exits
  const int rem = l % per_prime;
  const int c = (rem / nwg) * CG;  // the group's first ciphertext
  const int sg = (rem % nwg) * RPW + sl;
  const bool valid = sg < nsub_total && c + cs < a.cnum;
  const PrimeC pc = a.pc[p];
  const uint32_t q = pc.q, two_q = pc.two_q, qneg = pc.qneg;
  const TwTab tw = tw_table(a.tw, p), itw = tw_table(a.itw, p);
  // one sub-row per wave when CG = 4: the strided stages' twiddle index is then uniform
  const int tw_mul = CG > 1 ? __builtin_amdgcn_readfirstlane(nsub_total + sg) : nsub_total + sg;
  // The tensor and relinearization forms take their inverse twiddles from the forward
  // table at the mirrored multiplier (mirror_tw; sg taken inside the transform on lanes
  // past the last sub-row), so that a prime's inverse table is not read; the ring form
  // reads the inverse table.
  const int mi = 2 * nsub_total - min(sg, nsub_total - 1);
  const int tw_mi = CG > 1 ? __builtin_amdgcn_readfirstlane(mi) : mi;
  const long long KN = (long long)a.K * N;
  // Rows are addressed through buffer resources from the workgroup's first row of
  // prime p (and its first ciphertext): a lane's 32-bit offset selects its sub-row and
  // ciphertext, a slot or key row goes into the scalar offset, and the lanes of a
  // sub-row past the last take an offset beyond the buffer, so that their loads return
  // zero and their stores are dropped (the range check), with no branches and no 64-bit
  // addresses held in registers.
  const long long base = (long long)p * N + (long long)(rem % nwg) * RPW * n;
  const uint32_t lrow = 4u * (uint32_t)(sl * n + j);
  const uint32_t lane = valid ? lrow + 4u * (uint32_t)(cs * a.group_stride) : 0x7FFFFF00u;
  const uint32_t span = (uint32_t)((CG - 1) * a.group_stride);  // words before the last ciphertext's rows
  uint32_t* lb[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) lb[b] = lds[b] + s * SS;

  if (MODE == 0) {  // tensor, in place: slots 0..3 in, 0..2 out
    const __amdgpu_buffer_rsrc_t rs =
        row_buffer(wave_uniform(a.data + (long long)c * a.group_stride + base),
                   (uint32_t)((3 * KN + NSUB * n) * 4) + 4u * span);
    uint32_t x[4][16];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int u = 0; u < 16; ++u)
        x[r][u] = __builtin_amdgcn_raw_buffer_load_b32(rs, (int)(lane + 4u * u * T), (int)(4 * r * KN), 0);
    fwd_rows<S, 4, NB, HOIST>(x, lb, j, tw, tw_mul, q, two_q);
    RowTw<S> wi;
    if (HOIST) load_inv_tw<S, true>(wi, tw, tw_mi, j);  // in flight during the products
    // Montgomery products (Eq. ntt_mul) carry a factor 2^-32, compensated in the inverse
    // transform's final factor.  d1 is formed directly (the Karatsuba identity of
    // Section 5.4 gives the same value; with full-rate multiplies the direct form issues
    // fewer instructions).
    // Inputs in [0, 2q), outputs in [0, 2q) (what the inverse butterflies take): a
    // product below 4 q^2 < q 2^32 reduces to [0, 2q); d1's sum below 8 q^2 (< 2^63, and
    // T + m q < 2^64) reduces to [0, 3q), then one conditional subtraction of 2q.
    uint32_t d[3][16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      d[0][u] = redc_lazy(mad64(x[0][u], x[2][u], 0), q, qneg);
      d[1][u] = csub(redc_lazy(mad64(x[0][u], x[3][u], mad64(x[1][u], x[2][u], 0)), q, qneg), two_q);
      d[2][u] = redc_lazy(mad64(x[1][u], x[3][u], 0), q, qneg);
    }
    slot_sync();  // every lane has read the forward exchange before it is overwritten
    inv_rows<S, 3, NB, HOIST, true, (CG > 1)>(d, lb, j, tw, tw_mi, q, two_q, wi);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int u = 0; u < 16; ++u)
        __builtin_amdgcn_raw_buffer_store_b32(d[r][u], rs, (int)(lane + 4u * u * T), (int)(4 * r * KN), 0);
  } else if (MODE == 1) {  // relin: d2 row times the key's two rows, to out
    const uint32_t bytes = (uint32_t)((KN + NSUB * n) * 4);
    const __amdgpu_buffer_rsrc_t ri =
        row_buffer(wave_uniform(a.data + (long long)c * a.group_stride + base), bytes + 4u * span);
    const __amdgpu_buffer_rsrc_t rk = row_buffer(wave_uniform(a.key + base), bytes);
    const __amdgpu_buffer_rsrc_t ro = row_buffer(wave_uniform(a.out + (long long)c * a.out_stride + base),
                                                 bytes + 4u * (uint32_t)((CG - 1) * a.out_stride));
    // the key rows are the same for every ciphertext: lane offset without the ciphertext's
    const uint32_t lk = valid ? lrow : 0x7FFFFF00u;
    const uint32_t lo = valid ? lrow + 4u * (uint32_t)(cs * a.out_stride) : 0x7FFFFF00u;
    uint32_t x[1][16], k[2][16];
#pragma unroll
    for (int u = 0; u < 16; ++u) x[0][u] = __builtin_amdgcn_raw_buffer_load_b32(ri, (int)(lane + 4u * u * T), 0, 0);
    uint32_t* const lf[1] = {lb[0]};
    fwd_rows<S, 1, 1, HOIST>(x, lf, j, tw, tw_mul, q, two_q);
    RowTw<S> wi;
    if (HOIST) load_inv_tw<S, true>(wi, tw, tw_mi, j);
    // the key rows are stored transposed (launch_row_transpose): thread j's element
    // 16 j + u sits at u T + j, so that these loads are coalesced
    // all 32 key words issued together (left to the scheduler, they may be issued two
    // at a time, each pair waited for before the next)
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      k[0][u] = __builtin_amdgcn_raw_buffer_load_b32(rk, (int)(lk + 4u * u * T), 0, 0);
      k[1][u] = __builtin_amdgcn_raw_buffer_load_b32(rk, (int)(lk + 4u * u * T), (int)(4 * KN), 0);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      // x in [0, 2q), key canonical: products below 2 q^2, results in [0, 2q)
      k[0][u] = redc_lazy(mad64(x[0][u], k[0][u], 0), q, qneg);
      k[1][u] = redc_lazy(mad64(x[0][u], k[1][u], 0), q, qneg);
    }
    slot_sync();  // every lane has read the forward exchange before it is overwritten
    uint32_t* const li[1] = {lb[0]};
    inv_rows<S, 2, 1, HOIST, true, (CG > 1)>(k, li, j, tw, tw_mi, q, two_q, wi);
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int u = 0; u < 16; ++u)
        __builtin_amdgcn_raw_buffer_store_b32(k[r][u], ro, (int)(lo + 4u * u * T), (int)(4 * r * KN), 0);
  } else {  // ring: a times b, in place of a
    const uint32_t bytes = (uint32_t)(NSUB * n * 4);
    const __amdgpu_buffer_rsrc_t ra = row_buffer(wave_uniform(a.data + (long long)c * a.group_stride + base), bytes);
    const __amdgpu_buffer_rsrc_t rb =
        row_buffer(wave_uniform(a.data2 + (long long)(c % a.data2_groups) * a.data2_stride + base), bytes);
    uint32_t x[2][16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      x[0][u] = __builtin_amdgcn_raw_buffer_load_b32(ra, (int)(lane + 4u * u * T), 0, 0);
      x[1][u] = __builtin_amdgcn_raw_buffer_load_b32(rb, (int)(lane + 4u * u * T), 0, 0);
    }
    uint32_t* const lf[2] = {lb[0], lb[1]};
    fwd_rows<S, 2, 2>(x, lf, j, tw, tw_mul, q, two_q);
    uint32_t y[1][16];
#pragma unroll
    for (int u = 0; u < 16; ++u) y[0][u] = redc_lazy(mad64(x[0][u], x[1][u], 0), q, qneg);  // [0, 2q)
    slot_sync();  // the forward exchange's buffers are reused
    uint32_t* const li[1] = {lb[0]};
    RowTw<S> wi;  // unused: this form loads its twiddles in place
    inv_rows<S, 1, 1>(y, li, j, itw, tw_mul, q, two_q, wi);
#pragma unroll
    for (int u = 0; u < 16; ++u) __builtin_amdgcn_raw_buffer_store_b32(y[0][u], ra, (int)(lane + 4u * u * T), 0, 0);
  }
}

template <int S, int MODE, int CG>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(S >= 6 ? 3 : 2))) void rows_fused_kernel(
    RowsArgs a) {
  rows_fused_kernel_body<S, MODE, CG>(a, own_blk());
}

// The same over the cells of a stage-batched plan: one launch, each workgroup in its
// cell's segment (cell_of) with that cell's arguments.
template <int S, int MODE, int CG>
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(S >= 6 ? 3 : 2))) void rows_fused_kernel_multi(
    const RowsArgs* __restrict__ cells, const CellSeg* __restrict__ seg, int ncells) {
  Blk bk;
  const int c = cell_of(seg, ncells, bk);
  if (c < 0) return;
  rows_fused_kernel_body<S, MODE, CG>(cells[c], bk);
}

template <int S, int MODE, int CG>
static hipError_t rows_fused(const RowsArgs& a, hipStream_t st) {
  constexpr int n = 1 << S;
  constexpr int RPW = RowsShape<S>::NSUB / CG;
  const int nsub_total = (1 << a.logN) / n;
  const int nwg = (nsub_total + RPW - 1) / RPW;
  const int kx = (a.K + 7) / 8;
  const int ncg = (a.cnum + CG - 1) / CG;
  dim3 grid(8 * kx * ncg * nwg);
  // algorithmic HBM bytes per prime: tensor 4 rows in and 3 out per ciphertext; relin
  // 1 row in and 2 out per ciphertext plus the key's 2 rows once; ring 2 in (b once per
  // distinct operand) and 1 out per group
  const int b_rows = a.data2_stride ? std::min(a.data2_groups, a.cnum) : 1;
  const double rows = MODE == 0 ? 7.0 * a.cnum : (MODE == 1 ? 3.0 * a.cnum + 2.0 : 2.0 * a.cnum + b_rows);
  Bracket br(KID_ROWS_FUSED, st, 4.0 * rows * a.K * (double)(1 << a.logN));
  const hipError_t e = emit((const void*)rows_fused_kernel<S, MODE, CG>,
                            (const void*)rows_fused_kernel_multi<S, MODE, CG>, grid, dim3(128), 0, st, a);
  return e != hipSuccess ? e : hipGetLastError();
}

// Bytes a workgroup's buffers span from their base: they must stay below the
// out-of-range lane offset 0x7FFFFF00 (the tensor form's, the largest, spans 3 K N words
// past its group's last ciphertext; the relinearization output 1 K N past it), plus the
// workgroup's NSUB n = 2048 words.
static long long rows_span_bytes(const RowsArgs& a, int cg) {
  const long long KN = (long long)a.K << a.logN;
  const long long last = (long long)(cg - 1) * std::max(a.group_stride, a.out_stride);
  return (last + 3 * KN + 2048) * 4;
}

template <int MODE>
static hipError_t rows_fused_s(int S, const RowsArgs& a, hipStream_t st) {
  if (rows_span_bytes(a, 1) >= 0x70000000LL) return hipErrorInvalidValue;
  // four ciphertexts per sub-row where rows are 256 points and at most 1 slot in 8 idles
  if (MODE != 2 && S == 8 && 8 * (4 * ((a.cnum + 3) / 4) - a.cnum) <= 4 * ((a.cnum + 3) / 4) &&
      rows_span_bytes(a, 4) < 0x70000000LL)
    return rows_fused<8, MODE == 2 ? 0 : MODE, 4>(a, st);
  switch (S) {
    case 5: return rows_fused<5, MODE, 1>(a, st);
    case 6: return rows_fused<6, MODE, 1>(a, st);
    case 7: return rows_fused<7, MODE, 1>(a, st);
    case 8: return rows_fused<8, MODE, 1>(a, st);
    default: return hipErrorInvalidValue;
  }
}

template <int S, bool INV, bool ROWS, int BLK = ntt_pass_threads<S, ROWS>(), int CG = 1>
static hipError_t ntt_pass(const NttArgs& a, int ntr, hipStream_t st) {
  constexpr int n = 1 << S;
  constexpr int RPW = BLK / (n / 16) / CG;
  const int nsub_total = (1 << a.logN) / n;
  const int nwg = (nsub_total + RPW - 1) / RPW;
  const int kx = (a.K + 7) / 8;  // primes per XCD (the largest share)
  const int ncg = (ntr / a.K + CG - 1) / CG;
  dim3 grid(8 * kx * ncg * nwg);
  // algorithmic work: (N / 2) S butterflies per transform, one constant product each
  // algorithmic HBM bytes: every element of every transform read and written once
  Bracket br(INV ? (ROWS ? KID_NTT_INV_ROWS : KID_NTT_INV_COLS) : (ROWS ? KID_NTT_FWD_ROWS : KID_NTT_FWD_COLS), st,
             8.0 * ntr * (double)(1 << a.logN));
  const hipError_t e = emit((const void*)ntt_pass_kernel<S, INV, ROWS, BLK, CG>,
                             (const void*)ntt_pass_kernel_multi<S, INV, ROWS, BLK, CG>, grid, dim3(BLK), 0, st, a);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

// cols_threads: 0 for the default workgroup of a column pass, else 256 or 512 threads
// (16 or 32 columns of 2^8 points, 32 of 2^7) where it is smaller than the default.
template <bool INV, bool ROWS>
static hipError_t ntt_pass_s(int S, const NttArgs& a, int ntr, hipStream_t st, int cols_threads = 0) {
  // row passes of 256 points over blocks of four transforms one group apart (one
  // polynomial per group), where at most one slot in eight idles and the block's span
  // stays below the buffer's out-of-range offset
  const int npp = ntr / a.K, ncg4 = (npp + 3) / 4;
  if (ROWS && S == 8 && a.per_group == a.K && npp >= 4 && 8 * (4 * ncg4 - npp) <= 4 * ncg4 &&
      (3 * a.group_stride + (1LL << a.logN)) * 4 < 0x70000000LL)
    return ntt_pass<8, INV, true, 256, 4>(a, ntr, st);
  if (!ROWS && S == 8 && cols_threads == 256) return ntt_pass<8, INV, false, 256>(a, ntr, st);
  if (!ROWS && S == 8 && cols_threads == 512) return ntt_pass<8, INV, false, 512>(a, ntr, st);
  if (!ROWS && S == 7 && cols_threads == 256) return ntt_pass<7, INV, false, 256>(a, ntr, st);
  switch (S) {
    case 5: return ntt_pass<5, INV, ROWS>(a, ntr, st);
    case 6: return ntt_pass<6, INV, ROWS>(a, ntr, st);
    case 7: return ntt_pass<7, INV, ROWS>(a, ntr, st);
    case 8: return ntt_pass<8, INV, ROWS>(a, ntr, st);
    default: return hipErrorInvalidValue;
  }
}

// dst[r n + u T + j] = src[r n + 16 j + u] within rows of n = 2^S words (T = n / 16):
// a key in NTT form laid out in the order the fused relinearization pass holds it.
__global__ __launch_bounds__(256) void row_transpose_kernel(
    const uint32_t* src, uint32_t* dst, long long total, int S) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const int n = 1 << S, T = n >> 4;
  const int pos = (int)(i & (n - 1)), u = pos / T, j = pos % T;
  dst[i] = src[(i - pos) + 16 * j + u];
}

hipError_t launch_row_transpose(const uint32_t* src, uint32_t* dst, long long total, int S, hipStream_t st) {
  if (total <= 0) return hipSuccess;
  if (S < 4 || (total & ((1LL << S) - 1)) != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(row_transpose_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, src, dst, total, S);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void scale_rows_kernel(uint32_t* data, long long total, int K, int logN,
                                                        const uint2* scale, const PrimeC* pc) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= total) return;
  const int p = (int)((i >> logN) % K);
  const uint32_t q = pc[p].q;
  data[i] = csub(shoup_lazy(data[i], scale[p].x, scale[p].y, q), q);
}

hipError_t launch_scale_rows(uint32_t* data, long long rows, int K, int N, const uint2* scale, const PrimeC* pc,
                             hipStream_t st) {
  const long long total = rows * N;
  if (total <= 0) return hipSuccess;
  if (K <= 0 || (N & (N - 1)) != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(scale_rows_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, data, total, K,
                     __builtin_ctz((unsigned)N), scale, pc);
  return hipGetLastError();
}

int ntt_split_cols(int logN, const Tuning& tu) { return tu.ntt_cols_first ? logN - logN / 2 : logN / 2; }

hipError_t launch_ntt_cols(const NttArgs& a0, int ntr, bool inverse, hipStream_t st, const Tuning& tu) {
  if (ntr <= 0) return hipSuccess;
  if (ntr % a0.K != 0 || a0.per_group % a0.K != 0) return hipErrorInvalidValue;
  NttArgs a = a0;
  a.ntr = ntr;
  const int s_cols = ntt_split_cols(a.logN, tu);
  return inverse ? ntt_pass_s<true, false>(s_cols, a, ntr, st, tu.cols_threads)
                 : ntt_pass_s<false, false>(s_cols, a, ntr, st, tu.cols_threads);
}

hipError_t launch_rows_fused(const RowsArgs& a, int mode, hipStream_t st, const Tuning& tu) {
  if (a.cnum <= 0) return hipSuccess;
  const int s_rows = a.logN - ntt_split_cols(a.logN, tu);
  switch (mode) {
    case ROWS_TENSOR: return rows_fused_s<0>(s_rows, a, st);
    case ROWS_RELIN: return rows_fused_s<1>(s_rows, a, st);
    case ROWS_RING: return rows_fused_s<2>(s_rows, a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ntt(const NttArgs& a0, int ntr, bool inverse, hipStream_t st, const Tuning& tu) {
  if (ntr <= 0) return hipSuccess;
  if (ntr % a0.K != 0 || a0.per_group % a0.K != 0) return hipErrorInvalidValue;
  NttArgs a = a0;
  a.ntr = ntr;
  // the split groups the same stages differently and does not change the result
  const int s_cols = ntt_split_cols(a.logN, tu);
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

// The limbs of input polynomial z of a lift.
__device__ __forceinline__ const uint32_t* lift_source(const LiftArgs& a, uint32_t z) {
  if (a.interleave4) {
    const uint32_t i = z & 3u, c = z >> 2;
    return a.in_ptrs ? a.in_ptrs[i * (uint32_t)(a.npoly >> 2) + c] : a.in4[i] + (long long)c * a.in_stride;
  }
  return a.in_ptrs ? a.in_ptrs[z] : a.limbs + (long long)z * a.in_stride;
}

template <int PB>
__device__ __forceinline__ void lift_kernel_body(const LiftArgs& a, const Blk bk) {
  // Workgroup w runs on XCD w % 8.  The prime groups of one (polynomial,
  // coefficient block) unit are consecutive workgroups of one XCD, so the unit's
  // limbs are read from HBM once and then from that XCD's L2.
  const int G = (a.K + PB - 1) / PB;
  const int nb = (a.N + 255) / 256;
  const int w = bk.x, xcd = w & 7, l = w >> 3;
  const int unit = (l / G) * 8 + xcd;
  if (unit >= nb * a.npoly) return;
  const int p0 = (l % G) * PB;
  const int z = unit / nb;
  const int jc = (unit % nb) * 256 + threadIdx.x;  // coefficient
  if (jc >= a.N) return;
  const uint32_t* src = lift_source(a, (uint32_t)z) + jc;
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
__global__ __launch_bounds__(256) void lift_kernel(LiftArgs a) { lift_kernel_body<PB>(a, own_blk()); }

// The same over the cells of a stage-batched plan: one launch, each workgroup in its
// cell's segment (cell_of) with that cell's arguments.
template <int PB>
__global__ __launch_bounds__(256) void lift_kernel_multi(
    const LiftArgs* __restrict__ cells, const CellSeg* __restrict__ seg, int ncells) {
  Blk bk;
  const int c = cell_of(seg, ncells, bk);
  if (c < 0) return;
  lift_kernel_body<PB>(cells[c], bk);
}

template <int PB>
static void lift_launch(const LiftArgs& b, int npoly, hipStream_t st) {
  const int G = (b.K + PB - 1) / PB;
  const int units = ((b.N + 255) / 256) * npoly;
  dim3 grid(8 * ((units + 7) / 8) * G);
  (void)emit((const void*)lift_kernel<PB>, (const void*)lift_kernel_multi<PB>, grid, dim3(256), 0, st, b);
}

// The same projection on the i8 matrix cores.  A limb's four bytes minus 128 are
// signed digits s_(i,a), so A = sum_(i,a) s_(i,a) 2^(32 i + 8 a) + C0 with the
// constant C0 = 0x80808080 sum_(i<L) 2^(32 i): a limb word XOR 0x80808080 is its
// four digits as int8 bytes.  The digit index runs along the contraction, against
// the constants T_(i,a),p = [2^(32 i + 8 a) 2^32]_(q_p) split into four balanced
// byte planes b (rows of the tile: row = 8 b + p', prime 8 t + p').  The VALU adds
// the planes (sum_b 2^(8 b) C_b, |.| < 2^49), the per-prime constant
// [C0 2^32]_(q_p) + 2^20 q_p (makes it positive), and Montgomery-reduces.
// One wave per 32 coefficients; lane (c, h) supplies limbs 8 kb + 4 h + r (r < 4)
// of coefficient c as B register r of k-block kb.
// Workgroups are persistent: each wave takes groups of 32 coefficients in turn.
// With LDSA the A table is staged once per workgroup in LDS (else read from L2).
template <int NKB, bool LDSA, int BLK>
__device__ __forceinline__ void lift_mfma_kernel_body(const LiftArgs& a, const Blk bk) {
  extern __shared__ v4i sA[];
  __shared__ uint32_t s_q[kCrtMaxPrimes], s_qn[kCrtMaxPrimes], s_olo[kCrtMaxPrimes], s_ohi[kCrtMaxPrimes];
  const int nfrag = a.ntiles * NKB * 64;
  if (LDSA)
    for (int f = threadIdx.x; f < nfrag; f += BLK) sA[f] = a.A[f];
  for (int p = threadIdx.x; p < 8 * a.ntiles; p += BLK) {
    const int pl = min(p, a.K - 1);
    s_q[p] = a.pc[pl].q;
    s_qn[p] = a.pc[pl].qneg;
    const uint64_t o = a.off[pl];
    s_olo[p] = (uint32_t)o;
    s_ohi[p] = (uint32_t)(o >> 32);
  }
  __syncthreads();
  uint32_t one = 1, m8 = 256, m16 = 65536, m24 = 16777216;  // opaque multipliers of mad_i64
  opaque(one);
  opaque(m8);
  opaque(m16);
  opaque(m24);
  const v4i* At = LDSA ? sA : a.A;
  const int lane = threadIdx.x & 63, c = lane & 31, h = lane >> 5;
  const int lg = __builtin_ctz((unsigned)a.N) - 5;  // log2 of the 32-coefficient groups per poly
  const uint32_t total = (uint32_t)a.npoly << lg;
  const uint32_t row = 4u * (uint32_t)a.N;          // bytes between limb (or residue) rows
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (uint32_t unit = bk.x * (BLK / 64) + wave; unit < total; unit += bk.nx * (BLK / 64)) {
    // row 4 h, column c of a 32-coefficient group; recomputed per unit (opaque), or the
    // row offsets derived from it are hoisted out of the loop, each holding a register
    uint32_t lane_off = 4u * h * row + 4u * c;
    opaque(lane_off);
    const uint32_t z = unit >> lg, j0 = (unit & ((1u << lg) - 1u)) << 5;
    const uint32_t* src = wave_uniform(lift_source(a, z) + j0);
    // limbs 8 kb + 4 h + r; rows at or beyond L read as zero, where the table is zero too
    const __amdgpu_buffer_rsrc_t rs = row_buffer(src, 4u * ((uint32_t)a.L * (uint32_t)a.N - j0));
    v4i B[NKB];
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
      for (int r = 0; r < 4; ++r) B[kb][r] = (int)(buffer_word(rs, lane_off + (8 * kb + r) * row) ^ 0x80808080u);
    uint32_t* dst = wave_uniform(a.res + (long long)z * a.out_stride + j0);
    // one tile: residues 8 t + 4 h + i (i < 4); `last` guards the rows past K
    auto tile = [&](int t, bool last) {
      const v4i* Ap = At + (long long)t * NKB * 64 + lane;
      v4i Af[NKB];
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) Af[kb] = Ap[kb * 64];
      // two independent accumulation chains (a single dependent chain issues at 2/3 rate)
      v16i acc = {}, acc2 = {};
#pragma unroll
      for (int kb = 0; kb < NKB; kb += 2) acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(Af[kb], B[kb], acc, 0, 0, 0);
#pragma unroll
      for (int kb = 1; kb < NKB; kb += 2) acc2 = __builtin_amdgcn_mfma_i32_32x32x32_i8(Af[kb], B[kb], acc2, 0, 0, 0);
      if (NKB > 1) acc += acc2;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int p = 8 * t + 4 * h + i;
        const uint32_t q = s_q[p];
        int64_t v = (int64_t)(((uint64_t)s_ohi[p] << 32) | s_olo[p]);
        v = mad_i64(acc[i], one, v);
        v = mad_i64(acc[4 + i], m8, v);
        v = mad_i64(acc[8 + i], m16, v);
        v = mad_i64(acc[12 + i], m24, v);
        const uint32_t r = csub(redc_lazy((uint64_t)v, q, s_qn[p]), q);
        if (!last || p < a.K) store_at(dst, lane_off + i * row, r);
      }
    };
    for (int t = 0; t < a.ntiles - 1; ++t) {
      tile(t, false);
      dst += 8 * a.N;
    }
    tile(a.ntiles - 1, true);
  }
}

template <int NKB, bool LDSA, int BLK>
__global__ __launch_bounds__(BLK) void lift_mfma_kernel(LiftArgs a) {
  lift_mfma_kernel_body<NKB, LDSA, BLK>(a, own_blk());
}

// The same over the cells of a stage-batched plan: one launch, each workgroup in its
// cell's segment (cell_of) with that cell's arguments.
template <int NKB, bool LDSA, int BLK>
__global__ __launch_bounds__(BLK) void lift_mfma_kernel_multi(
    const LiftArgs* __restrict__ cells, const CellSeg* __restrict__ seg, int ncells) {
  Blk bk;
  const int c = cell_of(seg, ncells, bk);
  if (c < 0) return;
  lift_mfma_kernel_body<NKB, LDSA, BLK>(cells[c], bk);
}

// Persistent grid: enough workgroups to fill the chip, no more than the work needs.
static unsigned persistent_grid(long long units, int waves_per_block, int blocks_per_cu, int cus) {
  const long long need = (units + waves_per_block - 1) / waves_per_block;
  return (unsigned)std::max(1LL, std::min(need, (long long)blocks_per_cu * cus));
}

template <int NKB>
static void lift_mfma_launch(const LiftArgs& b, hipStream_t st) {
  const long long units = (long long)b.npoly * (b.N >> 5);
  const size_t lds = (size_t)b.ntiles * NKB * 64 * sizeof(v4i);
  const size_t lds_static = 4 * kCrtMaxPrimes * 4;
  if (NKB <= 7 && lds + lds_static <= (size_t)b.lds_max) {  // larger k-block counts spill at 768 threads
    static bool attr = false;  // allow the rest of the device's LDS for this instantiation (once)
    if (!attr)
      attr = hipFuncSetAttribute((const void*)lift_mfma_kernel<NKB, true, 768>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 b.lds_max - (int)lds_static) == hipSuccess;
    (void)emit((const void*)lift_mfma_kernel<NKB, true, 768>, (const void*)lift_mfma_kernel_multi<NKB, true, 768>,
               dim3(persistent_grid(units, 12, 1, b.cus)), dim3(768), lds, st, b);
  } else {
    (void)emit((const void*)lift_mfma_kernel<NKB, false, 256>, (const void*)lift_mfma_kernel_multi<NKB, false, 256>,
               dim3(persistent_grid(units, 4, 8, b.cus)), dim3(256), 0, st, b);
  }
}

hipError_t launch_lift(const LiftArgs& a, int npoly, hipStream_t st, const Tuning& t) {
  if (npoly <= 0) return hipSuccess;
  LiftArgs b = a;
  b.npoly = npoly;
  // algorithmic HBM bytes: L limbs read and K residues written per coefficient
  Bracket br(KID_LIFT, st, 4.0 * npoly * a.N * (double)(a.L + a.K));
  if (t.lift_primes == 0 && a.A) {
    // the table's k-block count: exact up to 16 (L <= 128), else padded to 32
    switch (b.nkb) {
      case 1: lift_mfma_launch<1>(b, st); break;
      case 2: lift_mfma_launch<2>(b, st); break;
      case 3: lift_mfma_launch<3>(b, st); break;
      case 4: lift_mfma_launch<4>(b, st); break;
      case 5: lift_mfma_launch<5>(b, st); break;
      case 6: lift_mfma_launch<6>(b, st); break;
      case 7: lift_mfma_launch<7>(b, st); break;
      case 8: lift_mfma_launch<8>(b, st); break;
      case 9: lift_mfma_launch<9>(b, st); break;
      case 10: lift_mfma_launch<10>(b, st); break;
      case 11: lift_mfma_launch<11>(b, st); break;
      case 12: lift_mfma_launch<12>(b, st); break;
      case 13: lift_mfma_launch<13>(b, st); break;
      case 14: lift_mfma_launch<14>(b, st); break;
      case 15: lift_mfma_launch<15>(b, st); break;
      case 16: lift_mfma_launch<16>(b, st); break;
      case 32: lift_mfma_launch<32>(b, st); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  switch (t.lift_primes) {
    case 8: lift_launch<8>(b, npoly, st); break;
    case 32: lift_launch<32>(b, npoly, st); break;
    default: lift_launch<16>(b, npoly, st); break;
  }
  return hipGetLastError();
}

// ============================================================================ CRT reconstruction
// Residues -> limbs (the reconstruction step of Section 5.1 / Eq. garner_mrc, here
// in its direct CRT form).  With M = q_0 ... q_(K-1), c_k = [(M/q_k)^-1]_(q_k) and
// the inverse NTT's final factor including c_k, a transform output x_k
// gives y_k = [x_k + d_k]_(q_k), d_k = [2^e c_k]_(q_k), the CRT coordinates of
// Y = X + 2^e in [0, 2^(e+1)) (X the signed exact product, |X| < 2^e).  Then
//   Y = sum_k y_k (M/q_k) - alpha M,   alpha = floor(sum_k y_k / q_k),
// and the output is X mod 2^outbits = (Y - 2^e) mod 2^outbits.  The prime count
// leaves Y / M < 2^-16, so alpha is exact from the sum in fixed point
// sum_k y_k floor(2^56 / q_k) (each term < 2^56, truncation error < K 2^-26 <
// 2^-18 in units of 2^56): alpha = (sum + 2^38) >> 56.
//
// The column sums sum_k y_k V_kl, V_kl = limb l of (M/q_k) mod 2^(32 Lout), are a
// dense integer contraction [coefficients x K] x [K x Lout] and run on the i8
// matrix cores: y_k - 0x80808080 and V_kl are split into 4 balanced base-256 digits
// each (digits in [-128, 127]; the digits of y_k - 0x80808080 are the bytes of
// y_k ^ 0x80808080, and limbs of V are taken in [-0x80808080, 0x7F7F7F7F]), the 16
// digit-plane products accumulate exactly in int32 (|sum| <= K 2^14), and the VALU
// recombines sum_(a,b) 2^(8(a+b)) C_ab per limb (the 7 diagonal sums in int32, then
// 64-bit multiply-adds), adds alpha [-M] + [0x80808080 sum_k V_k - 2^e] (both
// constants as limbs mod 2^(32 Lout)), and propagates the carries.
//
// One wave per 32 coefficients.  MFMA v_mfma_i32_32x32x32_i8: lane (c, h) = (lane
// mod 32, lane / 32) supplies B bytes k = 32 kb + 16 h + i (i < 16) of coefficient
// column c, and A bytes of row c for the same k; its accumulator holds rows
// 8 j + 4 h + i.  Rows of a tile are (digit plane b of V, limb 8 t + l'), row =
// 8 b + l', so lane half h ends with all four planes of limbs 8 t + 4 h + i.


// 4 x 32-bit words -> their byte plane a (a < 4) as 4 packed bytes, for all planes.
__device__ __forceinline__ void byte_planes(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, uint32_t& p0,
                                            uint32_t& p1, uint32_t& p2, uint32_t& p3) {
  // v_perm_b32: result byte i = byte sel_i of {src0 (bytes 4..7), src1 (bytes 0..3)}
  const uint32_t lo01 = __builtin_amdgcn_perm(w1, w0, 0x05010400u);  // w0.0 w1.0 w0.1 w1.1
  const uint32_t hi01 = __builtin_amdgcn_perm(w1, w0, 0x07030602u);  // w0.2 w1.2 w0.3 w1.3
  const uint32_t lo23 = __builtin_amdgcn_perm(w3, w2, 0x05010400u);
  const uint32_t hi23 = __builtin_amdgcn_perm(w3, w2, 0x07030602u);
  p0 = __builtin_amdgcn_perm(lo23, lo01, 0x05040100u);  // w0.0 w1.0 w2.0 w3.0
  p1 = __builtin_amdgcn_perm(lo23, lo01, 0x07060302u);
  p2 = __builtin_amdgcn_perm(hi23, hi01, 0x05040100u);
  p3 = __builtin_amdgcn_perm(hi23, hi01, 0x07060302u);
}

// Waves per workgroup: one persistent workgroup per CU holds the LDS table; 12 waves
// (3 per SIMD) where the registers allow it, else 8.
template <int NKB>
constexpr int crt_waves() { return NKB <= 4 ? 12 : 8; }

template <int NKB, bool LDSA>
__device__ __forceinline__ void crt_kernel_body(const CrtArgs& a, const Blk bk) {
  constexpr int kCrtWaves = crt_waves<NKB>();
  extern __shared__ v4i sA[];
  __shared__ uint32_t s_q[32 * NKB], s_d[32 * NKB], s_r[32 * NKB];
  __shared__ uint32_t s_mneg[kCrtMaxLimbs], s_eneg[kCrtMaxLimbs];
  for (int k = threadIdx.x; k < 32 * NKB; k += 64 * kCrtWaves) {
    const bool in = k < a.K;
    s_q[k] = in ? a.pc[k].q : 1u;
    s_d[k] = in ? a.d[k] : 0u;
    s_r[k] = in ? a.rq[k] : 0u;  // rows past K add nothing to the quotient
  }
  for (int l = threadIdx.x; l < 8 * a.ntiles; l += 64 * kCrtWaves) {
    s_mneg[l] = a.mneg[l];
    s_eneg[l] = a.eneg[l];
  }
  if (LDSA)
    for (int f = threadIdx.x; f < a.ntiles * NKB * 64; f += 64 * kCrtWaves) sA[f] = a.A[f];
  __syncthreads();
  const v4i* At = LDSA ? sA : a.A;
  const int lane = threadIdx.x & 63, c = lane & 31, h = lane >> 5;
  const int lg = __builtin_ctz((unsigned)a.N) - 5;  // log2 of the 32-coefficient groups per poly
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t total = (uint32_t)a.npoly << lg;
  // the waves sharing a SIMD start apart, so that one's loads overlap another's products
  if (wave >= 4) __builtin_amdgcn_s_sleep(63);
  if (wave >= 8) __builtin_amdgcn_s_sleep(63);
  for (uint32_t unit = bk.x * kCrtWaves + wave; unit < total; unit += bk.nx * kCrtWaves) {
  const uint32_t z = unit >> lg, j0 = (unit & ((1u << lg) - 1u)) << 5;
  const uint32_t row = 4u * (uint32_t)a.N;  // bytes between residue (or limb) rows
  const uint32_t* xb = wave_uniform(a.res + (long long)(z / a.per_group) * a.gstride +
                                    (long long)(z % a.per_group) * a.pstride + j0);
  // residue rows 32 kb + 16 h + i; rows at or beyond K read as zero
  const __amdgpu_buffer_rsrc_t rs = row_buffer(xb, 4u * ((uint32_t)a.K * (uint32_t)a.N - j0));
  // recomputed per unit (opaque): hoisted out of the unit loop, the 80-odd row offsets
  // derived from it would each hold a register for the whole kernel
  uint32_t in_off = 16u * h * row + 4u * c;
  opaque(in_off);

  // phase 1: y_k, the partial sum of y_k / q_k, and the four digit planes per k-block.
  // The digits are the bytes of y_k ^ 0x80808080, i.e. of y_k - 0x80808080 in balanced
  // base 256; the table's constant adds back 0x80808080 sum_k V_k.  The next block's
  // loads are in flight while a block is converted.
  v4i B[NKB][4];
  uint64_t frac = 0;  // sum_k y_k floor(2^56 / q_k)
  uint32_t xv[16], xn[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) xv[i] = buffer_word(rs, in_off + i * row);
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb) {
    if (kb + 1 < NKB) {
#pragma unroll
      for (int i = 0; i < 16; ++i) xn[i] = buffer_word(rs, in_off + (32 * (kb + 1) + i) * row);
    }
    uint32_t s[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int k = 32 * kb + 16 * h + i;
      uint32_t y = xv[i] + s_d[k];
      y = min(y, y - s_q[k]);
      frac += (uint64_t)y * s_r[k];
      s[i] = y ^ 0x80808080u;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      uint32_t p0, p1, p2, p3;
      byte_planes(s[4 * r], s[4 * r + 1], s[4 * r + 2], s[4 * r + 3], p0, p1, p2, p3);
      // materialised here: left to the compiler, the planes may be recomputed later
      opaque(p0);
      opaque(p1);
      opaque(p2);
      opaque(p3);
      B[kb][0][r] = (int)p0;
      B[kb][1][r] = (int)p1;
      B[kb][2][r] = (int)p2;
      B[kb][3][r] = (int)p3;
    }
    if (kb + 1 < NKB) {
#pragma unroll
      for (int i = 0; i < 16; ++i) xv[i] = xn[i];
    }
  }
  frac = sum_lane_halves(frac);
  const uint32_t alpha = (uint32_t)((frac + (1ull << 38)) >> 56);
  // opaque multipliers of mad_i64 (the unit multipliers distinct per term of a sum)
  uint32_t one0 = 1, one1 = 1, one2 = 1, one3 = 1, m8 = 256, m16 = 65536, m24 = 16777216;
  opaque(one0);
  opaque(one1);
  opaque(one2);
  opaque(one3);
  opaque(m8);
  opaque(m16);
  opaque(m24);

  // phase 2, per tile of 8 limbs: the digit-plane products, recombination, carries.
  // Lane half h holds limbs l = 8 t + 4 h + i (i < 4) with C_ab = acc_a[4 b + i] (y plane
  // a, V plane b) and diagonal sums S_p = sum_(a+b=p) C_ab.  S_4..S_6 weigh 2^0..2^16 in
  // limb l + 1: inside the lane they join the next limb's sums, from the top limb they
  // leave with the carry.
  uint32_t* o = wave_uniform(a.out + (long long)z * a.ostride + j0);
  uint32_t out_off = 4u * h * row + 4u * c;
  opaque(out_off);
  const int topbits = a.outbits - 32 * (a.Lout - 1);
  int64_t cin = 0;  // carry into the tile (used in lane half 0)
  v16i acc0, acc1, acc2, acc3;
  auto products = [&](int t) {
    const v4i* Ap = At + ((long long)t * NKB) * 64 + lane;
    v4i Af[NKB];
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) Af[kb] = Ap[kb * 64];
    acc0 = v16i{};
    acc1 = v16i{};
    acc2 = v16i{};
    acc3 = v16i{};
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
      acc0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(Af[kb], B[kb][0], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(Af[kb], B[kb][1], acc1, 0, 0, 0);
      acc2 = __builtin_amdgcn_mfma_i32_32x32x32_i8(Af[kb], B[kb][2], acc2, 0, 0, 0);
      acc3 = __builtin_amdgcn_mfma_i32_32x32x32_i8(Af[kb], B[kb][3], acc3, 0, 0, 0);
    }
  };
  // tile sums: tt[i][p] = T_p of limb i (S_p plus S_(p+4) of limb i - 1), s4..s6 of limb 3
  int32_t tt[4][4], s4, s5, s6;
  auto sums = [&]() {
    s4 = s5 = s6 = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      tt[i][0] = acc0[i] + s4;
      tt[i][1] = acc0[4 + i] + acc1[i] + s5;
      tt[i][2] = acc0[8 + i] + acc1[4 + i] + acc2[i] + s6;
      tt[i][3] = acc0[12 + i] + acc1[8 + i] + acc2[4 + i] + acc3[i];
      s4 = acc1[12 + i] + acc2[8 + i] + acc3[4 + i];
      s5 = acc2[12 + i] + acc3[8 + i];
      s6 = acc3[12 + i];
    }
  };
  auto finish = [&](int t, bool last) {
    uint32_t ol[4];
    int64_t u = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int limb = 8 * t + 4 * h + i;
      // |T_p| <= 4 K 2^14 < 2^25: the limb value fits 64 bits with the constant and carry
      int64_t v = (int64_t)((uint64_t)alpha * s_mneg[limb] + s_eneg[limb]);
      v = mad_i64(tt[i][0], one0, v);
      v = mad_i64(tt[i][1], m8, v);
      v = mad_i64(tt[i][2], m16, v);
      v = mad_i64(tt[i][3], m24, v);
      if (i > 0) v = mad_i64((int32_t)(u >> 32), one1, v);
      u = v;
      ol[i] = (uint32_t)v;
    }
    int64_t carry = mad_i64(s4, one0, 0);
    carry = mad_i64(s5, m8, carry);
    carry = mad_i64(s6, m16, carry);
    carry = mad_i64((int32_t)(u >> 32), one1, carry);
    // carry across the lane halves: half 0 takes the carry into the tile, passes its
    // carry out to half 1, whose carry out enters the next tile
    carry = mad_i64(add_carry4(ol, h == 0 ? cin : 0), one2, carry);
    const int64_t mid = from_lane_below(carry);
    carry = mad_i64(add_carry4(ol, h == 1 ? mid : 0), one3, carry);
    cin = from_lane_above(carry);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int limb = 8 * t + 4 * h + i;
      uint32_t w = ol[i];
      if (last) {
        if (limb >= a.Lout) continue;
        if (limb == a.Lout - 1 && topbits < 32) w &= (1u << topbits) - 1u;
      }
      store_at(o, out_off + i * row, w);
    }
  };
  for (int t = 0; t < a.ntiles - 1; ++t) {
    products(t);
    sums();
    finish(t, false);
    o += 8 * a.N;
  }
  products(a.ntiles - 1);
  sums();
  finish(a.ntiles - 1, true);
  }
}

template <int NKB, bool LDSA>
__global__ __launch_bounds__(64 * crt_waves<NKB>()) void crt_kernel(CrtArgs a) {
  crt_kernel_body<NKB, LDSA>(a, own_blk());
}

// The same over the cells of a stage-batched plan: one launch, each workgroup in its
// cell's segment (cell_of) with that cell's arguments.
template <int NKB, bool LDSA>
__global__ __launch_bounds__(64 * crt_waves<NKB>()) void crt_kernel_multi(
    const CrtArgs* __restrict__ cells, const CellSeg* __restrict__ seg, int ncells) {
  Blk bk;
  const int c = cell_of(seg, ncells, bk);
  if (c < 0) return;
  crt_kernel_body<NKB, LDSA>(cells[c], bk);
}

template <int NKB>
static void crt_launch(const CrtArgs& a, hipStream_t st) {
  constexpr int kCrtWaves = crt_waves<NKB>();
  const long long units = (long long)a.npoly * (a.N >> 5);
  const size_t lds = (size_t)a.ntiles * NKB * 64 * sizeof(v4i);
  const unsigned grid = persistent_grid(units, kCrtWaves, 1, a.cus);
  const size_t lds_static = 32 * NKB * 12 + 2 * kCrtMaxLimbs * 4;
  if (lds + lds_static <= (size_t)a.lds_max) {
    static bool attr = false;  // allow the full LDS of the device for this instantiation (once)
    if (!attr)
      attr = hipFuncSetAttribute((const void*)crt_kernel<NKB, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 a.lds_max - (int)lds_static) == hipSuccess;
    (void)emit((const void*)crt_kernel<NKB, true>, (const void*)crt_kernel_multi<NKB, true>, dim3(grid),
               dim3(64 * kCrtWaves), lds, st, a);
  } else {
    (void)emit((const void*)crt_kernel<NKB, false>, (const void*)crt_kernel_multi<NKB, false>, dim3(grid),
               dim3(64 * kCrtWaves), 0, st, a);
  }
}

hipError_t launch_crt(CrtArgs a, int npoly, hipStream_t st) {
  a.npoly = npoly;
  if (npoly == 0) return hipSuccess;
  const int nkb = (a.K + 31) / 32;
  // algorithmic HBM bytes: K residues read and Lout limbs written per coefficient
  Bracket br(KID_CRT, st, 4.0 * npoly * a.N * (double)(a.K + a.Lout));
  switch (nkb) {
    case 1: crt_launch<1>(a, st); break;
    case 2: crt_launch<2>(a, st); break;
    case 3: crt_launch<3>(a, st); break;
    case 4: crt_launch<4>(a, st); break;
    case 5: crt_launch<5>(a, st); break;
    case 6: crt_launch<6>(a, st); break;
    case 7: crt_launch<7>(a, st); break;
    case 8: crt_launch<8>(a, st); break;
    default: return hipErrorInvalidValue;
  }
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

__device__ __forceinline__ void compose_kernel_body(const ComposeArgs& a, const Blk bk) {
  const int jc = bk.x * 256 + threadIdx.x;
  const int z = bk.y;  // 2 c + i
  if (jc >= a.N) return;
  const int c = z >> 1, i = z & 1;
  const uint32_t* k = a.k + (long long)z * a.kstride + jc;
  const uint32_t* d = a.d + (long long)(3 * c + i) * a.dstride + jc;
  const bool dread = !(a.d1_zero && i);  // block-uniform
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
    const uint64_t sum = (uint64_t)(dread ? d[(long long)l * a.N] : 0u) + ks + cl + carry;
    uint32_t wv = (uint32_t)sum;
    carry = sum >> 32;
    if (l == a.L - 1 && topbits < 32) wv &= (1u << topbits) - 1u;
    o[(long long)l * a.N] = wv;
  }
}

__global__ __launch_bounds__(256) void compose_kernel(ComposeArgs a) { compose_kernel_body(a, own_blk()); }

// The same over the cells of a stage-batched plan: one launch, each workgroup in its
// cell's segment (cell_of) with that cell's arguments.
__global__ __launch_bounds__(256) void compose_kernel_multi(
    const ComposeArgs* __restrict__ cells, const CellSeg* __restrict__ seg, int ncells) {
  Blk bk;
  const int c = cell_of(seg, ncells, bk);
  if (c < 0) return;
  compose_kernel_body(cells[c], bk);
}

// compose and rescale in one pass (a HE-mult with rescale): c = [d + R_P(k)]_(2^logq)
// is produced limb by limb and never stored; the rescale's correction is collected
// from its low limbs as they appear (the round bit, or (c mod 2^bits) mod t), and
// output limb m of [R_B(c)]_(2^(logq - bits)) is emitted once c limbs sb + m and
// sb + m + 1 exist (sb = bits / 32).
__device__ __forceinline__ void compose_rescale_kernel_body(const ComposeArgs& a, const Blk bk) {
  const int jc = bk.x * 256 + threadIdx.x;
  const int z = bk.y;  // 2 c + i
  if (jc >= a.N) return;
  const int c = z >> 1, i = z & 1;
  const uint32_t* k = a.k + (long long)z * a.kstride + jc;
  const uint32_t* d = a.d + (long long)(3 * c + i) * a.dstride + jc;
  const bool dread = !(a.d1_zero && i);  // block-uniform
  uint32_t* o = (a.out0s ? (i ? a.out1s[c] : a.out0s[c]) : (i ? a.out1 : a.out0) + (long long)c * a.ostride) + jc;
  // compose state
  const int64_t corrP = round_correction(k, a.N, a.LK, a.logP, a.scheme, a.t, a.invP, a.pw);
  const int sl = a.logP >> 5, rs = a.logP & 31;
  const uint32_t extP = corrP < 0 ? 0xFFFFFFFFu : 0u;
  uint64_t carryP = 0;
  uint32_t klo = sl < a.LK ? k[(long long)sl * a.N] : 0u;
  const int topbits = a.logq - 32 * (a.L - 1);
  // rescale state
  const int sb = a.bits >> 5, rb = a.bits & 31;
  const int newq = a.logq - a.bits, Lout = (newq + 31) >> 5, otop = newq - 32 * (Lout - 1);
  uint64_t acc = 0;  // BGV: (c mod 2^bits) mod t, accumulated per limb
  uint32_t rbit = 0;  // CKKS: bit bits-1 of c
  int64_t corrB = 0;
  uint32_t extB = 0, cprev = 0;
  uint64_t carryB = 0;
  auto emit = [&](int m, uint32_t xs) {
    const uint32_t cl = m == 0 ? (uint32_t)corrB : extB;
    const uint64_t sum = (uint64_t)xs + cl + carryB;
    uint32_t w = (uint32_t)sum;
    carryB = sum >> 32;
    if (m == Lout - 1 && otop < 32) w &= (1u << otop) - 1u;
    o[(long long)m * a.N] = w;
  };
  for (int l = 0; l < a.L; ++l) {
    const uint32_t khi = (sl + l + 1 < a.LK) ? k[(long long)(sl + l + 1) * a.N] : 0u;
    const uint32_t ks = rs ? ((klo >> rs) | (khi << (32 - rs))) : klo;
    klo = khi;
    const uint32_t cp = l == 0 ? (uint32_t)corrP : extP;
    const uint64_t sum = (uint64_t)(dread ? d[(long long)l * a.N] : 0u) + ks + cp + carryP;
    uint32_t cv = (uint32_t)sum;
    carryP = sum >> 32;
    if (l == a.L - 1 && topbits < 32) cv &= (1u << topbits) - 1u;
    // the rescale's correction from the low bits of c
    if (a.scheme == 0) {
      if (l == ((a.bits - 1) >> 5)) rbit = (cv >> ((a.bits - 1) & 31)) & 1u;
    } else if (l < sb) {
      acc += (uint64_t)cv * a.pw[l];
    } else if (l == sb && rb) {
      acc += (uint64_t)(cv & ((1u << rb) - 1u)) * a.pw[sb];
    }
    if (l == sb) {
      if (a.scheme == 0) {
        corrB = rbit;
      } else {
        const uint64_t rr = (acc % a.t) * a.invB % a.t;
        corrB = (2 * rr > a.t) ? (int64_t)rr - (int64_t)a.t : (int64_t)rr;
      }
      extB = corrB < 0 ? 0xFFFFFFFFu : 0u;
    }
    if (l > sb) {
      const int m = l - sb - 1;
      if (m < Lout) emit(m, rb ? ((cprev >> rb) | (cv << (32 - rb))) : cprev);
    }
    if (l >= sb) cprev = cv;
  }
  const int m = a.L - sb - 1;  // the last output limb takes zeros above c
  if (m >= 0 && m < Lout) emit(m, rb ? (cprev >> rb) : cprev);
}

__global__ __launch_bounds__(256) void compose_rescale_kernel(ComposeArgs a) {
  compose_rescale_kernel_body(a, own_blk());
}

// The same over the cells of a stage-batched plan: one launch, each workgroup in its
// cell's segment (cell_of) with that cell's arguments.
__global__ __launch_bounds__(256) void compose_rescale_kernel_multi(
    const ComposeArgs* __restrict__ cells, const CellSeg* __restrict__ seg, int ncells) {
  Blk bk;
  const int c = cell_of(seg, ncells, bk);
  if (c < 0) return;
  compose_rescale_kernel_body(cells[c], bk);
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
  Bracket br(KID_COMPOSE, st, 8.0 * cnum * a.N * (double)(a.LK + 2 * a.L));  // bytes: k_i, d_i in, c_i out
  const hipError_t e = emit((const void*)compose_kernel, (const void*)compose_kernel_multi, grid, dim3(256), 0, st, a);
  return e != hipSuccess ? e : hipGetLastError();
}

hipError_t launch_compose_rescale(const ComposeArgs& a, int cnum, hipStream_t st) {
  dim3 grid((a.N + 255) / 256, 2 * cnum);
  // bytes: k_i and d_i in, the rescaled c_i out
  Bracket br(KID_COMPOSE_RESCALE, st,
             8.0 * cnum * a.N * (double)(a.LK + a.L + ((a.logq - a.bits + 31) >> 5)));
  const hipError_t e =
      emit((const void*)compose_rescale_kernel, (const void*)compose_rescale_kernel_multi, grid, dim3(256), 0, st, a);
  return e != hipSuccess ? e : hipGetLastError();
}

hipError_t launch_rescale(const RescaleArgs& a, int cnum, hipStream_t st) {
  dim3 grid((a.N + 255) / 256, 2 * cnum);
  // bytes: L limbs in, L - bits/32 limbs out, per polynomial
  Bracket br(KID_RESCALE, st, 8.0 * cnum * a.N * (double)(((a.logq + 31) >> 5) + ((a.logq - a.bits + 31) >> 5)));
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
