// Internal interfaces between the host layer (api.hip) and the kernels
// (kernels.hip).  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "modarith.h"

namespace fhe {

typedef int v4i_t __attribute__((ext_vector_type(4)));

constexpr int kLogNMax = 16;
constexpr int kNMax = 1 << kLogNMax;
constexpr int kLiftDigitBits = 28;    // lift input digits: 8 digits = 7 limbs
constexpr int kLiftPrimes = 32;       // largest primes-per-thread choice of the lift
constexpr int kCrtMarginBits = 16;    // prime product >= 2^(e + 1 + margin): exact alpha
constexpr int kCrtMaxPrimes = 256;    // k-blocks of 32 held in registers by the CRT kernel (<= 8)
constexpr int kCrtMaxLimbs = 512;     // output limbs of one reconstruction (tiles of 8)

// Negacyclic NTT over a set of transforms.  Transform (group g, row r) lives at
// data + g * group_stride + r * N and uses prime r % K; per_group (rows per group)
// and the number of transforms are multiples of K.
struct NttArgs {
  uint32_t* data = nullptr;
  int logN = 0;
  int K = 0;
  int per_group = 0;
  long long group_stride = 0;
  const uint2* tw = nullptr; // [prime][kNMax] (w, floor(w 2^32 / q)), bit-reversed powers
  const PrimeC* pc = nullptr;
  const uint2* scale = nullptr; // inverse only: per-prime final factor (w, w'); null: the
                                // inputs already carry it (only the canonical reduction)
  const uint2* scale_w = nullptr; // with scale: the factor times the last stage's twiddle
                                  // (table entry 1), folded into that stage
  int ntr = 0;         // number of transforms (set by launch_ntt; a multiple of K)
};

// Fused last forward row pass + pointwise products + first inverse row pass over
// cnum groups of transforms whose column passes ran separately.
enum { ROWS_TENSOR = 0, ROWS_RELIN = 1, ROWS_RING = 2 };
struct RowsArgs {
  uint32_t* data = nullptr;        // group c at data + c group_stride: tensor [4][K][N]; relin [K][N]; ring a [K][N]
  const uint32_t* data2 = nullptr; // ring: b, group c at data2 + (c % data2_groups) data2_stride
  long long group_stride = 0;
  long long data2_stride = 0;      // ring: 0 gives every group the same b (broadcast)
  int data2_groups = 1;            // ring: groups of b (c and c + data2_groups share one)
  const uint32_t* key = nullptr;   // relin: the key's [2][K][N] in NTT form
  uint32_t* out = nullptr;         // relin: group c at out + c out_stride, [2][K][N]
  long long out_stride = 0;
  int logN = 0, K = 0, cnum = 0;
  const uint2* tw = nullptr;       // forward and inverse twiddles, [prime][kNMax]
  const uint2* itw = nullptr;
  const PrimeC* pc = nullptr;
};

struct LiftArgs {
  const uint32_t* limbs = nullptr; // poly z at limbs + z * in_stride, uint32[L][N] (or in_ptrs[z])
  const uint32_t* const* in_ptrs = nullptr;  // optional device array of per-poly inputs
  // four interleaved inputs (the tensor's x0, x1, y0, y1): poly z = 4 c + i is ciphertext c
  // of input i, at in4[i] + c * in_stride, or in_ptrs[i * (npoly / 4) + c]
  const uint32_t* in4[4] = {nullptr, nullptr, nullptr, nullptr};
  bool interleave4 = false;
  uint32_t* res = nullptr;          // poly z at res + z * out_stride, uint32[K][N]
  long long in_stride = 0, out_stride = 0;
  int N = 0, L = 0, K = 0;
  int npoly = 0;          // set by launch_lift
  const uint32_t* T = nullptr; // [prime][TS]: 2^(28 i) 2^32 mod q (VALU lift)
  int TS = 0;
  const PrimeC* pc = nullptr;
  // matrix-core lift: A fragments [tile of 8 primes][k-block of 8 limbs][lane] and
  // per-prime offsets [C0 2^32]_(q_p) + 2^20 q_p (null: only the VALU lift)
  const v4i_t* A = nullptr;
  const uint64_t* off = nullptr;
  int nkb = 0, ntiles = 0;
  int lds_max = 0, cus = 0;  // device: LDS bytes per workgroup, compute units
};

// CRT reconstruction of `npoly` polynomials from canonical residues (the inverse
// NTT's output with the CRT factor c_k folded in).
struct CrtArgs {
  const uint32_t* res = nullptr; // poly z: res + (z / per_group) * gstride + (z % per_group) * pstride, [K][N]
  int per_group = 0;
  long long gstride = 0, pstride = 0;
  uint32_t* out = nullptr;  // poly z: out + z * ostride, uint32[Lout][N]
  long long ostride = 0;
  int N = 0, K = 0, outbits = 0, Lout = 0;
  int ntiles = 0;           // tiles of 8 output limbs
  const v4i_t* A = nullptr; // [tile][k-block][lane]: the 16 MFMA A bytes of each lane
  const PrimeC* pc = nullptr;
  const uint32_t* d = nullptr;    // [k] = [2^e c_k]_(q_k)
  const uint32_t* rq = nullptr;   // [k] = floor(2^56 / q_k)
  const uint32_t* mneg = nullptr; // [l < 8 ntiles] limbs of (-M) mod 2^(32 Lout), zero beyond Lout
  const uint32_t* eneg = nullptr; // [l < 8 ntiles] limbs of (-2^e) mod 2^(32 Lout), zero beyond Lout
  int npoly = 0;                  // set by launch_crt
  int lds_max = 0, cus = 0;       // device: LDS bytes per workgroup, compute units
};

struct ComposeArgs {
  const uint32_t* k = nullptr; // poly z (= 2 c + i): k + z * kstride, uint32[LK][N]
  long long kstride = 0;
  const uint32_t* d = nullptr; // d_i of ciphertext c at d + (3 c + i) * dstride, uint32[L][N]
  long long dstride = 0;
  uint32_t* out0 = nullptr;
  uint32_t* out1 = nullptr;
  long long ostride = 0;  // per ciphertext, uint32[L][N]
  uint32_t* const* out0s = nullptr;  // optional device arrays of per-ciphertext outputs
  uint32_t* const* out1s = nullptr;
  int N = 0, L = 0, LK = 0, logq = 0, logP = 0, scheme = 0;
  uint32_t t = 0, invP = 0;  // BGV: t and 2^-logP mod t
  const uint32_t* pw = nullptr; // BGV: pw[l] = 2^(32 l) mod t
  int bits = 0;              // compose + rescale: rescale bits (outputs hold logq - bits bits)
  uint32_t invB = 0;         // BGV: 2^-bits mod t
  int d1_zero = 0;           // key switch: d_1 is zero (slot 1 is not read)
};

struct RescaleArgs {
  const uint32_t* in0 = nullptr;
  const uint32_t* in1 = nullptr;
  uint32_t* out0 = nullptr;
  uint32_t* out1 = nullptr;
  long long istride = 0, ostride = 0;
  uint32_t* const* out0s = nullptr;  // optional device arrays of per-ciphertext outputs
  uint32_t* const* out1s = nullptr;
  int N = 0, logq = 0, bits = 0, scheme = 0;
  uint32_t t = 0, invB = 0;  // BGV: t and 2^-bits mod t
  const uint32_t* pw = nullptr;
};

// Coefficient-wise sums: polynomial z = 2 c + i (ciphertext c, component i) of
// x at (i ? x1 : x0) + c xstride, likewise y (null component: zero) and out.
// out = [(-1)^negx x + (-1)^negy y]_(2^logq), L limbs, the top one masked.
struct LimbSumArgs {
  const uint32_t* x0 = nullptr;
  const uint32_t* x1 = nullptr;
  const uint32_t* y0 = nullptr;
  const uint32_t* y1 = nullptr;
  uint32_t* out0 = nullptr;
  uint32_t* out1 = nullptr;
  long long xstride = 0, ystride = 0, ostride = 0;  // ystride 0: one y for every ciphertext
  int N = 0, L = 0;
  uint32_t topmask = 0xFFFFFFFFu;
  int negx = 0, negy = 0;
};

// Signed permutation: out[k] = +-in[i mod N] with i = (k mul + add) mod 2N, negated
// when i >= N (automorphism: mul = g^-1 mod 2N, add = 0; monomial X^s: mul = 1,
// add = 2N - s).  Components and strides as in LimbSumArgs.
struct PermArgs {
  const uint32_t* in0 = nullptr;
  const uint32_t* in1 = nullptr;
  uint32_t* out0 = nullptr;
  uint32_t* out1 = nullptr;
  long long istride = 0, ostride = 0;
  int logN = 0, L = 0;
  uint32_t topmask = 0xFFFFFFFFu;
  uint32_t mul = 1, add = 0;
  int comps = 2;  // components per ciphertext (1: in0 -> out0 only)
};

// out = [(-1)^neg in k]_(2^logq) for an integer constant k of klimbs limbs.
constexpr int kConstMaxLimbs = 8;
struct ConstMulArgs {
  const uint32_t* in0 = nullptr;
  const uint32_t* in1 = nullptr;
  uint32_t* out0 = nullptr;
  uint32_t* out1 = nullptr;
  long long istride = 0, ostride = 0;
  int N = 0, L = 0;
  uint32_t topmask = 0xFFFFFFFFu;
  uint32_t k[kConstMaxLimbs] = {};
  int klimbs = 0, neg = 0;
};

// Optional per-kernel timing: when a recorder is installed, every launcher records
// a HIP event pair around its kernel on the launch stream.
enum KernelId {
  KID_LIFT = 0,
  KID_NTT_FWD_COLS,
  KID_NTT_FWD_ROWS,
  KID_NTT_INV_ROWS,
  KID_NTT_INV_COLS,
  KID_POINTWISE,
  KID_CRT,
  KID_COMPOSE,
  KID_RESCALE,
  KID_ROWS_FUSED,
  KID_COMPOSE_RESCALE,
  KID_COEFFWISE,  // coefficient-wise ops, signed permutations, constant products
  KID_COUNT
};

struct EventRecorder {
  virtual void begin(int kid, hipStream_t s) = 0;
  virtual void end(int kid, hipStream_t s, double work) = 0;
  virtual ~EventRecorder() {}
};

void set_recorder(EventRecorder* r);  // host thread-local
long long kernel_launch_count();      // kernels launched by this host thread so far
void bracket_begin(int kid, hipStream_t s);
void bracket_end(int kid, hipStream_t s, double work);

// Brackets one kernel launch with the recorder's events; `work` is the kernel's
// algorithmic HBM bytes (what it must read and write at least once).
// One cell's segment of a stage-batched launch (see LaunchSink): its first workgroup
// (a multiple of 8) and the grid gx x gy of the cell's own launch.
struct CellSeg {
  uint32_t off = 0, gx = 0, gy = 0, pad = 0;
};

// A launch as recorded instead of issued while a sink is installed: the entry point
// that runs it as one cell of a stage-batched launch, its grid, workgroup, dynamic LDS
// and argument struct (raw bytes; every entry point takes one struct).
struct LaunchRec {
  const void* multi = nullptr;
  dim3 grid, block;
  size_t lds = 0;
  std::vector<char> args;
};
struct LaunchSink {
  std::vector<LaunchRec> recs;
};
// While a sink is installed on this thread, the pipeline launchers append to it and
// launch nothing.
void set_launch_sink(LaunchSink* s);

struct Bracket {
  int kid;
  hipStream_t s;
  double work;
  Bracket(int k, hipStream_t st, double w) : kid(k), s(st), work(w) { bracket_begin(kid, s); }
  ~Bracket() { bracket_end(kid, s, work); }
};

// Launch parameters chosen by the autotuner (defaults: 16 primes per lift thread,
// NTT column pass of ceil(logN / 2) stages).
struct Tuning {
  int lift_primes = 0;  // 0: matrix-core lift; 8, 16 or 32: VALU lift with that many primes per thread
  int ntt_cols_first = 1;  // 1: column pass takes ceil(logN/2) stages; 0: floor
  int cols_threads = 0;    // column-pass workgroup: 0 default (64 columns), or 256 / 512 threads
};

hipError_t launch_ntt(const NttArgs& a, int ntransforms, bool inverse, hipStream_t s,
                      const Tuning& t = Tuning());
hipError_t launch_ntt_cols(const NttArgs& a, int ntransforms, bool inverse, hipStream_t s,
                           const Tuning& t = Tuning());
hipError_t launch_rows_fused(const RowsArgs& a, int mode, hipStream_t s, const Tuning& t = Tuning());
// log2 of the column pass's length for a transform of 2^logN points
int ntt_split_cols(int logN, const Tuning& t);
// Transposes rows of 2^S words into the register order of the fused relinearization pass.
hipError_t launch_row_transpose(const uint32_t* src, uint32_t* dst, long long total, int S, hipStream_t s);
// data[r][j] <- data[r][j] scale[r mod K] mod q_(r mod K) for `rows` rows of N words
// (canonical in, canonical out).
hipError_t launch_scale_rows(uint32_t* data, long long rows, int K, int N, const uint2* scale, const PrimeC* pc,
                             hipStream_t s);
hipError_t launch_lift(const LiftArgs& a, int npoly, hipStream_t s, const Tuning& t = Tuning());
hipError_t launch_crt(CrtArgs a, int npoly, hipStream_t s);
hipError_t launch_compose(const ComposeArgs& a, int cnum, hipStream_t s);
hipError_t launch_rescale(const RescaleArgs& a, int cnum, hipStream_t s);
hipError_t launch_compose_rescale(const ComposeArgs& a, int cnum, hipStream_t s);
hipError_t launch_small_to_limbs(const int8_t* v, uint32_t* out, int N, int L, uint32_t topmask, hipStream_t s);
hipError_t launch_mask_rows(const uint32_t* in, uint32_t* out, int N, int L, uint32_t topmask, hipStream_t s);
hipError_t launch_add_small(const uint32_t* x, const uint32_t* y, const int32_t* e, long long mult, uint32_t* out,
                            int N, int L, uint32_t topmask, hipStream_t s);
hipError_t launch_bgv_decode(const uint32_t* ph, uint32_t* m, int N, int L, int logq, uint32_t t, uint32_t qmodt,
                             uint32_t ginv, hipStream_t s);
hipError_t launch_bitrev(uint32_t* data, int logN, long long rows, hipStream_t s);
hipError_t launch_limb_sum(const LimbSumArgs& a, int cnum, hipStream_t s);
hipError_t launch_signed_perm(const PermArgs& a, int cnum, hipStream_t s);
hipError_t launch_const_mul(const ConstMulArgs& a, int cnum, hipStream_t s);

}  // namespace fhe
