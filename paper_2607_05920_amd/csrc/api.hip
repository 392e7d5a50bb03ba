// Host layer of the C ABI: contexts, precomputed tables (Section 5.2), keys,
// scratch memory and the launch sequences of the HE-mult pipeline.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <deque>
#include <thread>
#include <tuple>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <queue>
#include <vector>

#include "fhe_internal.h"
#include "fhe_mi355x.h"
#include "queue_layout.h"
#include "srv_core.h"

using namespace fhe;

// Device scratch of fhe_ring_mul_noalloc: the residues of both operands of every pair
// (2 cnum K N words).  Each device the library runs on holds its own copy until the
// process ends; host code uses only the address hipGetSymbolAddress gives per device.
constexpr size_t kNoAllocWords = (size_t)16 << 20;  // 64 MiB
__device__ __align__(256) uint32_t scratch[kNoAllocWords];

namespace {

// Text of the last failing HIP call on this host thread (see fhe_error_detail).
thread_local char g_detail[256] = "";

void note(const char* what, hipError_t e) {
  snprintf(g_detail, sizeof g_detail, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

// Device address of `scratch` per device, set by fhe_ctx_create with the device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t* g_scratch_dev[kMaxDevices] = {};

// ---------------------------------------------------------------- host number theory

uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((unsigned __int128)a * b % m); }

uint64_t powmod(uint64_t b, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  b %= m;
  while (e) {
    if (e & 1) r = mulmod64(r, b, m);
    b = mulmod64(b, b, m);
    e >>= 1;
  }
  return r;
}

// a^-1 mod m for gcd(a, m) = 1 (extended Euclid; m need not be prime).
uint64_t invmod(uint64_t a, uint64_t m) {
  long long r0 = (long long)m, r1 = (long long)(a % m), s0 = 0, s1 = 1;
  while (r1 != 0) {
    const long long qt = r0 / r1;
    long long t = r0 - qt * r1;
    r0 = r1;
    r1 = t;
    t = s0 - qt * s1;
    s0 = s1;
    s1 = t;
  }
  return (uint64_t)(s0 < 0 ? s0 + (long long)m : s0);
}

bool is_prime32(uint32_t n) {
  if (n < 2) return false;
  for (uint32_t p : {2u, 3u, 5u, 7u, 11u, 13u}) {
    if (n % p == 0) return n == p;
  }
  uint32_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) {
    d >>= 1;
    ++s;
  }
  for (uint32_t a : {2u, 3u, 5u, 7u}) {  // deterministic below 3.2e9
    uint64_t x = powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s; ++r) {
      x = mulmod64(x, x, n);
      if (x == n - 1) {
        comp = false;
        break;
      }
    }
    if (comp) return false;
  }
  return true;
}

uint32_t bitrev(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

uint2 shoup_pair(uint32_t w, uint32_t q) {
  return make_uint2(w, (uint32_t)(((uint64_t)w << 32) / q));
}

// Unsigned big integer as little-endian 32-bit words.
struct Big {
  std::vector<uint32_t> w{1};
  void mul_small(uint32_t m) {
    uint64_t c = 0;
    for (auto& x : w) {
      uint64_t t = (uint64_t)x * m + c;
      x = (uint32_t)t;
      c = t >> 32;
    }
    if (c) w.push_back((uint32_t)c);
  }
  int bitlen() const {
    int n = (int)w.size();
    while (n > 0 && w[n - 1] == 0) --n;
    if (n == 0) return 0;
    return 32 * (n - 1) + (32 - __builtin_clz(w[n - 1]));
  }
  uint32_t bits_at(int pos, int nb) const {  // nb <= 32
    uint64_t v = 0;
    int wi = pos >> 5, sh = pos & 31;
    if (wi < (int)w.size()) v = w[wi];
    if (wi + 1 < (int)w.size()) v |= (uint64_t)w[wi + 1] << 32;
    return (uint32_t)((v >> sh) & ((nb == 32) ? 0xFFFFFFFFull : ((1ull << nb) - 1)));
  }
};

template <typename T>
hipError_t upload(T** dptr, const std::vector<T>& h) {
  hipError_t e = hipMalloc((void**)dptr, h.size() * sizeof(T));
  if (e != hipSuccess) {
    note("hipMalloc of a constant table", e);
    return e;
  }
  e = hipMemcpy(*dptr, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) note("hipMemcpy of a constant table", e);
  return e;
}

int ceil_log2(int x) {
  int r = 0;
  while ((1 << r) < x) ++r;
  return r;
}

int status_of(hipError_t e) {
  if (e == hipSuccess) return FHE_OK;
  note("HIP call", e);
  if (e == hipErrorOutOfMemory) return FHE_E_NOMEM;
  return FHE_E_DEVICE;
}

}  // namespace

// ---------------------------------------------------------------- objects

struct Workspace {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// Per-kernel HIP-event timing (instrumentation; off unless enabled).
struct Recorder : EventRecorder {
  struct Pending {
    int kid;
    hipEvent_t a, b;
    double work;
  };
  std::vector<hipEvent_t> pool;
  std::vector<Pending> pending;
  std::vector<std::pair<int, hipEvent_t>> open;
  double ms[KID_COUNT] = {}, work[KID_COUNT] = {};
  long long launches[KID_COUNT] = {};
  hipEvent_t take() {
    if (pool.empty()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      return e;
    }
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  void begin(int kid, hipStream_t s) override {
    hipEvent_t e = take();
    if (e) hipEventRecord(e, s);
    open.emplace_back(kid, e);
  }
  void end(int kid, hipStream_t s, double w) override {
    hipEvent_t a = open.back().second;
    open.pop_back();
    hipEvent_t b = take();
    if (b) hipEventRecord(b, s);
    pending.push_back({kid, a, b, w});
  }
  void collect() {
    for (auto& p : pending) {
      if (p.a && p.b && hipEventSynchronize(p.b) == hipSuccess) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
          ms[p.kid] += t;
          work[p.kid] += p.work;
          launches[p.kid] += 1;
        }
      }
      if (p.a) pool.push_back(p.a);
      if (p.b) pool.push_back(p.b);
    }
    pending.clear();
  }
  void clear() {
    collect();
    for (int k = 0; k < KID_COUNT; ++k) ms[k] = work[k] = 0, launches[k] = 0;
  }
  ~Recorder() override {
    collect();
    for (auto e : pool) hipEventDestroy(e);
  }
};

// Constant tables of the matrix-core lift of L limbs onto K primes.
struct LiftTab {
  v4i_t* A = nullptr;      // A fragments [tile][k-block][lane]
  uint64_t* off = nullptr; // [p] = [C0 2^32]_(q_p) + 2^20 q_p
  int nkb = 0, ntiles = 0;
};

// Constant tables of one CRT reconstruction (prime count K, offset exponent e,
// output limbs Lout).
struct CrtTab {
  v4i_t* A = nullptr;        // MFMA A fragments [tile][k-block][lane]
  uint32_t* d = nullptr;     // [k] = [2^e c_k]_(q_k)
  uint32_t* mneg = nullptr;  // limbs of (-M) mod 2^(32 Lout), 8 ntiles words
  uint32_t* eneg = nullptr;  // limbs of (-2^e) mod 2^(32 Lout), 8 ntiles words
  int ntiles = 0;
};

struct fhe_ctx {
  int device = 0;
  int logQ_max = 0, logP_max = 0;
  int K = 0;     // primes in the table
  int Kpad = 0;  // K + padding read by blocked kernels
  int lds_max = 0, cus = 0;  // LDS bytes per workgroup and compute units of the device
  std::vector<uint32_t> q, psi;
  std::vector<int> mbits;  // mbits[k] = bit length of M_k = prod_(i<k) q_i, k <= K
  // device tables
  PrimeC* pc = nullptr;
  uint2* tw = nullptr;
  uint2* itw = nullptr;
  uint2* nscale[kLogNMax + 1] = {};  // N^-1 per prime
  uint32_t* liftT = nullptr;
  int TS = 0, Lmax = 0;
  uint32_t* rq = nullptr;  // [k] = floor(2^56 / q_k)
  std::map<int, std::vector<uint32_t>> crt_c;             // per K: c_k = [(M/q_k)^-1]_(q_k)
  std::map<std::tuple<int, int, int>, CrtTab> crt;        // per (K, e, Lout)
  std::map<std::pair<int, int>, uint2*> cscale;           // per (logN, K): [N^-1 2^32 c_k]_(q_k), Shoup
  std::map<std::pair<int, int>, LiftTab> lifts;           // per (L, K)
  std::map<uint32_t, uint32_t*> pw;  // per BGV t: 2^(32 l) mod t
  std::map<std::pair<void*, int>, Workspace> ws;  // (stream, slot)
  std::recursive_mutex mu;
  int sticky = FHE_OK;
  Recorder* rec = nullptr;  // non-null while profiling is on
  uint32_t* noalloc = nullptr;  // this device's address of `scratch`
  std::map<std::vector<int>, Tuning> tuned;  // autotuner results by (logN, logq, logP, K_t, K_r)
};

// One cell of a batch plan: jobs sharing (key, logq, bits), run as a CipherTensor.
struct PlanCell {
  fhe_evk* evk = nullptr;
  int logN = 0, logq = 0, bits = 0, cnum = 0;
  uint32_t** ptrs = nullptr;  // device: x0s, x1s, y0s, y1s, out0s, out1s (cnum each)
  Tuning tune;
};

// Graph branches of a captured plan: cells run on up to kPlanBranches concurrent
// branches of the graph, each with its own scratch, so that small cells (which do not
// fill the device) overlap.
constexpr int kPlanBranches = 4;

// One launch of a stage-batched plan: a kernel variant's stage-batched entry point over
// the cells whose pipeline step uses that variant at this stage.
struct QueueLaunch {
  const void* multi = nullptr;
  unsigned blocks = 0;  // workgroups: the cells' grids, each rounded up to 8
  dim3 block;
  size_t lds = 0;       // dynamic LDS: the largest of the cells'
  void* args = nullptr;      // device: the cells' argument structs
  CellSeg* seg = nullptr;    // device: their segments
  int ncells = 0;
  int branch = 0;            // graph branch of its cells
};

struct fhe_plan {
  fhe_ctx* ctx = nullptr;
  std::vector<PlanCell> cells;
  // stage-batched (FHE_PLAN_QUEUE): the launches in order, each cell's own scratch, and
  // the one device buffer holding every launch's argument structs and segments
  std::vector<QueueLaunch> queue;
  std::vector<uint32_t*> cws;
  void* qmem = nullptr;
  std::vector<int> branch;         // per cell: its graph branch
  uint32_t* ws = nullptr;          // scratch of eager runs and of branch 0
  uint32_t* bws[kPlanBranches] = {nullptr, nullptr, nullptr, nullptr};  // scratch of branches 1..
  hipStream_t cap = nullptr;
  hipStream_t bst[kPlanBranches] = {nullptr, nullptr, nullptr, nullptr};  // capture streams 1..
  hipEvent_t fork = nullptr, join[kPlanBranches] = {nullptr, nullptr, nullptr, nullptr};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int kernels = 0;
};

struct fhe_evk {
  fhe_ctx* ctx = nullptr;
  int scheme = 0;
  uint32_t t = 0;
  uint32_t g = 0;  // 0: relinearization key (of s^2); odd g: switching key of kappa_g(s)
  int logN = 0, logQ = 0, logP = 0;
  std::vector<uint32_t> hb, ha;  // host limbs [L_PQ][N]
  // per logq: [2][K_r][N] in NTT form, each row of the fused pass transposed into its
  // register order (launch_row_transpose) for rows of 2^(logN/2) points; for odd logN,
  // ntt_alt holds the same for rows of 2^(logN - logN/2) points
  std::map<int, uint32_t*> ntt, ntt_alt;
};

namespace {

// Installs the context's recorder (if profiling) for the duration of one call.
struct RecGuard {
  explicit RecGuard(fhe_ctx* c) { set_recorder(c->rec); }
  ~RecGuard() { set_recorder(nullptr); }
};

int set_sticky(fhe_ctx* c, hipError_t e) {
  int st = status_of(e);
  if (st != FHE_OK && c->sticky == FHE_OK) c->sticky = st;
  return st;
}

// Smallest K with M_K >= 2^(e + 1 + margin), i.e. bitlen(M_K) >= e + 2 + margin:
// |X| < 2^e is recovered from its residues, and Y = X + 2^e satisfies Y / M_K <
// 2^-margin, which keeps the CRT quotient alpha exact in double precision.
int primes_for_e(const fhe_ctx* c, int e) {
  for (int k = 0; k <= c->K; ++k)
    if (c->mbits[k] >= e + 2 + kCrtMarginBits) return k;
  return -1;
}

// c_k = [(M/q_k)^-1]_(q_k) for the first K primes.
const std::vector<uint32_t>& crt_c(fhe_ctx* c, int K) {
  auto it = c->crt_c.find(K);
  if (it != c->crt_c.end()) return it->second;
  std::vector<uint32_t> v(K);
  for (int k = 0; k < K; ++k) {
    uint64_t m = 1;
    for (int j = 0; j < K; ++j)
      if (j != k) m = mulmod64(m, c->q[j], c->q[k]);
    v[k] = (uint32_t)invmod(m, c->q[k]);
  }
  return c->crt_c[K] = std::move(v);
}

// The inverse transform's last-stage twiddle of prime k (inverse table entry 1):
// psi_k^-bitrev(1) over the table's 16 bits, i.e. psi_k^-(2^15).
uint64_t last_inv_twiddle(const fhe_ctx* c, int k) {
  return powmod(invmod(c->psi[k], c->q[k]), 1ull << (kLogNMax - 1), c->q[k]);
}

// Final inverse-NTT factors [N^-1 2^32 c_k]_(q_k) (Shoup pairs) for transforms whose
// output goes to a K-prime CRT reconstruction: 2^32 undoes the 2^-32 of the
// Montgomery pointwise products, c_k is the CRT factor.  Entries Kpad + k hold the
// factor times the last stage's twiddle (NttArgs::scale_w).
const uint2* crt_scale(fhe_ctx* c, int logN, int K, hipError_t* err) {
  auto it = c->cscale.find(std::make_pair(logN, K));
  if (it != c->cscale.end()) return it->second;
  const std::vector<uint32_t>& ck = crt_c(c, K);
  std::vector<uint2> h(2 * (size_t)c->Kpad, make_uint2(0, 0));
  for (int k = 0; k < K; ++k) {
    const uint32_t q = c->q[k];
    const uint64_t f = mulmod64(mulmod64(invmod(1ull << logN, q), (1ull << 32) % q, q), ck[k], q);
    h[k] = shoup_pair((uint32_t)f, q);
    h[c->Kpad + k] = shoup_pair((uint32_t)mulmod64(f, last_inv_twiddle(c, k), q), q);
  }
  uint2* d = nullptr;
  *err = upload(&d, h);
  if (*err != hipSuccess) return nullptr;
  c->cscale[std::make_pair(logN, K)] = d;
  return d;
}

// x mod 2^(32 n) as n limbs, for x given by its limbs (truncating or zero-padding).
std::vector<uint32_t> limbs_mod(const std::vector<uint32_t>& x, int n) {
  std::vector<uint32_t> r(n, 0);
  for (int i = 0; i < n && i < (int)x.size(); ++i) r[i] = x[i];
  return r;
}

// r = r * m mod 2^(32 n) in place.
void mul_small_trunc(std::vector<uint32_t>& r, uint32_t m) {
  uint64_t carry = 0;
  for (auto& w : r) {
    const uint64_t t = (uint64_t)w * m + carry;
    w = (uint32_t)t;
    carry = t >> 32;
  }
}

// -x mod 2^(32 n) in place.
void negate_trunc(std::vector<uint32_t>& r) {
  uint64_t carry = 1;
  for (auto& w : r) {
    const uint64_t t = (uint64_t)(uint32_t)~w + carry;
    w = (uint32_t)t;
    carry = t >> 32;
  }
}

// r += x mod 2^(32 n) in place (equal lengths).
void add_trunc(std::vector<uint32_t>& r, const std::vector<uint32_t>& x) {
  uint64_t carry = 0;
  for (size_t i = 0; i < r.size(); ++i) {
    const uint64_t t = (uint64_t)r[i] + x[i] + carry;
    r[i] = (uint32_t)t;
    carry = t >> 32;
  }
}

// Tables of the K-prime CRT reconstruction with offset 2^e into Lout output limbs.
const CrtTab* crt_table(fhe_ctx* c, int K, int e, int Lout, hipError_t* err) {
  const auto key = std::make_tuple(K, e, Lout);
  auto it = c->crt.find(key);
  if (it != c->crt.end()) return &it->second;
  if (8 * ((Lout + 7) / 8) > kCrtMaxLimbs || K > kCrtMaxPrimes) {
    *err = hipErrorInvalidValue;
    return nullptr;
  }
  const std::vector<uint32_t>& ck = crt_c(c, K);
  const int nkb = (K + 31) / 32, ntiles = (Lout + 7) / 8, Lp = 8 * ntiles;
  CrtTab t;
  t.ntiles = ntiles;
  std::vector<uint32_t> d(c->Kpad, 0);
  for (int k = 0; k < K; ++k) d[k] = (uint32_t)mulmod64(powmod(2, e, c->q[k]), ck[k], c->q[k]);
  // V_k = (M / q_k) mod 2^(32 Lout) in balanced limbs D_kl in [-0x80808080, 0x7F7F7F7F];
  // vsum = sum_k V_k mod 2^(32 Lout)
  std::vector<int64_t> D((size_t)K * Lp, 0);
  std::vector<uint32_t> vsum(Lout, 0);
  for (int k = 0; k < K; ++k) {
    std::vector<uint32_t> v(Lout, 0);
    v[0] = 1;
    for (int j = 0; j < K; ++j)
      if (j != k) mul_small_trunc(v, c->q[j]);
    add_trunc(vsum, v);
    int64_t carry = 0;
    for (int l = 0; l < Lout; ++l) {
      const int64_t u = (int64_t)v[l] + carry;
      carry = u > 0x7F7F7F7FLL ? 1 : 0;
      D[(size_t)k * Lp + l] = u - (carry << 32);
    }
  }
  // A fragments: lane (r, h) of tile t, k-block kb holds bytes i < 16 of row r
  // (digit plane b = r / 8 of limb 8 t + r % 8) at k = 32 kb + 16 h + i
  std::vector<v4i_t> A((size_t)ntiles * nkb * 64);
  for (int tt = 0; tt < ntiles; ++tt)
    for (int kb = 0; kb < nkb; ++kb)
      for (int lane = 0; lane < 64; ++lane) {
        const int r = lane & 31, hh = lane >> 5, b = r >> 3, limb = 8 * tt + (r & 7);
        uint32_t w[4] = {0, 0, 0, 0};
        for (int i = 0; i < 16; ++i) {
          const int k = 32 * kb + 16 * hh + i;
          if (k >= K || limb >= Lout) continue;
          const uint32_t digits = ((uint32_t)(D[(size_t)k * Lp + limb] + 0x80808080LL)) ^ 0x80808080u;
          w[i >> 2] |= ((digits >> (8 * b)) & 0xFFu) << (8 * (i & 3));
        }
        v4i_t f;
        f[0] = (int)w[0];
        f[1] = (int)w[1];
        f[2] = (int)w[2];
        f[3] = (int)w[3];
        A[((size_t)tt * nkb + kb) * 64 + lane] = f;
      }
  std::vector<uint32_t> mneg(Lout, 0);
  mneg[0] = 1;
  for (int j = 0; j < K; ++j) mul_small_trunc(mneg, c->q[j]);
  negate_trunc(mneg);
  // [0x80808080 sum_k V_k - 2^e]: the digits of y_k ^ 0x80808080 stand for y_k - 0x80808080
  std::vector<uint32_t> eneg(Lout, 0);
  if (e < 32 * Lout) {
    eneg[e >> 5] = 1u << (e & 31);
    negate_trunc(eneg);
  }
  mul_small_trunc(vsum, 0x80808080u);
  add_trunc(eneg, vsum);
  mneg.resize(Lp, 0);
  eneg.resize(Lp, 0);
  *err = upload(&t.A, A);
  if (*err == hipSuccess) *err = upload(&t.d, d);
  if (*err == hipSuccess) *err = upload(&t.mneg, mneg);
  if (*err == hipSuccess) *err = upload(&t.eneg, eneg);
  if (*err != hipSuccess) {
    for (void* p : {(void*)t.A, (void*)t.d, (void*)t.mneg, (void*)t.eneg})
      if (p) hipFree(p);
    return nullptr;
  }
  return &(c->crt[key] = t);
}

uint32_t* pow_table(fhe_ctx* c, uint32_t t, hipError_t* err) {
  auto it = c->pw.find(t);
  if (it != c->pw.end()) return it->second;
  std::vector<uint32_t> h(512);
  uint64_t x = 1 % t;
  const uint64_t w32 = ((uint64_t)1 << 32) % t;
  for (auto& v : h) {
    v = (uint32_t)x;
    x = x * w32 % t;
  }
  uint32_t* d = nullptr;
  *err = upload(&d, h);
  if (*err != hipSuccess) return nullptr;
  c->pw[t] = d;
  return d;
}

// Scratch memory of a (context, stream, slot), grown on demand.
void* stream_scratch(fhe_ctx* c, void* stream, int slot, size_t bytes, hipError_t* err) {
  Workspace& w = c->ws[std::make_pair(stream, slot)];
  if (w.bytes < bytes) {
    if (w.ptr) {
      hipStreamSynchronize((hipStream_t)stream);
      hipFree(w.ptr);
      w.ptr = nullptr;
      w.bytes = 0;
    }
    *err = hipMalloc(&w.ptr, bytes);
    if (*err != hipSuccess) return nullptr;
    w.bytes = bytes;
  }
  *err = hipSuccess;
  return w.ptr;
}

int check_logN(int logN) { return (logN >= FHE_LOGN_MIN && logN <= FHE_LOGN_MAX) ? FHE_OK : FHE_E_RANGE; }

NttArgs ntt_args(fhe_ctx* c, uint32_t* data, int logN, int K, int per_group, long long gstride,
                 bool inverse, const uint2* scale) {
  NttArgs a{};
  a.data = data;
  a.logN = logN;
  a.K = K;
  a.per_group = per_group;
  a.group_stride = gstride;
  a.tw = inverse ? c->itw : c->tw;
  a.pc = c->pc;
  a.scale = scale;
  a.scale_w = scale ? scale + c->Kpad : nullptr;  // the tables hold both halves
  return a;
}

// Tables of the matrix-core lift of L limbs onto K primes (built on first use).
const LiftTab* lift_table(fhe_ctx* c, int L, int K, hipError_t* err) {
  const auto key = std::make_pair(L, K);
  auto it = c->lifts.find(key);
  if (it != c->lifts.end()) return &it->second;
  LiftTab t;
  t.nkb = (L + 7) / 8;
  if (t.nkb > 16) t.nkb = 32;  // the kernel is instantiated for 1..16 and 32 k-blocks (zero-padded)
  if (L > 256) {
    *err = hipErrorInvalidValue;
    return nullptr;
  }
  t.ntiles = (K + 7) / 8;
  // T_(i,a),p = [2^(32 i + 8 a + 32)]_(q_p), i < 8 nkb, a < 4
  std::vector<uint32_t> T((size_t)K * 32 * t.nkb, 0);
  std::vector<uint64_t> off(c->Kpad, 0);
  for (int p = 0; p < K; ++p) {
    const uint32_t q = c->q[p];
    const uint64_t r32 = (1ull << 32) % q;
    uint64_t v = r32;
    for (int i = 0; i < 32 * t.nkb; ++i) {
      T[(size_t)p * 32 * t.nkb + i] = (uint32_t)v;
      v = mulmod64(v, 256, q);
    }
    // C0 = 0x80808080 sum_(i<L) 2^(32 i), in Montgomery form, plus 2^20 q
    uint64_t sum = 0, pw = 1;
    for (int i = 0; i < L; ++i) {
      sum = (sum + pw) % q;
      pw = mulmod64(pw, r32, q);
    }
    const uint64_t c0 = mulmod64(mulmod64(0x80808080ull % q, sum, q), r32, q);
    off[p] = c0 + ((uint64_t)q << 20);
  }
  std::vector<v4i_t> A((size_t)t.ntiles * t.nkb * 64);
  for (int tt = 0; tt < t.ntiles; ++tt)
    for (int kb = 0; kb < t.nkb; ++kb)
      for (int lane = 0; lane < 64; ++lane) {
        const int r = lane & 31, hh = lane >> 5, b = r >> 3, p = 8 * tt + (r & 7);
        uint32_t w[4] = {0, 0, 0, 0};
        for (int i = 0; i < 16; ++i) {
          const int li = 8 * kb + 4 * hh + (i >> 2), dg = i & 3;
          if (li >= L || p >= K) continue;
          const uint32_t tv = T[(size_t)p * 32 * t.nkb + 4 * li + dg];
          const uint32_t digits = (tv + 0x80808080u) ^ 0x80808080u;
          w[i >> 2] |= ((digits >> (8 * b)) & 0xFFu) << (8 * (i & 3));
        }
        v4i_t f;
        f[0] = (int)w[0];
        f[1] = (int)w[1];
        f[2] = (int)w[2];
        f[3] = (int)w[3];
        A[((size_t)tt * t.nkb + kb) * 64 + lane] = f;
      }
  *err = upload(&t.A, A);
  if (*err == hipSuccess) *err = upload(&t.off, off);
  if (*err != hipSuccess) {
    if (t.A) hipFree(t.A);
    if (t.off) hipFree(t.off);
    return nullptr;
  }
  return &(c->lifts[key] = t);
}

RowsArgs rows_args(fhe_ctx* c, int logN, int K, int cnum) {
  RowsArgs a{};
  a.logN = logN;
  a.K = K;
  a.cnum = cnum;
  a.tw = c->tw;
  a.itw = c->itw;
  a.pc = c->pc;
  return a;
}

LiftArgs lift_args(fhe_ctx* c, const uint32_t* limbs, uint32_t* res, long long in_stride,
                   long long out_stride, int N, int L, int K) {
  LiftArgs a{};
  hipError_t err = hipSuccess;
  if (const LiftTab* t = lift_table(c, L, K, &err)) {  // else only the VALU lift is available
    a.A = t->A;
    a.off = t->off;
    a.nkb = t->nkb;
    a.ntiles = t->ntiles;
  }
  a.lds_max = c->lds_max;
  a.cus = c->cus;
  a.limbs = limbs;
  a.res = res;
  a.in_stride = in_stride;
  a.out_stride = out_stride;
  a.N = N;
  a.L = L;
  a.K = K;
  a.T = c->liftT;
  a.TS = c->TS;
  a.pc = c->pc;
  return a;
}

// CRT reconstruction of npoly polynomials: residues of X (with |X| < 2^e) on K
// primes -> X mod 2^outbits.  Poly z reads res + (z / per_group) gstride +
// (z % per_group) pstride and writes out + z ostride.
hipError_t run_crt(fhe_ctx* c, const uint32_t* res, int per_group, long long gstride, long long pstride,
                   uint32_t* out, long long ostride, int N, int K, int e, int outbits, int npoly, hipStream_t st) {
  hipError_t err = hipSuccess;
  const int Lout = (outbits + 31) / 32;
  const CrtTab* t = crt_table(c, K, e, Lout, &err);
  if (!t) return err;
  CrtArgs a{};
  a.res = res;
  a.per_group = per_group;
  a.gstride = gstride;
  a.pstride = pstride;
  a.out = out;
  a.ostride = ostride;
  a.N = N;
  a.K = K;
  a.outbits = outbits;
  a.Lout = Lout;
  a.ntiles = t->ntiles;
  a.A = t->A;
  a.pc = c->pc;
  a.d = t->d;
  a.rq = c->rq;
  a.mneg = t->mneg;
  a.eneg = t->eneg;
  a.lds_max = c->lds_max;
  a.cus = c->cus;
  return launch_crt(a, npoly, st);
}

// Creates the lift and CRT tables one pipeline run at (key, logN, logq) uses, so that a run
// under stream capture allocates and uploads nothing.
bool tables_prewarm(fhe_ctx* c, const fhe_evk* k, int logN, int logq, hipError_t* err) {
  const int Kt = primes_for_e(c, 2 * logq + logN + 1), Kr = primes_for_e(c, logN + 2 * logq + k->logP);
  if (Kt < 0 || Kr < 0) {
    *err = hipErrorInvalidValue;
    return false;
  }
  const int L = (logq + 31) / 32;
  return lift_table(c, L, Kt, err) && lift_table(c, L, Kr, err) && crt_scale(c, logN, Kt, err) &&
         crt_scale(c, logN, Kr, err) &&
         crt_table(c, Kt, 2 * logq + logN + 1, (logq + 31) / 32, err) &&
         crt_table(c, Kr, logN + 2 * logq + k->logP, (k->logP + logq + 31) / 32, err);
}

// Build the relinearization key's NTT form for level logq.
int evk_prepare_locked(fhe_evk* k, int logq, hipStream_t stream) {
  fhe_ctx* c = k->ctx;
  if (k->ntt.count(logq)) return FHE_OK;
  if (logq < 1 || logq > k->logQ) return FHE_E_RANGE;
  const int N = 1 << k->logN;
  const int bits = k->logP + logq;
  const int Lk = (bits + 31) / 32;
  const int Lfull = (k->logP + k->logQ + 31) / 32;
  const int Kr = primes_for_e(c, k->logN + 2 * logq + k->logP);
  if (Kr < 0) return FHE_E_RANGE;
  // key limbs reduced mod P 2^logq
  std::vector<uint32_t> h((size_t)2 * Lk * N);
  for (int part = 0; part < 2; ++part) {
    const std::vector<uint32_t>& src = part ? k->ha : k->hb;
    for (int l = 0; l < Lk; ++l) {
      uint32_t mask = 0xFFFFFFFFu;
      if (l == Lk - 1 && (bits & 31)) mask = (1u << (bits & 31)) - 1u;
      for (int j = 0; j < N; ++j)
        h[((size_t)part * Lk + l) * N + j] = (l < Lfull ? src[(size_t)l * N + j] : 0u) & mask;
    }
  }
  uint32_t* limbs = nullptr;
  uint32_t* out = nullptr;
  hipError_t e = hipMalloc(&limbs, h.size() * 4);
  if (e != hipSuccess) return set_sticky(c, e);
  e = hipMalloc(&out, (size_t)2 * Kr * N * 4);
  if (e != hipSuccess) {
    hipFree(limbs);
    return set_sticky(c, e);
  }
  e = hipMemcpyAsync(limbs, h.data(), h.size() * 4, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = launch_lift(lift_args(c, limbs, out, (long long)Lk * N, (long long)Kr * N, N, Lk, Kr), 2, stream);
  if (e == hipSuccess)
    e = launch_ntt(ntt_args(c, out, k->logN, Kr, 2 * Kr, 0, false, nullptr), 2 * Kr, false, stream);
  // the relinearization's inverse transforms take their final factor (N^-1 2^32 c_k,
  // see crt_scale) from the key: multiplied in here once
  const uint2* scr = e == hipSuccess ? crt_scale(c, k->logN, Kr, &e) : nullptr;
  if (e == hipSuccess) e = launch_scale_rows(out, 2LL * Kr, Kr, N, scr, c->pc, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  hipFree(limbs);
  if (e != hipSuccess) {
    hipFree(out);
    return set_sticky(c, e);
  }
  // the fused relinearization pass reads each row in its transposed register order; the
  // row length depends on the column/row split, which differs by tuning for odd logN
  const long long words = 2LL * Kr * N;
  const int Sa = k->logN / 2, Sb = k->logN - k->logN / 2;
  uint32_t* perm[2] = {nullptr, nullptr};
  for (int v = 0; v < (Sa == Sb ? 1 : 2) && e == hipSuccess; ++v) {
    e = hipMalloc(&perm[v], (size_t)words * 4);
    if (e == hipSuccess) e = launch_row_transpose(out, perm[v], words, v ? Sb : Sa, stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  hipFree(out);
  if (e != hipSuccess) {
    for (uint32_t* q : perm)
      if (q) hipFree(q);
    return set_sticky(c, e);
  }
  k->ntt[logq] = perm[0];
  if (perm[1]) k->ntt_alt[logq] = perm[1];
  return FHE_OK;
}

// Inputs and outputs of one HE-mult pipeline run over cnum ciphertext pairs: either
// CipherTensor base pointers ([cnum][L][N], outputs [cnum][L'][N]) or device arrays of
// per-ciphertext pointers (x0s[c] ...), as used by batch plans.
struct PipeIO {
  const uint32_t *x0 = nullptr, *x1 = nullptr, *y0 = nullptr, *y1 = nullptr;
  uint32_t *out0 = nullptr, *out1 = nullptr;
  const uint32_t* const* ins = nullptr;  // device: x0s, x1s, y0s, y1s (4 cnum pointers)
  uint32_t* const* outs = nullptr;       // device: out0s, out1s (2 cnum pointers)
};

// Scratch words of one pipeline run.
struct PipeSize {
  int Kt = 0, Kr = 0, L = 0, LK = 0;
  long long main_words = 0;
};

PipeSize pipe_size(const fhe_ctx* c, const fhe_evk* k, int logN, int logq, int cnum) {
  PipeSize z;
  const long long NN = 1LL << logN;
  z.L = (logq + 31) / 32;
  z.LK = (k->logP + logq + 31) / 32;
  z.Kt = primes_for_e(c, 2 * logq + logN + 1);
  z.Kr = primes_for_e(c, logN + 2 * logq + k->logP);
  if (z.Kt < 0 || z.Kr < 0) return z;
  z.main_words = (long long)cnum * NN * (4LL * z.Kt + 3LL * z.L + z.Kr + 2LL * z.Kr + 2LL * z.LK);
  return z;
}

// The relinearization half of the HE-mult, shared with the Galois key switch: per
// ciphertext c, Dl + 3 c L N holds d0, d1, d2 (uint32[3][L][N]).  Lift d2 onto Kr
// primes, NTT, products with the resident key, iNTT, CRT (k0, k1 mod 2^(logP+logq));
// c_i = [d_i + R(k_i)]_(2^logq), rescaled in the same pass if bits > 0.  With d1_zero
// slot 1 is not read and d1 is taken as zero (the key switch).
int relin_part(fhe_ctx* c, fhe_evk* k, int logN, int logq, int bits, const PipeIO& io, int cnum, hipStream_t st,
               uint32_t* Dl, uint32_t* Rr, uint32_t* Rk, uint32_t* Kl, const Tuning& tu, bool d1_zero) {
  const int N = 1 << logN;
  const PipeSize z = pipe_size(c, k, logN, logq, cnum);
  if (z.Kt < 0 || z.Kr < 0) return FHE_E_RANGE;
  const int Kr = z.Kr, L = z.L, LK = z.LK;
  const int logP = k->logP;
  const int rows_log = logN - ntt_split_cols(logN, tu);  // the fused pass's row length
  const uint32_t* evk_ntt = rows_log == logN / 2 ? k->ntt.at(logq) : k->ntt_alt.at(logq);
  hipError_t e = hipSuccess;
  const int er = logN + 2 * logq + logP;  // |k_i| < 2^er
  const long long NN = N;
  const long long polyw = (long long)L * NN;
  // 6. lift d2 onto Kr primes; 7. forward NTT
  e = launch_lift(lift_args(c, Dl + 2 * polyw, Rr, 3 * polyw, (long long)Kr * NN, N, L, Kr), cnum, st, tu);
  if (e == hipSuccess)
    e = launch_ntt_cols(ntt_args(c, Rr, logN, Kr, Kr, (long long)Kr * NN, false, nullptr), cnum * Kr, false, st,
                        tu);
  // 8. forward row pass, products with the resident key into Rk[c][0..1][Kr][N],
  // first inverse row pass
  if (e == hipSuccess) {
    RowsArgs ra = rows_args(c, logN, Kr, cnum);
    ra.data = Rr;
    ra.group_stride = (long long)Kr * NN;
    ra.key = evk_ntt;
    ra.out = Rk;
    ra.out_stride = 2LL * Kr * NN;
    e = launch_rows_fused(ra, ROWS_RELIN, st, tu);
  }
  // 9. inverse NTT column pass; 10. CRT -> k0, k1 mod 2^(logP + logq)
  if (e == hipSuccess)
    e = launch_ntt_cols(ntt_args(c, Rk, logN, Kr, 2 * Kr, 2LL * Kr * NN, true, nullptr), cnum * 2 * Kr, true, st,
                        tu);  // the factor is in the prepared key
  if (e == hipSuccess)
    e = run_crt(c, Rk, 2, 2LL * Kr * NN, (long long)Kr * NN, Kl, (long long)LK * NN, N, Kr, er, logP + logq,
                cnum * 2, st);
  // 11. c_i = [d_i + R(k_i)]_(2^logq), to the outputs or (rescale follows) the staging area
  const uint32_t* pwt = nullptr;
  if (e == hipSuccess && k->scheme == FHE_BGV) pwt = pow_table(c, k->t, &e);
  if (e == hipSuccess) {
    ComposeArgs ca{};
    ca.k = Kl;
    ca.kstride = (long long)LK * NN;
    ca.d = Dl;
    ca.dstride = polyw;
    ca.d1_zero = d1_zero ? 1 : 0;
    if (io.outs) {
      ca.out0s = io.outs;
      ca.out1s = io.outs + cnum;
    } else {
      ca.out0 = io.out0;
      ca.out1 = io.out1;
      ca.ostride = (long long)((logq - bits + 31) / 32) * NN;  // polyw when there is no rescale
    }
    ca.N = N;
    ca.L = L;
    ca.LK = LK;
    ca.logq = logq;
    ca.logP = logP;
    ca.scheme = k->scheme;
    if (k->scheme == FHE_BGV) {
      ca.t = k->t;
      ca.invP = (uint32_t)invmod(powmod(2, logP, k->t), k->t);
      ca.pw = pwt;
    }
    // 12. with a rescale, both in one pass: the relinearized c_i is never stored
    ca.bits = bits;
    if (bits > 0 && k->scheme == FHE_BGV) ca.invB = (uint32_t)invmod(powmod(2, bits, k->t), k->t);
    e = bits > 0 ? launch_compose_rescale(ca, cnum, st) : launch_compose(ca, cnum, st);
  }
  return set_sticky(c, e);
}

// The HE-mult pipeline: lift, NTT, tensor products, iNTT, CRT (d0, d1, d2 mod
// 2^logq); then the relinearization half (relin_part).
int pipeline(fhe_ctx* c, fhe_evk* k, int logN, int logq, int bits, const PipeIO& io, int cnum, hipStream_t st,
             uint32_t* ws, const Tuning& tu) {
  const int N = 1 << logN;
  const PipeSize z = pipe_size(c, k, logN, logq, cnum);
  if (z.Kt < 0 || z.Kr < 0) return FHE_E_RANGE;
  const int Kt = z.Kt, Kr = z.Kr, L = z.L;
  hipError_t e = hipSuccess;
  const int et = 2 * logq + logN + 1;  // |d_i| < 2^et
  const uint2* sct = crt_scale(c, logN, Kt, &e);
  if (!sct) return set_sticky(c, e);
  const long long NN = N;
  uint32_t* Rt = ws;                                    // [cnum][4][Kt][N]
  uint32_t* Dl = Rt + (long long)cnum * 4 * Kt * NN;    // [cnum][3][L][N]
  uint32_t* Rr = Dl + (long long)cnum * 3 * L * NN;     // [cnum][Kr][N]
  uint32_t* Rk = Rr + (long long)cnum * Kr * NN;        // [cnum][2][Kr][N]
  uint32_t* Kl = Rk + (long long)cnum * 2 * Kr * NN;    // [cnum][2][LK][N]
  const long long polyw = (long long)L * NN;
  // 1. lift the four inputs in one launch: Rt[c][i][Kt][N], i = x0, x1, y0, y1
  {
    LiftArgs la = lift_args(c, io.x0, Rt, polyw, (long long)Kt * NN, N, L, Kt);
    la.interleave4 = true;
    la.in4[0] = io.x0;
    la.in4[1] = io.x1;
    la.in4[2] = io.y0;
    la.in4[3] = io.y1;
    la.in_ptrs = io.ins;
    e = launch_lift(la, 4 * cnum, st, tu);
  }
  // 2. forward NTT column pass of all 4 cnum Kt transforms
  if (e == hipSuccess)
    e = launch_ntt_cols(ntt_args(c, Rt, logN, Kt, 4 * Kt, 4LL * Kt * NN, false, nullptr), cnum * 4 * Kt, false, st,
                        tu);
  // 3. forward row pass, tensor products into slots 0..2, first inverse row pass
  if (e == hipSuccess) {
    RowsArgs ra = rows_args(c, logN, Kt, cnum);
    ra.data = Rt;
    ra.group_stride = 4LL * Kt * NN;
    e = launch_rows_fused(ra, ROWS_TENSOR, st, tu);
  }
  // 4. inverse NTT column pass of slots 0..2 (final factor N^-1 2^32 c_k)
  if (e == hipSuccess)
    e = launch_ntt_cols(ntt_args(c, Rt, logN, Kt, 3 * Kt, 4LL * Kt * NN, true, sct), cnum * 3 * Kt, true, st, tu);
  // 5. CRT -> d0, d1, d2 mod 2^logq: Dl[c][i][L][N]
  if (e == hipSuccess)
    e = run_crt(c, Rt, 3, 4LL * Kt * NN, (long long)Kt * NN, Dl, polyw, N, Kt, et, logq, cnum * 3, st);
  if (e != hipSuccess) return set_sticky(c, e);
  return relin_part(c, k, logN, logq, bits, io, cnum, st, Dl, Rr, Rk, Kl, tu, false);
}

// Per-op entry: scratch from the stream's slots, key prepared for the level.
int mul_relin_locked(fhe_ctx* c, fhe_evk* k, int logN, int logq, int bits, const PipeIO& io, int cnum,
                     hipStream_t st) {
  int rc = evk_prepare_locked(k, logq, st);
  if (rc != FHE_OK) return rc;
  const PipeSize z = pipe_size(c, k, logN, logq, cnum);
  if (z.Kt < 0 || z.Kr < 0) return FHE_E_RANGE;
  hipError_t e = hipSuccess;
  uint32_t* ws = (uint32_t*)stream_scratch(c, st, 0, (size_t)z.main_words * 4, &e);
  if (!ws) return set_sticky(c, e);
  return pipeline(c, k, logN, logq, bits, io, cnum, st, ws, Tuning());
}

int rescale_locked(fhe_ctx* c, int scheme, uint32_t t, int logN, int logq, int bits,
                   const uint32_t* in0, const uint32_t* in1, long long istride, uint32_t* out0,
                   uint32_t* out1, long long ostride, int cnum, hipStream_t st) {
  RescaleArgs ra{};
  ra.in0 = in0;
  ra.in1 = in1;
  ra.out0 = out0;
  ra.out1 = out1;
  ra.istride = istride;
  ra.ostride = ostride;
  ra.N = 1 << logN;
  ra.logq = logq;
  ra.bits = bits;
  ra.scheme = scheme;
  hipError_t e = hipSuccess;
  if (scheme == FHE_BGV) {
    ra.t = t;
    ra.invB = (uint32_t)invmod(powmod(2, bits, t), t);
    ra.pw = pow_table(c, t, &e);
    if (!ra.pw) return set_sticky(c, e);
  }
  e = launch_rescale(ra, cnum, st);
  return set_sticky(c, e);
}

// Runs every cell of a plan on `st` (no graph).
int plan_run_cells(fhe_plan* pl, hipStream_t st) {
  for (PlanCell& cell : pl->cells) {
    PipeIO io;
    io.ins = cell.ptrs;
    io.outs = cell.ptrs + 4LL * cell.cnum;
    const int rc =
        pipeline(pl->ctx, cell.evk, cell.logN, cell.logq, cell.bits, io, cell.cnum, st, pl->ws, cell.tune);
    if (rc != FHE_OK) return rc;
  }
  return FHE_OK;
}

// Autotuner: times each candidate launch configuration of one cell (one warm-up, then
// the median of three runs) and keeps the fastest.
// Stage-batched plan: each cell's pipeline is recorded (a LaunchSink: nothing runs),
// every cell with scratch of its own; then step s of every cell's pipeline, which is
// the same stage of the same pipeline for all cells, becomes one launch per graph
// branch and kernel variant (template instance and workgroup) over the cells that use
// it (queue_layout.h: the grouping, the cells' order, and the segments, each cell's
// grid rounded up to a multiple of 8 workgroups so that every workgroup keeps the XCD
// its own launch would give it, the kernels' prime-to-XCD assignment).
int plan_build_queue(fhe_plan* pl, hipStream_t st) {
  fhe_ctx* c = pl->ctx;
  const size_t nc = pl->cells.size();
  pl->cws.assign(nc, nullptr);
  std::vector<std::vector<LaunchRec>> recs(nc);
  for (size_t ci = 0; ci < nc; ++ci) {
    PlanCell& cell = pl->cells[ci];
    const PipeSize z = pipe_size(c, cell.evk, cell.logN, cell.logq, cell.cnum);
    hipError_t e = hipMalloc((void**)&pl->cws[ci], (size_t)std::max(z.main_words, 1LL) * 4);
    if (e != hipSuccess) return set_sticky(c, e);
    PipeIO io;
    io.ins = cell.ptrs;
    io.outs = cell.ptrs + 4LL * cell.cnum;
    LaunchSink sink;
    set_launch_sink(&sink);
    const int rc = pipeline(c, cell.evk, cell.logN, cell.logq, cell.bits, io, cell.cnum, st, pl->cws[ci], cell.tune);
    set_launch_sink(nullptr);
    if (rc != FHE_OK) return rc;
    recs[ci] = std::move(sink.recs);
  }
  // which cells go into which launch (queue_layout.h), then the host image of the
  // device buffer: argument structs and segments, 256-byte aligned
  std::vector<std::vector<QRec>> q(nc);
  for (size_t ci = 0; ci < nc; ++ci)
    for (const LaunchRec& r : recs[ci]) {
      QRec x;
      x.variant = r.multi;
      x.bx = r.block.x;
      x.by = r.block.y;
      x.bz = r.block.z;
      x.gx = r.grid.x;
      x.gy = r.grid.y;
      x.gz = r.grid.z;
      x.arg_bytes = (uint32_t)r.args.size();
      x.branch = pl->branch[ci];
      q[ci].push_back(x);
    }
  std::vector<QLaunch> lay;
  const int lr = queue_layout(q, &lay);
  if (lr != QL_OK) return lr == QL_TOO_BIG ? FHE_E_RANGE : FHE_E_STATE;
  std::vector<char> img;
  auto put = [&](const void* p, size_t n) {
    const size_t at = (img.size() + 255) & ~(size_t)255;
    img.resize(at + n);
    memcpy(img.data() + at, p, n);
    return at;
  };
  struct Pending {
    QueueLaunch q;
    size_t args_at = 0, seg_at = 0;
  };
  std::vector<Pending> pend;
  std::map<const void*, size_t> lds_need;
  for (const QLaunch& L : lay) {
    std::vector<char> args;
    std::vector<CellSeg> segs;
    Pending pd;
    for (const QSeg& g : L.segs) {
      const LaunchRec& r = recs[g.cell][L.step];
      CellSeg sg;
      sg.off = g.off;
      sg.gx = g.gx;
      sg.gy = g.gy;
      segs.push_back(sg);
      args.insert(args.end(), r.args.begin(), r.args.end());
      pd.q.lds = std::max(pd.q.lds, r.lds);
    }
    const LaunchRec& r0 = recs[L.segs[0].cell][L.step];
    pd.q.multi = L.variant;
    pd.q.branch = L.branch;
    pd.q.block = r0.block;
    pd.q.blocks = L.blocks;
    pd.q.ncells = (int)segs.size();
    pd.args_at = put(args.data(), args.size());
    pd.seg_at = put(segs.data(), segs.size() * sizeof(CellSeg));
    if (pd.q.lds) lds_need[pd.q.multi] = std::max(lds_need[pd.q.multi], pd.q.lds);
    pend.push_back(pd);
  }
  hipError_t e = hipSuccess;
  for (const auto& kv : lds_need)  // dynamic LDS beyond the default for these entry points
    if (e == hipSuccess)
      e = hipFuncSetAttribute(kv.first, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kv.second);
  if (e == hipSuccess && !img.empty()) e = hipMalloc(&pl->qmem, img.size());
  if (e == hipSuccess && !img.empty()) e = hipMemcpy(pl->qmem, img.data(), img.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return set_sticky(c, e);
  for (Pending& pd : pend) {
    pd.q.args = (char*)pl->qmem + pd.args_at;
    pd.q.seg = (CellSeg*)((char*)pl->qmem + pd.seg_at);
    pl->queue.push_back(pd.q);
  }
  return FHE_OK;
}

// The launches of `branch` (all of them for branch -1), in order, on st.
int plan_run_queue(fhe_plan* pl, hipStream_t st, int branch = -1) {
  for (QueueLaunch& q : pl->queue) {
    if (branch >= 0 && q.branch != branch) continue;
    void* kargs[] = {(void*)&q.args, (void*)&q.seg, (void*)&q.ncells};
    hipError_t e = hipLaunchKernel(q.multi, dim3(q.blocks), q.block, kargs, q.lds, st);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return set_sticky(pl->ctx, e);
  }
  return FHE_OK;
}

// Under capture on pl->cap: each graph branch's launches on its own stream, forked from
// and joined back into the capture stream, as for a plan of cell pipelines.
int plan_capture_queue(fhe_plan* pl) {
  hipError_t e = hipEventRecord(pl->fork, pl->cap);
  for (int b = 1; b < kPlanBranches && e == hipSuccess; ++b)
    if (pl->bst[b]) e = hipStreamWaitEvent(pl->bst[b], pl->fork, 0);
  if (e != hipSuccess) return set_sticky(pl->ctx, e);
  for (int b = 0; b < kPlanBranches; ++b) {
    if (b > 0 && !pl->bst[b]) continue;
    const int rc = plan_run_queue(pl, b ? pl->bst[b] : pl->cap, b);
    if (rc != FHE_OK) return rc;
  }
  for (int b = 1; b < kPlanBranches && e == hipSuccess; ++b)
    if (pl->bst[b]) {
      e = hipEventRecord(pl->join[b], pl->bst[b]);
      if (e == hipSuccess) e = hipStreamWaitEvent(pl->cap, pl->join[b], 0);
    }
  return e == hipSuccess ? FHE_OK : set_sticky(pl->ctx, e);
}

int plan_autotune(fhe_plan* pl, PlanCell& cell, hipStream_t st) {
  fhe_ctx* c = pl->ctx;
  const PipeSize z = pipe_size(c, cell.evk, cell.logN, cell.logq, cell.cnum);
  const std::vector<int> key = {cell.logN, cell.logq, cell.evk->logP, z.Kt, z.Kr, cell.cnum};
  auto it = c->tuned.find(key);
  if (it != c->tuned.end()) {
    cell.tune = it->second;
    return FHE_OK;
  }
  // Candidates: the lift on the matrix cores or the VALU (16 primes per thread); for odd
  // logN, which pass takes the extra stage; the column passes' workgroup width (64, 32
  // or 16 columns of 2^8 points, 64 or 32 of 2^7).
  std::vector<Tuning> cands;
  for (int lp : {0, 16})
    for (int cf : {1, 0}) {
      if (cf == 0 && (cell.logN % 2 == 0)) continue;  // same split either way
      Tuning t;
      t.lift_primes = lp;
      t.ntt_cols_first = cf;
      const int s_cols = ntt_split_cols(cell.logN, t);
      std::vector<int> widths = {0};  // the default: 64 columns per workgroup
      if (s_cols == 8) widths = {0, 512, 256};
      if (s_cols == 7) widths = {0, 256};
      for (int ct : widths) {
        t.cols_threads = ct;
        cands.push_back(t);
      }
    }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return FHE_E_DEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return FHE_E_DEVICE;
  }
  PipeIO io;
  io.ins = cell.ptrs;
  io.outs = cell.ptrs + 4LL * cell.cnum;
  float best = 1e30f;
  Tuning bt = cands[0];
  int rc = FHE_OK;
  for (const Tuning& t : cands) {
    float ts[3];
    rc = pipeline(c, cell.evk, cell.logN, cell.logq, cell.bits, io, cell.cnum, st, pl->ws, t);
    for (int r = 0; r < 3 && rc == FHE_OK; ++r) {
      hipEventRecord(e0, st);
      rc = pipeline(c, cell.evk, cell.logN, cell.logq, cell.bits, io, cell.cnum, st, pl->ws,
                    t);
      hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ts[r], e0, e1) != hipSuccess)
        rc = FHE_E_DEVICE;
    }
    if (rc != FHE_OK) break;
    std::sort(ts, ts + 3);
    if (ts[1] < best) {
      best = ts[1];
      bt = t;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc != FHE_OK) return rc;
  cell.tune = bt;
  c->tuned[key] = bt;
  return FHE_OK;
}

void plan_free(fhe_plan* pl) {
  if (pl->exec) hipGraphExecDestroy(pl->exec);
  if (pl->graph) hipGraphDestroy(pl->graph);
  if (pl->cap) hipStreamDestroy(pl->cap);
  for (int b = 0; b < kPlanBranches; ++b) {
    if (pl->bst[b]) hipStreamDestroy(pl->bst[b]);
    if (pl->join[b]) hipEventDestroy(pl->join[b]);
    if (pl->bws[b]) hipFree(pl->bws[b]);
  }
  if (pl->fork) hipEventDestroy(pl->fork);
  for (PlanCell& cell : pl->cells)
    if (cell.ptrs) hipFree(cell.ptrs);
  for (uint32_t* w : pl->cws)
    if (w) hipFree(w);
  for (void* p : {(void*)pl->ws, pl->qmem})
    if (p) hipFree(p);
  delete pl;
}

// Captures the plan's cells as concurrent graph branches on `cap`: branch 0 on `cap`
// itself, branches 1.. on their own streams, forked from and joined back into `cap`.
int plan_capture_branches(fhe_plan* pl) {
  hipError_t e = hipEventRecord(pl->fork, pl->cap);
  for (int b = 1; b < kPlanBranches && e == hipSuccess; ++b)
    if (pl->bst[b]) e = hipStreamWaitEvent(pl->bst[b], pl->fork, 0);
  if (e != hipSuccess) return set_sticky(pl->ctx, e);
  for (size_t ci = 0; ci < pl->cells.size(); ++ci) {
    PlanCell& cell = pl->cells[ci];
    const int b = pl->branch[ci];
    PipeIO io;
    io.ins = cell.ptrs;
    io.outs = cell.ptrs + 4LL * cell.cnum;
    const int rc = pipeline(pl->ctx, cell.evk, cell.logN, cell.logq, cell.bits, io, cell.cnum,
                            b ? pl->bst[b] : pl->cap, b ? pl->bws[b] : pl->ws, cell.tune);
    if (rc != FHE_OK) return rc;
  }
  for (int b = 1; b < kPlanBranches && e == hipSuccess; ++b)
    if (pl->bst[b]) {
      e = hipEventRecord(pl->join[b], pl->bst[b]);
      if (e == hipSuccess) e = hipStreamWaitEvent(pl->cap, pl->join[b], 0);
    }
  return e == hipSuccess ? FHE_OK : set_sticky(pl->ctx, e);
}

// ---------------------------------------------------------------- serving loop

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// A served request: the job and the event recorded on the submitter's stream after the
// work that writes its inputs (the batch's stream waits for it).
struct SrvJob {
  fhe_job job{};
  hipEvent_t ready = nullptr;
};

// The HIP side of the request loop (the executor of SrvCore): one non-blocking stream
// per slot, scratch carved from one arena allocated at creation, pointer arrays staged
// through pinned host memory.  The scheduler thread calls launch and poll; nothing on
// that path allocates device memory.
struct SrvExec {
  using Job = SrvJob;
  using Cell = std::tuple<const fhe_evk*, int, int>;  // (key, logq, rescale bits)
  struct Slot {
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;
    const uint32_t** hptr = nullptr;  // pinned host staging of the pointer arrays
    uint32_t** dptr = nullptr;        // device pointer arrays (6 max_batch)
  };
  fhe_ctx* ctx = nullptr;
  uint8_t* arena = nullptr;
  std::vector<Slot> slots;
  std::mutex evm;                  // guards the pool of ready events
  std::vector<hipEvent_t> events;  // recycled ready events

  Cell cell_of(const Job& j) const { return Cell(j.job.evk, j.job.logq, j.job.bits); }
  // Scratch bytes per request: the pipeline's scratch is linear in the batch size.
  size_t unit_bytes(const Job& j) const {
    return (size_t)pipe_size(ctx, j.job.evk, j.job.evk->logN, j.job.logq, 1).main_words * 4;
  }
  uint64_t now() { return now_ns(); }

  hipEvent_t take_event() {
    std::lock_guard<std::mutex> lk(evm);
    if (!events.empty()) {
      hipEvent_t e = events.back();
      events.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    return hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess ? e : nullptr;
  }
  void give_event(hipEvent_t e) {
    if (!e) return;
    std::lock_guard<std::mutex> lk(evm);
    events.push_back(e);
  }

  int launch(int s, const std::vector<const Job*>& batch, size_t off) {
    fhe_ctx* c = ctx;
    Slot& sl = slots[s];
    const int cnum = (int)batch.size();
    const fhe_job& j0 = batch[0]->job;
    std::lock_guard<std::recursive_mutex> g(c->mu);
    hipSetDevice(c->device);
    hipError_t e = hipSuccess;
    // the inputs are ready once the submitters' streams reached their events; a wait
    // holds the event's state when it is queued, so the event can be reused right after
    for (const Job* j : batch) {
      if (j->ready && e == hipSuccess && c->sticky == FHE_OK) e = hipStreamWaitEvent(sl.st, j->ready, 0);
      give_event(j->ready);
    }
    if (c->sticky != FHE_OK) return c->sticky;
    if (e != hipSuccess) return set_sticky(c, e);
    // the previous batch of this slot has completed, so its staging may be rewritten
    for (int m = 0; m < cnum; ++m) {
      const fhe_job& j = batch[m]->job;
      sl.hptr[m] = j.x0;
      sl.hptr[cnum + m] = j.x1;
      sl.hptr[2 * cnum + m] = j.y0;
      sl.hptr[3 * cnum + m] = j.y1;
      sl.hptr[4 * cnum + m] = j.out0;
      sl.hptr[5 * cnum + m] = j.out1;
    }
    e = hipMemcpyAsync(sl.dptr, sl.hptr, 6 * (size_t)cnum * sizeof(void*), hipMemcpyHostToDevice, sl.st);
    if (e != hipSuccess) return set_sticky(c, e);
    PipeIO io;
    io.ins = sl.dptr;
    io.outs = sl.dptr + 4LL * cnum;
    const int rc = pipeline(c, j0.evk, j0.evk->logN, j0.logq, j0.bits, io, cnum, sl.st, (uint32_t*)(arena + off),
                            Tuning());
    if (rc != FHE_OK) return rc;
    return set_sticky(c, hipEventRecord(sl.done, sl.st));
  }

  // A request completed without a launch (rejected or cancelled): its event goes back.
  void discard(const Job& j) { give_event(j.ready); }

  int poll(int s) {
    const hipError_t e = hipEventQuery(slots[s].done);
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) return 0;
    std::lock_guard<std::recursive_mutex> g(ctx->mu);
    return set_sticky(ctx, e);
  }
};

}  // namespace

struct fhe_server {
  SrvExec ex;
  SrvCore<SrvExec>* core = nullptr;
};

namespace {

// c = a b in Z_(2^logq)[X]/(X^N + 1) for cnum pairs (lift, NTT, pointwise, iNTT,
// CRT reconstruction); the caller holds the context lock and has checked the arguments.
int ring_mul_locked(fhe_ctx* c, int logN, int logq, const uint32_t* a, const uint32_t* b, uint32_t* out, int cnum,
                    void* stream, uint32_t* R = nullptr) {
  hipStream_t st = (hipStream_t)stream;
  const int N = 1 << logN;
  const int L = (logq + 31) / 32;
  const int eb = 2 * logq + logN;
  const int K = primes_for_e(c, eb);
  if (K < 0) return FHE_E_RANGE;
  hipError_t e = hipSuccess;
  const uint2* sc = crt_scale(c, logN, K, &e);
  if (!sc) return set_sticky(c, e);
  const long long KN = (long long)K * N;
  if (!R) R = (uint32_t*)stream_scratch(c, stream, 0, (size_t)2 * cnum * KN * 4, &e);
  if (!R) return set_sticky(c, e);
  uint32_t* Ra = R;
  uint32_t* Rb = R + (long long)cnum * KN;
  e = launch_lift(lift_args(c, a, Ra, (long long)L * N, KN, N, L, K), cnum, st);
  if (e == hipSuccess) e = launch_lift(lift_args(c, b, Rb, (long long)L * N, KN, N, L, K), cnum, st);
  if (e == hipSuccess) e = launch_ntt_cols(ntt_args(c, R, logN, K, K, KN, false, nullptr), 2 * cnum * K, false, st);
  if (e == hipSuccess) {
    RowsArgs ra = rows_args(c, logN, K, cnum);
    ra.data = Ra;
    ra.data2 = Rb;
    ra.group_stride = KN;
    ra.data2_stride = KN;
    ra.data2_groups = cnum;
    e = launch_rows_fused(ra, ROWS_RING, st);
  }
  if (e == hipSuccess) e = launch_ntt_cols(ntt_args(c, Ra, logN, K, K, KN, true, sc), cnum * K, true, st);
  if (e == hipSuccess) e = run_crt(c, Ra, 1, KN, 0, out, (long long)L * N, N, K, eb, logq, cnum, st);
  return set_sticky(c, e);
}

bool valid_t(int scheme, uint32_t t) {
  if (scheme == FHE_CKKS) return true;
  return scheme == FHE_BGV && t >= 3 && (t & 1) && t < (1u << 24);
}

uint32_t top_mask(int logq) { return (logq & 31) ? (1u << (logq & 31)) - 1u : 0xFFFFFFFFu; }

// Key switch of cnum ciphertexts by the automorphism kappa_g of a Galois key (Section
// 2.5): u = kappa_g(c1), c0' = [kappa_g(c0) + R(u b')]_(2^logq), c1' = [R(u a')].  The
// signed permutation writes kappa_g(c0) and kappa_g(c1) into slots 0 and 2 of the
// relinearization half's limb area; slot 1 (d1) is taken as zero.
int key_switch_locked(fhe_ctx* c, fhe_evk* k, int logN, int logq, const uint32_t* in0, const uint32_t* in1,
                      uint32_t* out0, uint32_t* out1, int cnum, hipStream_t st) {
  int rc = evk_prepare_locked(k, logq, st);
  if (rc != FHE_OK) return rc;
  const PipeSize z = pipe_size(c, k, logN, logq, cnum);
  if (z.Kt < 0 || z.Kr < 0) return FHE_E_RANGE;
  const long long NN = 1LL << logN;
  const long long polyw = (long long)z.L * NN;
  const long long words = (long long)cnum * NN * (3LL * z.L + 3LL * z.Kr + 2LL * z.LK);
  hipError_t e = hipSuccess;
  uint32_t* ws = (uint32_t*)stream_scratch(c, st, 0, (size_t)words * 4, &e);
  if (!ws) return set_sticky(c, e);
  uint32_t* Dl = ws;                                  // [cnum][3][L][N]
  uint32_t* Rr = Dl + (long long)cnum * 3 * polyw;    // [cnum][Kr][N]
  uint32_t* Rk = Rr + (long long)cnum * z.Kr * NN;    // [cnum][2][Kr][N]
  uint32_t* Kl = Rk + (long long)cnum * 2 * z.Kr * NN;  // [cnum][2][LK][N]
  PermArgs pa{};
  pa.in0 = in0;
  pa.in1 = in1;
  pa.out0 = Dl;
  pa.out1 = Dl + 2 * polyw;
  pa.istride = polyw;
  pa.ostride = 3 * polyw;
  pa.logN = logN;
  pa.L = z.L;
  pa.topmask = top_mask(logq);
  pa.mul = (uint32_t)invmod(k->g, 2ull << logN);
  pa.add = 0;
  e = launch_signed_perm(pa, cnum, st);
  if (e != hipSuccess) return set_sticky(c, e);
  PipeIO io;
  io.out0 = out0;
  io.out1 = out1;
  return relin_part(c, k, logN, logq, 0, io, cnum, st, Dl, Rr, Rk, Kl, Tuning(), true);
}

// out_i = m * x_i in Z_(2^logq)[X]/(X^N+1) for both components of cnum ciphertexts,
// with m_c = m + (c mod mcount) L N (mcount = cnum: pairwise; 1: broadcast).  One ring
// product pipeline: the components and the plaintexts are lifted and transformed
// together, the fused row pass multiplies component group g by plaintext g mod mcount.
int plain_mul_locked(fhe_ctx* c, int logN, int logq, const uint32_t* x0, const uint32_t* x1, const uint32_t* m,
                     int mcount, uint32_t* out0, uint32_t* out1, int cnum, hipStream_t st) {
  const int N = 1 << logN;
  const int L = (logq + 31) / 32;
  const int eb = 2 * logq + logN;
  const int K = primes_for_e(c, eb);
  if (K < 0) return FHE_E_RANGE;
  hipError_t e = hipSuccess;
  const uint2* sc = crt_scale(c, logN, K, &e);
  if (!sc) return set_sticky(c, e);
  const long long KN = (long long)K * N, LN = (long long)L * N;
  uint32_t* R = (uint32_t*)stream_scratch(c, st, 0, (size_t)(2LL * cnum + mcount) * KN * 4, &e);
  if (!R) return set_sticky(c, e);
  uint32_t* Rm = R + 2LL * cnum * KN;
  e = launch_lift(lift_args(c, x0, R, LN, KN, N, L, K), cnum, st);
  if (e == hipSuccess) e = launch_lift(lift_args(c, x1, R + cnum * KN, LN, KN, N, L, K), cnum, st);
  if (e == hipSuccess) e = launch_lift(lift_args(c, m, Rm, LN, KN, N, L, K), mcount, st);
  if (e == hipSuccess)
    e = launch_ntt_cols(ntt_args(c, R, logN, K, K, KN, false, nullptr), (2 * cnum + mcount) * K, false, st);
  if (e == hipSuccess) {
    RowsArgs ra = rows_args(c, logN, K, 2 * cnum);
    ra.data = R;
    ra.data2 = Rm;
    ra.group_stride = KN;
    ra.data2_stride = mcount > 1 ? KN : 0;
    ra.data2_groups = mcount > 1 ? mcount : 1;
    e = launch_rows_fused(ra, ROWS_RING, st);
  }
  if (e == hipSuccess) e = launch_ntt_cols(ntt_args(c, R, logN, K, K, KN, true, sc), 2 * cnum * K, true, st);
  if (e == hipSuccess) e = run_crt(c, R, 1, KN, 0, out0, LN, N, K, eb, logq, cnum, st);
  if (e == hipSuccess) e = run_crt(c, R + cnum * KN, 1, KN, 0, out1, LN, N, K, eb, logq, cnum, st);
  return set_sticky(c, e);
}

// ---------------------------------------------------------------- fhe_ct checks

bool ct_valid(const fhe_ctx* c, const fhe_ct* x) {
  if (!x || !x->c0 || !x->c1 || x->cnum < 0 || x->logq < 1) return false;
  if (x->scheme != FHE_CKKS && x->scheme != FHE_BGV) return false;
  if (!valid_t(x->scheme, x->t)) return false;
  if (x->scheme == FHE_BGV && (x->gamma == 0 || x->gamma >= x->t || std::gcd((uint64_t)x->gamma, (uint64_t)x->t) != 1))
    return false;
  (void)c;
  return true;
}

// Argument checks shared by the fhe_ct entry points: status, or FHE_OK.
int ct_check(const fhe_ctx* c, const fhe_ct* x, const fhe_ct* out) {
  if (!c || !ct_valid(c, x) || !out || !out->c0 || !out->c1) return FHE_E_INVAL;
  if (check_logN(x->logN) != FHE_OK || x->logq > c->logQ_max + c->logP_max) return FHE_E_RANGE;
  return FHE_OK;
}

// Same ring, level, scheme and t (and, with scale, the same logp and gamma).
bool ct_same(const fhe_ct* x, const fhe_ct* y, bool scale) {
  if (x->logN != y->logN || x->logq != y->logq || x->scheme != y->scheme || x->t != y->t) return false;
  return !scale || (x->logp == y->logp && x->gamma == y->gamma);
}

void ct_meta(fhe_ct* o, const fhe_ct* x, int logq, int logp, uint32_t gamma) {
  o->cnum = x->cnum;
  o->logN = x->logN;
  o->logq = logq;
  o->logp = logp;
  o->scheme = x->scheme;
  o->t = x->t;
  o->gamma = x->scheme == FHE_BGV ? gamma : 1u;
}

// Buffers [cnum][L][N] of a and b overlap (either component).
bool ct_overlap(const fhe_ct* a, int La, const fhe_ct* b, int Lb) {
  const size_t na = (size_t)a->cnum * La << a->logN, nb = (size_t)b->cnum * Lb << b->logN;
  auto ov = [](const uint32_t* p, size_t n, const uint32_t* q, size_t m) { return p < q + m && q < p + n; };
  return ov(a->c0, na, b->c0, nb) || ov(a->c0, na, b->c1, nb) || ov(a->c1, na, b->c0, nb) ||
         ov(a->c1, na, b->c1, nb);
}

}  // namespace

// ================================================================ C ABI

extern "C" {

const char* fhe_error_detail(void) { return g_detail; }

const char* fhe_strerror(int status) {
  switch (status) {
    case FHE_OK: return "ok";
    case FHE_E_INVAL: return "invalid argument";
    case FHE_E_SHAPE: return "operand shape or parameter mismatch";
    case FHE_E_RANGE: return "beyond context limits or key level";
    case FHE_E_NOMEM: return "out of memory";
    case FHE_E_DEVICE: return "HIP device error";
    case FHE_E_STATE: return "object in the wrong state";
    default: return "unknown status";
  }
}

int fhe_ctx_create(int device, int logQ_max, int logP_max, fhe_ctx** out) {
  if (!out || logQ_max < 1 || logP_max < 1 || logQ_max > 8192 || logP_max > 8192) return FHE_E_INVAL;
  *out = nullptr;
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) {
    note("hipSetDevice", e);
    return FHE_E_DEVICE;
  }
  fhe_ctx* c = new (std::nothrow) fhe_ctx();
  if (!c) return FHE_E_NOMEM;
  c->device = device;
  if (hipDeviceGetAttribute(&c->lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess ||
      hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
    delete c;
    return FHE_E_DEVICE;
  }
  c->logQ_max = logQ_max;
  c->logP_max = logP_max;
  if (device < 0 || device >= kMaxDevices) {
    delete c;
    return FHE_E_RANGE;
  }
  {
    // once per device, with the device current: the address of this device's copy of
    // `scratch` (the symbol itself is a host-side stand-in, not a device address)
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
      void* p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) {
        note("hipGetSymbolAddress(scratch)", e);
        delete c;
        return FHE_E_DEVICE;
      }
      g_scratch_dev[device] = (uint32_t*)p;
    }
    c->noalloc = g_scratch_dev[device];
  }
  // primes q = 1 mod 2^17 below 2^30, largest first, until the largest relinearization
  // product (logN 16, logq = logQ_max, logP = logP_max) is covered with the CRT margin.
  const int e_max = kLogNMax + 2 * logQ_max + logP_max + kCrtMarginBits;
  Big M;
  c->mbits.push_back(M.bitlen());
  for (uint32_t cand = (1u << 30) - (1u << 17) + 1; cand > (1u << 29); cand -= (1u << 17)) {
    if (c->mbits.back() >= e_max + 2) break;
    if (!is_prime32(cand)) continue;
    c->q.push_back(cand);
    M.mul_small(cand);
    c->mbits.push_back(M.bitlen());
  }
  if (c->mbits.back() < e_max + 2) {
    delete c;
    return FHE_E_RANGE;
  }
  const int K = (int)c->q.size();
  c->K = K;
  if (K > kCrtMaxPrimes) {
    delete c;
    return FHE_E_RANGE;
  }
  c->Kpad = K + 16 + kLiftPrimes;  // blocked kernels read per-prime constants past K
  const int Kpad = c->Kpad;
  // psi: g^((q-1)/2^17) for the smallest g with order exactly 2^17
  for (int k = 0; k < K; ++k) {
    const uint32_t q = c->q[k];
    for (uint32_t g = 2;; ++g) {
      uint64_t r = powmod(g, (q - 1) >> 17, q);
      if (powmod(r, 1u << 16, q) == q - 1) {
        c->psi.push_back((uint32_t)r);
        break;
      }
    }
  }
  // per-prime constants
  std::vector<PrimeC> pc(Kpad);
  for (int k = 0; k < Kpad; ++k) {
    const uint32_t q = k < K ? c->q[k] : c->q[0];
    uint32_t inv = 1;  // q^-1 mod 2^32 by Newton iteration
    for (int it = 0; it < 5; ++it) inv *= 2u - q * inv;
    pc[k].q = q;
    pc[k].qneg = (uint32_t)(0u - inv);
    pc[k].c32 = (uint32_t)((1ull << 32) % q);
    pc[k].two_q = 2 * q;
  }
  std::vector<uint32_t> rq(Kpad, 0);
  for (int k = 0; k < K; ++k) rq[k] = (uint32_t)((1ull << 56) / c->q[k]);
  // lift constants 2^(28 i) 2^32 mod q_p (Montgomery form)
  c->Lmax = (std::max(logQ_max, logP_max + logQ_max) + 31) / 32;
  c->TS = 8 * ((c->Lmax + 6) / 7);
  std::vector<uint32_t> T((size_t)Kpad * c->TS, 0);
  for (int p = 0; p < K; ++p) {
    const uint32_t q = c->q[p];
    uint64_t v = (1ull << 32) % q;
    const uint64_t step = (1ull << kLiftDigitBits) % q;
    for (int i = 0; i < c->TS; ++i) {
      T[(size_t)p * c->TS + i] = (uint32_t)v;
      v = mulmod64(v, step, q);
    }
  }
  // twiddles psi^bitrev(k) and psi^-bitrev(k), k < 2^16
  std::vector<uint2> tw((size_t)K * kNMax), itw((size_t)K * kNMax);
  {
    std::vector<uint32_t> pw(kNMax), ipw(kNMax);
    for (int p = 0; p < K; ++p) {
      const uint32_t q = c->q[p];
      const uint64_t ps = c->psi[p], ips = invmod(ps, q);
      uint64_t a = 1, b = 1;
      for (int i = 0; i < kNMax; ++i) {
        pw[i] = (uint32_t)a;
        ipw[i] = (uint32_t)b;
        a = mulmod64(a, ps, q);
        b = mulmod64(b, ips, q);
      }
      for (int i = 0; i < kNMax; ++i) {
        const uint32_t br = bitrev((uint32_t)i, kLogNMax);
        tw[(size_t)p * kNMax + i] = shoup_pair(pw[br], q);
        tw[(size_t)p * kNMax + i].x = 0u - tw[(size_t)p * kNMax + i].x;  // forward butterflies take -w
        itw[(size_t)p * kNMax + i] = shoup_pair(ipw[br], q);
      }
    }
  }
  // final inverse factors N^-1 per logN (standalone transforms), then the same times
  // the last stage's twiddle (NttArgs::scale_w)
  std::vector<std::vector<uint2>> ns(kLogNMax + 1);
  for (int lg = FHE_LOGN_MIN; lg <= kLogNMax; ++lg) {
    ns[lg].assign(2 * (size_t)Kpad, make_uint2(0, 0));
    for (int p = 0; p < K; ++p) {
      const uint64_t f = invmod(1ull << lg, c->q[p]);
      ns[lg][p] = shoup_pair((uint32_t)f, c->q[p]);
      ns[lg][Kpad + p] = shoup_pair((uint32_t)mulmod64(f, last_inv_twiddle(c, p), c->q[p]), c->q[p]);
    }
  }
  // upload
  if ((e = upload(&c->pc, pc)) == hipSuccess && (e = upload(&c->tw, tw)) == hipSuccess &&
      (e = upload(&c->itw, itw)) == hipSuccess && (e = upload(&c->liftT, T)) == hipSuccess &&
      (e = upload(&c->rq, rq)) == hipSuccess) {
    for (int lg = FHE_LOGN_MIN; lg <= kLogNMax && e == hipSuccess; ++lg) e = upload(&c->nscale[lg], ns[lg]);
  }
  if (e != hipSuccess) {
    const int st = e == hipErrorOutOfMemory ? FHE_E_NOMEM : FHE_E_DEVICE;
    fhe_ctx_destroy(c);
    return st;
  }
  *out = c;
  return FHE_OK;
}

void fhe_ctx_destroy(fhe_ctx* c) {
  if (!c) return;
  hipSetDevice(c->device);
  hipDeviceSynchronize();
  for (void* p : {(void*)c->pc, (void*)c->tw, (void*)c->itw, (void*)c->liftT, (void*)c->rq})
    if (p) hipFree(p);
  for (int lg = 0; lg <= kLogNMax; ++lg)
    if (c->nscale[lg]) hipFree(c->nscale[lg]);
  for (auto& kv : c->cscale) hipFree(kv.second);
  for (auto& kv : c->lifts)
    for (void* p : {(void*)kv.second.A, (void*)kv.second.off})
      if (p) hipFree(p);
  for (auto& kv : c->crt)
    for (void* p : {(void*)kv.second.A, (void*)kv.second.d, (void*)kv.second.mneg, (void*)kv.second.eneg})
      if (p) hipFree(p);
  for (auto& kv : c->pw) hipFree(kv.second);
  for (auto& kv : c->ws)
    if (kv.second.ptr) hipFree(kv.second.ptr);
  delete c->rec;
  delete c;
}

int fhe_ctx_reset_error(fhe_ctx* c) {
  if (!c) return FHE_E_INVAL;
  std::lock_guard<std::recursive_mutex> g(c->mu);
  int s = c->sticky;
  c->sticky = FHE_OK;
  (void)hipGetLastError();
  return s;
}

int fhe_ctx_profile(fhe_ctx* c, int enable) {
  if (!c || (enable != 0 && enable != 1)) return FHE_E_INVAL;
  std::lock_guard<std::recursive_mutex> g(c->mu);
  if (enable) {
    if (!c->rec) c->rec = new (std::nothrow) Recorder();
    if (!c->rec) return FHE_E_NOMEM;
    c->rec->clear();
  } else if (c->rec) {
    c->rec->collect();
    delete c->rec;
    c->rec = nullptr;
  }
  return FHE_OK;
}

int fhe_ctx_profile_read(fhe_ctx* c, int kernel, double* ms, double* work, long long* launches) {
  if (!c || !ms || !work || !launches || kernel < 0 || kernel >= KID_COUNT) return FHE_E_INVAL;
  std::lock_guard<std::recursive_mutex> g(c->mu);
  if (!c->rec) return FHE_E_STATE;
  c->rec->collect();
  *ms = c->rec->ms[kernel];
  *work = c->rec->work[kernel];
  *launches = c->rec->launches[kernel];
  return FHE_OK;
}

int fhe_prime_count(const fhe_ctx* c, int* count) {
  if (!c || !count) return FHE_E_INVAL;
  *count = c->K;
  return FHE_OK;
}

int fhe_prime_info(const fhe_ctx* c, int idx, uint32_t* q, uint32_t* psi) {
  if (!c || !q || !psi) return FHE_E_INVAL;
  if (idx < 0 || idx >= c->K) return FHE_E_RANGE;
  *q = c->q[idx];
  *psi = c->psi[idx];
  return FHE_OK;
}

int fhe_primes_needed(const fhe_ctx* c, int logN, int bits_a, int bits_b, int terms, int* K) {
  if (!c || !K || bits_a < 1 || bits_b < 1 || terms < 1) return FHE_E_INVAL;
  if (check_logN(logN) != FHE_OK) return FHE_E_RANGE;
  const int k = primes_for_e(c, bits_a + bits_b + logN + ceil_log2(terms));
  if (k < 0) return FHE_E_RANGE;
  *K = k;
  return FHE_OK;
}

int fhe_lift(fhe_ctx* c, int logN, int L, int nprimes, const uint32_t* limbs, uint32_t* res, int count,
             void* stream) {
  if (!c || !limbs || !res || count < 0 || L < 1 || nprimes < 1) return FHE_E_INVAL;
  if (check_logN(logN) != FHE_OK || nprimes > c->K || L > c->Lmax) return FHE_E_RANGE;
  std::lock_guard<std::recursive_mutex> g(c->mu);
  if (c->sticky != FHE_OK) return c->sticky;
  hipSetDevice(c->device);
  RecGuard rg(c);
  const int N = 1 << logN;
  hipError_t e = launch_lift(lift_args(c, limbs, res, (long long)L * N, (long long)nprimes * N, N, L, nprimes),
                             count, (hipStream_t)stream);
  return set_sticky(c, e);
}

int fhe_ntt(fhe_ctx* c, int logN, int prime0, int nprimes, int flags, uint32_t* data, int count, void* stream) {
  if (!c || !data || count < 0 || nprimes < 1 || prime0 < 0 || (flags & ~(FHE_NTT_INVERSE | FHE_NTT_BITREV)))
    return FHE_E_INVAL;
  if (check_logN(logN) != FHE_OK || prime0 + nprimes > c->K) return FHE_E_RANGE;
  if (count == 0) return FHE_OK;
  std::lock_guard<std::recursive_mutex> g(c->mu);
  if (c->sticky != FHE_OK) return c->sticky;
  hipSetDevice(c->device);
  RecGuard rg(c);
  hipStream_t st = (hipStream_t)stream;
  const long long N = 1LL << logN;
  const bool inverse = (flags & FHE_NTT_INVERSE) != 0, natural = !(flags & FHE_NTT_BITREV);
  const long long rows = (long long)count * nprimes;
  NttArgs a = ntt_args(c, data, logN, nprimes, nprimes, (long long)nprimes * N, inverse, c->nscale[logN] + prime0);
  a.tw += (long long)prime0 * kNMax;
  a.pc += prime0;
  hipError_t e = hipSuccess;
  if (inverse && natural) e = launch_bitrev(data, logN, rows, st);
  if (e == hipSuccess) e = launch_ntt(a, (int)rows, inverse, st);
  if (e == hipSuccess && !inverse && natural) e = launch_bitrev(data, logN, rows, st);
  return set_sticky(c, e);
}

int fhe_ring_mul(fhe_ctx* c, int logN, int logq, const uint32_t* a, const uint32_t* b, uint32_t* out, int cnum,
                 void* stream) {
  if (!c || !a || !b || !out || cnum < 0 || logq < 1) return FHE_E_INVAL;
  if (check_logN(logN) != FHE_OK || logq > c->logQ_max + c->logP_max) return FHE_E_RANGE;
  if (cnum == 0) return FHE_OK;
  std::lock_guard<std::recursive_mutex> g(c->mu);
  if (c->sticky != FHE_OK) return c->sticky;
  hipSetDevice(c->device);
  RecGuard rg(c);
  return ring_mul_locked(c, logN, logq, a, b, out, cnum, stream);
}

int fhe_ring_mul_noalloc(fhe_ctx* c, int logN, int logq, const uint32_t* a, const uint32_t* b, uint32_t* out,
                         int cnum, void* stream) {
  if (!c || !a || !b || !out || cnum < 0 || logq < 1) return FHE_E_INVAL;
  if (check_logN(logN) != FHE_OK || logq > c->logQ_max + c->logP_max) return FHE_E_RANGE;
  if (cnum == 0) return FHE_OK;
  const int N = 1 << logN, L = (logq + 31) / 32, eb = 2 * logq + logN;
  std::lock_guard<std::recursive_mutex> g(c->mu);
  if (c->sticky != FHE_OK) return c->sticky;
  const int K = primes_for_e(c, eb);
  if (K < 0) return FHE_E_RANGE;
  if ((size_t)2 * cnum * K * N > kNoAllocWords) return FHE_E_RANGE;  // beyond the fixed scratch
  // every table the product uses must exist already (built by an fhe_ring_mul of this
  // shape): lookups only, nothing is created here
  if (!c->cscale.count(std::make_pair(logN, K)) || !c->lifts.count(std::make_pair(L, K)) ||
      !c->crt.count(std::make_tuple(K, eb, L)) || c->rec)
    return FHE_E_STATE;
  hipSetDevice(c->device);
  return ring_mul_locked(c, logN, logq, a, b, out, cnum, stream, c->noalloc);
}

int fhe_encrypt(fhe_ctx* c, int scheme, uint32_t t, int logN, int logq, const uint32_t* pk_b, const uint32_t* pk_a,
                const uint32_t* m, const int8_t* v, const int32_t* e0, const int32_t* e1, uint32_t* c0, uint32_t* c1,
                void* stream) {
  if (!c || !pk_b || !pk_a || !m || !v || !e0 || !e1 || !c0 || !c1 || logq < 1) return FHE_E_INVAL;
  if (!valid_t(scheme, t)) return FHE_E_INVAL;
  if (check_logN(logN) != FHE_OK || logq > c->logQ_max + c->logP_max) return FHE_E_RANGE;
  std::lock_guard<std::recursive_mutex> g(c->mu);
  if (c->sticky != FHE_OK) return c->sticky;
  hipSetDevice(c->device);
  RecGuard rg(c);
  hipStream_t st = (hipStream_t)stream;
  const int N = 1 << logN, L = (logq + 31) / 32;
  const uint32_t top = (logq & 31) ? (1u << (logq & 31)) - 1u : 0xFFFFFFFFu;
  const long long LN = (long long)L * N;
  hipError_t e = hipSuccess;
  // [v, v] against [pk_b, pk_a] mod Q_l as one pair of ring products
  uint32_t* S = (uint32_t*)stream_scratch(c, stream, 3, (size_t)6 * LN * 4, &e);
  if (!S) return set_sticky(c, e);
  uint32_t *A = S, *B = S + 2 * LN, *P = S + 4 * LN;
  e = launch_small_to_limbs(v, A, N, L, top, st);
  if (e == hipSuccess) e = launch_small_to_limbs(v, A + LN, N, L, top, st);
  if (e == hipSuccess) e = launch_mask_rows(pk_b, B, N, L, top, st);
  if (e == hipSuccess) e = launch_mask_rows(pk_a, B + LN, N, L, top, st);
  if (e != hipSuccess) return set_sticky(c, e);
  int rc = ring_mul_locked(c, logN, logq, A, B, P, 2, stream);
  if (rc != FHE_OK) return rc;
  const long long mult = scheme == FHE_BGV ? (long long)t : 1;
  e = launch_add_small(P, m, e0, mult, c0, N, L, top, st);
  if (e == hipSuccess) e = launch_add_small(P + LN, nullptr, e1, mult, c1, N, L, top, st);
  return set_sticky(c, e);
}

int fhe_decrypt(fhe_ctx* c, int scheme, uint32_t t, uint32_t gamma, int logN, int logq, const uint32_t* c0,
                const uint32_t* c1, const int8_t* s, uint32_t* out, void* stream) {
  if (!c || !c0 || !c1 || !s || !out || logq < 1) return FHE_E_INVAL;
  if (!valid_t(scheme, t)) return FHE_E_INVAL;
  if (scheme == FHE_BGV && (gamma % t == 0 || std::gcd((uint64_t)gamma, (uint64_t)t) != 1)) return FHE_E_INVAL;
  if (check_logN(logN) != FHE_OK || logq > c->logQ_max + c->logP_max) return FHE_E_RANGE;
  std::lock_guard<std::recursive_mutex> g(c->mu);
  if (c->sticky != FHE_OK) return c->sticky;
  hipSetDevice(c->device);
  RecGuard rg(c);
  hipStream_t st = (hipStream_t)stream;
  const int N = 1 << logN, L = (logq + 31) / 32;
  const uint32_t top = (logq & 31) ? (1u << (logq & 31)) - 1u : 0xFFFFFFFFu;
  const long long LN = (long long)L * N;
  hipError_t e = hipSuccess;
  uint32_t* S = (uint32_t*)stream_scratch(c, stream, 3, (size_t)3 * LN * 4, &e);
  if (!S) return set_sticky(c, e);
  uint32_t *SL = S, *P = S + LN, *PH = S + 2 * LN;
  e = launch_small_to_limbs(s, SL, N, L, top, st);
  if (e != hipSuccess) return set_sticky(c, e);
  int rc = ring_mul_locked(c, logN, logq, c1, SL, P, 1, stream);
  if (rc != FHE_OK) return rc;
  if (scheme == FHE_CKKS) return set_sticky(c, launch_add_small(P, c0, nullptr, 0, out, N, L, top, st));
  e = launch_add_small(P, c0, nullptr, 0, PH, N, L, top, st);
  if (e == hipSuccess)
    e = launch_bgv_decode(PH, out, N, L, logq, t, (uint32_t)powmod(2, logq, t), (uint32_t)invmod(gamma, t), st);
  return set_sticky(c, e);
}

int fhe_evk_create(fhe_ctx* c, int scheme, uint32_t t, int logN, int logQ_key, int logP, const uint32_t* b_host,
                   const uint32_t* a_host, fhe_evk** out) {
  if (!c || !b_host || !a_host || !out || logQ_key < 1 || logP < 1) return FHE_E_INVAL;
  if (scheme != FHE_CKKS && scheme != FHE_BGV) return FHE_E_INVAL;
  if (!valid_t(scheme, t)) return FHE_E_INVAL;
  if (check_logN(logN) != FHE_OK || logQ_key > c->logQ_max || logP > c->logP_max) return FHE_E_RANGE;
  *out = nullptr;
  fhe_evk* k = new (std::nothrow) fhe_evk();
  if (!k) return FHE_E_NOMEM;
  k->ctx = c;
  k->scheme = scheme;
  k->t = scheme == FHE_BGV ? t : 0;
  k->logN = logN;
  k->logQ = logQ_key;
  k->logP = logP;
  const size_t n = (size_t)((logP + logQ_key + 31) / 32) << logN;
  k->hb.assign(b_host, b_host + n);
  k->ha.assign(a_host, a_host + n);
  *out = k;
  return FHE_OK;
}

int fhe_evk_prepare(fhe_evk* k, int logq, void* stream) {
  if (!k || !k->ctx) return FHE_E_INVAL;
  fhe_ctx* c = k->ctx;
  std::lock_guard<std::recursive_mutex> g(c->mu);
  if (c->sticky != FHE_OK) return c->sticky;
  hipSetDevice(c->device);
  RecGuard rg(c);
  return evk_prepare_locked(k, logq, (hipStream_t)stream);
}

void fhe_evk_destroy(fhe_evk* k) {
  if (!k) return;
  if (k->ctx) {
    hipSetDevice(k->ctx->device);
    hipDeviceSynchronize();
  }
  for (auto& kv : k->ntt) hipFree(kv.second);
  for (auto& kv : k->ntt_alt) hipFree(kv.second);
  delete k;
}

int fhe_mul_relin(fhe_ctx* c, fhe_evk* k, int logN, int logq, const uint32_t* x0, const uint32_t* x1,
                  const uint32_t* y0, const uint32_t* y1, uint32_t* out0, uint32_t* out1, int cnum, void* stream) {
  if (!c || !k || !x0 || !x1 || !y0 || !y1 || !out0 || !out1 || cnum < 0 || logq < 1) return FHE_E_INVAL;
  if (k->ctx != c || k->g != 0) return FHE_E_STATE;
  if (logN != k->logN) return FHE_E_SHAPE;
  if (logq > k->logQ) return FHE_E_RANGE;
  if (cnum == 0) return FHE_OK;
  std::lock_guard<std::recursive_mutex> g(c->mu);
  if (c->sticky != FHE_OK) return c->sticky;
  hipSetDevice(c->device);
  RecGuard rg(c);
  PipeIO io;
  io.x0 = x0;
  io.x1 = x1;
  io.y0 = y0;
  io.y1 = y1;
  io.out0 = out0;
  io.out1 = out1;
  return mul_relin_locked(c, k, logN, logq, 0, io, cnum, (hipStream_t)stream);
}

int fhe_rescale(fhe_ctx* c, int scheme, uint32_t t, int logN, int logq, int bits, const uint32_t* in0,
                const uint32_t* in1, uint32_t* out0, uint32_t* out1, int cnum, void* stream) {
  if (!c || !in0 || !in1 || !out0 || !out1 || cnum < 0 || logq < 2 || bits < 1 || bits >= logq) return FHE_E_INVAL;
  if (scheme != FHE_CKKS && scheme != FHE_BGV) return FHE_E_INVAL;
  if (!valid_t(scheme, t)) return FHE_E_INVAL;
  if (check_logN(logN) != FHE_OK) return FHE_E_RANGE;
  const int L = (logq + 31) / 32, Lo = (logq - bits + 31) / 32;
  if (cnum > 1 && Lo != L && ((const void*)in0 == (void*)out0 || (const void*)in1 == (void*)out1))
    return FHE_E_INVAL;  // in place needs equal strides
  if (cnum == 0) return FHE_OK;
  std::lock_guard<std::recursive_mutex> g(c->mu);
  if (c->sticky != FHE_OK) return c->sticky;
  hipSetDevice(c->device);
  RecGuard rg(c);
  return rescale_locked(c, scheme, t, logN, logq, bits, in0, in1, (long long)L << logN, out0, out1,
                        (long long)Lo << logN, cnum, (hipStream_t)stream);
}

int fhe_mul_relin_rescale(fhe_ctx* c, fhe_evk* k, int logN, int logq, int bits, const uint32_t* x0,
                          const uint32_t* x1, const uint32_t* y0, const uint32_t* y1, uint32_t* out0,
                          uint32_t* out1, int cnum, void* stream) {
  if (!c || !k || !x0 || !x1 || !y0 || !y1 || !out0 || !out1 || cnum < 0 || logq < 2) return FHE_E_INVAL;
  if (bits < 1 || bits >= logq) return FHE_E_INVAL;
  if (k->ctx != c || k->g != 0) return FHE_E_STATE;
  if (logN != k->logN) return FHE_E_SHAPE;
  if (logq > k->logQ) return FHE_E_RANGE;
  if (cnum == 0) return FHE_OK;
  std::lock_guard<std::recursive_mutex> g(c->mu);
  if (c->sticky != FHE_OK) return c->sticky;
  hipSetDevice(c->device);
  RecGuard rg(c);
  PipeIO io;
  io.x0 = x0;
  io.x1 = x1;
  io.y0 = y0;
  io.y1 = y1;
  io.out0 = out0;
  io.out1 = out1;
  return mul_relin_locked(c, k, logN, logq, bits, io, cnum, (hipStream_t)stream);
}

int fhe_batch_plan(fhe_ctx* c, const fhe_job* jobs, int njobs, int flags, void* stream, fhe_plan** out) {
  if (!c || !out || njobs < 0 || (njobs > 0 && !jobs) || (flags & ~(FHE_PLAN_GRAPH | FHE_PLAN_AUTOTUNE | FHE_PLAN_QUEUE)))
    return FHE_E_INVAL;
  *out = nullptr;
  for (int i = 0; i < njobs; ++i) {
    const fhe_job& j = jobs[i];
    if (!j.evk || !j.x0 || !j.x1 || !j.y0 || !j.y1 || !j.out0 || !j.out1) return FHE_E_INVAL;
    if (j.evk->ctx != c || j.evk->g != 0) return FHE_E_STATE;
    if (j.logq < 1 || j.logq > j.evk->logQ) return FHE_E_RANGE;
    if (j.bits < 0 || j.bits >= j.logq) return FHE_E_INVAL;
  }
  std::lock_guard<std::recursive_mutex> g(c->mu);
  if (c->sticky != FHE_OK) return c->sticky;
  hipSetDevice(c->device);
  hipStream_t st = (hipStream_t)stream;
  fhe_plan* pl = new (std::nothrow) fhe_plan();
  if (!pl) return FHE_E_NOMEM;
  pl->ctx = c;
  // cells in order of first appearance
  std::vector<std::vector<int>> members;
  for (int i = 0; i < njobs; ++i) {
    size_t ci = 0;
    for (; ci < pl->cells.size(); ++ci) {
      const PlanCell& cc = pl->cells[ci];
      if (cc.evk == jobs[i].evk && cc.logq == jobs[i].logq && cc.bits == jobs[i].bits) break;
    }
    if (ci == pl->cells.size()) {
      PlanCell nc;
      nc.evk = jobs[i].evk;
      nc.logN = jobs[i].evk->logN;
      nc.logq = jobs[i].logq;
      nc.bits = jobs[i].bits;
      pl->cells.push_back(nc);
      members.emplace_back();
    }
    members[ci].push_back(i);
  }
  int rc = FHE_OK;
  long long mw = 0;
  for (size_t ci = 0; ci < pl->cells.size() && rc == FHE_OK; ++ci) {
    PlanCell& cell = pl->cells[ci];
    cell.cnum = (int)members[ci].size();
    rc = evk_prepare_locked(cell.evk, cell.logq, st);
    if (rc != FHE_OK) break;
    {
      // tables the pipeline would otherwise upload lazily (not allowed under capture)
      hipError_t e = hipSuccess;
      if (!tables_prewarm(c, cell.evk, cell.logN, cell.logq, &e) ||
          (cell.evk->scheme == FHE_BGV && !pow_table(c, cell.evk->t, &e))) {
        rc = set_sticky(c, e);
        break;
      }
    }
    const PipeSize z = pipe_size(c, cell.evk, cell.logN, cell.logq, cell.cnum);
    if (z.Kt < 0 || z.Kr < 0) {
      rc = FHE_E_RANGE;
      break;
    }
    mw = std::max(mw, z.main_words);
    std::vector<const uint32_t*> h(6 * (size_t)cell.cnum);
    for (int m = 0; m < cell.cnum; ++m) {
      const fhe_job& j = jobs[members[ci][m]];
      h[m] = j.x0;
      h[cell.cnum + m] = j.x1;
      h[2 * cell.cnum + m] = j.y0;
      h[3 * cell.cnum + m] = j.y1;
      h[4 * cell.cnum + m] = j.out0;
      h[5 * cell.cnum + m] = j.out1;
    }
    hipError_t e = hipMalloc((void**)&cell.ptrs, h.size() * sizeof(void*));
    if (e == hipSuccess) e = hipMemcpy(cell.ptrs, h.data(), h.size() * sizeof(void*), hipMemcpyHostToDevice);
    if (e != hipSuccess) rc = set_sticky(c, e);
  }
  if (rc == FHE_OK) {
    hipError_t e = hipMalloc((void**)&pl->ws, (size_t)std::max(mw, 1LL) * 4);
    if (e != hipSuccess) rc = set_sticky(c, e);
  }
  // graph branches: cells by decreasing scratch size (a proxy for their work), each to
  // the branch with the least so far; branches 1.. get scratch for their largest cell
  pl->branch.assign(pl->cells.size(), 0);
  const bool queue = (flags & FHE_PLAN_QUEUE) != 0;
  if (rc == FHE_OK && (flags & FHE_PLAN_GRAPH)) {
    std::vector<long long> words(pl->cells.size());
    std::vector<int> order(pl->cells.size());
    for (size_t ci = 0; ci < pl->cells.size(); ++ci) {
      const PlanCell& cell = pl->cells[ci];
      words[ci] = pipe_size(c, cell.evk, cell.logN, cell.logq, cell.cnum).main_words;
      order[ci] = (int)ci;
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return words[x] > words[y]; });
    long long load[kPlanBranches] = {0, 0, 0, 0}, need[kPlanBranches] = {0, 0, 0, 0};
    for (int ci : order) {
      int b = 0;
      for (int v = 1; v < kPlanBranches; ++v)
        if (load[v] < load[b]) b = v;
      pl->branch[ci] = b;
      load[b] += words[ci];
      need[b] = std::max(need[b], words[ci]);
    }
    hipError_t e = hipEventCreateWithFlags(&pl->fork, hipEventDisableTiming);
    for (int b = 1; b < kPlanBranches && e == hipSuccess; ++b) {
      if (need[b] == 0) continue;  // an empty branch
      // a stage-batched plan gives every cell scratch of its own instead
      if (!queue) e = hipMalloc((void**)&pl->bws[b], (size_t)need[b] * 4);
      if (e == hipSuccess) e = hipStreamCreateWithFlags(&pl->bst[b], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->join[b], hipEventDisableTiming);
    }
    if (e != hipSuccess) rc = set_sticky(c, e);
  }
  if (rc == FHE_OK && (flags & FHE_PLAN_AUTOTUNE)) {
    set_recorder(nullptr);
    for (PlanCell& cell : pl->cells)
      if ((rc = plan_autotune(pl, cell, st)) != FHE_OK) break;
  }
  if (rc == FHE_OK && queue) {
    set_recorder(nullptr);
    rc = plan_build_queue(pl, st);
    if (rc == FHE_OK && (flags & FHE_PLAN_GRAPH)) {
      hipError_t e = hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipStreamBeginCapture(pl->cap, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        rc = plan_capture_queue(pl);
        hipGraph_t gr = nullptr;
        const hipError_t e2 = hipStreamEndCapture(pl->cap, &gr);
        pl->graph = gr;
        if (rc == FHE_OK && e2 != hipSuccess) e = e2;
      }
      if (rc == FHE_OK && e == hipSuccess) e = hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0);
      if (rc == FHE_OK && e != hipSuccess) rc = set_sticky(c, e);
    } else if (rc == FHE_OK) {
      rc = plan_run_queue(pl, st);  // the first execution, as for an eager plan
    }
    pl->kernels = (int)pl->queue.size();
  } else if (rc == FHE_OK) {
    const long long k0 = kernel_launch_count();
    set_recorder(nullptr);
    if (flags & FHE_PLAN_GRAPH) {
      hipError_t e = hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipStreamBeginCapture(pl->cap, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        rc = plan_capture_branches(pl);
        hipGraph_t gr = nullptr;
        const hipError_t e2 = hipStreamEndCapture(pl->cap, &gr);
        pl->graph = gr;
        if (rc == FHE_OK && e2 != hipSuccess) e = e2;
      }
      if (rc == FHE_OK && e == hipSuccess) e = hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0);
      if (rc == FHE_OK && e != hipSuccess) rc = set_sticky(c, e);
      pl->kernels = (int)(kernel_launch_count() - k0);
    } else {
      // count the launches of one run without running it twice: plan runs are
      // deterministic, so run once now (the first execution)
      rc = plan_run_cells(pl, st);
      pl->kernels = (int)(kernel_launch_count() - k0);
    }
  }
  if (rc == FHE_OK) {
    const hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) rc = set_sticky(c, e);
  }
  if (rc != FHE_OK) {
    plan_free(pl);
    return rc;
  }
  *out = pl;
  return FHE_OK;
}

int fhe_batch_run(fhe_plan* pl, void* stream) {
  if (!pl || !pl->ctx) return FHE_E_INVAL;
  fhe_ctx* c = pl->ctx;
  std::lock_guard<std::recursive_mutex> g(c->mu);
  if (c->sticky != FHE_OK) return c->sticky;
  hipSetDevice(c->device);
  if (pl->exec) return set_sticky(c, hipGraphLaunch(pl->exec, (hipStream_t)stream));
  if (!pl->queue.empty()) return plan_run_queue(pl, (hipStream_t)stream);
  RecGuard rg(c);
  return plan_run_cells(pl, (hipStream_t)stream);
}

int fhe_batch_info(const fhe_plan* pl, int* cells, int* kernels, int* graphed) {
  if (!pl || !cells || !kernels || !graphed) return FHE_E_INVAL;
  *cells = (int)pl->cells.size();
  *kernels = pl->kernels;
  *graphed = pl->exec != nullptr;
  return FHE_OK;
}

void fhe_batch_destroy(fhe_plan* pl) {
  if (!pl) return;
  if (pl->ctx) {
    hipSetDevice(pl->ctx->device);
    hipDeviceSynchronize();
  }
  plan_free(pl);
}

uint64_t fhe_clock_ns(void) { return now_ns(); }

int fhe_server_create(fhe_ctx* c, size_t hbm_budget, int nstreams, int max_batch, fhe_server** out) {
  if (!c || !out || nstreams < 1 || nstreams > 16 || max_batch < 1 || max_batch > 256) return FHE_E_INVAL;
  *out = nullptr;
  hipSetDevice(c->device);
  fhe_server* sv = new (std::nothrow) fhe_server();
  if (!sv) return FHE_E_NOMEM;
  SrvExec& ex = sv->ex;
  ex.ctx = c;
  ex.slots.resize(nstreams);
  hipError_t e = hipSuccess;
  const size_t arena = hbm_budget & ~(size_t)255;
  if (arena) e = hipMalloc((void**)&ex.arena, arena);
  for (SrvExec::Slot& sl : ex.slots) {
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl.hptr, 6 * (size_t)max_batch * sizeof(void*), 0);
    if (e == hipSuccess) e = hipMalloc((void**)&sl.dptr, 6 * (size_t)max_batch * sizeof(void*));
  }
  if (e == hipSuccess) sv->core = new (std::nothrow) SrvCore<SrvExec>(ex, arena, nstreams, max_batch);
  if (e != hipSuccess || !sv->core) {
    if (e == hipSuccess) e = hipErrorOutOfMemory;
    note("fhe_server_create", e);
    fhe_server_destroy(sv);
    return status_of(e);
  }
  sv->core->start();
  *out = sv;
  return FHE_OK;
}

int fhe_server_submit(fhe_server* sv, const fhe_job* j, uint64_t arrival_ns, void* stream, uint64_t* ticket) {
  if (!sv || !j || !ticket) return FHE_E_INVAL;
  if (!j->evk || !j->x0 || !j->x1 || !j->y0 || !j->y1 || !j->out0 || !j->out1) return FHE_E_INVAL;
  fhe_ctx* c = sv->ex.ctx;
  if (j->evk->ctx != c || j->evk->g != 0) return FHE_E_STATE;
  if (j->logq < 1 || j->logq > j->evk->logQ) return FHE_E_RANGE;
  if (j->bits < 0 || j->bits >= j->logq) return FHE_E_INVAL;
  SrvJob sj;
  sj.job = *j;
  {
    // the key level must be resident already; the context's tables for this shape are
    // built here, outside the scheduler (nothing on its path allocates)
    std::lock_guard<std::recursive_mutex> g(c->mu);
    if (c->sticky != FHE_OK) return c->sticky;
    if (!j->evk->ntt.count(j->logq)) return FHE_E_STATE;
    hipSetDevice(c->device);
    hipError_t e = hipSuccess;
    if (!tables_prewarm(c, j->evk, j->evk->logN, j->logq, &e)) return set_sticky(c, e);
    if (j->evk->scheme == FHE_BGV && !pow_table(c, j->evk->t, &e)) return set_sticky(c, e);
    sj.ready = sv->ex.take_event();
    if (!sj.ready) return FHE_E_NOMEM;
    e = hipEventRecord(sj.ready, (hipStream_t)stream);
    if (e != hipSuccess) {
      sv->ex.give_event(sj.ready);
      return set_sticky(c, e);
    }
  }
  const uint64_t t = sv->core->submit(sj, arrival_ns);
  if (!t) {
    sv->ex.give_event(sj.ready);
    return FHE_E_STATE;
  }
  *ticket = t;
  return FHE_OK;
}

int fhe_server_poll(fhe_server* sv, fhe_done* out, int max, int* n) {
  if (!sv || !n || max < 0 || (max > 0 && !out)) return FHE_E_INVAL;
  static_assert(sizeof(fhe_done) == sizeof(SrvDone), "fhe_done and SrvDone share a layout");
  *n = sv->core->poll(reinterpret_cast<SrvDone*>(out), max);
  return FHE_OK;
}

int fhe_server_drain(fhe_server* sv) {
  if (!sv) return FHE_E_INVAL;
  sv->core->drain();
  return FHE_OK;
}

int fhe_server_cancel(fhe_server* sv) {
  if (!sv) return FHE_E_INVAL;
  sv->core->cancel();
  return FHE_OK;
}

void fhe_server_destroy(fhe_server* sv) {
  if (!sv) return;
  if (sv->core) sv->core->stop();  // once every submitted request has completed
  delete sv->core;
  SrvExec& ex = sv->ex;
  hipSetDevice(ex.ctx->device);
  for (SrvExec::Slot& sl : ex.slots) {
    if (sl.st) hipStreamSynchronize(sl.st);
    if (sl.dptr) hipFree(sl.dptr);
    if (sl.hptr) hipHostFree(sl.hptr);
    if (sl.done) hipEventDestroy(sl.done);
    if (sl.st) hipStreamDestroy(sl.st);
  }
  if (ex.arena) hipFree(ex.arena);
  for (hipEvent_t e : ex.events) hipEventDestroy(e);
  delete sv;
}

// ---------------------------------------------------------------- Galois keys and automorphisms

int fhe_galois_key_create(fhe_ctx* c, int scheme, uint32_t t, int logN, int logQ_key, int logP, uint32_t g,
                          const uint32_t* b_host, const uint32_t* a_host, fhe_evk** out) {
  if (!out) return FHE_E_INVAL;
  *out = nullptr;
  if (check_logN(logN) == FHE_OK && ((g & 1u) == 0 || g >= (2u << logN))) return FHE_E_INVAL;
  fhe_evk* k = nullptr;
  const int rc = fhe_evk_create(c, scheme, t, logN, logQ_key, logP, b_host, a_host, &k);
  if (rc != FHE_OK) return rc;
  k->g = g;
  *out = k;
  return FHE_OK;
}

int fhe_automorphism(fhe_ctx* c, int logN, int logq, uint32_t g, const uint32_t* in, uint32_t* out, int count,
                     void* stream) {
  if (!c || !in || !out || count < 0 || logq < 1) return FHE_E_INVAL;
  if (check_logN(logN) != FHE_OK || logq > c->logQ_max + c->logP_max) return FHE_E_RANGE;
  if ((g & 1u) == 0 || g >= (2u << logN)) return FHE_E_INVAL;
  const int L = (logq + 31) / 32;
  const size_t n = (size_t)count * L << logN;
  if (count > 0 && in < out + n && out < in + n) return FHE_E_INVAL;
  if (count == 0) return FHE_OK;
  std::lock_guard<std::recursive_mutex> lg(c->mu);
  if (c->sticky != FHE_OK) return c->sticky;
  hipSetDevice(c->device);
  RecGuard rg(c);
  // `count` one-component polynomials
  const long long LN = (long long)L << logN;
  PermArgs pa{};
  pa.in0 = in;
  pa.out0 = out;
  pa.istride = LN;
  pa.ostride = LN;
  pa.logN = logN;
  pa.L = L;
  pa.topmask = top_mask(logq);
  pa.mul = (uint32_t)invmod(g, 2ull << logN);
  pa.comps = 1;
  return set_sticky(c, launch_signed_perm(pa, count, (hipStream_t)stream));
}

int fhe_key_switch(fhe_ctx* c, fhe_evk* k, int logN, int logq, const uint32_t* in0, const uint32_t* in1,
                   uint32_t* out0, uint32_t* out1, int cnum, void* stream) {
  if (!c || !k || !in0 || !in1 || !out0 || !out1 || cnum < 0 || logq < 1) return FHE_E_INVAL;
  if (k->ctx != c || k->g == 0) return FHE_E_STATE;
  if (logN != k->logN) return FHE_E_SHAPE;
  if (logq > k->logQ) return FHE_E_RANGE;
  if (cnum == 0) return FHE_OK;
  std::lock_guard<std::recursive_mutex> lg(c->mu);
  if (c->sticky != FHE_OK) return c->sticky;
  hipSetDevice(c->device);
  RecGuard rg(c);
  return key_switch_locked(c, k, logN, logq, in0, in1, out0, out1, cnum, (hipStream_t)stream);
}

// ---------------------------------------------------------------- ciphertexts with metadata

int fhe_ct_mul_relin_rescale(fhe_ctx* c, fhe_evk* k, const fhe_ct* x, const fhe_ct* y, int bits, fhe_ct* out,
                             void* stream) {
  int rc = ct_check(c, x, out);
  if (rc != FHE_OK) return rc;
  if (!k || !ct_valid(c, y) || bits < 0 || bits >= x->logq) return FHE_E_INVAL;
  if (k->ctx != c || k->g != 0) return FHE_E_STATE;
  if (!ct_same(x, y, false) || x->cnum != y->cnum || x->logN != k->logN || x->scheme != k->scheme ||
      (x->scheme == FHE_BGV && x->t != k->t))
    return FHE_E_SHAPE;
  if (x->logq > k->logQ) return FHE_E_RANGE;
  const int L = (x->logq + 31) / 32, Lo = (x->logq - bits + 31) / 32;
  if (ct_overlap(out, Lo, x, L) || ct_overlap(out, Lo, y, L)) return FHE_E_INVAL;
  if (x->cnum > 0) {
    rc = bits > 0 ? fhe_mul_relin_rescale(c, k, x->logN, x->logq, bits, x->c0, x->c1, y->c0, y->c1, out->c0,
                                          out->c1, x->cnum, stream)
                  : fhe_mul_relin(c, k, x->logN, x->logq, x->c0, x->c1, y->c0, y->c1, out->c0, out->c1, x->cnum,
                                  stream);
    if (rc != FHE_OK) return rc;
  }
  // mult: logp adds, gamma multiplies; rescale: logq and (CKKS) logp drop by bits,
  // (BGV) gamma picks up 2^-bits mod t
  uint32_t gamma = 1;
  if (x->scheme == FHE_BGV) {
    gamma = (uint32_t)((uint64_t)x->gamma * y->gamma % x->t);
    if (bits > 0) gamma = (uint32_t)((uint64_t)gamma * invmod(powmod(2, bits, x->t), x->t) % x->t);
  }
  const int logp = x->logp + y->logp - (x->scheme == FHE_CKKS ? bits : 0);
  ct_meta(out, x, x->logq - bits, logp, gamma);
  return FHE_OK;
}

int fhe_ct_mul_relin(fhe_ctx* c, fhe_evk* k, const fhe_ct* x, const fhe_ct* y, fhe_ct* out, void* stream) {
  return fhe_ct_mul_relin_rescale(c, k, x, y, 0, out, stream);
}

int fhe_ct_rescale(fhe_ctx* c, const fhe_ct* x, int bits, fhe_ct* out, void* stream) {
  int rc = ct_check(c, x, out);
  if (rc != FHE_OK) return rc;
  if (bits < 1 || bits >= x->logq) return FHE_E_INVAL;
  if (x->cnum > 0) {
    rc = fhe_rescale(c, x->scheme, x->t, x->logN, x->logq, bits, x->c0, x->c1, out->c0, out->c1, x->cnum, stream);
    if (rc != FHE_OK) return rc;
  }
  uint32_t gamma = 1;
  if (x->scheme == FHE_BGV) gamma = (uint32_t)((uint64_t)x->gamma * invmod(powmod(2, bits, x->t), x->t) % x->t);
  ct_meta(out, x, x->logq - bits, x->scheme == FHE_CKKS ? x->logp - bits : x->logp, gamma);
  return FHE_OK;
}

// Coefficient-wise sum with signs (add, sub, negate, addconst, moddown) on the context.
static int ct_limb_sum(fhe_ctx* c, const fhe_ct* x, const uint32_t* y0, const uint32_t* y1, long long ystride,
                       int negx, int negy, int logq_out, fhe_ct* out, void* stream) {
  if (x->cnum == 0) return FHE_OK;
  std::lock_guard<std::recursive_mutex> lg(c->mu);
  if (c->sticky != FHE_OK) return c->sticky;
  hipSetDevice(c->device);
  RecGuard rg(c);
  const int L = (x->logq + 31) / 32, Lo = (logq_out + 31) / 32;
  LimbSumArgs a{};
  a.x0 = x->c0;
  a.x1 = x->c1;
  a.y0 = y0;
  a.y1 = y1;
  a.out0 = out->c0;
  a.out1 = out->c1;
  a.xstride = (long long)L << x->logN;
  a.ystride = ystride;
  a.ostride = (long long)Lo << x->logN;
  a.N = 1 << x->logN;
  a.L = Lo;
  a.topmask = top_mask(logq_out);
  a.negx = negx;
  a.negy = negy;
  return set_sticky(c, launch_limb_sum(a, x->cnum, (hipStream_t)stream));
}

// In place is allowed when the output is the input itself; partial overlaps are not.
static bool ct_alias_ok(const fhe_ct* out, int Lo, const fhe_ct* x, int L) {
  if (out->c0 == x->c0 && out->c1 == x->c1 && Lo == L) return true;
  return !ct_overlap(out, Lo, x, L);
}

static int ct_add_sub(fhe_ctx* c, const fhe_ct* x, const fhe_ct* y, fhe_ct* out, int sub, void* stream) {
  int rc = ct_check(c, x, out);
  if (rc != FHE_OK) return rc;
  if (!ct_valid(c, y)) return FHE_E_INVAL;
  if (!ct_same(x, y, true) || !(y->cnum == x->cnum || y->cnum == 1)) return FHE_E_SHAPE;
  const int L = (x->logq + 31) / 32;
  if (!ct_alias_ok(out, L, x, L) || !ct_alias_ok(out, L, y, L)) return FHE_E_INVAL;
  const long long ystride = y->cnum == x->cnum ? (long long)L << x->logN : 0;  // 1: broadcast
  rc = ct_limb_sum(c, x, y->c0, y->c1, ystride, 0, sub, x->logq, out, stream);
  if (rc == FHE_OK) ct_meta(out, x, x->logq, x->logp, x->gamma);
  return rc;
}

int fhe_ct_add(fhe_ctx* c, const fhe_ct* x, const fhe_ct* y, fhe_ct* out, void* stream) {
  return ct_add_sub(c, x, y, out, 0, stream);
}

int fhe_ct_sub(fhe_ctx* c, const fhe_ct* x, const fhe_ct* y, fhe_ct* out, void* stream) {
  return ct_add_sub(c, x, y, out, 1, stream);
}

int fhe_ct_negate(fhe_ctx* c, const fhe_ct* x, fhe_ct* out, void* stream) {
  int rc = ct_check(c, x, out);
  if (rc != FHE_OK) return rc;
  const int L = (x->logq + 31) / 32;
  if (!ct_alias_ok(out, L, x, L)) return FHE_E_INVAL;
  rc = ct_limb_sum(c, x, nullptr, nullptr, 0, 1, 0, x->logq, out, stream);
  if (rc == FHE_OK) ct_meta(out, x, x->logq, x->logp, x->gamma);
  return rc;
}

int fhe_ct_moddown(fhe_ctx* c, const fhe_ct* x, int bits, fhe_ct* out, void* stream) {
  int rc = ct_check(c, x, out);
  if (rc != FHE_OK) return rc;
  if (bits < 0 || bits >= x->logq) return FHE_E_INVAL;
  const int L = (x->logq + 31) / 32, Lo = (x->logq - bits + 31) / 32;
  if (!(out->c0 == x->c0 && out->c1 == x->c1 && (x->cnum <= 1 || Lo == L)) && ct_overlap(out, Lo, x, L))
    return FHE_E_INVAL;
  rc = ct_limb_sum(c, x, nullptr, nullptr, 0, 0, 0, x->logq - bits, out, stream);
  if (rc == FHE_OK) ct_meta(out, x, x->logq - bits, x->logp, x->gamma);
  return rc;
}

int fhe_ct_addconst(fhe_ctx* c, const fhe_ct* x, const uint32_t* m, int mcount, fhe_ct* out, void* stream) {
  int rc = ct_check(c, x, out);
  if (rc != FHE_OK) return rc;
  if (!m || !(mcount == 1 || mcount == x->cnum)) return FHE_E_INVAL;
  const int L = (x->logq + 31) / 32;
  if (!ct_alias_ok(out, L, x, L)) return FHE_E_INVAL;
  const long long ystride = mcount > 1 ? (long long)L << x->logN : 0;
  rc = ct_limb_sum(c, x, m, nullptr, ystride, 0, 0, x->logq, out, stream);
  if (rc == FHE_OK) ct_meta(out, x, x->logq, x->logp, x->gamma);
  return rc;
}

int fhe_ct_imult(fhe_ctx* c, const fhe_ct* x, fhe_ct* out, void* stream) {
  int rc = ct_check(c, x, out);
  if (rc != FHE_OK) return rc;
  if (x->scheme != FHE_CKKS) return FHE_E_INVAL;
  const int L = (x->logq + 31) / 32;
  if (ct_overlap(out, L, x, L)) return FHE_E_INVAL;
  if (x->cnum > 0) {
    std::lock_guard<std::recursive_mutex> lg(c->mu);
    if (c->sticky != FHE_OK) return c->sticky;
    hipSetDevice(c->device);
    RecGuard rg(c);
    // X^(N/2): output position k takes input k - N/2 (mod 2N, negated below zero)
    PermArgs pa{};
    pa.in0 = x->c0;
    pa.in1 = x->c1;
    pa.out0 = out->c0;
    pa.out1 = out->c1;
    pa.istride = pa.ostride = (long long)L << x->logN;
    pa.logN = x->logN;
    pa.L = L;
    pa.topmask = top_mask(x->logq);
    pa.mul = 1;
    pa.add = (2u << x->logN) - (1u << (x->logN - 1));
    rc = set_sticky(c, launch_signed_perm(pa, x->cnum, (hipStream_t)stream));
    if (rc != FHE_OK) return rc;
  }
  ct_meta(out, x, x->logq, x->logp, x->gamma);
  return FHE_OK;
}

int fhe_ct_multconst(fhe_ctx* c, const fhe_ct* x, const uint32_t* k_host, int klimbs, int negative, int logp_k,
                     fhe_ct* out, void* stream) {
  int rc = ct_check(c, x, out);
  if (rc != FHE_OK) return rc;
  if (!k_host || klimbs < 1 || klimbs > kConstMaxLimbs || logp_k < 0) return FHE_E_INVAL;
  const int L = (x->logq + 31) / 32;
  if (!ct_alias_ok(out, L, x, L)) return FHE_E_INVAL;
  if (x->cnum > 0) {
    std::lock_guard<std::recursive_mutex> lg(c->mu);
    if (c->sticky != FHE_OK) return c->sticky;
    hipSetDevice(c->device);
    RecGuard rg(c);
    ConstMulArgs a{};
    a.in0 = x->c0;
    a.in1 = x->c1;
    a.out0 = out->c0;
    a.out1 = out->c1;
    a.istride = a.ostride = (long long)L << x->logN;
    a.N = 1 << x->logN;
    a.L = L;
    a.topmask = top_mask(x->logq);
    for (int i = 0; i < klimbs; ++i) a.k[i] = k_host[i];
    a.klimbs = klimbs;
    a.neg = negative ? 1 : 0;
    rc = set_sticky(c, launch_const_mul(a, x->cnum, (hipStream_t)stream));
    if (rc != FHE_OK) return rc;
  }
  ct_meta(out, x, x->logq, x->scheme == FHE_CKKS ? x->logp + logp_k : x->logp, x->gamma);
  return FHE_OK;
}

int fhe_ct_multconstvec(fhe_ctx* c, const fhe_ct* x, const uint32_t* m, int mcount, int logp_m, fhe_ct* out,
                        void* stream) {
  int rc = ct_check(c, x, out);
  if (rc != FHE_OK) return rc;
  if (!m || !(mcount == 1 || mcount == x->cnum) || logp_m < 0) return FHE_E_INVAL;
  const int L = (x->logq + 31) / 32;
  if (!ct_alias_ok(out, L, x, L)) return FHE_E_INVAL;
  if (x->cnum > 0) {
    std::lock_guard<std::recursive_mutex> lg(c->mu);
    if (c->sticky != FHE_OK) return c->sticky;
    hipSetDevice(c->device);
    RecGuard rg(c);
    rc = plain_mul_locked(c, x->logN, x->logq, x->c0, x->c1, m, mcount, out->c0, out->c1, x->cnum,
                          (hipStream_t)stream);
    if (rc != FHE_OK) return rc;
  }
  ct_meta(out, x, x->logq, x->scheme == FHE_CKKS ? x->logp + logp_m : x->logp, x->gamma);
  return FHE_OK;
}

int fhe_ct_key_switch(fhe_ctx* c, fhe_evk* k, const fhe_ct* x, fhe_ct* out, void* stream) {
  int rc = ct_check(c, x, out);
  if (rc != FHE_OK) return rc;
  if (!k) return FHE_E_INVAL;
  if (k->ctx != c || k->g == 0) return FHE_E_STATE;
  if (x->logN != k->logN || x->scheme != k->scheme || (x->scheme == FHE_BGV && x->t != k->t)) return FHE_E_SHAPE;
  if (x->logq > k->logQ) return FHE_E_RANGE;
  const int L = (x->logq + 31) / 32;
  if (ct_overlap(out, L, x, L)) return FHE_E_INVAL;
  if (x->cnum > 0) {
    rc = fhe_key_switch(c, k, x->logN, x->logq, x->c0, x->c1, out->c0, out->c1, x->cnum, stream);
    if (rc != FHE_OK) return rc;
  }
  ct_meta(out, x, x->logq, x->logp, x->gamma);
  return FHE_OK;
}

int fhe_ct_leftrotate(fhe_ctx* c, fhe_evk* k, int r, const fhe_ct* x, fhe_ct* out, void* stream) {
  if (!k || !x || r < 0) return FHE_E_INVAL;
  if (check_logN(x->logN) != FHE_OK) return FHE_E_RANGE;
  if (k->g != (uint32_t)powmod(5, (uint64_t)r, 2ull << x->logN)) return FHE_E_STATE;
  return fhe_ct_key_switch(c, k, x, out, stream);
}

int fhe_ct_conjugate(fhe_ctx* c, fhe_evk* k, const fhe_ct* x, fhe_ct* out, void* stream) {
  if (!k || !x) return FHE_E_INVAL;
  if (check_logN(x->logN) != FHE_OK) return FHE_E_RANGE;
  if (k->g != (2u << x->logN) - 1u) return FHE_E_STATE;
  return fhe_ct_key_switch(c, k, x, out, stream);
}

}  // extern "C"
