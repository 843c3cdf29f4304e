// C ABI of libbmlp (declared in include/bmlp.h) and the host fixpoint drivers
// of the BMLP algorithms.  Host code only: every step of the computation runs
// in the kernels of k_bits.hip, k_gemm.hip and k_smp.hip.
#include <hip/hip_runtime.h>

#include <dlfcn.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bmlp.h"
#include "bmlp_batch.h"
#include "bmlp_mlp.h"
#include "bmlp_internal.h"
#include "rms_cost.h"
#include "features.h"

using namespace bmlp;

namespace {

thread_local std::string g_last_error;

struct Fail {
  bmlp_status st;
};

[[noreturn]] void fail(bmlp_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  throw Fail{st};
}

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(BMLP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

struct bmlp_ctx {
  int device = 0;
  static constexpr int kSlots = 22;
  void* slot[kSlots] = {};
  size_t slot_bytes[kSlots] = {};
  u32* d_flags = nullptr;  // device flags / counters
  unsigned char* scratch = nullptr;  // this device's address of the file-scope scratch array (bmlp_smp_noalloc)
  u32* h_flags = nullptr;  // pinned host mirror
  hipEvent_t ev0 = nullptr, ev1 = nullptr, evp0 = nullptr, evp1 = nullptr;
  // timed products awaiting their readback (statistics): event pairs and matrix-core work counters
  static constexpr int kPend = 64;
  hipEvent_t pe0[kPend] = {}, pe1[kPend] = {};
  unsigned long long* d_exec = nullptr;  // kPend counters on the device
  unsigned long long* h_exec = nullptr;  // pinned mirror
  // batched launch: the captured kernel chain, reused while the batch is unchanged
  hipStream_t capture_stream = nullptr;
  hipGraph_t bgraph = nullptr;
  hipGraphExec_t bexec = nullptr;
  uint64_t bkey = 0;
  // dispatcher model on the device: params (5,508) | mu (16) | sd (16); host copy beside it
  float* d_model = nullptr;
  bool model = false;
  std::vector<float> h_model;
  bmlp_trace* trace = nullptr;
  // autotuned tile code per (tuned kernel, bucket): a candidate index, or -1 for the built-in default
  static constexpr int kTuneKernels = 2, kTuneBuckets = 16;
  int32_t tune[kTuneKernels][kTuneBuckets];
  float tune_ms[kTuneKernels][kTuneBuckets];
};

namespace {

// ------------------------------------------------------------ allocation-free selection
// bmlp_smp_noalloc builds the relation's edge index in this file-scope device array instead of the
// handle's workspace.  Each device the library runs on holds its own copy until the process ends; host
// code never uses the array's name as an address (it is a host-side stand-in): bmlp_create looks up the
// device address once per device with hipGetSymbolAddress and keeps it.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_dev[kMaxScratchDevices] = {};

// The scratch array's address on `device`, which must be the current device.  Null if it cannot be found.
unsigned char* scratch_address(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_dev[device] = (unsigned char*)p;
  }
  return g_scratch_dev[device];
}

// Kernels with autotuned tile code (bmlp_ctx::tune): the matrix-core product, the VALU product.
enum TuneKernel { TK_MFMA = 0, TK_VALU = 1 };

// Slots of the handle's small device flag buffer (and its pinned host mirror), in 32-bit words.
enum FlagSlot {
  F_CHANGED = 0,   // change flag of the current product / round
  F_PAD = 1,       // padding check
  F_ROUNDS = 2,    // rounds of the one-launch sparse selection
  F_COO = 3,       // out-of-range fact in packing
  F_CNT = 4,       // 64-bit bit count
  F_NEW = 6,       // 64-bit count of new bits of a round
  F_DEC = 8,       // dispatcher decision
  F_PRED = 12,     // 4 predicted log times
  F_FEAT = 16,     // 16 features
  F_GSTATS = 32,   // 3 x 64-bit graph statistics
  F_EXEC = 40,     // 64-bit count of matrix-core ops issued by a timed product
  F_LIST = 44,     // length of a device row list
  F_QUEUE = 46,    // 64-bit piece counter of the gathers' overflow queue
  F_ROUNDS_OUT = 48,  // host side only: a one-launch selection's round count, read at the end of the call
  F_TOT0 = 50,        // host side only: the first running bit count of an RMS chain, uploaded from here
  F_DEFER = 54,       // an out-of-range fact given to bmlp_pack_coo_async (latched until bmlp_deferred_error)
  F_VBITS = 56,       // 64-bit count of a gather's query-row bits, from which the device sizes its pieces
  F_RELABEL = 58,     // 9 x 64-bit: the relabelling's class counts (k_relabel_classes)
  F_CHAIN = 128,      // BMLP-RMS: one record of kRmsRecWords words per squaring (rms_core)
  F_WORDS = 512
};
constexpr int kChainRecords = (F_WORDS - F_CHAIN) / kRmsRecWords;

// S_RD .. S_RL: the semi-naive squarings of rms_core (delta, its row-list, the column gather and the rows;
// the transposed route also takes S_RA, S_RX and S_BT for D^T, R^T and the gathered product); S_GQ: the
// overflow queue of the row gathers; S_RPT, S_CIT: the CSC (in-edges) of the one-launch selection (through
// R^T in S_BT for a dense relation); S_PERM: a relabelling of the nodes and its inverse (rms_core); S_QV: the
// query rows of a session query given by its source indices
enum Slot { S_W0 = 0, S_W1, S_W2, S_W3, S_W4, S_DEG, S_RP, S_CI, S_T0, S_T1, S_T2, S_BT, S_BATCH, S_RD, S_RA, S_RX, S_RL,
            S_GQ, S_RPT, S_CIT, S_PERM, S_QV };

// Restores the caller's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    hip_check(hipSetDevice(dev), "hipSetDevice");
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

size_t ws_total(const bmlp_ctx* c) {
  size_t t = 0;
  for (int i = 0; i < bmlp_ctx::kSlots; ++i) t += c->slot_bytes[i];
  return t;
}

void* ws(bmlp_ctx* c, int s, size_t bytes, const bmlp_opts& o) {
  bytes = (bytes + 255) & ~(size_t)255;
  if (bytes == 0) bytes = 256;
  if (c->slot_bytes[s] >= bytes) return c->slot[s];
  if (o.workspace_limit > 0 && ws_total(c) - c->slot_bytes[s] + bytes > (size_t)o.workspace_limit)
    fail(BMLP_ENOMEM, "workspace would exceed limit (%lld bytes)", (long long)o.workspace_limit);
  if (c->slot[s]) {
    hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
    hip_check(hipFree(c->slot[s]), "hipFree");
    c->slot[s] = nullptr;
    c->slot_bytes[s] = 0;
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    fail(BMLP_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
  }
  c->slot[s] = p;
  c->slot_bytes[s] = bytes;
  return p;
}

u64* ws_bits(bmlp_ctx* c, int s, i64 rows, i64 ld, const bmlp_opts& o) {
  return (u64*)ws(c, s, (size_t)std::max<i64>(rows * ld, 1) * sizeof(u64), o);
}

// The overflow queue for a gather of k rows of n bits (heavy rows split over waves), or none when it
// would take the workspace past the caller's limit.
GatherQueue gather_queue(bmlp_ctx* c, i64 k, i64 n, const bmlp_opts& o) {
  GatherQueue q{nullptr, nullptr, 0};
  if (words_for(n) > 256) return q;  // the wide-row gather kernel takes no queue
  const i64 cap = gather_queue_capacity(k, n);
  const size_t bytes = ((size_t)std::max<i64>(cap, 1) * sizeof(int2) + 255) & ~(size_t)255;
  if (c->slot_bytes[S_GQ] < bytes && o.workspace_limit > 0 &&
      ws_total(c) - c->slot_bytes[S_GQ] + bytes > (size_t)o.workspace_limit)
    return q;
  q.e = (int2*)ws(c, S_GQ, bytes, o);
  q.n = (unsigned long long*)(c->d_flags + F_QUEUE);
  q.cap = cap;
  q.piece = 64;
  return q;
}

// The queue for a gather whose query rows hold `bits` set bits over `rows` rows: only rows beyond twice
// the mean are split (splitting rows of about the mean size buys no balance and costs the atomics).
GatherQueue sized(GatherQueue q, i64 bits, i64 rows) {
  const i64 mean = bits / std::max<i64>(rows, 1);
  q.piece = (int)std::min<i64>(std::max<i64>(64, 2 * mean), 1 << 24);
  return q;
}

bmlp_opts opts_or_default(const bmlp_opts* o) {
  bmlp_opts d;
  bmlp_opts_init(&d);
  if (!o) return d;
  if (o->size != sizeof(bmlp_opts)) fail(BMLP_EINVAL, "bmlp_opts.size mismatch (%u != %zu)", o->size, sizeof(bmlp_opts));
  return *o;
}

// ------------------------------------------------------------ validation
void need(bool c, bmlp_status st, const char* fmt, ...) {
  if (c) return;
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  throw Fail{st};
}

void check_bits_arg(const void* p, const char* name, i64 rows, i64 cols, i64 ld) {
  need(rows >= 0 && cols >= 0, BMLP_EINVAL, "%s: negative size", name);
  need(ld >= words_for(cols), BMLP_EINVAL, "%s: ld %lld < ceil(%lld/64)", name, (long long)ld, (long long)cols);
  if (rows == 0 || ld == 0) return;
  need(p != nullptr, BMLP_EINVAL, "%s: null pointer", name);
  need(((uintptr_t)p & 7u) == 0, BMLP_EALIGN, "%s: not 8-byte aligned", name);
}

struct Range {
  uintptr_t lo, hi;
};
Range range_of(const void* p, i64 rows, i64 ld) {
  uintptr_t lo = (uintptr_t)p;
  return {lo, lo + (uintptr_t)(rows * ld) * sizeof(u64)};
}
bool overlap(Range a, Range b) { return a.lo < b.hi && b.lo < a.hi && a.hi > a.lo && b.hi > b.lo; }

void check_padding(bmlp_ctx* c, const u64* a, i64 rows, i64 n, i64 ld, hipStream_t s, const char* name) {
  hip_check(hipMemsetAsync(c->d_flags + 1, 0, sizeof(u32), s), "hipMemsetAsync");
  hip_check(launch_check_pad(a, rows, n, ld, c->d_flags + 1, s), "check_pad");
  hip_check(hipMemcpyAsync(c->h_flags + 1, c->d_flags + 1, sizeof(u32), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
  hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
  need(c->h_flags[1] == 0, BMLP_EPAD, "%s: nonzero padding bits (columns >= %lld)", name, (long long)n);
}

// ------------------------------------------------------------ stats
struct StatsRec {
  bmlp_stats* st;
  bmlp_ctx* c;
  hipStream_t s;
  const bmlp_opts* o = nullptr;  // options of the call (workspace limit)
  explicit StatsRec(bmlp_stats* st_, bmlp_ctx* c_, hipStream_t s_, const bmlp_opts* o_ = nullptr)
      : st(st_), c(c_), s(s_), o(o_) {
    if (!st) return;
    std::memset(st, 0, sizeof *st);
    for (int i = 0; i < 64; ++i) st->arm_trace[i] = -1;
    hip_check(hipEventRecord(c->ev0, s), "hipEventRecord");
  }
  void trace(int round, int arm) {
    if (st && round >= 0 && round < 64) st->arm_trace[round] = arm;
  }
  // The timed products of a call are read back together (at the end of the call, or when kPend of them
  // are waiting), so that timing a product adds no host synchronisation of its own.
  struct Pending {
    i64 m, k, n;
    int arm;
    int kind;   // 0 a product, 1 a squaring by row gathers
    i64 bytes;  // a gather squaring's algorithmic bytes (-1 until known)
    bool valid; // false once cancelled: it was enqueued ahead and its predicate was off
  };
  Pending pend[bmlp_ctx::kPend];
  int npend = 0;
  void pool() {
    if (c->d_exec) return;
    for (int i = 0; i < bmlp_ctx::kPend; ++i) {
      hip_check(hipEventCreate(&c->pe0[i]), "hipEventCreate");
      hip_check(hipEventCreate(&c->pe1[i]), "hipEventCreate");
    }
    hip_check(hipHostMalloc((void**)&c->h_exec, bmlp_ctx::kPend * sizeof(unsigned long long), hipHostMallocDefault),
              "hipHostMalloc");
    hip_check(hipMalloc((void**)&c->d_exec, bmlp_ctx::kPend * sizeof(unsigned long long)), "hipMalloc");
  }
  // counter of matrix-core work for the next timed product (null when no statistics are kept)
  unsigned long long* exec_counter() {
    if (!st) return nullptr;
    pool();
    return c->d_exec + npend;
  }
  void product_begin() {
    if (!st) return;
    pool();
    if (npend == bmlp_ctx::kPend) flush();  // a full batch is read back before the next product is timed
    // the counters of a batch are cleared together before its first product and copied back together
    if (npend == 0)
      hip_check(hipMemsetAsync(c->d_exec, 0, bmlp_ctx::kPend * sizeof(unsigned long long), s), "hipMemsetAsync");
    hip_check(hipEventRecord(c->pe0[npend], s), "hipEventRecord");
  }
  void product(i64 m, i64 k, i64 n, int arm) {
    if (!st) return;
    hip_check(hipEventRecord(c->pe1[npend], s), "hipEventRecord");
    pend[npend++] = Pending{m, k, n, arm, 0, 0, true};
  }
  // A squaring by row gathers, timed like a product.  gather_begin keeps room for it and the dense product
  // enqueued beside it, so that both are still pending when the route is read back.  Returns its index
  // (-1 without statistics).
  int gather_begin() {
    if (!st) return -1;
    if (npend + 2 > bmlp_ctx::kPend) flush();
    product_begin();
    return npend;
  }
  void gather_end(int idx, i64 bytes) {
    if (!st || idx < 0) return;
    hip_check(hipEventRecord(c->pe1[npend], s), "hipEventRecord");
    pend[npend++] = Pending{0, 0, 0, BMLP_ARM_PRODUCT_GATHER, 1, bytes, true};
  }
  void set_bytes(int idx, i64 bytes) {
    if (st && idx >= 0 && idx < npend) pend[idx].bytes = bytes;
  }
  void cancel(int idx) {
    if (st && idx >= 0 && idx < npend) pend[idx].valid = false;
  }
  // forget the last timed product: it was enqueued ahead under a device-side condition that did not hold,
  // so it ran no work.  Batches are read back before the next timed launch, so it is still pending.
  void cancel_last() {
    if (st && npend > 0) pend[npend - 1].valid = false;
  }
  void flush() {
    if (!st || npend == 0) return;
    hip_check(hipMemcpyAsync(c->h_exec, c->d_exec, (size_t)npend * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                             s),
              "hipMemcpyAsync");
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    for (int i = 0; i < npend; ++i) {
      const Pending& p = pend[i];
      if (!p.valid) continue;
      float ms = 0.f;
      hip_check(hipEventElapsedTime(&ms, c->pe0[i], c->pe1[i]), "hipEventElapsedTime");
      if (p.kind == 1) {
        if (p.bytes < 0) continue;
        st->gathers += 1;
        st->gather_ms += ms;
        st->gather_bytes += (uint64_t)p.bytes;
        continue;
      }
      const uint64_t ops = (uint64_t)2 * (uint64_t)p.m * (uint64_t)p.k * (uint64_t)p.n;
      st->products += 1;
      st->bool_ops += ops;
      st->product_bool_ops += ops;
      st->product_ms += ms;
      if (p.arm == BMLP_ARM_PRODUCT_MFMA) {
        st->products_mfma += 1;
        st->product_bool_ops_mfma += ops;
        st->product_ms_mfma += ms;
        st->mfma_ops_issued += c->h_exec[i];
      }
      st->bytes_moved += (uint64_t)(p.m * words_for(p.k) + p.k * words_for(p.n) + 2 * p.m * words_for(p.n)) * 8u;
    }
    npend = 0;
  }
  // a one-launch selection's round count, copied back with the end-of-call readback
  i64 rounds_n = -1;
  int rounds_arm = 0;
  void defer_rounds(i64 n, int arm) {
    if (!st) return;
    hip_check(hipMemcpyAsync(c->h_flags + F_ROUNDS_OUT, c->d_flags + F_ROUNDS, sizeof(u32), hipMemcpyDeviceToHost,
                             s),
              "hipMemcpyAsync");
    rounds_n = n;
    rounds_arm = arm;
  }
  void finish() {
    if (!st) return;
    flush();
    hip_check(hipEventRecord(c->ev1, s), "hipEventRecord");
    hip_check(hipEventSynchronize(c->ev1), "hipEventSynchronize");
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, c->ev0, c->ev1), "hipEventElapsedTime");
    st->device_ms = ms;
    if (rounds_n >= 0) {
      const u32 rounds = c->h_flags[F_ROUNDS_OUT];
      need((i64)rounds <= rounds_n + 2, BMLP_EITER, "SMP exceeded the round cap");
      st->iterations = (int32_t)rounds;
      for (u32 r = 0; r < rounds && r < 64; ++r) trace((int)r, rounds_arm);
      rounds_n = -1;
    }
  }
};

// ------------------------------------------------------------ helpers
void zero_flag(bmlp_ctx* c, hipStream_t s) {
  hip_check(hipMemsetAsync(c->d_flags, 0, sizeof(u32), s), "hipMemsetAsync");
}
u32 read_flag(bmlp_ctx* c, hipStream_t s, int idx = 0) {
  hip_check(hipMemcpyAsync(c->h_flags + idx, c->d_flags + idx, sizeof(u32), hipMemcpyDeviceToHost, s),
            "hipMemcpyAsync");
  hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
  return c->h_flags[idx];
}

// transpose of B (K x N) into the S_BT workspace, for the MFMA arm
const u64* transpose_b(bmlp_ctx* c, const u64* B, i64 ldb, i64 K, i64 N, const bmlp_opts& o, hipStream_t s,
                       i64* ldbt, const u32* pred = nullptr, u32 pred_val = 0) {
  *ldbt = std::max<i64>(words_for(K), 1);
  *ldbt += *ldbt & 1;  // even, so that rows are 16-byte aligned (the tile codes that load 16-byte pieces)
  u64* bt = ws_bits(c, S_BT, N, *ldbt, o);
  hip_check(launch_transpose(B, K, N, ldb, bt, *ldbt, s, pred, pred_val), "transpose");
  return bt;
}

// ------------------------------------------------------------ autotuned tile code
// Buckets of a product (M x K).(K x N): four sizes by the dense operation count 2 M K N (up to about
// 2 x 2,048^3, 2 x 4,096^3, 2 x 8,192^3, beyond) times four classes of the left operand: bits below
// 1/4,096 (words of k often zero across a whole row block, skipped), below 1/64, denser or not known,
// and block-structured (the squarings of a relabelled relation, whose bits crowd into one corner).
int tune_bucket(i64 M, i64 K, i64 N, double density, bool structured = false) {
  const double ops = 2.0 * (double)M * (double)K * (double)N;
  const int sb = ops < 3.4e10 ? 0 : ops < 2.7e11 ? 1 : ops < 2.2e12 ? 2 : 3;
  const int db = structured ? 3 : density < 0.0 ? 2 : density < 1.0 / 4096.0 ? 0 : density < 1.0 / 64.0 ? 1 : 2;
  return 4 * sb + db;
}
// Candidates the autotuner chooses among, and the built-in defaults (measured on MI355X at n = 16,384)
constexpr int kTuneCandidates[bmlp_ctx::kTuneKernels] = {kMfmaVariants, kValuVariants};
static_assert(kMfmaVariants <= BMLP_TUNE_MAX_CANDIDATES && kValuVariants <= BMLP_TUNE_MAX_CANDIDATES,
              "the tuning report holds BMLP_TUNE_MAX_CANDIDATES candidates per bucket");
constexpr int kTuneDefault[bmlp_ctx::kTuneKernels] = {0, 0};
int tuned_variant(const bmlp_ctx* c, int kernel, i64 M, i64 K, i64 N, double density, bool structured = false) {
  const int v = c->tune[kernel][tune_bucket(M, K, N, density, structured)];
  return v >= 0 ? v : kTuneDefault[kernel];
}

// One Boolean product C = Cold | A.B (D, changed optional) with the chosen arm.  The MFMA arm reads B
// transposed: pass BT when the caller has it, else B is transposed into workspace first.
// `density`: the fraction of set bits of A when the caller knows it (else -1); with `structured` (A is a
// relabelled, block-structured relation) it picks the tuned tile code.  `early` (or a nonzero *early_flag
// on the device): A.B likely saturates within the first chunk of k (a squaring of a dense relation,
// rms_early_votes), so the matrix-core tiles vote before loading ahead.
void product(bmlp_ctx* c, const u64* A, i64 lda, const u64* B, i64 ldb, const u64* Cold, i64 ldco, u64* C, i64 ldc,
             u64* D, i64 ldd, i64 M, i64 K, i64 N, u32* changed, int arm, hipStream_t s, StatsRec& sr,
             const u64* BT = nullptr, i64 ldbt = 0, unsigned long long* newbits = nullptr, double density = -1.0,
             bool structured = false, const u32* pred = nullptr, u32 pred_val = 0, const u32* early_flag = nullptr,
             bool early = false) {
  GemmArgs g{A, lda, B, ldb, Cold, ldco, C, ldc, D, ldd, M, K, N, changed};
  g.executed = sr.exec_counter();
  g.newbits = newbits;
  g.early_flag = early_flag;
  g.early = early;
  g.pred = pred;  // with pred, the product (and the transpose it needs) runs only when *pred == pred_val
  g.pred_val = pred_val;
  if (arm == BMLP_ARM_PRODUCT_MFMA) {
    bmlp_opts dflt;
    bmlp_opts_init(&dflt);
    if (!BT) BT = transpose_b(c, B, ldb, K, N, sr.o ? *sr.o : dflt, s, &ldbt, pred, pred_val);
    sr.product_begin();
    hip_check(launch_gemm_mfma(g, BT, ldbt, s, tuned_variant(c, TK_MFMA, M, K, N, density, structured)), "gemm_mfma");
  } else {
    sr.product_begin();
    hip_check(launch_gemm_valu(g, s, tuned_variant(c, TK_VALU, M, K, N, density, structured)), "gemm_valu");
  }
  sr.product(M, K, N, arm);
}

int ceil_log2(i64 x) {
  int r = 0;
  while (((i64)1 << r) < x) ++r;
  return r;
}

// Plain choice of the product kernel for an (M x K).(K x N) product: the matrix-core arm once both
// output dimensions fill its 256 x 256 workgroup tiles (measured faster from n = 4,096 up) and K is
// within its exact int32 range, the bit-packed VALU arm (which also splits K) for thin or small products.
int product_arm(const bmlp_opts& o, i64 M, i64 N, i64 K) {
  if (o.product_arm == BMLP_ARM_PRODUCT_MFMA)
    need(words_for(K) <= gemm_mfma_max_kwords(), BMLP_EINVAL, "the MFMA product arm supports K <= %lld",
         (long long)(64 * gemm_mfma_max_kwords()));
  if (o.product_arm == BMLP_ARM_PRODUCT_VALU || o.product_arm == BMLP_ARM_PRODUCT_MFMA) return o.product_arm;
  // The matrix cores pay from K = 512 on: below it the tile's fixed staging and epilogue dominate
  // (measured at M = N = 14,541: K = 64, 256, 512 took 30, 93, 159 us on the VALU kernel and 98,
  // 108, 136 us on the matrix cores).
  return (M >= 1024 && N >= 1024 && K >= 512 && words_for(K) <= gemm_mfma_max_kwords()) ? BMLP_ARM_PRODUCT_MFMA
                                                                                          : BMLP_ARM_PRODUCT_VALU;
}

i64 count_bits(bmlp_ctx* c, const u64* R, i64 rows, i64 n, i64 ld, hipStream_t s);

// The cost model of the squarings (rms_cost.h) with the gather kernel's size limit
bool rms_gather_pays(i64 n, i64 bits, int arm) {
  return bmlp::rms_gather_pays(n, bits, arm == BMLP_ARM_PRODUCT_MFMA, gather_rows_max_n());
}
SemiCost rms_semi_cost(i64 n, i64 dbits, int arm) { return bmlp::rms_semi_cost(n, dbits, arm == BMLP_ARM_PRODUCT_MFMA); }

struct GraphInfo {
  i64 n = 0, m = 0, maxdeg = 0, nonempty = 0;
  // the per-row counts graph_info left in the S_DEG workspace: valid only until that slot is reused, so
  // only the code that called graph_info just before may hand them on (Csr::deg)
  const int32_t* deg = nullptr;
};

// Algorithmic bytes of a squaring of an n x n R with `bits` set bits by row gathers: the n rows of R read as
// query rows, one source row read per set bit, the n rows of the result written (n / 8 bytes a row).
i64 gather_bytes(i64 n, i64 bits) { return (2 * n + bits) * ((n + 7) / 8); }

// Up to this n the statistics come from the per-row counts (one pass that fills the whole GPU, plus a
// one-workgroup reduction over n counts, 9 us at n = 16,384 against 17 us for the combined pass); the
// counts stay in S_DEG, where a CSR build that follows can take them.
constexpr i64 kDegStatsMaxN = 262144;

GraphInfo graph_info(bmlp_ctx* c, const u64* R, i64 ld, i64 n, const bmlp_opts& o, hipStream_t s) {
  GraphInfo g;
  g.n = n;
  if (n <= 0) return g;
  unsigned long long* out = (unsigned long long*)(c->d_flags + F_GSTATS);
  if (n <= kDegStatsMaxN) {
    int32_t* deg = (int32_t*)ws(c, S_DEG, (size_t)n * sizeof(int32_t), o);
    hip_check(launch_row_popcount(R, n, n, ld, deg, nullptr, s), "row_popcount");
    hip_check(launch_deg_stats(deg, n, out, s), "deg_stats");
    g.deg = deg;
  } else {
    hip_check(hipMemsetAsync(out, 0, 3 * sizeof(unsigned long long), s), "hipMemsetAsync");
    hip_check(launch_graph_stats(R, n, n, ld, out, s), "graph_stats");
  }
  hip_check(hipMemcpyAsync(c->h_flags + F_GSTATS, out, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s),
            "memcpy");
  hip_check(hipStreamSynchronize(s), "sync");
  unsigned long long v[3];
  std::memcpy(v, c->h_flags + F_GSTATS, sizeof v);
  g.m = (i64)v[0];
  g.maxdeg = (i64)v[1];
  g.nonempty = (i64)v[2];
  return g;
}

// Relabelling before the dense squarings.  Where a relation's closure is one big block -- the rows that
// reach a giant strongly connected part times the columns it reaches, the sparse random digraphs just
// above the percolation threshold -- the block is spread over every 256 x 256 output tile in the given
// node order, so no tile is all ones (copied), saturates early or has all-zero rows (skipped).  With the
// nodes ordered by class (heavy row and light column, heavy both, light row and heavy column, light
// both; heavy = at least a quarter of the largest popcount) the block becomes a few contiguous
// rectangles.  The squarings are the same up to the relabelling, (P R P^T)^2 = P R^2 P^T, and the
// closure is mapped back at the end.  Relabels when the rows or the columns split into the two classes
// with at least 2% heavy and 10% light.
//
// Failing that, the few dead nodes of a denser relation (a row or a column with almost no bits: out- or
// in-degree 0 in a random digraph of mean degree 8 -- a handful of nodes) are moved to the end.  A 256 x
// 256 output tile with such a row or column never saturates, so it runs the whole K loop, and a few dead
// nodes scattered over the order touch a tenth of all tiles; gathered at the end they touch the last
// tile row and column only.  This is done when at most 2% of the nodes are dead and it frees at least
// 5% of the tiles.  Returns 1 for the classes, 2 for the dead nodes, 0 (nothing to gain) otherwise.
int rms_relabel(bmlp_ctx* c, const u64* cur, i64 ld, i64 n, const bmlp_opts& o, hipStream_t s, int32_t** perm_out,
                 int32_t** inv_out) {
  const i64 nw = words_for(n);
  int32_t* rowpop = (int32_t*)ws(c, S_DEG, (size_t)n * sizeof(int32_t), o);
  int32_t* colpop = (int32_t*)ws(c, S_RL, (size_t)n * sizeof(int32_t), o);
  u64* ct = ws_bits(c, S_BT, n, nw, o);
  hip_check(launch_row_popcount(cur, n, n, ld, rowpop, nullptr, s), "row_popcount");
  hip_check(launch_transpose(cur, n, n, ld, ct, nw, s), "transpose");
  hip_check(launch_row_popcount(ct, n, n, nw, colpop, nullptr, s), "row_popcount");
  // the classes are counted and the permutation formed on the device; the host reads the counts alone
  unsigned long long* sum = (unsigned long long*)(c->d_flags + F_RELABEL);
  hip_check(launch_relabel_classes(rowpop, colpop, n, sum, s), "relabel_classes");
  hip_check(hipMemcpyAsync(c->h_flags + F_RELABEL, sum, 7 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s),
            "memcpy");
  hip_check(hipStreamSynchronize(s), "sync");
  unsigned long long v[7];
  std::memcpy(v, c->h_flags + F_RELABEL, sizeof v);
  const i64 rmax = (i64)v[0], cmax = (i64)v[1], hin = (i64)v[2], hout = (i64)v[3], dead = (i64)v[4];
  const i64 drt = (i64)v[5], dct = (i64)v[6];
  if (rmax <= 0 || cmax <= 0) return 0;
  auto splits = [&](i64 h) { return h * 50 >= n && h * 10 <= 9 * n; };  // a light class of at least 10%
  int mode = 1;
  if (!splits(hin) && !splits(hout)) {
    // dead nodes: a row or a column with fewer than 1/64 of the largest count's bits
    const i64 tiles = (n + 255) / 256;
    const i64 dirty = drt * tiles + dct * tiles - drt * dct;  // tiles with a dead row or column now
    const i64 last = (n - 1) / 256 - (n - dead) / 256 + 1;     // tile rows the dead nodes take at the end
    const i64 after = 2 * last * tiles - last * last;
    if (dead == 0 || dead * 50 > n || (dirty - after) * 20 < tiles * tiles) return 0;
    mode = 2;
  }
  int32_t* d = (int32_t*)ws(c, S_PERM, (size_t)(2 * n) * sizeof(int32_t), o);
  hip_check(launch_relabel_perm(rowpop, colpop, n, mode, sum, d, d + n, s), "relabel_perm");
  *perm_out = d;
  *inv_out = d + n;
  return mode;
}

// R1+ into `out` (n x ldo) -- the RMS fixpoint driver shared by rms, the closure arm of smp and the RMS
// route of compose.  `R1` has leading dimension ld1.  With the product arm left to the library, each
// squaring of a still sparse R is done by row gathers (the bit count of R is kept from the kernels'
// new-bit counts).
void rms_core(bmlp_ctx* c, const u64* R1, i64 ld1, u64* out, i64 ldo, i64 n, const bmlp_opts& o, hipStream_t s,
              StatsRec& sr) {
  const i64 nw = words_for(n);
  const i64 ldi = nw;
  u64* cur = ws_bits(c, S_W0, n, ldi, o);
  u64* nxt = ws_bits(c, S_W1, n, ldi, o);
  const int arm = product_arm(o, n, n, n);
  hip_check(launch_ewise(4, R1, ld1, nullptr, 0, cur, ldi, n, n, s), "copy");
  if (o.rms_variant == 1) hip_check(launch_set_diag(cur, ldi, n, n, s), "set_diag");
  bool may_gather = o.product_arm == BMLP_ARM_AUTO && n <= gather_rows_max_n();
  const GraphInfo g0 = may_gather ? graph_info(c, cur, ldi, n, o, s) : GraphInfo{};
  i64 bits = g0.m;
  // Semi-naive squarings need D = R_t & ~R_{t-1}: it is formed at the start of a squaring (the other
  // buffer still holds R_{t-1}) when the new-bit count of the last squaring says it may pay.
  const bool may_semi = o.product_arm == BMLP_ARM_AUTO && n <= gather_rows_max_n() && n <= gather_cols_max_n();
  bool have_prev = false;
  i64 dbits = 0;
  const GatherQueue gq = may_gather ? gather_queue(c, n, n, o) : GatherQueue{nullptr, nullptr, 0};
  // relabel (once) before the first dense squaring on the matrix cores, when a tenth or more of the rows
  // are empty (a light class is certain) and the squarings are large enough to repay the passes over the
  // matrix (at n = 8,192 they do not); inv maps the closure back
  // relabel before the first dense squaring where R1 has empty rows: many (the block of a closure just above
  // the percolation threshold) or a few dead nodes (rms_relabel)
  bool may_relabel = may_gather && o.rms_variant == 0 && arm == BMLP_ARM_PRODUCT_MFMA && n >= 16384 &&
                     g0.nonempty < n;
  const int32_t* inv = nullptr;
  int relabel_mode = 0;  // rms_relabel: 1 block classes (the products are block-structured), 2 dead nodes
  const int cap = ceil_log2(std::max<i64>(n, 2)) + 2;
  // Squaring t records its new-bit count (and the device's running bit count and route) in record t of the
  // chain.  While the host reads squaring t's count back, squaring t + 1 is already queued: a one-thread
  // kernel picks its route from that count on the device (the rules below, rms_cost.h), and its row
  // gathers and its dense product are both enqueued, each running only when the route names it.  The
  // device thus never waits for the host between squarings that stay on those two routes; the semi-naive
  // form and the relabelling are left to the host (route "host"), which then runs the squaring itself.
  need(cap + 1 < kChainRecords, BMLP_EINVAL, "n too large for the squaring chain");
  u32* recs = c->d_flags + F_CHAIN;
  auto rec_nb = [&](int t) { return (unsigned long long*)(recs + (i64)t * kRmsRecWords); };
  hip_check(launch_fill_zero((u64*)recs, (i64)(F_WORDS - F_CHAIN) / 2, s), "fill_zero");
  if (g0.n == n) {
    // the running count starts from the bits of R1 (counted above)
    const unsigned long long m0 = (unsigned long long)g0.m;
    std::memcpy(c->h_flags + F_TOT0, &m0, sizeof m0);
    hip_check(hipMemcpyAsync(recs + 2, c->h_flags + F_TOT0, sizeof m0, hipMemcpyHostToDevice, s), "memcpy");
  }
  const bool mfma = arm == BMLP_ARM_PRODUCT_MFMA;
  int it = 0;
  u32 queued = RR_HOST;  // route of squaring `it` when it was enqueued ahead (gathers or dense), else RR_HOST
  int ahead_gather = -1; // the timing entry of the gathers enqueued ahead, until their route is known
  for (;;) {
    unsigned long long* nb = rec_nb(it);
    int tarm = arm;
    bool count_after = false;  // new bits = popcount of the result - bits of cur
    int semi = 0;              // semi-naive squaring: 0 none, 1 columns route, 2 transposed route
    if (queued == RR_GATHER) {
      if (sr.st) sr.st->bool_ops += (uint64_t)2 * (uint64_t)n * (uint64_t)n * (uint64_t)n;
      tarm = BMLP_ARM_PRODUCT_GATHER;
    } else if (queued != RR_DENSE) {
      // the host runs this squaring.  variant 0: R <- R | R.R ; variant 1: R' = R.R (I is in R, so
      // R | R.R = R.R).  R only grows, so once gathers stop paying they never pay again and the bit
      // count is no longer needed.
      may_gather = may_gather && rms_gather_pays(n, bits, arm);
      const bool gather = may_gather;  // the gathers count the new bits, which keeps `bits` exact
      u64* dl = nullptr;
      int32_t* list = nullptr;
      i64 drows = 0;
      if (!gather && may_semi && have_prev && dbits > 0) {
        const SemiCost sc = rms_semi_cost(n, dbits, arm);
        // D has at least ceil(dbits / n) nonempty rows
        const double cols_lb = rms_semi_cols_s(sc, (dbits + n - 1) / n);
        if (sc.common + std::min(sc.transposed, cols_lb) + kSemiOverheadS < sc.dense) {
          dl = ws_bits(c, S_RD, n, ldi, o);
          hip_check(launch_ewise(2, cur, ldi, nxt, ldi, dl, ldi, n, n, s), "andnot");
          semi = 2;
          if (cols_lb < sc.transposed) {
            list = (int32_t*)ws(c, S_RL, (size_t)n * sizeof(int32_t), o);
            hip_check(launch_fill_zero((u64*)(c->d_flags + F_LIST), 1, s), "fill_zero");
            hip_check(launch_nonempty_rows(dl, n, n, ldi, list, c->d_flags + F_LIST, s), "nonempty_rows");
            drows = (i64)read_flag(c, s, F_LIST);
            const double tc = rms_semi_cols_s(sc, drows);
            if (drows > 0 && tc < sc.transposed) semi = 1;
            if (sc.common + std::min(tc, sc.transposed) + kSemiOverheadS >= sc.dense) semi = 0;
          }
        }
      }
      if (gather) {
        const GatherQueue q = sized(gq, bits, n);
        const int gi = sr.gather_begin();
        hip_check(launch_gather_rows(cur, ldi, n, cur, ldi, n, 1, nxt, ldi, s, nullptr, nb, &q), "gather_rows");
        sr.gather_end(gi, gather_bytes(n, bits));
        if (sr.st) sr.st->bool_ops += (uint64_t)2 * (uint64_t)n * (uint64_t)n * (uint64_t)n;
        tarm = BMLP_ARM_PRODUCT_GATHER;
      } else if (semi == 1) {
        // nxt = cur | D.cur (rows of cur gathered over the bits of D), then nxt |= cur.D over the rows of D
        // with a bit: A = those columns of cur, X = those rows of D
        const i64 kw = words_for(drows);
        u64* am = ws_bits(c, S_RA, n, kw, o);
        u64* xm = ws_bits(c, S_RX, drows, ldi, o);
        hip_check(launch_ewise(4, cur, ldi, nullptr, 0, nxt, ldi, n, n, s), "copy");
        const GatherQueue q = sized(gq, dbits, n);
        hip_check(launch_gather_rows(dl, ldi, n, cur, ldi, n, 2, nxt, ldi, s, nullptr, nb, &q), "gather_rows");
        hip_check(launch_gather_cols(cur, ldi, n, n, list, drows, 0, am, kw, s), "gather_cols");
        hip_check(launch_copy_rows(dl, ldi, list, drows, n, xm, ldi, s), "copy_rows");
        product(c, am, kw, xm, ldi, nxt, ldi, nxt, ldi, nullptr, 0, n, drows, n, nullptr, product_arm(o, n, n, drows),
                s, sr, nullptr, 0, nb);
        if (sr.st) sr.st->bool_ops += (uint64_t)2 * (uint64_t)n * (uint64_t)n * (uint64_t)n;
        tarm = BMLP_ARM_PRODUCT_SEMINAIVE;
      } else if (semi == 2) {
        // cur.D = (D^T . cur^T)^T: rows of cur^T gathered over the bits of D^T and transposed back; then
        // nxt (R_{t-1} is no longer needed once D is formed) = cur | cur.D, and nxt |= D.cur
        u64* dt = ws_bits(c, S_RX, n, ldi, o);
        u64* ct = ws_bits(c, S_BT, n, ldi, o);
        u64* yt = ws_bits(c, S_RA, n, ldi, o);
        hip_check(launch_transpose(dl, n, n, ldi, dt, ldi, s), "transpose");
        hip_check(launch_transpose(cur, n, n, ldi, ct, ldi, s), "transpose");
        const GatherQueue q = sized(gq, dbits, n);
        hip_check(launch_gather_rows(dt, ldi, n, ct, ldi, n, 0, yt, ldi, s, nullptr, nullptr, &q), "gather_rows");
        hip_check(launch_transpose(yt, n, n, ldi, dt, ldi, s), "transpose");  // dt now holds cur.D
        hip_check(launch_ewise(0, dt, ldi, cur, ldi, nxt, ldi, n, n, s), "or");
        hip_check(launch_gather_rows(dl, ldi, n, cur, ldi, n, 2, nxt, ldi, s, nullptr, nullptr, &q), "gather_rows");
        hip_check(launch_popcount_total(nxt, n, n, ldi, nb, s), "popcount_total");
        count_after = true;
        if (sr.st) sr.st->bool_ops += (uint64_t)2 * (uint64_t)n * (uint64_t)n * (uint64_t)n;
        tarm = BMLP_ARM_PRODUCT_SEMINAIVE_T;
      } else {
        if (may_relabel) {
          may_relabel = false;
          int32_t* perm;
          int32_t* pinv;
          relabel_mode = rms_relabel(c, cur, ldi, n, o, s, &perm, &pinv);
          if (relabel_mode) {
            // P R P^T, from the R^T that rms_relabel left in S_BT: its rows gathered in the new order (P R^T),
            // transposed (R P^T), the rows gathered again -- two row gathers and a transpose cost half the
            // bit-level permutation.  R_{t-1} in nxt is not needed by a dense squaring.
            u64* ct = ws_bits(c, S_BT, n, ldi, o);
            hip_check(launch_copy_rows(ct, ldi, perm, n, n, nxt, ldi, s), "copy_rows");
            hip_check(launch_transpose(nxt, n, n, ldi, ct, ldi, s), "transpose");
            hip_check(launch_copy_rows(ct, ldi, perm, n, n, nxt, ldi, s), "copy_rows");
            std::swap(cur, nxt);
            inv = pinv;
          }
        }
        const double dens = g0.n == n ? (double)bits / ((double)n * (double)n) : -1.0;  // kept once counted
        product(c, cur, ldi, cur, ldi, cur, ldi, nxt, ldi, nullptr, 0, n, n, n, nullptr, arm, s, sr, nullptr, 0, nb,
                dens, relabel_mode == 1, nullptr, 0, nullptr, g0.n == n && rms_early_votes(n, bits));
      }
    }
    sr.trace(it, tarm);
    ++it;
    // enqueue squaring `it` ahead (it reads nxt and writes cur), unless this one was semi-naive (its count
    // is a total, not the new bits) or the cap is reached
    const bool ahead = semi == 0 && it < cap;
    if (ahead) {
      hip_check(launch_rms_decide(recs, it, n, mfma ? 1 : 0, may_gather ? 1 : 0, (may_semi && dbits >= 0) ? 1 : 0,
                                  may_relabel ? 0 : 1, gather_rows_max_n(), s),
                "rms_decide");
      const u32* route = recs + (i64)it * kRmsRecWords + 4;
      unsigned long long* nb2 = rec_nb(it);
      if (may_gather) {
        // the pieces are sized on the device from R_it's bit count, which the decision kernel has just
        // written into record it (the host's count is R_{it-1}'s)
        GatherQueue q = sized(gq, bits, n);
        q.bits = (const unsigned long long*)(recs + (i64)it * kRmsRecWords) + 1;
        ahead_gather = sr.gather_begin();
        hip_check(launch_gather_rows(nxt, ldi, n, nxt, ldi, n, 1, cur, ldi, s, nullptr, nb2, &q, route, RR_GATHER),
                  "gather_rows");
        sr.gather_end(ahead_gather, -1);  // its bytes are known once this squaring's count is read back
      }
      // the bit count of R_it is not known on the host yet: a squaring that falls to the dense product
      // counts as dense for the tuned tile code (sparser ones go to the gathers)
      // (the decision kernel also flags a dense R, whose tiles vote after their first chunk: rms_early_votes)
      product(c, nxt, ldi, nxt, ldi, nxt, ldi, cur, ldi, nullptr, 0, n, n, n, nullptr, arm, s, sr, nullptr, 0, nb2, -1.0,
              relabel_mode == 1, route, RR_DENSE, recs + (i64)it * kRmsRecWords + kRmsRecEarly);
    }
    // read back this squaring's count and, when the next one was enqueued, its route (one contiguous copy)
    const size_t words = ahead ? (size_t)kRmsRecWords + 5 : 2;
    hip_check(hipMemcpyAsync(c->h_flags + F_CHAIN + (i64)(it - 1) * kRmsRecWords, recs + (i64)(it - 1) * kRmsRecWords,
                             words * sizeof(u32), hipMemcpyDeviceToHost, s),
              "memcpy");
    hip_check(hipStreamSynchronize(s), "sync");
    unsigned long long added = 0;
    std::memcpy(&added, c->h_flags + F_CHAIN + (i64)(it - 1) * kRmsRecWords, sizeof added);
    if (count_after) {
      need((i64)added >= bits, BMLP_EDEVICE, "RMS bit count went down");
      added -= (unsigned long long)bits;
    }
    bits += (i64)added;
    dbits = (i64)added;
    have_prev = true;
    const bool changed = added != 0;
    // an all-ones R is its own square (the count is exact once R1's bits were counted)
    const bool full = g0.n == n && bits >= n * n;
    std::swap(cur, nxt);
    queued = ahead ? c->h_flags[F_CHAIN + (i64)it * kRmsRecWords + 4] : (u32)RR_HOST;
    if (ahead && queued != RR_DENSE) sr.cancel_last();  // the product enqueued ahead did not run
    if (ahead_gather >= 0) {
      // the gathers enqueued ahead square R_it, whose bit count is now known
      if (queued == RR_GATHER) sr.set_bytes(ahead_gather, gather_bytes(n, bits));
      else sr.cancel(ahead_gather);
      ahead_gather = -1;
    }
    if (!changed || full) break;
    need(queued != RR_STOP, BMLP_EDEVICE, "RMS: the device saw no new bits");
    if (ahead && queued != RR_GATHER) may_gather = false;  // the device found that gathers no longer pay
    need(it < cap, BMLP_EITER, "RMS exceeded %d products (n=%lld)", cap, (long long)n);
  }
  if (sr.st) sr.st->iterations = it;
  if (o.rms_variant == 1) {
    // Algorithm 1, last line: R2* = R2* R1
    product(c, cur, ldi, R1, ld1, nullptr, 0, out, ldo, nullptr, 0, n, n, n, nullptr, arm, s, sr);
  } else if (inv) {
    // back to the given labels, P^T C P: rows gathered by the inverse, transposed, gathered, transposed
    u64* t2 = ws_bits(c, S_BT, n, ldi, o);
    hip_check(launch_copy_rows(cur, ldi, inv, n, n, nxt, ldi, s), "copy_rows");
    hip_check(launch_transpose(nxt, n, n, ldi, t2, ldi, s), "transpose");
    hip_check(launch_copy_rows(t2, ldi, inv, n, n, nxt, ldi, s), "copy_rows");
    hip_check(launch_transpose(nxt, n, n, ldi, out, ldo, s), "transpose");
  } else {
    hip_check(launch_ewise(4, cur, ldi, nullptr, 0, out, ldo, n, n, s), "copy");
  }
  hip_check(launch_zero_pad(out, n, n, ldo, s), "zero_pad");
}

// CSR of the bit matrix R (n x n, ld) in workspace slots S_DEG/S_RP/S_CI.
// With m_known >= 0 (the number of set bits of R, counted by the caller) the size needs no readback.
// With deg_ready (R's per-row counts, already in S_DEG) the counting pass is skipped.
void build_csr(bmlp_ctx* c, const u64* R, i64 ld, i64 n, const bmlp_opts& o, hipStream_t s, i64** rp_out,
               int32_t** ci_out, i64* m_out = nullptr, i64 m_known = -1, const int32_t* deg_ready = nullptr) {
  int32_t* deg = (int32_t*)ws(c, S_DEG, (size_t)n * sizeof(int32_t), o);
  i64* rp = (i64*)ws(c, S_RP, (size_t)(n + 1) * sizeof(i64), o);
  if (deg_ready != deg) hip_check(launch_row_popcount(R, n, n, ld, deg, nullptr, s), "row_popcount");
  hip_check(launch_scan_rowptr(deg, n, rp, s), "scan");
  i64 m = m_known;
  if (m < 0) {
    // the scan's last entry is the number of set bits
    hip_check(hipMemcpyAsync(c->h_flags + 4, rp + n, sizeof(i64), hipMemcpyDeviceToHost, s), "memcpy");
    hip_check(hipStreamSynchronize(s), "sync");
    std::memcpy(&m, c->h_flags + 4, sizeof m);
  }
  int32_t* ci = (int32_t*)ws(c, S_CI, (size_t)std::max<i64>(m, 1) * sizeof(int32_t), o);
  hip_check(launch_bits_to_csr(R, n, n, ld, rp, ci, s), "bits_to_csr");
  *rp_out = rp;
  *ci_out = ci;
  if (m_out) *m_out = m;
}

// CSC of R (the in-edges) in S_RPT/S_CIT, R given as bits (R, ld) and as its CSR (rp, ci; m edges).  A
// sparse R is inverted from its CSR in O(n + m) with atomics; a denser one through R^T (formed in S_BT),
// whose passes over n^2 bits beat m contended atomics once m passes about n^2 / 480 (n = 16,384: 45 us
// against some 200 us at 2.7 M edges; n = 65,536 with 262,144 edges: 20 us against 0.7 ms).
void build_csc(bmlp_ctx* c, const u64* R, i64 ld, const i64* rp, const int32_t* ci, i64 n, i64 m,
               const bmlp_opts& o, hipStream_t s, i64** rpt_out, int32_t** cit_out) {
  int32_t* degt = (int32_t*)ws(c, S_DEG, (size_t)(n + 1) * sizeof(int32_t), o);
  i64* rpt = (i64*)ws(c, S_RPT, (size_t)(n + 1) * sizeof(i64), o);
  int32_t* cit = (int32_t*)ws(c, S_CIT, (size_t)std::max<i64>(m, 1) * sizeof(int32_t), o);
  if ((double)m * 480.0 < (double)n * (double)n) {
    int32_t* cursor = (int32_t*)ws(c, S_RL, (size_t)(n + 1) * sizeof(int32_t), o);
    hip_check(launch_csc_from_csr(rp, ci, n, m, degt, cursor, rpt, cit, s), "csc_from_csr");
  } else {
    const i64 nw = words_for(n);
    u64* rt = ws_bits(c, S_BT, n, nw, o);
    hip_check(launch_transpose(R, n, n, ld, rt, nw, s), "transpose");
    hip_check(launch_row_popcount(rt, n, n, nw, degt, nullptr, s), "row_popcount");
    hip_check(launch_scan_rowptr(degt, n, rpt, s), "scan");
    hip_check(launch_bits_to_csr(rt, n, n, nw, rpt, cit, s), "bits_to_csr");
  }
  *rpt_out = rpt;
  *cit_out = cit;
}

// The one-launch selection turns bottom-up in rounds whose frontier is large next to the unvisited set;
// below this mean out-degree such rounds are too rare to pay for the in-edge index.
constexpr double kBottomUpMinDegree = 4.0;

// number of set bits of a bit matrix (device popcount, one readback)
i64 count_bits(bmlp_ctx* c, const u64* R, i64 rows, i64 n, i64 ld, hipStream_t s) {
  unsigned long long* tot = (unsigned long long*)(c->d_flags + 4);
  hip_check(hipMemsetAsync(tot, 0, sizeof(unsigned long long), s), "hipMemsetAsync");
  hip_check(launch_popcount_total(R, rows, n, ld, tot, s), "popcount_total");
  hip_check(hipMemcpyAsync(c->h_flags + 4, tot, sizeof(unsigned long long), hipMemcpyDeviceToHost, s), "memcpy");
  hip_check(hipStreamSynchronize(s), "sync");
  unsigned long long m = 0;
  std::memcpy(&m, c->h_flags + 4, sizeof m);
  return (i64)m;
}

// Plain schedule for the selection, from a timing sweep of the two arms on random digraphs with
// n = 4,096, 16,384 and 65,536, mean out-degree 1.6 .. 164 and k = 1 .. 1,024 query rows.  The
// one-launch sparse arm turns bottom-up once the frontier is large, so its time hardly grows with the
// degree; what it pays up front is the edge index (CSR, and CSC from degree 4), which grows with n.
// It wins whenever 64 or more rows share the launch (n = 65,536, degree 40, k = 1,024: 1.3 ms against
// 7.9 dense; n = 16,384, degree 164: 0.22 against 0.60) and at every k while the degree is low.  A few
// rows of a moderately dense relation are served faster by the dense rounds: at n = 16,384 for degree
// 30 .. 128 below k = 16 (degree 82, k = 1: 0.23 ms dense, 0.28 sparse; at degree 164 the hubs' bit rows
// make the sparse arm faster again, 0.19 against 0.23), and above that size from degree 12 below k = 16
// and from degree 30 below k = 64 (n = 65,536, degree 40, k = 16: 0.88 against 1.09).  At n = 4,096 the
// sparse arm wins nearly everywhere.
int smp_plain_arm(i64 n, i64 k, i64 m) {
  if (n > smp_rows_max_n()) return BMLP_ARM_SMP_DENSE;
  const double deg = n > 0 ? (double)m / (double)n : 0.0;
  if (k >= 64 || n <= 4096) return BMLP_ARM_SMP_SPARSE;
  if (n <= 16384) return (k >= 16 || deg < 30.0 || deg >= 128.0) ? BMLP_ARM_SMP_SPARSE : BMLP_ARM_SMP_DENSE;
  return (deg < 12.0 || (deg < 30.0 && k >= 16)) ? BMLP_ARM_SMP_SPARSE : BMLP_ARM_SMP_DENSE;
}

// ------------------------------------------------------------ dispatcher features

// The 16 dispatcher features (features.h), all O(1) from counters the drivers keep
void make_features(float* f, const GraphInfo& g, i64 k, int compose, int call_level, int round, double delta,
                   double prev_delta, double vis, int reflexive) {
  bmlp::make_features(f, (double)g.n, (double)g.m, (double)g.maxdeg, (double)g.nonempty, (double)k,
                      compose ? 1.f : 0.f, call_level, round, delta, prev_delta, vis, reflexive);
}

struct Csr {
  const i64* rp = nullptr;
  const int32_t* ci = nullptr;
  const i64* rpt = nullptr;  // CSC (in-edges), optional
  const int32_t* cit = nullptr;
  const int32_t* deg = nullptr;  // without rp: R1's per-row counts already in S_DEG (GraphInfo::deg, same call)
};

// model inference for one feature vector on the device; returns the chosen output index
int model_decide(bmlp_ctx* c, const float* f, u32 allowed, hipStream_t s, float* pred_out) {
  std::memcpy(c->h_flags + F_FEAT, f, kIn * sizeof(float));
  hip_check(hipMemcpyAsync(c->d_flags + F_FEAT, c->h_flags + F_FEAT, kIn * sizeof(float), hipMemcpyHostToDevice, s),
            "memcpy");
  hip_check(launch_mlp_decide(c->d_model, c->d_model + kParams, c->d_model + kParams + kIn,
                              (const float*)(c->d_flags + F_FEAT), (float*)(c->d_flags + F_PRED), c->d_flags + F_DEC,
                              allowed, s),
            "mlp_decide");
  hip_check(hipMemcpyAsync(c->h_flags + F_DEC, c->d_flags + F_DEC, 8 * sizeof(u32), hipMemcpyDeviceToHost, s),
            "memcpy");
  hip_check(hipStreamSynchronize(s), "sync");
  if (pred_out) std::memcpy(pred_out, c->h_flags + F_PRED, 4 * sizeof(float));
  return (int)c->h_flags[F_DEC];
}

enum RoundMode { RM_DENSE = 0, RM_SPARSE = 1, RM_LEARNED = 2 };

// The selection by semi-naive rounds: the selection of Eq. 5 pushed into the sum (v R1, v R1^2, ...),
// with every new bit expanded exactly once.  State in global memory: the frontier fr (k x nw) and the
// visited set vis, kept in Vstar.  Round: nxt = fr . R1, fr' = nxt & ~vis, vis |= fr'; it stops when
// fr' is empty (Algorithm 2's v* = v' test, the iterates being monotone).  The state is the same
// whichever arm serves a round, so each round may be served by the dense product or by sparse-frontier
// expansion; in learned mode the model chooses on the device, round by round.
void smp_rounds(bmlp_ctx* c, const u64* R1, i64 ld, i64 n, const u64* V, u64* Vstar, i64 k, i64 ldv, int reflexive,
                int mode, const GraphInfo& gi, int compose, Csr csr, const bmlp_opts& o, hipStream_t s,
                StatsRec& sr) {
  const i64 nw = words_for(n);
  u64* fa = ws_bits(c, S_W3, k, nw, o);
  u64* fb = ws_bits(c, S_W4, k, nw, o);
  const int parm = product_arm(o, k, n, n);
  const bool learned = mode == RM_LEARNED;
  if ((mode == RM_SPARSE || learned) && !csr.rp) {
    i64* rp;
    int32_t* ci;
    build_csr(c, R1, ld, n, o, s, &rp, &ci);
    csr.rp = rp;
    csr.ci = ci;
  }
  const u64* r1t = nullptr;
  i64 ldr1t = 0;
  if (mode != RM_SPARSE && parm == BMLP_ARM_PRODUCT_MFMA) r1t = transpose_b(c, R1, ld, n, n, o, s, &ldr1t);
  // state 0: fr = V, vis = 0 (or V for the reflexive answer)
  hip_check(launch_ewise(4, V, ldv, nullptr, 0, fa, nw, k, n, s), "copy");
  if (reflexive) hip_check(launch_ewise(4, V, ldv, nullptr, 0, Vstar, ldv, k, n, s), "copy");
  else hip_check(launch_fill_zero(Vstar, k * ldv, s), "fill_zero");
  double delta = (double)count_bits(c, V, k, n, ldv, s);
  double prev = delta, vis = reflexive ? delta : 0.0;
  bmlp_trace* tr = c->trace;
  float f[kIn];
  int t = 0;
  for (;; ++t) {
    need(t <= n + 1, BMLP_EITER, "selection exceeded %lld rounds", (long long)(n + 1));
    hip_check(hipMemsetAsync(c->d_flags, 0, 8 * sizeof(u32), s), "hipMemsetAsync");
    if (tr) hip_check(hipEventRecord(c->evp0, s), "hipEventRecord");
    make_features(f, gi, k, compose, 0, t, delta, prev, vis, reflexive);
    const u32* pred = nullptr;
    if (learned) {
      std::memcpy(c->h_flags + F_FEAT, f, kIn * sizeof(float));
      hip_check(hipMemcpyAsync(c->d_flags + F_FEAT, c->h_flags + F_FEAT, kIn * sizeof(float), hipMemcpyHostToDevice,
                               s),
                "memcpy");
      hip_check(launch_mlp_decide(c->d_model, c->d_model + kParams, c->d_model + kParams + kIn,
                                  (const float*)(c->d_flags + F_FEAT), (float*)(c->d_flags + F_PRED),
                                  c->d_flags + F_DEC, 0x3u, s),
                "mlp_decide");
      pred = c->d_flags + F_DEC;
    }
    unsigned long long* nb = (unsigned long long*)(c->d_flags + F_NEW);
    // an all-dense schedule times each product launch (the round events serve traces instead)
    const bool timed = mode == RM_DENSE && !tr;
    if (mode != RM_SPARSE) {
      GemmArgs g{fa, nw, R1, ld, Vstar, ldv, Vstar, ldv, fb, nw, k, n, n, c->d_flags + F_CHANGED};
      g.newbits = nb;
      g.pred = pred;
      g.pred_val = 0;
      if (timed) g.executed = sr.exec_counter();
      if (timed) sr.product_begin();
      if (parm == BMLP_ARM_PRODUCT_MFMA)
        hip_check(launch_gemm_mfma(g, r1t, ldr1t, s, tuned_variant(c, TK_MFMA, k, n, n, -1.0)), "gemm_mfma");
      else
        hip_check(launch_gemm_valu(g, s, tuned_variant(c, TK_VALU, k, n, n, -1.0)), "gemm_valu");
      if (timed) sr.product(k, n, n, parm);
    }
    if (mode != RM_DENSE)
      hip_check(launch_smp_round(fa, fb, nw, Vstar, ldv, k, csr.rp, csr.ci, R1, ld, n, c->d_flags + F_CHANGED, nb,
                                 pred, 1u, s),
                "smp_round");
    if (tr) hip_check(hipEventRecord(c->evp1, s), "hipEventRecord");
    hip_check(hipMemcpyAsync(c->h_flags, c->d_flags, 16 * sizeof(u32), hipMemcpyDeviceToHost, s), "memcpy");
    hip_check(hipStreamSynchronize(s), "sync");
    const u32 changed = c->h_flags[F_CHANGED];
    unsigned long long newbits = 0;
    std::memcpy(&newbits, c->h_flags + F_NEW, sizeof newbits);
    const int arm = learned ? (c->h_flags[F_DEC] == 0 ? BMLP_ARM_SMP_DENSE : BMLP_ARM_SMP_SPARSE)
                            : (mode == RM_DENSE ? BMLP_ARM_SMP_DENSE : BMLP_ARM_SMP_SPARSE);
    sr.trace(t, arm);
    if (sr.st && arm == BMLP_ARM_SMP_DENSE && !timed) {
      sr.st->products += 1;
      sr.st->bool_ops += (uint64_t)2 * (uint64_t)k * (uint64_t)n * (uint64_t)n;
    }
    if (tr && t < 64) {
      float ms = 0.f;
      hip_check(hipEventElapsedTime(&ms, c->evp0, c->evp1), "hipEventElapsedTime");
      tr->round_ms[t] = ms;
      tr->arm[t] = arm;
      std::memcpy(tr->features[t], f, sizeof f);
      if (learned) std::memcpy(tr->pred[t], c->h_flags + F_PRED, 4 * sizeof(float));
      tr->rounds = t + 1;
    }
    prev = delta;
    delta = (double)newbits;
    vis += (double)newbits;
    std::swap(fa, fb);
    if (!changed) break;
  }
  if (sr.st) sr.st->iterations = t + 1;
  hip_check(launch_zero_pad(Vstar, k, n, ldv, s), "zero_pad");
}

// Vstar = V . C for a closure C = R1+ (| V when reflexive): rows of the closure gathered for the set
// bits of each query row, or a product when n is beyond the gather kernel.
void read_off_closure(bmlp_ctx* c, const u64* V, i64 ldv, i64 k, const u64* clo, i64 ldc, i64 n, int reflexive,
                      u64* Vstar, const bmlp_opts& o, hipStream_t s, StatsRec& sr) {
  if (n <= gather_rows_max_n()) {
    const GatherQueue gq = gather_queue(c, k, n, o);
    hip_check(launch_gather_rows(V, ldv, k, clo, ldc, n, reflexive, Vstar, ldv, s, nullptr, nullptr, &gq),
              "gather_rows");
    return;
  }
  product(c, V, ldv, clo, ldc, reflexive ? V : nullptr, ldv, Vstar, ldv, nullptr, 0, k, n, n, nullptr,
          product_arm(o, k, n, n), s, sr);
  hip_check(launch_zero_pad(Vstar, k, n, ldv, s), "zero_pad");
}

void smp_core(bmlp_ctx* c, const u64* R1, i64 ld, i64 n, const u64* V, u64* Vstar, i64 k, i64 ldv, int reflexive,
              int arm, const GraphInfo& gi, int compose, Csr csr, const bmlp_opts& o, hipStream_t s, StatsRec& sr);

// R1+ (n x n, leading dimension ldo) by the one-launch selection from every source: row i of R1+ is the
// selection from the one-hot row e_i (the selection with V = I, whose rows the kernel forms itself).
// The same closure BMLP-RMS reaches, by per-source frontier expansion instead of squarings, which is
// cheaper where the closure rows cost less to expand than the squarings of a dense product.
void closure_by_selection(bmlp_ctx* c, const u64* R1, i64 ld, i64 n, u64* out, i64 ldo, const GraphInfo& gi, Csr csr,
                          const bmlp_opts& o, hipStream_t s, StatsRec& sr) {
  need(n <= smp_rows_max_n(), BMLP_EINVAL, "the closure by selection supports n <= %lld",
       (long long)smp_rows_max_n());
  const int keep = sr.st ? sr.st->arm : 0;
  const int keep_trace = c->trace ? c->trace->call_arm : 0;
  smp_core(c, R1, ld, n, nullptr, out, n, ldo, 0, BMLP_ARM_SMP_SPARSE, gi, 0, csr, o, s, sr);
  if (sr.st) sr.st->arm = keep;
  if (c->trace) c->trace->call_arm = keep_trace;
}

// Vstar = V . R1+ (or V . R1* when reflexive) by the given call-level arm.
void smp_core(bmlp_ctx* c, const u64* R1, i64 ld, i64 n, const u64* V, u64* Vstar, i64 k, i64 ldv, int reflexive,
              int arm, const GraphInfo& gi, int compose, Csr csr, const bmlp_opts& o, hipStream_t s, StatsRec& sr) {
  const i64 nw = words_for(n);
  if (sr.st) sr.st->arm = arm;
  if (c->trace) c->trace->call_arm = arm;
  if (arm == BMLP_ARM_SMP_SPARSE) {
    need(n <= smp_rows_max_n(), BMLP_EINVAL, "sparse SMP arm supports n <= %lld", (long long)smp_rows_max_n());
    i64 m = gi.m;
    if (!csr.rp) {
      i64* rp;
      int32_t* ci;
      // gi describes R1 when it was counted (gi.n == n); its bit count then sizes the CSR
      build_csr(c, R1, ld, n, o, s, &rp, &ci, &m, gi.n == n && gi.m > 0 ? gi.m : -1, csr.deg);
      csr.rp = rp;
      csr.ci = ci;
    }
    const i64* rpt = csr.rpt;
    const int32_t* cit = csr.cit;
    if (!rpt && m > 0 && (double)m >= kBottomUpMinDegree * (double)n) {
      i64* t;
      int32_t* ct;
      build_csc(c, R1, ld, csr.rp, csr.ci, n, m, o, s, &t, &ct);
      rpt = t;
      cit = ct;
    }
    hip_check(hipMemsetAsync(c->d_flags + F_ROUNDS, 0, sizeof(u32), s), "hipMemsetAsync");
    hip_check(launch_smp_rows(V, ldv, k, csr.rp, csr.ci, rpt, cit, R1, ld, n, reflexive, Vstar, ldv,
                              c->d_flags + F_ROUNDS, s),
              "smp_rows");
    // the round count only feeds the statistics: it is read with them at the end of the call (the kernel
    // stops by itself after n + 1 rounds)
    if (sr.st) sr.defer_rounds(n, arm);
    return;
  }
  if (arm == BMLP_ARM_SMP_CLOSURE || arm == BMLP_ARM_SMP_CLOSURE_SELECT) {
    u64* clo = ws_bits(c, S_W2, n, nw, o);
    if (arm == BMLP_ARM_SMP_CLOSURE)
      rms_core(c, R1, ld, clo, nw, n, o, s, sr);
    else
      closure_by_selection(c, R1, ld, n, clo, nw, gi, csr, o, s, sr);
    read_off_closure(c, V, ldv, k, clo, nw, n, reflexive, Vstar, o, s, sr);
    return;
  }
  const int mode = arm == BMLP_ARM_SMP_DENSE ? RM_DENSE : arm == BMLP_ARM_SMP_SPARSE_ROUNDS ? RM_SPARSE : RM_LEARNED;
  need(mode != RM_LEARNED || c->model, BMLP_EMODEL, "the adaptive arm needs a dispatcher model");
  smp_rounds(c, R1, ld, n, V, Vstar, k, ldv, reflexive, mode, gi, compose, csr, o, s, sr);
}

// Call-level arm of a selection: forced, plain rule, or the model's choice among the rounds arm
// (per-round choice), the closure arm and the one-launch sparse arm.
int smp_choose_arm(bmlp_ctx* c, const bmlp_opts& o, const GraphInfo& gi, i64 k, int compose, int reflexive,
                   double delta0, hipStream_t s, float* pred_out) {
  float f[kIn];
  make_features(f, gi, k, compose, 1, 0, delta0, delta0, reflexive ? delta0 : 0.0, reflexive);
  if (c->trace) std::memcpy(c->trace->call_features, f, sizeof f);
  if (o.dispatch == BMLP_DISPATCH_FORCED && o.smp_arm != BMLP_ARM_AUTO) return o.smp_arm;
  if (o.dispatch == BMLP_DISPATCH_LEARNED && c->model) {
    u32 allowed = 0x5u;  // rounds, closure
    if (gi.n <= smp_rows_max_n()) allowed |= 0x8u;  // one-launch sparse
    float pred[4];
    const int d = model_decide(c, f, allowed, s, pred);
    if (pred_out) std::memcpy(pred_out, pred, sizeof pred);
    if (c->trace) std::memcpy(c->trace->call_pred, pred, sizeof pred);
    return d == 2 ? BMLP_ARM_SMP_CLOSURE : d == 3 ? BMLP_ARM_SMP_SPARSE : BMLP_ARM_SMP_ADAPTIVE;
  }
  return smp_plain_arm(gi.n, k, gi.m);
}

// The call-level inputs of a dispatcher choice, computed on the device and read back together (one host
// wait): the statistics of R (n x n), the set bits of the query rows Q (qrows x n; Q null: *delta0 gives
// them), the 16 features (features.h) and, with allowed != 0, the model's decision among the allowed
// outputs.  Returns the decision, or -1 when the model is not asked.
int call_stats_decide(bmlp_ctx* c, const u64* R, i64 ld, i64 n, const u64* Q, i64 qrows, i64 ldq, i64 k,
                      float context, int reflexive, u32 allowed, const bmlp_opts& o, hipStream_t s, GraphInfo* gi,
                      double* delta0) {
  unsigned long long* gst = (unsigned long long*)(c->d_flags + F_GSTATS);
  unsigned long long* cnt = (unsigned long long*)(c->d_flags + F_CNT);
  float* feat = (float*)(c->d_flags + F_FEAT);
  const int32_t* deg = nullptr;
  if (n <= kDegStatsMaxN) {  // as graph_info: the statistics from the per-row counts, which stay in S_DEG
    int32_t* d = (int32_t*)ws(c, S_DEG, (size_t)n * sizeof(int32_t), o);
    hip_check(launch_row_popcount(R, n, n, ld, d, nullptr, s), "row_popcount");
    hip_check(launch_deg_stats(d, n, gst, s), "deg_stats");
    deg = d;
  } else {
    hip_check(hipMemsetAsync(gst, 0, 3 * sizeof(unsigned long long), s), "hipMemsetAsync");
    hip_check(launch_graph_stats(R, n, n, ld, gst, s), "graph_stats");
  }
  if (Q) {
    hip_check(hipMemsetAsync(cnt, 0, sizeof(unsigned long long), s), "hipMemsetAsync");
    hip_check(launch_popcount_total(Q, qrows, n, ldq, cnt, s), "popcount_total");
  } else {
    // no query rows given: *delta0 holds their bit count (the identity's n for a closure)
    const unsigned long long d = (unsigned long long)*delta0;
    std::memcpy(c->h_flags + F_CNT, &d, sizeof d);
    hip_check(hipMemcpyAsync(cnt, c->h_flags + F_CNT, sizeof d, hipMemcpyHostToDevice, s), "memcpy");
  }
  hip_check(launch_call_features(gst, cnt, n, k, context, reflexive, feat, s), "call_features");
  if (allowed)
    hip_check(launch_mlp_decide(c->d_model, c->d_model + kParams, c->d_model + kParams + kIn, feat,
                                (float*)(c->d_flags + F_PRED), c->d_flags + F_DEC, allowed, s),
              "mlp_decide");
  // words F_CNT .. F_GSTATS + 6: the bit count, the decision, the predictions, the features, the statistics
  hip_check(hipMemcpyAsync(c->h_flags + F_CNT, c->d_flags + F_CNT, (F_GSTATS + 6 - F_CNT) * sizeof(u32),
                           hipMemcpyDeviceToHost, s),
            "memcpy");
  hip_check(hipStreamSynchronize(s), "sync");
  unsigned long long v[3], d0 = 0;
  std::memcpy(v, c->h_flags + F_GSTATS, sizeof v);
  std::memcpy(&d0, c->h_flags + F_CNT, sizeof d0);
  gi->n = n;
  gi->m = (i64)v[0];
  gi->maxdeg = (i64)v[1];
  gi->nonempty = (i64)v[2];
  gi->deg = deg;
  *delta0 = (double)d0;
  if (c->trace) std::memcpy(c->trace->call_features, c->h_flags + F_FEAT, kIn * sizeof(float));
  if (!allowed) return -1;
  if (c->trace) std::memcpy(c->trace->call_pred, c->h_flags + F_PRED, 4 * sizeof(float));
  return (int)c->h_flags[F_DEC];
}

template <class F>
bmlp_status guarded(F&& f) {
  try {
    f();
    return BMLP_OK;
  } catch (const Fail& e) {
    return e.st;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return BMLP_ENOMEM;
  } catch (...) {
    g_last_error = "unexpected exception";
    return BMLP_EDEVICE;
  }
}

void need_handle(bmlp_handle h) { need(h != nullptr, BMLP_EINVAL, "null handle"); }

}  // namespace

extern "C" {

void bmlp_opts_init(bmlp_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->size = sizeof(bmlp_opts);
  o->dispatch = BMLP_DISPATCH_PLAIN;
  o->product_arm = BMLP_ARM_AUTO;
  o->smp_arm = BMLP_ARM_AUTO;
  o->compose_arm = BMLP_ARM_AUTO;
  o->rms_variant = 0;
  o->smp_reflexive = 0;
  o->check_padding = 0;
  o->workspace_limit = 0;
}

int32_t bmlp_version(void) { return 100; }

const char* bmlp_last_error(void) { return g_last_error.c_str(); }

bmlp_status bmlp_create(bmlp_handle* h, int device) {
  g_last_error.clear();
  return guarded([&] {
    need(h != nullptr, BMLP_EINVAL, "null handle pointer");
    *h = nullptr;
    int count = 0;
    hip_check(hipGetDeviceCount(&count), "hipGetDeviceCount");
    need(device >= 0 && device < count, BMLP_EINVAL, "device %d out of range (%d devices)", device, count);
    DeviceGuard dg(device);
    bmlp_ctx* c = new bmlp_ctx;
    c->device = device;
    for (int k = 0; k < bmlp_ctx::kTuneKernels; ++k)
      for (int b = 0; b < bmlp_ctx::kTuneBuckets; ++b) {
        c->tune[k][b] = -1;
        c->tune_ms[k][b] = 0.f;
      }
    if (hipMalloc((void**)&c->d_flags, F_WORDS * sizeof(u32)) != hipSuccess ||
        hipHostMalloc((void**)&c->h_flags, F_WORDS * sizeof(u32), hipHostMallocDefault) != hipSuccess ||
        hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
        hipEventCreate(&c->evp0) != hipSuccess || hipEventCreate(&c->evp1) != hipSuccess) {
      (void)hipGetLastError();
      bmlp_destroy(c);
      fail(BMLP_ENOMEM, "handle allocation failed");
    }
    hip_check(hipMemset(c->d_flags, 0, F_WORDS * sizeof(u32)), "hipMemset");
    c->scratch = scratch_address(device);
    *h = c;
    // default dispatcher model: $BMLP_DISPATCHER_MODEL, else dispatcher_model.bin beside the library
    // (an empty variable disables it); a missing or bad file leaves the plain schedule in force
    std::string path;
    if (const char* env = std::getenv("BMLP_DISPATCHER_MODEL")) {
      path = env;
    } else {
      Dl_info info;
      if (dladdr((const void*)&bmlp_create, &info) && info.dli_fname) {
        path = info.dli_fname;
        const size_t slash = path.find_last_of('/');
        path = (slash == std::string::npos ? std::string(".") : path.substr(0, slash)) + "/dispatcher_model.bin";
      }
    }
    if (!path.empty() && bmlp_dispatcher_load(c, path.c_str()) != BMLP_OK) g_last_error.clear();
    // tuning cache: $BMLP_AUTOTUNE_CACHE, else autotune_cache.json beside the library (an empty variable
    // disables it); a missing, bad or foreign cache leaves the built-in defaults
    std::string tpath;
    if (const char* env = std::getenv("BMLP_AUTOTUNE_CACHE")) {
      tpath = env;
    } else {
      Dl_info info;
      if (dladdr((const void*)&bmlp_create, &info) && info.dli_fname) {
        tpath = info.dli_fname;
        const size_t slash = tpath.find_last_of('/');
        tpath = (slash == std::string::npos ? std::string(".") : tpath.substr(0, slash)) + "/autotune_cache.json";
      }
    }
    if (!tpath.empty() && bmlp_tune_load(c, tpath.c_str()) != BMLP_OK) g_last_error.clear();
  });
}

bmlp_status bmlp_destroy(bmlp_handle h) {
  if (!h) return BMLP_OK;
  return guarded([&] {
    {
      DeviceGuard dg(h->device);
      (void)hipDeviceSynchronize();
      for (int i = 0; i < bmlp_ctx::kSlots; ++i)
        if (h->slot[i]) (void)hipFree(h->slot[i]);
      if (h->d_flags) (void)hipFree(h->d_flags);
      if (h->h_flags) (void)hipHostFree(h->h_flags);
      if (h->ev0) (void)hipEventDestroy(h->ev0);
      if (h->ev1) (void)hipEventDestroy(h->ev1);
      if (h->evp0) (void)hipEventDestroy(h->evp0);
      if (h->evp1) (void)hipEventDestroy(h->evp1);
      for (int i = 0; i < bmlp_ctx::kPend; ++i) {
        if (h->pe0[i]) (void)hipEventDestroy(h->pe0[i]);
        if (h->pe1[i]) (void)hipEventDestroy(h->pe1[i]);
      }
      if (h->d_exec) (void)hipFree(h->d_exec);
      if (h->h_exec) (void)hipHostFree(h->h_exec);
      if (h->d_model) (void)hipFree(h->d_model);
      if (h->bexec) (void)hipGraphExecDestroy(h->bexec);
      if (h->bgraph) (void)hipGraphDestroy(h->bgraph);
      if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
    }
    delete h;
  });
}

int32_t bmlp_tune_candidates(int32_t kernel) {
  return (kernel >= 0 && kernel < bmlp_ctx::kTuneKernels) ? kTuneCandidates[kernel] : 0;
}

int32_t bmlp_tune_buckets(int32_t kernel) {
  return (kernel >= 0 && kernel < bmlp_ctx::kTuneKernels) ? bmlp_ctx::kTuneBuckets : 0;
}

int32_t bmlp_tune_bucket_of(int32_t kernel, int64_t m, int64_t kdim, int64_t n, double density, int32_t structured) {
  if (kernel < 0 || kernel >= bmlp_ctx::kTuneKernels || m < 0 || kdim < 0 || n < 0) return -1;
  return tune_bucket(m, kdim, n, density, structured != 0);
}

bmlp_status bmlp_tune_get(bmlp_handle h, int32_t kernel, int32_t bucket, int32_t* variant, float* ms) {
  return guarded([&] {
    need_handle(h);
    need(kernel >= 0 && kernel < bmlp_ctx::kTuneKernels, BMLP_EINVAL, "unknown tuned kernel %d", kernel);
    need(bucket >= 0 && bucket < bmlp_ctx::kTuneBuckets, BMLP_EINVAL, "bucket %d out of range", bucket);
    need(variant != nullptr, BMLP_EINVAL, "variant: null pointer");
    *variant = h->tune[kernel][bucket];
    if (ms) *ms = h->tune_ms[kernel][bucket];
  });
}

bmlp_status bmlp_tune_set(bmlp_handle h, int32_t kernel, int32_t bucket, int32_t variant) {
  return guarded([&] {
    need_handle(h);
    need(kernel >= 0 && kernel < bmlp_ctx::kTuneKernels, BMLP_EINVAL, "unknown tuned kernel %d", kernel);
    need(bucket >= -1 && bucket < bmlp_ctx::kTuneBuckets, BMLP_EINVAL, "bucket %d out of range", bucket);
    need(variant >= -1 && variant < kTuneCandidates[kernel], BMLP_EINVAL, "candidate %d out of range", variant);
    for (int b = 0; b < bmlp_ctx::kTuneBuckets; ++b)
      if (bucket == -1 || b == bucket) {
        h->tune[kernel][b] = variant;
        h->tune_ms[kernel][b] = 0.f;
      }
  });
}

// The autotuner.  Every candidate of the selected kernels is timed on the squarings C = R | R.R that a
// closure goes through, at four sizes (n = 2,048, 4,096, 8,192, 16,384):
//   * the states of a seeded random digraph of mean out-degree 8 on its way to its closure (they fill
//     the "below 1/64" and "denser" classes);
//   * the states of one of mean out-degree 2, just above the percolation threshold, once they are dense
//     enough for the matrix cores, relabelled as the RMS driver relabels such a relation (the
//     block-structured class);
//   * uniform random bits for a class no state fell into (density 2^-13 for the sparsest).
// The random bits are drawn on the device (k_fill_random).  A candidate's score in a bucket is its median
// time summed over the bucket's states; the fastest is kept.  Candidates return identical bits (checked
// by the tests), so the choice changes speed only.
bmlp_status bmlp_autotune(bmlp_handle h, int32_t kernel_mask, int32_t reps, const char* cache_out, float* report) {
  return guarded([&] {
    need_handle(h);
    need(reps >= 1 && reps <= 100, BMLP_EINVAL, "reps must be 1..100");
    need((kernel_mask & ~((1 << bmlp_ctx::kTuneKernels) - 1)) == 0, BMLP_EINVAL, "unknown kernel in mask");
    DeviceGuard dg(h->device);
    hipStream_t s = nullptr;
    bmlp_opts o;
    bmlp_opts_init(&o);
    constexpr int NK = bmlp_ctx::kTuneKernels, NC = BMLP_TUNE_MAX_CANDIDATES;
    if (report)
      for (int i = 0; i < NK * bmlp_ctx::kTuneBuckets * NC; ++i) report[i] = -1.f;
    hipEvent_t e0 = h->evp0, e1 = h->evp1;
    unsigned long long* nbc = (unsigned long long*)(h->d_flags + F_NEW);
    u64 seed = 0x5EED5EEDull;
    for (int sb = 0; sb < 4; ++sb) {
      const i64 n = (i64)2048 << sb, nw = words_for(n);
      const int logn = 11 + sb;
      u64* R = ws_bits(h, S_T0, n, nw, o);
      u64* C = ws_bits(h, S_T1, n, nw, o);
      u64* P = ws_bits(h, S_T2, n, nw, o);
      u64* RT = ws_bits(h, S_BT, n, nw, o);
      double sum[NK][4][NC] = {};
      int states[4] = {0, 0, 0, 0};
      auto time_state = [&](const u64* A, int cls) {
        hip_check(launch_transpose(A, n, n, nw, RT, nw, s), "transpose");
        for (int k = 0; k < NK; ++k) {
          if (!((kernel_mask >> k) & 1)) continue;
          for (int v = 0; v < kTuneCandidates[k]; ++v) {
            GemmArgs g{A, nw, A, nw, A, nw, C, nw, nullptr, 0, n, n, n, nullptr};
            std::vector<float> ts;
            for (int r = 0; r <= reps; ++r) {
              hip_check(hipEventRecord(e0, s), "hipEventRecord");
              if (k == TK_MFMA) hip_check(launch_gemm_mfma(g, RT, nw, s, v), "gemm_mfma");
              else hip_check(launch_gemm_valu(g, s, v), "gemm_valu");
              hip_check(hipEventRecord(e1, s), "hipEventRecord");
              hip_check(hipEventSynchronize(e1), "hipEventSynchronize");
              float ms = 0.f;
              hip_check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
              if (r > 0) ts.push_back(ms);  // the first launch warms up
            }
            std::sort(ts.begin(), ts.end());
            sum[k][cls][v] += ts[ts.size() / 2];
          }
        }
        ++states[cls];
      };
      // R <- R | R.R (the first matrix-core candidate), returning the bits it added
      auto square = [&]() -> i64 {
        hip_check(launch_transpose(R, n, n, nw, RT, nw, s), "transpose");
        hip_check(launch_fill_zero((u64*)nbc, 1, s), "fill_zero");
        GemmArgs g{R, nw, R, nw, R, nw, C, nw, nullptr, 0, n, n, n, nullptr};
        g.newbits = nbc;
        hip_check(launch_gemm_mfma(g, RT, nw, s, 0), "gemm_mfma");
        std::swap(R, C);
        return (i64)read_flag(h, s, F_NEW) | ((i64)read_flag(h, s, F_NEW + 1) << 32);
      };
      auto cls_of = [&](i64 bits) {
        const double d = (double)bits / ((double)n * (double)n);
        return d < 1.0 / 4096.0 ? 0 : d < 1.0 / 64.0 ? 1 : 2;
      };
      // 1. mean out-degree 8, squared to its closure
      hip_check(launch_fill_random(R, n, n, nw, ++seed, logn - 3, logn - 3, n, nw, s), "fill_random");
      i64 bits = count_bits(h, R, n, n, nw, s);
      for (int step = 0; step < 8; ++step) {
        time_state(R, cls_of(bits));
        const i64 added = square();
        if (added == 0) break;
        bits += added;
      }
      // 2. mean out-degree 2: squared until dense, relabelled, then its squarings timed as block-structured
      hip_check(launch_fill_random(R, n, n, nw, ++seed, logn - 1, logn - 1, n, nw, s), "fill_random");
      bits = count_bits(h, R, n, n, nw, s);
      for (int step = 0; step < 8 && cls_of(bits) < 2; ++step) {
        const i64 added = square();
        if (added == 0) break;
        bits += added;
      }
      int32_t* perm;
      int32_t* pinv;
      if (rms_relabel(h, R, nw, n, o, s, &perm, &pinv) == 1) {
        hip_check(launch_permute(R, nw, perm, n, P, nw, s), "permute");
        std::swap(R, P);
        for (int step = 0; step < 3; ++step) {
          time_state(R, 3);
          if (square() == 0) break;
        }
      }
      // 3. uniform random bits for the classes no state fell into: 2^-13, 2^-8, 2^-(logn/2 - 1), and a
      //    dense corner block of 40% of the rows and columns in a sparse rest
      for (int cls = 0; cls < 4; ++cls) {
        if (states[cls] > 0) continue;
        const int s_in = cls == 0 ? 13 : cls == 1 ? 8 : cls == 2 ? logn / 2 - 1 : 4;
        const int s_out = cls == 3 ? 13 : s_in;
        const i64 brows = cls == 3 ? (2 * n) / 5 : n, bwords = cls == 3 ? (2 * nw) / 5 : nw;
        hip_check(launch_fill_random(R, n, n, nw, ++seed, s_in, s_out, brows, bwords, s), "fill_random");
        time_state(R, cls);
      }
      for (int k = 0; k < NK; ++k) {
        if (!((kernel_mask >> k) & 1)) continue;
        for (int cls = 0; cls < 4; ++cls) {
          const int bucket = 4 * sb + cls;
          int bestv = 0;
          for (int v = 0; v < kTuneCandidates[k]; ++v) {
            if (report) report[(k * bmlp_ctx::kTuneBuckets + bucket) * NC + v] = (float)(sum[k][cls][v] / states[cls]);
            if (sum[k][cls][v] < sum[k][cls][bestv]) bestv = v;
          }
          h->tune[k][bucket] = bestv;
          h->tune_ms[k][bucket] = (float)(sum[k][cls][bestv] / states[cls]);
        }
      }
    }
    if (cache_out) {
      const bmlp_status st = bmlp_tune_save(h, cache_out);
      need(st == BMLP_OK, st, "%s", g_last_error.c_str());
    }
  });
}

// The tuning cache: JSON with the device's architecture name and compute-unit count (a cache is used only
// on the same kind of device) and, per tuned kernel, the candidate and its time for every bucket.
namespace {
const char* kTuneNames[bmlp_ctx::kTuneKernels] = {"mfma_product", "valu_product"};
void device_key(int device, std::string* arch, int* cus) {
  hipDeviceProp_t prop;
  hip_check(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
  *arch = prop.gcnArchName;
  *cus = prop.multiProcessorCount;
}
}  // namespace

bmlp_status bmlp_tune_save(bmlp_handle h, const char* path) {
  return guarded([&] {
    need_handle(h);
    need(path != nullptr, BMLP_EINVAL, "path: null pointer");
    std::string arch;
    int cus = 0;
    device_key(h->device, &arch, &cus);
    FILE* fp = std::fopen(path, "w");
    need(fp != nullptr, BMLP_EINVAL, "cannot write %s", path);
    std::fprintf(fp, "{\n  \"format\": \"bmlp-autotune\",\n  \"version\": 1,\n  \"arch\": \"%s\",\n  \"cus\": %d,\n",
                 arch.c_str(), cus);
    std::fprintf(fp, "  \"buckets\": \"4 * size + class; size by 2 m k n below 3.4e10, 2.7e11, 2.2e12, beyond; class: "
                     "left operand bits below 1/4096, below 1/64, denser or unknown, block-structured\",\n");
    std::fprintf(fp, "  \"kernels\": [\n");
    for (int k = 0; k < bmlp_ctx::kTuneKernels; ++k) {
      std::fprintf(fp, "    {\"kernel\": %d, \"name\": \"%s\", \"candidates\": %d,\n     \"choice\": [", k, kTuneNames[k],
                   kTuneCandidates[k]);
      for (int b = 0; b < bmlp_ctx::kTuneBuckets; ++b) std::fprintf(fp, "%s%d", b ? ", " : "", h->tune[k][b]);
      std::fprintf(fp, "],\n     \"ms\": [");
      for (int b = 0; b < bmlp_ctx::kTuneBuckets; ++b) std::fprintf(fp, "%s%.4f", b ? ", " : "", h->tune_ms[k][b]);
      std::fprintf(fp, "]}%s\n", k + 1 < bmlp_ctx::kTuneKernels ? "," : "");
    }
    std::fprintf(fp, "  ]\n}\n");
    const bool ok = std::ferror(fp) == 0;
    std::fclose(fp);
    need(ok, BMLP_EINVAL, "short write to %s", path);
  });
}

bmlp_status bmlp_tune_load(bmlp_handle h, const char* path) {
  return guarded([&] {
    need_handle(h);
    need(path != nullptr, BMLP_EINVAL, "path: null pointer");
    FILE* fp = std::fopen(path, "r");
    need(fp != nullptr, BMLP_EMODEL, "cannot open tuning cache %s", path);
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, fp)) > 0) text.append(buf, got);
    std::fclose(fp);
    // a small reader for the format bmlp_tune_save writes
    auto str_after = [&](const char* key, size_t from, std::string* out) -> size_t {
      const size_t k = text.find(key, from);
      if (k == std::string::npos) return k;
      const size_t a = text.find('"', text.find(':', k) + 1);
      const size_t b = a == std::string::npos ? a : text.find('"', a + 1);
      if (b == std::string::npos) return b;
      *out = text.substr(a + 1, b - a - 1);
      return b;
    };
    auto int_after = [&](const char* key, size_t from, long* out) -> size_t {
      const size_t k = text.find(key, from);
      if (k == std::string::npos) return k;
      const size_t c = text.find(':', k);
      if (c == std::string::npos) return c;
      char* end = nullptr;
      *out = std::strtol(text.c_str() + c + 1, &end, 10);
      return end == text.c_str() + c + 1 ? std::string::npos : (size_t)(end - text.c_str());
    };
    std::string fmt, arch;
    long version = 0, cus = 0;
    need(str_after("\"format\"", 0, &fmt) != std::string::npos && fmt == "bmlp-autotune" &&
             int_after("\"version\"", 0, &version) != std::string::npos && version == 1,
         BMLP_EMODEL, "%s is not a tuning cache of this format", path);
    need(str_after("\"arch\"", 0, &arch) != std::string::npos && int_after("\"cus\"", 0, &cus) != std::string::npos,
         BMLP_EMODEL, "%s: no device key", path);
    std::string my_arch;
    int my_cus = 0;
    DeviceGuard dg(h->device);
    device_key(h->device, &my_arch, &my_cus);
    need(arch == my_arch && cus == my_cus, BMLP_EMODEL, "%s was tuned on %s with %ld CUs, this device is %s with %d",
         path, arch.c_str(), cus, my_arch.c_str(), my_cus);
    int32_t tune[bmlp_ctx::kTuneKernels][bmlp_ctx::kTuneBuckets];
    float ms[bmlp_ctx::kTuneKernels][bmlp_ctx::kTuneBuckets];
    size_t at = 0;
    for (int k = 0; k < bmlp_ctx::kTuneKernels; ++k) {
      long kk = -1;
      at = int_after("\"kernel\"", at, &kk);
      need(at != std::string::npos && kk == k, BMLP_EMODEL, "%s: kernel %d missing", path, k);
      size_t c = text.find("\"choice\"", at);
      need(c != std::string::npos, BMLP_EMODEL, "%s: kernel %d has no choice", path, k);
      c = text.find('[', c);
      const char* q = text.c_str() + c + 1;
      for (int b = 0; b < bmlp_ctx::kTuneBuckets; ++b) {
        char* end = nullptr;
        const long v = std::strtol(q, &end, 10);
        need(end != q && v >= -1 && v < kTuneCandidates[k], BMLP_EMODEL, "%s: bad choice for kernel %d", path, k);
        tune[k][b] = (int32_t)v;
        q = end;
        while (*q == ',' || *q == ' ') ++q;
      }
      size_t m = text.find("\"ms\"", at);
      need(m != std::string::npos, BMLP_EMODEL, "%s: kernel %d has no times", path, k);
      q = text.c_str() + text.find('[', m) + 1;
      for (int b = 0; b < bmlp_ctx::kTuneBuckets; ++b) {
        char* end = nullptr;
        ms[k][b] = std::strtof(q, &end);
        need(end != q, BMLP_EMODEL, "%s: bad time for kernel %d", path, k);
        q = end;
        while (*q == ',' || *q == ' ') ++q;
      }
      at = (size_t)(q - text.c_str());
    }
    std::memcpy(h->tune, tune, sizeof tune);
    std::memcpy(h->tune_ms, ms, sizeof ms);
  });
}

bmlp_status bmlp_pack_u8(bmlp_handle h, const uint8_t* dense, int64_t rows, int64_t n, int64_t ldd, uint64_t* bits,
                         int64_t ld, void* stream) {
  return guarded([&] {
    need_handle(h);
    check_bits_arg(bits, "bits", rows, n, ld);
    need(ldd >= n, BMLP_EINVAL, "ldd < n");
    if (rows == 0) return;
    need(n == 0 || dense != nullptr, BMLP_EINVAL, "dense: null pointer");
    DeviceGuard dg(h->device);
    hip_check(launch_pack_u8(dense, rows, n, ldd, bits, ld, (hipStream_t)stream), "pack_u8");
  });
}

bmlp_status bmlp_pack_coo(bmlp_handle h, const int32_t* row, const int32_t* col, int64_t m, int64_t rows, int64_t n,
                          uint64_t* bits, int64_t ld, void* stream) {
  return guarded([&] {
    need_handle(h);
    check_bits_arg(bits, "bits", rows, n, ld);
    need(m >= 0, BMLP_EINVAL, "m < 0");
    if (m > 0) {
      need(row && col, BMLP_EINVAL, "row/col: null pointer");
      need(((uintptr_t)row & 3u) == 0 && ((uintptr_t)col & 3u) == 0, BMLP_EALIGN, "row/col: not 4-byte aligned");
    }
    DeviceGuard dg(h->device);
    hipStream_t s = (hipStream_t)stream;
    hip_check(launch_fill_zero(bits, rows * ld, s), "fill_zero");
    hip_check(hipMemsetAsync(h->d_flags + 3, 0, sizeof(u32), s), "hipMemsetAsync");
    hip_check(launch_pack_coo(row, col, m, rows, n, bits, ld, h->d_flags + 3, s), "pack_coo");
    need(read_flag(h, s, 3) == 0, BMLP_EINVAL, "pack_coo: index outside [0,%lld) x [0,%lld)", (long long)rows,
         (long long)n);
  });
}

bmlp_status bmlp_pack_coo_async(bmlp_handle h, const int32_t* row, const int32_t* col, int64_t m, int64_t rows,
                                int64_t n, uint64_t* bits, int64_t ld, void* stream) {
  return guarded([&] {
    need_handle(h);
    check_bits_arg(bits, "bits", rows, n, ld);
    need(m >= 0, BMLP_EINVAL, "m < 0");
    if (m > 0) {
      need(row && col, BMLP_EINVAL, "row/col: null pointer");
      need(((uintptr_t)row & 3u) == 0 && ((uintptr_t)col & 3u) == 0, BMLP_EALIGN, "row/col: not 4-byte aligned");
    }
    DeviceGuard dg(h->device);
    hipStream_t s = (hipStream_t)stream;
    hip_check(launch_fill_zero(bits, rows * ld, s), "fill_zero");
    hip_check(launch_pack_coo(row, col, m, rows, n, bits, ld, h->d_flags + F_DEFER, s), "pack_coo");
  });
}

bmlp_status bmlp_deferred_error(bmlp_handle h, void* stream) {
  return guarded([&] {
    need_handle(h);
    DeviceGuard dg(h->device);
    hipStream_t s = (hipStream_t)stream;
    const u32 bad = read_flag(h, s, F_DEFER);
    if (bad) hip_check(launch_fill_zero((u64*)(h->d_flags + F_DEFER - (F_DEFER & 1)), 1, s), "fill_zero");
    need(bad == 0, BMLP_EINVAL, "a fact given to bmlp_pack_coo_async lay outside its matrix (it was skipped)");
  });
}

bmlp_status bmlp_unpack_coo(bmlp_handle h, const uint64_t* bits, int64_t rows, int64_t n, int64_t ld,
                            int32_t* row_out, int32_t* col_out, int64_t cap, int64_t* count, void* stream) {
  return guarded([&] {
    need_handle(h);
    check_bits_arg(bits, "bits", rows, n, ld);
    need(count != nullptr, BMLP_EINVAL, "count: null pointer");
    need(cap >= 0, BMLP_EINVAL, "cap < 0");
    need(((uintptr_t)row_out & 3u) == 0 && ((uintptr_t)col_out & 3u) == 0, BMLP_EALIGN,
         "row_out/col_out: not 4-byte aligned");
    *count = 0;
    if (rows == 0 || n == 0) return;
    DeviceGuard dg(h->device);
    hipStream_t s = (hipStream_t)stream;
    bmlp_opts o;
    bmlp_opts_init(&o);
    int32_t* deg = (int32_t*)ws(h, S_DEG, (size_t)rows * sizeof(int32_t), o);
    i64* rp = (i64*)ws(h, S_RP, (size_t)(rows + 1) * sizeof(i64), o);
    hip_check(launch_row_popcount(bits, rows, n, ld, deg, nullptr, s), "row_popcount");
    hip_check(launch_scan_rowptr(deg, rows, rp, s), "scan");
    hip_check(hipMemcpyAsync(h->h_flags + 4, rp + rows, sizeof(i64), hipMemcpyDeviceToHost, s), "memcpy");
    hip_check(hipStreamSynchronize(s), "sync");
    i64 m = 0;
    std::memcpy(&m, h->h_flags + 4, sizeof m);
    *count = m;
    if (!row_out && !col_out) return;  // the count only
    need(cap >= m, BMLP_EINVAL, "unpack_coo: %lld facts do not fit in cap = %lld", (long long)m, (long long)cap);
    if (col_out) hip_check(launch_bits_to_csr(bits, rows, n, ld, rp, col_out, s), "bits_to_csr");
    if (row_out) hip_check(launch_rows_from_rp(rp, rows, row_out, s), "rows_from_rp");
  });
}

bmlp_status bmlp_unpack_u8(bmlp_handle h, const uint64_t* bits, int64_t rows, int64_t n, int64_t ld, uint8_t* dense,
                           int64_t ldd, void* stream) {
  return guarded([&] {
    need_handle(h);
    check_bits_arg(bits, "bits", rows, n, ld);
    need(ldd >= n, BMLP_EINVAL, "ldd < n");
    if (rows == 0 || n == 0) return;
    need(dense != nullptr, BMLP_EINVAL, "dense: null pointer");
    DeviceGuard dg(h->device);
    hip_check(launch_unpack_u8(bits, rows, n, ld, dense, ldd, (hipStream_t)stream), "unpack_u8");
  });
}

static bmlp_status ewise_api(int op, bmlp_handle h, const uint64_t* A, const uint64_t* B, uint64_t* C, int64_t rows,
                             int64_t n, int64_t ld, void* stream) {
  return guarded([&] {
    need_handle(h);
    check_bits_arg(A, "A", rows, n, ld);
    if (op <= 2) check_bits_arg(B, "B", rows, n, ld);
    check_bits_arg(C, "C", rows, n, ld);
    if (rows == 0 || ld == 0) return;
    DeviceGuard dg(h->device);
    hip_check(launch_ewise(op, A, ld, B, ld, C, ld, rows, n, (hipStream_t)stream), "ewise");
  });
}

bmlp_status bmlp_or(bmlp_handle h, const uint64_t* A, const uint64_t* B, uint64_t* C, int64_t rows, int64_t n,
                    int64_t ld, void* stream) {
  return ewise_api(0, h, A, B, C, rows, n, ld, stream);
}
bmlp_status bmlp_and(bmlp_handle h, const uint64_t* A, const uint64_t* B, uint64_t* C, int64_t rows, int64_t n,
                     int64_t ld, void* stream) {
  return ewise_api(1, h, A, B, C, rows, n, ld, stream);
}
bmlp_status bmlp_andnot(bmlp_handle h, const uint64_t* A, const uint64_t* B, uint64_t* C, int64_t rows, int64_t n,
                        int64_t ld, void* stream) {
  return ewise_api(2, h, A, B, C, rows, n, ld, stream);
}
bmlp_status bmlp_not(bmlp_handle h, const uint64_t* A, uint64_t* C, int64_t rows, int64_t n, int64_t ld,
                     void* stream) {
  return ewise_api(3, h, A, nullptr, C, rows, n, ld, stream);
}

bmlp_status bmlp_transpose(bmlp_handle h, const uint64_t* A, int64_t rows, int64_t cols, int64_t lda, uint64_t* AT,
                           int64_t ldat, void* stream) {
  return guarded([&] {
    need_handle(h);
    check_bits_arg(A, "A", rows, cols, lda);
    check_bits_arg(AT, "AT", cols, rows, ldat);
    need(!overlap(range_of(A, rows, lda), range_of(AT, cols, ldat)), BMLP_EALIAS, "AT overlaps A");
    if (cols == 0) return;
    DeviceGuard dg(h->device);
    hipStream_t s = (hipStream_t)stream;
    if (rows == 0) {
      hip_check(launch_fill_zero(AT, cols * ldat, s), "fill_zero");
      return;
    }
    hip_check(launch_transpose(A, rows, cols, lda, AT, ldat, s), "transpose");
  });
}

bmlp_status bmlp_product(bmlp_handle h, const uint64_t* A, int64_t lda, const uint64_t* B, int64_t ldb,
                         const uint64_t* Cold, uint64_t* C, int64_t ldc, int64_t m, int64_t kdim, int64_t n,
                         const bmlp_opts* opts, void* stream, bmlp_stats* stats) {
  return guarded([&] {
    need_handle(h);
    const bmlp_opts o = opts_or_default(opts);
    check_bits_arg(A, "A", m, kdim, lda);
    check_bits_arg(B, "B", kdim, n, ldb);
    check_bits_arg(C, "C", m, n, ldc);
    if (Cold) check_bits_arg(Cold, "Cold", m, n, ldc);
    const Range rc = range_of(C, m, ldc);
    need(!overlap(rc, range_of(A, m, lda)), BMLP_EALIAS, "C overlaps A");
    need(!overlap(rc, range_of(B, kdim, ldb)), BMLP_EALIAS, "C overlaps B");
    need(!Cold || Cold == C || !overlap(rc, range_of(Cold, m, ldc)), BMLP_EALIAS, "C partially overlaps Cold");
    DeviceGuard dg(h->device);
    hipStream_t s = (hipStream_t)stream;
    if (o.check_padding) {
      check_padding(h, A, m, kdim, lda, s, "A");
      check_padding(h, B, kdim, n, ldb, s, "B");
      if (Cold) check_padding(h, Cold, m, n, ldc, s, "Cold");
    }
    StatsRec sr(stats, h, s, &o);
    if (m > 0 && n > 0) {
      if (kdim == 0) {
        if (Cold) hip_check(launch_ewise(4, Cold, ldc, nullptr, 0, C, ldc, m, n, s), "copy");
        else hip_check(launch_fill_zero(C, m * ldc, s), "fill_zero");
      } else {
        product(h, A, lda, B, ldb, Cold, ldc, C, ldc, nullptr, 0, m, kdim, n, nullptr, product_arm(o, m, n, kdim), s,
                sr);
      }
    }
    if (m > 0) hip_check(launch_zero_pad(C, m, n, ldc, s), "zero_pad");
    if (stats) stats->arm = product_arm(o, m, n, kdim);
    sr.finish();
  });
}

bmlp_status bmlp_rms(bmlp_handle h, const uint64_t* R1, uint64_t* Rstar, int64_t n, int64_t ld, const bmlp_opts* opts,
                     void* stream, bmlp_stats* stats) {
  return guarded([&] {
    need_handle(h);
    const bmlp_opts o = opts_or_default(opts);
    need(o.rms_variant == 0 || o.rms_variant == 1, BMLP_EINVAL, "rms_variant must be 0 or 1");
    check_bits_arg(R1, "R1", n, n, ld);
    check_bits_arg(Rstar, "Rstar", n, n, ld);
    need(!overlap(range_of(R1, n, ld), range_of(Rstar, n, ld)), BMLP_EALIAS, "Rstar overlaps R1");
    DeviceGuard dg(h->device);
    hipStream_t s = (hipStream_t)stream;
    if (o.check_padding) check_padding(h, R1, n, n, ld, s, "R1");
    StatsRec sr(stats, h, s, &o);
    if (stats) stats->arm = product_arm(o, n, n, n);
    if (n > 0) {
      // The closure by squaring (BMLP-RMS), or -- forced, or where the learned model predicts it cheaper --
      // by the selection from every source (Eq. 5 with V = I): the same bits.
      const bool sel_ok = o.rms_variant == 0 && n <= smp_rows_max_n();
      bool by_sel = sel_ok && o.dispatch == BMLP_DISPATCH_FORCED && o.smp_arm == BMLP_ARM_SMP_CLOSURE_SELECT;
      GraphInfo gi;
      if (sel_ok && o.dispatch == BMLP_DISPATCH_LEARNED && h->model) {
        // outputs 2 (the closure by squaring, then its rows read) and 3 (the one-launch selection of the n
        // identity rows), as for a session's closure
        double delta0 = (double)n;
        by_sel = call_stats_decide(h, R1, ld, n, nullptr, 0, 0, n, 0.f, 0, 0x4u | 0x8u, o, s, &gi, &delta0) == 3;
      }
      if (by_sel) {
        if (gi.n != n) gi = graph_info(h, R1, ld, n, o, s);
        if (stats) stats->arm = BMLP_ARM_SMP_CLOSURE_SELECT;
        if (h->trace) h->trace->call_arm = BMLP_ARM_SMP_CLOSURE_SELECT;
        Csr pre;
        pre.deg = gi.deg;  // R1's row counts, just left in S_DEG by the statistics pass
        closure_by_selection(h, R1, ld, n, Rstar, ld, gi, pre, o, s, sr);
      } else {
        rms_core(h, R1, ld, Rstar, ld, n, o, s, sr);
      }
    }
    sr.finish();
  });
}

bmlp_status bmlp_smp(bmlp_handle h, const uint64_t* R1, int64_t n, int64_t ld, const uint64_t* V, uint64_t* Vstar,
                     int64_t k, int64_t ldv, const bmlp_opts* opts, void* stream, bmlp_stats* stats) {
  return guarded([&] {
    need_handle(h);
    const bmlp_opts o = opts_or_default(opts);
    check_bits_arg(R1, "R1", n, n, ld);
    check_bits_arg(V, "V", k, n, ldv);
    check_bits_arg(Vstar, "Vstar", k, n, ldv);
    const Range rv = range_of(Vstar, k, ldv);
    need(!overlap(rv, range_of(V, k, ldv)), BMLP_EALIAS, "Vstar overlaps V");
    need(!overlap(rv, range_of(R1, n, ld)), BMLP_EALIAS, "Vstar overlaps R1");
    const bool forced = o.dispatch == BMLP_DISPATCH_FORCED && o.smp_arm != BMLP_ARM_AUTO;
    if (forced)
      need(o.smp_arm == BMLP_ARM_SMP_DENSE || o.smp_arm == BMLP_ARM_SMP_SPARSE || o.smp_arm == BMLP_ARM_SMP_CLOSURE ||
               o.smp_arm == BMLP_ARM_SMP_SPARSE_ROUNDS || o.smp_arm == BMLP_ARM_SMP_ADAPTIVE ||
               o.smp_arm == BMLP_ARM_SMP_CLOSURE_SELECT,
           BMLP_EINVAL, "smp_arm %d is not a selection arm", o.smp_arm);
    DeviceGuard dg(h->device);
    hipStream_t s = (hipStream_t)stream;
    if (o.check_padding) {
      check_padding(h, R1, n, n, ld, s, "R1");
      check_padding(h, V, k, n, ldv, s, "V");
    }
    StatsRec sr(stats, h, s, &o);
    int arm = BMLP_ARM_SMP_SPARSE;
    const int refl = o.smp_reflexive ? 1 : 0;
    if (k > 0) {
      if (n == 0) {
        hip_check(launch_fill_zero(Vstar, k * ldv, s), "fill_zero");
      } else {
        // the source count is a feature of the model's call-level choice (and of the trace) only
        const bool model_call = !forced && o.dispatch == BMLP_DISPATCH_LEARNED && h->model;
        GraphInfo gi;
        if (model_call || h->trace) {
          // the statistics, the source bits, the features and the model's choice in one device pass
          u32 allowed = 0x5u;  // rounds, closure
          if (n <= smp_rows_max_n()) allowed |= 0x8u;  // one-launch sparse
          double delta0 = 0.0;
          const int d = call_stats_decide(h, R1, ld, n, V, k, ldv, k, 0.f, refl, model_call ? allowed : 0u, o, s, &gi,
                                          &delta0);
          if (forced) arm = o.smp_arm;
          else if (model_call) arm = d == 2 ? BMLP_ARM_SMP_CLOSURE : d == 3 ? BMLP_ARM_SMP_SPARSE : BMLP_ARM_SMP_ADAPTIVE;
          else arm = smp_plain_arm(gi.n, k, gi.m);
        } else {
          gi = graph_info(h, R1, ld, n, o, s);
          arm = smp_choose_arm(h, o, gi, k, 0, refl, 0.0, s, nullptr);
        }
        // R1's row counts, when graph_info just left them in S_DEG, spare the CSR build its counting pass
        Csr pre;
        pre.deg = gi.deg;
        smp_core(h, R1, ld, n, V, Vstar, k, ldv, refl, arm, gi, 0, pre, o, s, sr);
      }
    }
    if (stats) stats->arm = arm;
    sr.finish();
    if (h->trace && stats) h->trace->total_ms = (float)stats->device_ms;
  });
}

// The selection of bmlp_smp by its one-launch sparse kernel with the relation's CSR (and, from mean degree
// 4, its CSC) built in the file-scope scratch array: no allocation of any kind.  Layout of the scratch
// (256-byte aligned parts): the round counter, out-degrees, row offsets, in-degrees, fill cursors,
// in-edge offsets, then the column indices of the CSR and the CSC.
bmlp_status bmlp_smp_noalloc(bmlp_handle h, const uint64_t* R1, int64_t n, int64_t ld, const uint64_t* V,
                             uint64_t* Vstar, int64_t k, int64_t ldv, int32_t reflexive, void* stream) {
  return guarded([&] {
    need_handle(h);
    need(n <= smp_rows_max_n(), BMLP_EINVAL, "bmlp_smp_noalloc supports n <= %lld", (long long)smp_rows_max_n());
    check_bits_arg(R1, "R1", n, n, ld);
    check_bits_arg(V, "V", k, n, ldv);
    check_bits_arg(Vstar, "Vstar", k, n, ldv);
    const Range rv = range_of(Vstar, k, ldv);
    need(!overlap(rv, range_of(V, k, ldv)), BMLP_EALIAS, "Vstar overlaps V");
    need(!overlap(rv, range_of(R1, n, ld)), BMLP_EALIAS, "Vstar overlaps R1");
    if (k == 0) return;
    DeviceGuard dg(h->device);
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
      hip_check(launch_fill_zero(Vstar, k * ldv, s), "fill_zero");
      return;
    }
    need(h->scratch != nullptr, BMLP_EDEVICE, "the scratch array has no address on device %d", h->device);
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t n1 = (size_t)n + 1;
    const size_t o_deg = 256, o_rp = o_deg + up(4 * n1), o_degt = o_rp + up(8 * n1), o_cur = o_degt + up(4 * n1),
                 o_rpt = o_cur + up(4 * n1), o_ci = o_rpt + up(8 * n1);
    need(o_ci <= kScratchBytes, BMLP_ENOMEM, "scratch (%zu bytes) too small for n = %lld", kScratchBytes, (long long)n);
    unsigned char* sp = h->scratch;
    u32* rounds = (u32*)sp;
    int32_t* deg = (int32_t*)(sp + o_deg);
    i64* rp = (i64*)(sp + o_rp);
    hip_check(launch_row_popcount(R1, n, n, ld, deg, nullptr, s), "row_popcount");
    hip_check(launch_scan_rowptr(deg, n, rp, s), "scan");
    // the edge count sizes the index: one readback into the handle's pinned flag words
    hip_check(hipMemcpyAsync(h->h_flags + F_CNT, rp + n, sizeof(i64), hipMemcpyDeviceToHost, s), "memcpy");
    hip_check(hipStreamSynchronize(s), "sync");
    i64 m = 0;
    std::memcpy(&m, h->h_flags + F_CNT, sizeof m);
    const bool csc = m > 0 && (double)m >= kBottomUpMinDegree * (double)n;
    const size_t o_cit = o_ci + up(4 * (size_t)std::max<i64>(m, 1));
    const size_t end = csc ? o_cit + up(4 * (size_t)m) : o_cit;
    need(end <= kScratchBytes, BMLP_ENOMEM, "scratch (%zu bytes) too small for n = %lld with %lld edges (%zu bytes)",
         kScratchBytes, (long long)n, (long long)m, end);
    int32_t* ci = (int32_t*)(sp + o_ci);
    hip_check(launch_bits_to_csr(R1, n, n, ld, rp, ci, s), "bits_to_csr");
    const i64* rpt = nullptr;
    const int32_t* cit = nullptr;
    if (csc) {
      i64* t_rp = (i64*)(sp + o_rpt);
      int32_t* t_ci = (int32_t*)(sp + o_cit);
      hip_check(launch_csc_from_csr(rp, ci, n, m, (int32_t*)(sp + o_degt), (int32_t*)(sp + o_cur), t_rp, t_ci, s),
                "csc_from_csr");
      rpt = t_rp;
      cit = t_ci;
    }
    hip_check(launch_fill_zero((u64*)rounds, 1, s), "fill_zero");  // a kernel, not a memset node
    hip_check(launch_smp_rows(V, ldv, k, rp, ci, rpt, cit, R1, ld, n, reflexive ? 1 : 0, Vstar, ldv, rounds, s),
              "smp_rows");
  });
}

// Closure under insertions (dynamic databases, a direction the conclusion names as future work).  With
// T = R+ and U = T | I, a path of R | E either avoids E (it is in T) or runs x ->U u_i ->E v_i ->U ...
// ->E v_j ->U y.  Hence (R | E)+ = T | A . M* . B, where for the b inserted edges (u_i, v_i)
//   A = columns u_i of U (n x b), B = rows v_j of U (b x n), M[i][j] = U[v_i][u_j] (b x b),
// and M* = I | M+ is the closure of the small relation among the inserted edges.  Every step is a
// product, a gather, a transpose or a closure of the library; T is updated in place.
bmlp_status bmlp_closure_insert(bmlp_handle h, uint64_t* Rplus, int64_t n, int64_t ld, const int32_t* src,
                                const int32_t* dst, int64_t b, const bmlp_opts* opts, void* stream,
                                bmlp_stats* stats) {
  return guarded([&] {
    need_handle(h);
    const bmlp_opts o = opts_or_default(opts);
    check_bits_arg(Rplus, "Rplus", n, n, ld);
    need(b >= 0, BMLP_EINVAL, "b < 0");
    if (b > 0) {
      need(src && dst, BMLP_EINVAL, "src/dst: null pointer");
      need(((uintptr_t)src & 3u) == 0 && ((uintptr_t)dst & 3u) == 0, BMLP_EALIGN, "src/dst: not 4-byte aligned");
      need(n > 0, BMLP_EINVAL, "closure_insert: edges given for an empty relation");
    }
    DeviceGuard dg(h->device);
    hipStream_t s = (hipStream_t)stream;
    if (o.check_padding) check_padding(h, Rplus, n, n, ld, s, "Rplus");
    StatsRec sr(stats, h, s, &o);
    if (b > 0) {
      const i64 nw = words_for(n), bw = words_for(b);
      hip_check(hipMemsetAsync(h->d_flags + F_COO, 0, sizeof(u32), s), "hipMemsetAsync");
      hip_check(launch_check_index(src, b, n, h->d_flags + F_COO, s), "check_index");
      hip_check(launch_check_index(dst, b, n, h->d_flags + F_COO, s), "check_index");
      need(read_flag(h, s, F_COO) == 0, BMLP_EINVAL, "closure_insert: edge endpoint outside [0,%lld)", (long long)n);
      // B = rows v_j of U (b x n): the one-hot rows of the targets, each OR-ed with its row of T
      u64* ev = ws_bits(h, S_T1, b, nw, o);
      hip_check(launch_fill_zero(ev, b * nw, s), "fill_zero");
      hip_check(launch_set_onehot(ev, nw, dst, b, n, nullptr, s), "set_onehot");
      u64* bm = ws_bits(h, S_W2, b, nw, o);
      if (n <= gather_rows_max_n())
        hip_check(launch_gather_rows(ev, nw, b, Rplus, ld, n, 1, bm, nw, s), "gather_rows");
      else
        product(h, ev, nw, Rplus, ld, ev, nw, bm, nw, nullptr, 0, b, n, n, nullptr, product_arm(o, b, n, n), s, sr);
      hip_check(launch_zero_pad(bm, b, n, nw, s), "zero_pad");
      // A = columns u_i of U (n x b); M[i][j] = B[i][u_j] (b x b)
      u64* am = ws_bits(h, S_W3, n, bw, o);
      u64* mm = ws_bits(h, S_W4, b, bw, o);
      if (n <= gather_cols_max_n()) {
        hip_check(launch_gather_cols(Rplus, ld, n, n, src, b, 1, am, bw, s), "gather_cols");
        hip_check(launch_gather_cols(bm, nw, b, n, src, b, 0, mm, bw, s), "gather_cols");
      } else {
        // P[x][i] = (x == u_i), then A = P | T . P and M = B . P
        u64* eu = ws_bits(h, S_T0, b, nw, o);
        hip_check(launch_fill_zero(eu, b * nw, s), "fill_zero");
        hip_check(launch_set_onehot(eu, nw, src, b, n, nullptr, s), "set_onehot");
        u64* pt = ws_bits(h, S_T2, n, bw, o);
        hip_check(launch_transpose(eu, b, n, nw, pt, bw, s), "transpose");
        product(h, Rplus, ld, pt, bw, pt, bw, am, bw, nullptr, 0, n, n, b, nullptr, product_arm(o, n, b, n), s, sr);
        product(h, bm, nw, pt, bw, nullptr, 0, mm, bw, nullptr, 0, b, n, b, nullptr, product_arm(o, b, b, n), s, sr);
        hip_check(launch_zero_pad(am, n, b, bw, s), "zero_pad");
        hip_check(launch_zero_pad(mm, b, b, bw, s), "zero_pad");
      }
      // M* = I | M+ (b x b)
      u64* ms = ws_bits(h, S_T0, b, bw, o);
      if (b <= 64) {
        hip_check(launch_closure64(mm, bw, b, ms, bw, s), "closure64");  // one wave, no host round trip
      } else {
        rms_core(h, mm, bw, ms, bw, b, o, s, sr);
        hip_check(launch_set_diag(ms, bw, b, b, s), "set_diag");
      }
      // X = M* . B (b x n), then T |= A . X
      u64* xm = ws_bits(h, S_T1, b, nw, o);  // the one-hot targets are no longer needed
      product(h, ms, bw, bm, nw, nullptr, 0, xm, nw, nullptr, 0, b, b, n, nullptr, product_arm(o, b, n, b), s, sr);
      hip_check(launch_zero_pad(xm, b, n, nw, s), "zero_pad");
      product(h, am, bw, xm, nw, Rplus, ld, Rplus, ld, nullptr, 0, n, b, n, nullptr, product_arm(o, n, n, b), s, sr);
      hip_check(launch_zero_pad(Rplus, n, n, ld, s), "zero_pad");
    }
    sr.finish();
  });
}

// Two-sided linear recursion p(X,Y) <- b(X,Y).  p(X,Y) <- l(X,X1), p(X1,Y1), r(Y1,Y): the least P with
// P = B | L . P . R, i.e. P = OR over k of L^k . B . R^k (same-generation when l = up, r = down; one
// of the multilinear programs the paper names as future work).  Unlike P = Rs* . Rb it has no closure
// form, so it runs semi-naive rounds: W = D . R, then P |= L . W with D the new bits.  Each of the
// two products is done by row gathers while its left operand is sparse (the rule of the RMS
// squarings), else by the product kernel, which also yields the new bits.
bmlp_status bmlp_compose_two_sided(bmlp_handle h, const uint64_t* Rbase, const uint64_t* Rleft, const uint64_t* Rright,
                                   uint64_t* P, int64_t n, int64_t ld, const bmlp_opts* opts, void* stream,
                                   bmlp_stats* stats) {
  return guarded([&] {
    need_handle(h);
    const bmlp_opts o = opts_or_default(opts);
    check_bits_arg(Rbase, "Rbase", n, n, ld);
    check_bits_arg(Rleft, "Rleft", n, n, ld);
    check_bits_arg(Rright, "Rright", n, n, ld);
    check_bits_arg(P, "P", n, n, ld);
    const Range rp = range_of(P, n, ld);
    need(!overlap(rp, range_of(Rbase, n, ld)), BMLP_EALIAS, "P overlaps Rbase");
    need(!overlap(rp, range_of(Rleft, n, ld)), BMLP_EALIAS, "P overlaps Rleft");
    need(!overlap(rp, range_of(Rright, n, ld)), BMLP_EALIAS, "P overlaps Rright");
    DeviceGuard dg(h->device);
    hipStream_t s = (hipStream_t)stream;
    if (o.check_padding) {
      check_padding(h, Rbase, n, n, ld, s, "Rbase");
      check_padding(h, Rleft, n, n, ld, s, "Rleft");
      check_padding(h, Rright, n, n, ld, s, "Rright");
    }
    StatsRec sr(stats, h, s, &o);
    int rounds = 0;
    if (n > 0) {
      const i64 nw = words_for(n);
      const int arm = product_arm(o, n, n, n);
      const bool may_gather = o.product_arm == BMLP_ARM_AUTO && n <= gather_rows_max_n();
      u64* dl = ws_bits(h, S_T0, n, nw, o);   // the new bits of the last round
      u64* wm = ws_bits(h, S_T1, n, nw, o);   // D . R
      u64* aux = ws_bits(h, S_T2, n, nw, o);  // P before the round (gathers) or the next D (products)
      hip_check(launch_ewise(4, Rbase, ld, nullptr, 0, P, ld, n, n, s), "copy");
      hip_check(launch_ewise(4, Rbase, ld, nullptr, 0, dl, nw, n, n, s), "copy");
      i64 dbits = count_bits(h, dl, n, n, nw, s);
      const i64 lbits = may_gather ? count_bits(h, Rleft, n, n, ld, s) : 0;
      unsigned long long* nb = (unsigned long long*)(h->d_flags + F_NEW);
      const GatherQueue gq = may_gather ? gather_queue(h, n, n, o) : GatherQueue{nullptr, nullptr, 0};
      const i64 cap = n * n + 1;  // every round but the last adds a fact
      while (dbits > 0) {
        need(rounds < cap, BMLP_EITER, "two-sided recursion exceeded %lld rounds", (long long)cap);
        hip_check(hipMemsetAsync(h->d_flags, 0, 8 * sizeof(u32), s), "hipMemsetAsync");
        // W = D . R
        if (may_gather && rms_gather_pays(n, dbits, arm)) {
          const GatherQueue q = sized(gq, dbits, n);
          hip_check(launch_gather_rows(dl, nw, n, Rright, ld, n, 0, wm, nw, s, nullptr, nullptr, &q), "gather_rows");
        } else {
          product(h, dl, nw, Rright, ld, nullptr, 0, wm, nw, nullptr, 0, n, n, n, nullptr, arm, s, sr);
        }
        // P |= L . W, D = the bits new to P
        if (may_gather && rms_gather_pays(n, lbits, arm)) {
          hip_check(launch_ewise(4, P, ld, nullptr, 0, aux, nw, n, n, s), "copy");
          const GatherQueue q = sized(gq, lbits, n);
          hip_check(launch_gather_rows(Rleft, ld, n, wm, nw, n, 2, P, ld, s, nullptr, nb, &q), "gather_rows");
          hip_check(launch_ewise(2, P, ld, aux, nw, dl, nw, n, n, s), "andnot");
        } else {
          product(h, Rleft, ld, wm, nw, P, ld, P, ld, aux, nw, n, n, n, nullptr, arm, s, sr, nullptr, 0, nb);
          std::swap(dl, aux);
        }
        if (sr.st) sr.st->bool_ops += (uint64_t)4 * (uint64_t)n * (uint64_t)n * (uint64_t)n;
        hip_check(hipMemcpyAsync(h->h_flags, h->d_flags, 8 * sizeof(u32), hipMemcpyDeviceToHost, s), "memcpy");
        hip_check(hipStreamSynchronize(s), "sync");
        unsigned long long added = 0;
        std::memcpy(&added, h->h_flags + F_NEW, sizeof added);
        dbits = (i64)added;
        ++rounds;
      }
      hip_check(launch_zero_pad(P, n, n, ld, s), "zero_pad");
    }
    if (sr.st) sr.st->iterations = rounds;
    sr.finish();
  });
}

bmlp_status bmlp_compose_linear(bmlp_handle h, const uint64_t* Rbase, const uint64_t* Rstep, uint64_t* P, int64_t n,
                                int64_t ld, const bmlp_opts* opts, void* stream, bmlp_stats* stats) {
  return guarded([&] {
    need_handle(h);
    const bmlp_opts o = opts_or_default(opts);
    check_bits_arg(Rbase, "Rbase", n, n, ld);
    check_bits_arg(Rstep, "Rstep", n, n, ld);
    check_bits_arg(P, "P", n, n, ld);
    const Range rp = range_of(P, n, ld);
    need(!overlap(rp, range_of(Rbase, n, ld)), BMLP_EALIAS, "P overlaps Rbase");
    need(!overlap(rp, range_of(Rstep, n, ld)), BMLP_EALIAS, "P overlaps Rstep");
    const bool forced = o.dispatch == BMLP_DISPATCH_FORCED && o.compose_arm != BMLP_ARM_AUTO;
    if (forced) {
      need(o.compose_arm == BMLP_ARM_COMPOSE_RMS || o.compose_arm == BMLP_ARM_COMPOSE_SEMINAIVE ||
               o.compose_arm == BMLP_ARM_COMPOSE_ROWWISE,
           BMLP_EINVAL, "compose_arm %d is not a composition arm", o.compose_arm);
      need(o.compose_arm != BMLP_ARM_COMPOSE_ROWWISE || n <= gather_rows_max_n(), BMLP_EINVAL,
           "the row-wise composition arm supports n <= %lld", (long long)gather_rows_max_n());
    }
    if (o.dispatch == BMLP_DISPATCH_FORCED && o.smp_arm != BMLP_ARM_AUTO)
      need(o.smp_arm == BMLP_ARM_SMP_DENSE || o.smp_arm == BMLP_ARM_SMP_SPARSE || o.smp_arm == BMLP_ARM_SMP_CLOSURE ||
               o.smp_arm == BMLP_ARM_SMP_SPARSE_ROUNDS || o.smp_arm == BMLP_ARM_SMP_ADAPTIVE ||
               o.smp_arm == BMLP_ARM_SMP_CLOSURE_SELECT,
           BMLP_EINVAL, "smp_arm %d is not a selection arm", o.smp_arm);
    DeviceGuard dg(h->device);
    hipStream_t s = (hipStream_t)stream;
    if (o.check_padding) {
      check_padding(h, Rbase, n, n, ld, s, "Rbase");
      check_padding(h, Rstep, n, n, ld, s, "Rstep");
    }
    StatsRec sr(stats, h, s, &o);
    int arm = forced ? o.compose_arm : BMLP_ARM_COMPOSE_SEMINAIVE;
    if (n > 0) {
      const i64 nw = words_for(n);
      // Three routes to P = Rs* . Rb:
      //  (i)   closure: Rs+ by BMLP-RMS, then P = Rb | Rs+ . Rb;
      //  (ii)  columns: P^T = Rb^T . (Rs^T)*, the columns of P as reflexive selections over the
      //        transposed step relation (n query rows);
      //  (iii) rows: P[X] = Rb[X] | OR of Rb[Z] over Z in e_X . Rs+, a strict selection from each
      //        row X that has a step edge, then the rows of Rb gathered; other rows are Rb's.
      GraphInfo gs;
      gs.n = n;
      const bool learned = o.dispatch == BMLP_DISPATCH_LEARNED && h->model && !forced;
      const bool rowwise_ok = n <= gather_rows_max_n();
      int sarm = (o.dispatch == BMLP_DISPATCH_FORCED && o.smp_arm != BMLP_ARM_AUTO) ? o.smp_arm : BMLP_ARM_AUTO;
      if (learned || h->trace) {
        // outputs: 0 columns by adaptive rounds, 1 rows, 2 closure, 3 columns by the one-launch kernel
        u32 allowed = 0x5u;
        if (rowwise_ok) allowed |= 0x2u;
        if (n <= smp_rows_max_n()) allowed |= 0x8u;
        double delta0 = 0.0;
        const int d = call_stats_decide(h, Rstep, ld, n, Rbase, n, ld, n, 1.f, 1, learned ? allowed : 0u, o, s, &gs,
                                        &delta0);
        if (learned) {
          arm = d == 1 ? BMLP_ARM_COMPOSE_ROWWISE : d == 2 ? BMLP_ARM_COMPOSE_RMS : BMLP_ARM_COMPOSE_SEMINAIVE;
          if (d == 0) sarm = BMLP_ARM_SMP_ADAPTIVE;
          if (d == 3) sarm = BMLP_ARM_SMP_SPARSE;
        }
      } else {
        gs = graph_info(h, Rstep, ld, n, o, s);
      }
      if (arm == BMLP_ARM_COMPOSE_SEMINAIVE) {
        u64* rbt = ws_bits(h, S_T0, n, nw, o);
        u64* rst = ws_bits(h, S_T1, n, nw, o);
        u64* pt = ws_bits(h, S_T2, n, nw, o);
        hip_check(launch_transpose(Rbase, n, n, ld, rbt, nw, s), "transpose");
        hip_check(launch_transpose(Rstep, n, n, ld, rst, nw, s), "transpose");
        if (sarm == BMLP_ARM_AUTO) sarm = smp_plain_arm(n, n, gs.m);
        smp_core(h, rst, nw, n, rbt, pt, n, nw, 1, sarm, gs, 1, Csr{}, o, s, sr);
        hip_check(launch_transpose(pt, n, n, nw, P, ld, s), "transpose");
      } else if (arm == BMLP_ARM_COMPOSE_ROWWISE) {
        i64* rp;
        int32_t* ci;
        build_csr(h, Rstep, ld, n, o, s, &rp, &ci);
        const int32_t* deg = (const int32_t*)ws(h, S_DEG, (size_t)n * sizeof(int32_t), o);
        std::vector<int32_t> hdeg((size_t)n), rows;
        hip_check(hipMemcpyAsync(hdeg.data(), deg, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost, s), "memcpy");
        hip_check(hipStreamSynchronize(s), "sync");
        rows.reserve((size_t)gs.nonempty);
        for (i64 i = 0; i < n; ++i)
          if (hdeg[(size_t)i] > 0) rows.push_back((int32_t)i);
        const i64 kr = (i64)rows.size();
        hip_check(launch_ewise(4, Rbase, ld, nullptr, 0, P, ld, n, n, s), "copy");
        if (kr > 0) {
          int32_t* drows = (int32_t*)ws(h, S_T2, (size_t)kr * sizeof(int32_t), o);
          u64* v1 = ws_bits(h, S_T0, kr, nw, o);
          u64* sel = ws_bits(h, S_T1, kr, nw, o);
          hip_check(hipMemcpyAsync(drows, rows.data(), (size_t)kr * sizeof(int32_t), hipMemcpyHostToDevice, s),
                    "memcpy");
          hip_check(launch_fill_zero(v1, kr * nw, s), "fill_zero");
          hip_check(launch_set_onehot(v1, nw, drows, kr, n, nullptr, s), "set_onehot");
          if (sarm == BMLP_ARM_AUTO || sarm == BMLP_ARM_SMP_ADAPTIVE) sarm = smp_plain_arm(n, kr, gs.m);
          smp_core(h, Rstep, ld, n, v1, sel, kr, nw, 0, sarm, gs, 1, Csr{rp, ci}, o, s, sr);
          // the selected rows hold as many bits as Rstep's closure rows (thousands where it is large): the
          // pieces are sized on the device from their count, twice the mean row, instead of the default 64,
          // which split such rows into many pieces merged with atomics
          GatherQueue gq = gather_queue(h, kr, n, o);
          if (gq.e) {
            unsigned long long* vb = (unsigned long long*)(h->d_flags + F_VBITS);
            hip_check(launch_fill_zero((u64*)vb, 1, s), "fill_zero");
            hip_check(launch_popcount_total(sel, kr, n, nw, vb, s), "popcount_total");
            gq.bits = vb;
          }
          hip_check(launch_gather_rows(sel, nw, kr, Rbase, ld, n, 2, P, ld, s, drows, nullptr, &gq), "gather_rows");
          // the host list is read by the upload above; wait before it goes out of scope
          hip_check(hipStreamSynchronize(s), "sync");
        }
        hip_check(launch_zero_pad(P, n, n, ld, s), "zero_pad");
      } else {
        u64* sp = ws_bits(h, S_W2, n, nw, o);
        bmlp_opts o2 = o;
        o2.rms_variant = 0;
        rms_core(h, Rstep, ld, sp, nw, n, o2, s, sr);
        product(h, sp, nw, Rbase, ld, Rbase, ld, P, ld, nullptr, 0, n, n, n, nullptr, product_arm(o, n, n, n), s, sr);
        hip_check(launch_zero_pad(P, n, n, ld, s), "zero_pad");
      }
      if (h->trace) h->trace->call_arm = arm;
    }
    if (stats) stats->arm = arm;
    sr.finish();
    if (h->trace && stats) h->trace->total_ms = (float)stats->device_ms;
  });
}

bmlp_status bmlp_batched(bmlp_handle h, const bmlp_graph_desc* graphs, int32_t count, const bmlp_opts* opts,
                         void* stream, bmlp_stats* stats) {
  return guarded([&] {
    need_handle(h);
    const bmlp_opts o = opts_or_default(opts);
    need(count >= 0, BMLP_EINVAL, "count < 0");
    if (count == 0) return;
    need(graphs != nullptr, BMLP_EINVAL, "graphs: null pointer");
    for (int32_t i = 0; i < count; ++i) {
      const bmlp_graph_desc& d = graphs[i];
      need(d.n >= 0 && d.k >= 0, BMLP_EINVAL, "graph %d: negative size", i);
      check_bits_arg(d.R1, "R1", d.n, d.n, d.ld);
      if (d.closure) {
        check_bits_arg(d.closure, "closure", d.n, d.n, d.ldc);
        need(!overlap(range_of(d.closure, d.n, d.ldc), range_of(d.R1, d.n, d.ld)), BMLP_EALIAS,
             "graph %d: closure overlaps R1", i);
      }
      if (d.k > 0) {
        check_bits_arg(d.V, "V", d.k, d.n, d.ldv);
        check_bits_arg(d.Vstar, "Vstar", d.k, d.n, d.ldv);
        const Range rv = range_of(d.Vstar, d.k, d.ldv);
        need(!overlap(rv, range_of(d.V, d.k, d.ldv)) && !overlap(rv, range_of(d.R1, d.n, d.ld)), BMLP_EALIAS,
             "graph %d: Vstar overlaps an input", i);
      }
    }
    DeviceGuard dg(h->device);
    hipStream_t s = (hipStream_t)stream;

    // biggest graphs first: their tiles are claimed first in every round (longest-processing-time order)
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return graphs[a].n > graphs[b].n; });
    BatchPlan plan{0, 0, 0, 0, 0, 0, 0, 0, 0};
    // Query answers: the plain schedule takes the paper's mapping of a partially grounded query to
    // BMLP-SMP (a selection per query row); forced, all by selection or all off the closures; learned, a
    // graph whose closure is an output reads its answers off it (the closure is computed anyway), and
    // for the others the dispatcher model chooses on the device between the closure and selection (a
    // graph whose closure is neither an output nor read is not squared at all).  Graphs beyond the
    // selection kernel's size always read the closure.
    const bool forced_sel = o.dispatch == BMLP_DISPATCH_FORCED && o.smp_arm != BMLP_ARM_AUTO;
    need(!forced_sel || o.smp_arm != BMLP_ARM_SMP_CLOSURE_SELECT, BMLP_EINVAL,
         "the batched launch squares its closures (smp_arm %d is not available there)", o.smp_arm);
    const bool learned = o.dispatch == BMLP_DISPATCH_LEARNED && h->model;
    plan.qmode = forced_sel ? (o.smp_arm == BMLP_ARM_SMP_CLOSURE ? 0 : 1) : learned ? 2 : 1;
    if (plan.qmode == 2) {
      // the model has a choice only for graphs with query rows, no closure output and a size the selection
      // kernels take; without one, every graph reads its answers off its closure and the model is not run
      bool choice = false;
      for (int i = 0; i < count; ++i)
        choice |= graphs[i].k > 0 && graphs[i].closure == nullptr && graphs[i].n <= batch_bfs_max_n();
      if (!choice) plan.qmode = 0;
    }
    size_t buf_words = 0;
    BatchPlan sizes{0, 0, 0, 0, 0, 0, 0, 0, 0};  // the totals the flag area depends on
    for (int i = 0; i < count; ++i) {
      const bmlp_graph_desc& d = graphs[i];
      plan.rounds = std::max(plan.rounds, ceil_log2(std::max<int64_t>(d.n, 2)) + 2);
      // ping-pong pair, plus R^T for the graphs that square on the matrix cores
      const bool mfma = d.n >= batch_mfma_min_n();
      buf_words += (size_t)((mfma ? 3 : 2) * d.n * words_for(d.n));
      if (mfma) sizes.total_mblocks += (d.n + 255) / 256;
      sizes.total_sgroups += (std::max<int64_t>(d.n, d.k) + 63) / 64;
    }
    sizes.rounds = plan.rounds;
    const size_t table_bytes = ((size_t)count * sizeof(BatchGraph) + 255) & ~(size_t)255;
    const size_t nflags = (size_t)batch_flag_words(count, sizes);
    const size_t flag_bytes = (nflags * sizeof(u32) + 255) & ~(size_t)255;
    char* base = (char*)ws(h, S_BATCH, table_bytes + flag_bytes + buf_words * sizeof(u64), o);
    BatchGraph* d_table = (BatchGraph*)base;
    u32* d_flags = (u32*)(base + table_bytes);
    u64* bufs = (u64*)(base + table_bytes + flag_bytes);

    std::vector<BatchGraph> tab(count);
    size_t off = 0;
    for (int j = 0; j < count; ++j) {
      const bmlp_graph_desc& d = graphs[order[j]];
      BatchGraph& G = tab[j];
      G.n = d.n;
      G.nw = words_for(d.n);
      G.closure_req = d.closure ? 1 : 0;
      G.R1 = d.R1;
      G.ld = d.ld;
      G.closure = d.closure;
      G.ldc = d.closure ? d.ldc : 0;
      G.V = d.V;
      G.k = d.k;
      G.ldv = d.ldv;
      G.Vstar = d.Vstar;
      G.buf0 = bufs + off;
      G.buf1 = bufs + off + (size_t)(d.n * G.nw);
      off += (size_t)(2 * d.n * G.nw);
      G.row_begin = plan.total_rows;
      G.tile_begin = plan.total_tiles;
      G.rtiles = batch_rtiles(d.n);
      G.smp_tile_begin = plan.total_select_tiles;
      G.qrow_begin = plan.total_qrows;
      G.mfma_tile_begin = plan.total_mfma_tiles;
      G.tblock_begin = plan.total_tblocks;
      G.mblock_begin = plan.total_mblocks;
      G.sgroup_begin = plan.total_sgroups;
      plan.total_sgroups += (std::max<int64_t>(d.n, d.k) + 63) / 64;
      const bool mfma = d.n >= batch_mfma_min_n();
      G.bt = mfma ? bufs + off : nullptr;
      G.mfma_rtiles = mfma ? (d.n + 255) / 256 : 0;
      if (mfma) {
        off += (size_t)(d.n * G.nw);
        plan.total_mfma_tiles += G.mfma_rtiles * G.mfma_rtiles;
        plan.total_tblocks += G.nw * G.nw;
        plan.total_mblocks += G.mfma_rtiles;
      }
      plan.total_rows += (std::max<int64_t>(d.n, d.k) + 7) / 8 * 8;  // groups of 8 rows never span two graphs
      plan.total_tiles += mfma ? 4 * G.mfma_rtiles : batch_tiles(d.n);  // 64-row tiles of an MFMA graph
      plan.total_select_tiles += d.k > 0 ? batch_select_tiles(d.k, d.n) : 0;
      plan.total_qrows += d.k;
      if (d.k > 0 && d.n > 0 && d.n <= batch_ms_max_n()) {
        plan.ms_max_n = std::max<i64>(plan.ms_max_n, d.n);
        plan.ms_qrows += d.k;
      }
    }
    need((size_t)batch_flag_words(count, plan) == nflags, BMLP_EDEVICE, "batched plan: flag area mismatch");
    // the captured chain is reused while the batch (and its workspace) is unchanged
    uint64_t key = 1469598103934665603ull;
    auto mix = [&](const void* p, size_t nb) {
      const unsigned char* b = (const unsigned char*)p;
      for (size_t i = 0; i < nb; ++i) key = (key ^ b[i]) * 1099511628211ull;
    };
    mix(graphs, sizeof(bmlp_graph_desc) * (size_t)count);
    mix(&base, sizeof base);
    mix(&plan.qmode, sizeof plan.qmode);
    if (!h->bexec || key != h->bkey) {
      if (h->bexec) {
        hip_check(hipGraphExecDestroy(h->bexec), "hipGraphExecDestroy");
        h->bexec = nullptr;
      }
      if (h->bgraph) {
        hip_check(hipGraphDestroy(h->bgraph), "hipGraphDestroy");
        h->bgraph = nullptr;
      }
      hip_check(hipMemcpyAsync(d_table, tab.data(), sizeof(BatchGraph) * (size_t)count, hipMemcpyHostToDevice, s),
                "hipMemcpyAsync");
      hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
      if (!h->capture_stream)
        hip_check(hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking), "hipStreamCreate");
      hip_check(hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
      const hipError_t le =
          launch_batch_chain(d_table, count, plan, d_flags, learned ? h->d_model : nullptr, h->capture_stream);
      hipGraph_t graph = nullptr;
      const hipError_t ce = hipStreamEndCapture(h->capture_stream, &graph);
      hip_check(le, "batch chain");
      hip_check(ce, "hipStreamEndCapture");
      h->bgraph = graph;
      hip_check(hipGraphInstantiate(&h->bexec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
      h->bkey = key;
    }
    StatsRec sr(stats, h, s, &o);
    hip_check(hipGraphLaunch(h->bexec, s), "hipGraphLaunch");
    if (stats) {
      sr.finish();
      std::vector<u32> fl(nflags);
      hip_check(hipMemcpyAsync(fl.data(), d_flags, nflags * sizeof(u32), hipMemcpyDeviceToHost, s), "memcpy");
      hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
      int max_rounds = 0, by_closure = 0, by_selection = 0;
      const u32* qsel = fl.data() + batch_qsel_offset(count, plan);
      const u32* needc = qsel + count;
      for (int j = 0; j < count; ++j) {
        const uint64_t nn = (uint64_t)tab[j].n;
        const bool sel = qsel[j] != 0;
        if (tab[j].k > 0) ++(sel ? by_selection : by_closure);
        if (!needc[j]) continue;  // not squared
        int r = 0;
        while (r < plan.rounds && fl[(size_t)j * plan.rounds + r]) ++r;
        need(r < plan.rounds, BMLP_EITER, "batched RMS exceeded %d rounds (graph of n=%lld)", plan.rounds,
             (long long)tab[j].n);
        const int prods = r + 1;  // the rounds that changed plus the one that found the fixpoint
        max_rounds = std::max(max_rounds, prods);
        const bool gathered = tab[j].k > 0 && !sel;
        stats->products += prods + (gathered ? 1 : 0);
        stats->bool_ops += (uint64_t)prods * 2u * nn * nn * nn + (gathered ? 2u * (uint64_t)tab[j].k * nn * nn : 0u);
      }
      stats->iterations = max_rounds;
      stats->arm = by_selection == 0 ? BMLP_ARM_SMP_CLOSURE : by_closure == 0 ? BMLP_ARM_SMP_SPARSE : BMLP_ARM_AUTO;
      stats->arm_trace[0] = by_closure;  // graphs (with queries) answered off their closure
      stats->arm_trace[1] = by_selection;  // graphs answered by per-row selection
      stats->product_bool_ops = stats->bool_ops;
      stats->product_ms = stats->device_ms;
    }
  });
}

}  // extern "C"

// ------------------------------------------------------------ sessions over one relation
struct bmlp_graph_s {
  bmlp_ctx* c = nullptr;
  const u64* R1 = nullptr;
  i64 n = 0, ld = 0;
  GraphInfo gi;
  i64* rp = nullptr;        // owned CSR of R1
  int32_t* ci = nullptr;
  i64* rpt = nullptr;       // owned CSC of R1 (when the mean degree makes bottom-up rounds pay)
  int32_t* cit = nullptr;
  u64* closure = nullptr;   // owned R1+ (n x ceil(n/64)) once computed
  double spent_ms = 0.0;    // device time spent answering queries without the closure
  double p_sel_all_ms = -1; // the model's predicted time of the closure by selection (learned sessions)
  int32_t closure_arm = -1; // how the closure was built, until the query that built it has reported it
  int32_t last_arm = -1;    // the arm that served the last query
};

namespace {

// ------------------------------------------------------------ model file
uint32_t crc32_bytes(const void* data, size_t n, uint32_t crc = 0) {
  // CRC-32 (IEEE 802.3, reflected polynomial 0xEDB88320), bit by bit
  const unsigned char* p = (const unsigned char*)data;
  crc = ~crc;
  for (size_t i = 0; i < n; ++i) {
    crc ^= p[i];
    for (int b = 0; b < 8; ++b) crc = (crc >> 1) ^ (0xEDB88320u & (0u - (crc & 1u)));
  }
  return ~crc;
}

constexpr char kMagic[8] = {'B', 'M', 'L', 'P', 'M', 'L', 'P', '1'};
struct ModelHeader {
  char magic[8];
  uint32_t version, n_in, h1, h2, n_out, n_params;
};

void model_to_device(bmlp_ctx* c) {
  if (!c->d_model) hip_check(hipMalloc((void**)&c->d_model, (kParams + 2 * kIn) * sizeof(float)), "hipMalloc");
  hip_check(hipMemcpy(c->d_model, c->h_model.data(), (kParams + 2 * kIn) * sizeof(float), hipMemcpyHostToDevice),
            "hipMemcpy");
  c->model = true;
}

// splitmix64: a small counter-based generator for the initial weights
uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

struct DevBuf {
  void* p = nullptr;
  DevBuf() = default;
  explicit DevBuf(size_t bytes) {
    if (hipMalloc(&p, std::max<size_t>(bytes, 16)) != hipSuccess) {
      (void)hipGetLastError();
      fail(BMLP_ENOMEM, "hipMalloc of %zu bytes failed", bytes);
    }
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  DevBuf(DevBuf&& o) noexcept : p(o.p) { o.p = nullptr; }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  float* f() const { return (float*)p; }
};

// one forward + backward pass over (X, T, M) with parameters P; returns the loss, G receives the gradient
float mlp_pass(const float* P, const float* mu, const float* sd, const float* X, const float* T, const float* M,
               i64 rows, float inv_m, DevBuf* act, float* G, hipStream_t s) {
  float* H1 = act[0].f();
  float* H2 = act[1].f();
  float* Y = act[2].f();
  float* dY = act[3].f();
  float* dH2 = act[4].f();
  float* dH1 = act[5].f();
  float* loss = act[6].f();
  hip_check(launch_mlp_forward(P, mu, sd, X, rows, H1, H2, Y, s), "mlp_forward");
  hip_check(hipMemsetAsync(loss, 0, sizeof(float), s), "hipMemsetAsync");
  hip_check(launch_mlp_backward(P, mu, sd, X, H1, H2, Y, T, M, rows, inv_m, dY, dH2, dH1, G, loss, s), "mlp_backward");
  float l = 0.f;
  hip_check(hipMemcpyAsync(&l, loss, sizeof(float), hipMemcpyDeviceToHost, s), "memcpy");
  hip_check(hipStreamSynchronize(s), "sync");
  return l;
}

void alloc_acts(DevBuf* act, i64 rows) {
  new (&act[0]) DevBuf((size_t)rows * kH1 * sizeof(float));
  new (&act[1]) DevBuf((size_t)rows * kH2 * sizeof(float));
  new (&act[2]) DevBuf((size_t)rows * kOut * sizeof(float));
  new (&act[3]) DevBuf((size_t)rows * kOut * sizeof(float));
  new (&act[4]) DevBuf((size_t)rows * kH2 * sizeof(float));
  new (&act[5]) DevBuf((size_t)rows * kH1 * sizeof(float));
  new (&act[6]) DevBuf(sizeof(float));
}

DevBuf upload(const float* host, size_t count, hipStream_t s) {
  DevBuf b(count * sizeof(float));
  if (count) hip_check(hipMemcpyAsync(b.p, host, count * sizeof(float), hipMemcpyHostToDevice, s), "memcpy");
  return b;
}

}  // namespace

extern "C" {

bmlp_status bmlp_set_trace(bmlp_handle h, bmlp_trace* trace) {
  return guarded([&] {
    need_handle(h);
    h->trace = trace;
    if (trace) {
      std::memset(trace, 0, sizeof *trace);
      trace->call_arm = -1;
    }
  });
}

int32_t bmlp_dispatcher_loaded(bmlp_handle h) { return (h && h->model) ? 1 : 0; }

bmlp_status bmlp_dispatcher_load(bmlp_handle h, const char* path) {
  return guarded([&] {
    need_handle(h);
    need(path != nullptr, BMLP_EINVAL, "path: null pointer");
    FILE* fp = std::fopen(path, "rb");
    need(fp != nullptr, BMLP_EMODEL, "cannot open model file %s", path);
    std::vector<unsigned char> buf;
    unsigned char tmp[4096];
    size_t got;
    while ((got = std::fread(tmp, 1, sizeof tmp, fp)) > 0) buf.insert(buf.end(), tmp, tmp + got);
    std::fclose(fp);
    const size_t body = sizeof(ModelHeader) + (size_t)(kParams + 2 * kIn) * sizeof(float);
    need(buf.size() == body + 4, BMLP_EMODEL, "model file %s has %zu bytes, expected %zu", path, buf.size(), body + 4);
    ModelHeader hd;
    std::memcpy(&hd, buf.data(), sizeof hd);
    need(std::memcmp(hd.magic, kMagic, 8) == 0 && hd.version == 1 && hd.n_in == (uint32_t)kIn &&
             hd.h1 == (uint32_t)kH1 && hd.h2 == (uint32_t)kH2 && hd.n_out == (uint32_t)kOut &&
             hd.n_params == (uint32_t)kParams,
         BMLP_EMODEL, "model file %s: wrong header", path);
    uint32_t crc;
    std::memcpy(&crc, buf.data() + body, 4);
    need(crc32_bytes(buf.data(), body) == crc, BMLP_EMODEL, "model file %s: checksum mismatch", path);
    std::vector<float> m((size_t)(kParams + 2 * kIn));
    std::memcpy(m.data(), buf.data() + sizeof(ModelHeader), m.size() * sizeof(float));
    // file layout: mu | sd | params; device layout: params | mu | sd
    std::vector<float> dev((size_t)(kParams + 2 * kIn));
    std::memcpy(dev.data(), m.data() + 2 * kIn, kParams * sizeof(float));
    std::memcpy(dev.data() + kParams, m.data(), 2 * kIn * sizeof(float));
    for (int i = 0; i < kIn; ++i) need(dev[kParams + kIn + i] > 0.f, BMLP_EMODEL, "model file %s: bad scale", path);
    DeviceGuard dg(h->device);
    h->h_model = dev;
    model_to_device(h);
  });
}

bmlp_status bmlp_dispatcher_save(bmlp_handle h, const char* path) {
  return guarded([&] {
    need_handle(h);
    need(path != nullptr, BMLP_EINVAL, "path: null pointer");
    need(h->model, BMLP_EMODEL, "no model to save");
    ModelHeader hd;
    std::memcpy(hd.magic, kMagic, 8);
    hd.version = 1;
    hd.n_in = kIn;
    hd.h1 = kH1;
    hd.h2 = kH2;
    hd.n_out = kOut;
    hd.n_params = kParams;
    std::vector<unsigned char> buf(sizeof hd + (size_t)(kParams + 2 * kIn) * sizeof(float));
    std::memcpy(buf.data(), &hd, sizeof hd);
    std::memcpy(buf.data() + sizeof hd, h->h_model.data() + kParams, 2 * kIn * sizeof(float));
    std::memcpy(buf.data() + sizeof hd + 2 * kIn * sizeof(float), h->h_model.data(), kParams * sizeof(float));
    const uint32_t crc = crc32_bytes(buf.data(), buf.size());
    FILE* fp = std::fopen(path, "wb");
    need(fp != nullptr, BMLP_EINVAL, "cannot write %s", path);
    const bool ok = std::fwrite(buf.data(), 1, buf.size(), fp) == buf.size() && std::fwrite(&crc, 4, 1, fp) == 1;
    std::fclose(fp);
    need(ok, BMLP_EINVAL, "short write to %s", path);
  });
}

bmlp_status bmlp_dispatcher_train(bmlp_handle h, const float* X, const float* T, const float* M, int64_t rows,
                                  int32_t epochs, float lr, uint64_t seed, float* loss_out) {
  return guarded([&] {
    need_handle(h);
    need(rows > 0 && X && T && M, BMLP_EINVAL, "training data: empty or null");
    need(epochs >= 0 && lr > 0.f, BMLP_EINVAL, "bad epochs / learning rate");
    // standardisation of the inputs from the data
    std::vector<float> model((size_t)(kParams + 2 * kIn), 0.f);
    float* mu = model.data() + kParams;
    float* sd = mu + kIn;
    for (int f = 0; f < kIn; ++f) {
      double a = 0.0, b = 0.0;
      for (int64_t i = 0; i < rows; ++i) {
        a += X[i * kIn + f];
        b += (double)X[i * kIn + f] * X[i * kIn + f];
      }
      const double mean = a / rows, var = std::max(0.0, b / rows - mean * mean);
      mu[f] = (float)mean;
      sd[f] = (float)std::max(std::sqrt(var), 1e-3);
    }
    // Glorot-uniform weights, zero biases
    uint64_t st = seed;
    auto uni = [&]() { return (double)(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0); };
    auto fill = [&](float* w, int fan_out, int fan_in) {
      const double a = std::sqrt(6.0 / (fan_in + fan_out));
      for (int i = 0; i < fan_out * fan_in; ++i) w[i] = (float)((2.0 * uni() - 1.0) * a);
    };
    float* P = model.data();
    fill(P, kH1, kIn);
    fill(P + kH1 * kIn + kH1, kH2, kH1);
    fill(P + kH1 * kIn + kH1 + kH2 * kH1 + kH2, kOut, kH2);
    double msum = 0.0;
    for (int64_t i = 0; i < rows * kOut; ++i) msum += M[i];
    need(msum > 0.0, BMLP_EINVAL, "training data: empty mask");
    DeviceGuard dg(h->device);
    hipStream_t s = nullptr;
    DevBuf dX = upload(X, (size_t)rows * kIn, s), dT = upload(T, (size_t)rows * kOut, s),
           dM = upload(M, (size_t)rows * kOut, s), dP = upload(model.data(), model.size(), s);
    DevBuf dG((size_t)kParams * sizeof(float)), m1((size_t)kParams * sizeof(float)), m2((size_t)kParams * sizeof(float));
    hip_check(hipMemsetAsync(m1.p, 0, kParams * sizeof(float), s), "hipMemsetAsync");
    hip_check(hipMemsetAsync(m2.p, 0, kParams * sizeof(float), s), "hipMemsetAsync");
    DevBuf act[7];
    alloc_acts(act, rows);
    const float inv_m = (float)(1.0 / msum);
    const float* dmu = dP.f() + kParams;
    const float* dsd = dmu + kIn;
    float loss = 0.f;
    for (int e = 1; e <= epochs; ++e) {
      hip_check(launch_mlp_forward(dP.f(), dmu, dsd, dX.f(), rows, act[0].f(), act[1].f(), act[2].f(), s), "forward");
      hip_check(launch_mlp_backward(dP.f(), dmu, dsd, dX.f(), act[0].f(), act[1].f(), act[2].f(), dT.f(), dM.f(), rows,
                                    inv_m, act[3].f(), act[4].f(), act[5].f(), dG.f(), act[6].f(), s),
                "backward");
      hip_check(launch_adam(dP.f(), dG.f(), m1.f(), m2.f(), lr, 0.9f, 0.999f, 1e-8f, e, s), "adam");
    }
    loss = mlp_pass(dP.f(), dmu, dsd, dX.f(), dT.f(), dM.f(), rows, inv_m, act, dG.f(), s);
    hip_check(hipMemcpy(model.data(), dP.p, model.size() * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy");
    h->h_model = model;
    model_to_device(h);
    if (loss_out) *loss_out = loss;
  });
}

bmlp_status bmlp_dispatcher_forward(bmlp_handle h, const float* X, int64_t rows, float* Y) {
  return guarded([&] {
    need_handle(h);
    need(h->model, BMLP_EMODEL, "no model");
    need(rows >= 0 && (rows == 0 || (X && Y)), BMLP_EINVAL, "bad arguments");
    if (rows == 0) return;
    DeviceGuard dg(h->device);
    hipStream_t s = nullptr;
    DevBuf dX = upload(X, (size_t)rows * kIn, s);
    DevBuf dY((size_t)rows * kOut * sizeof(float));
    hip_check(launch_mlp_forward(h->d_model, h->d_model + kParams, h->d_model + kParams + kIn, dX.f(), rows, nullptr,
                                 nullptr, dY.f(), s),
              "forward");
    hip_check(hipMemcpy(Y, dY.p, (size_t)rows * kOut * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy");
  });
}

bmlp_status bmlp_mlp_loss_grad(bmlp_handle h, const float* params, const float* mu, const float* sd, const float* X,
                               const float* T, const float* M, int64_t rows, float* loss, float* grad) {
  return guarded([&] {
    need_handle(h);
    need(rows > 0 && params && mu && sd && X && T && M && loss && grad, BMLP_EINVAL, "bad arguments");
    double msum = 0.0;
    for (int64_t i = 0; i < rows * kOut; ++i) msum += M[i];
    need(msum > 0.0, BMLP_EINVAL, "empty mask");
    DeviceGuard dg(h->device);
    hipStream_t s = nullptr;
    DevBuf dP = upload(params, kParams, s), dmu = upload(mu, kIn, s), dsd = upload(sd, kIn, s),
           dX = upload(X, (size_t)rows * kIn, s), dT = upload(T, (size_t)rows * kOut, s),
           dM = upload(M, (size_t)rows * kOut, s);
    DevBuf dG((size_t)kParams * sizeof(float));
    DevBuf act[7];
    alloc_acts(act, rows);
    *loss = mlp_pass(dP.f(), dmu.f(), dsd.f(), dX.f(), dT.f(), dM.f(), rows, (float)(1.0 / msum), act, dG.f(), s);
    hip_check(hipMemcpy(grad, dG.p, kParams * sizeof(float), hipMemcpyDeviceToHost), "hipMemcpy");
  });
}

bmlp_status bmlp_graph_open(bmlp_handle h, const uint64_t* R1, int64_t n, int64_t ld, void* stream, bmlp_graph* g) {
  return guarded([&] {
    need_handle(h);
    need(g != nullptr, BMLP_EINVAL, "g: null pointer");
    *g = nullptr;
    check_bits_arg(R1, "R1", n, n, ld);
    DeviceGuard dg(h->device);
    hipStream_t s = (hipStream_t)stream;
    bmlp_graph_s* G = new bmlp_graph_s;
    G->c = h;
    G->R1 = R1;
    G->n = n;
    G->ld = ld;
    try {
      if (n > 0) {
        bmlp_opts o;
        bmlp_opts_init(&o);
        G->gi = graph_info(h, R1, ld, n, o, s);
        i64* rp;
        int32_t* ci;
        build_csr(h, R1, ld, n, o, s, &rp, &ci);
        DevBuf b1((size_t)(n + 1) * sizeof(i64)), b2((size_t)std::max<i64>(G->gi.m, 1) * sizeof(int32_t));
        hip_check(hipMemcpyAsync(b1.p, rp, (size_t)(n + 1) * sizeof(i64), hipMemcpyDeviceToDevice, s), "memcpy");
        hip_check(hipMemcpyAsync(b2.p, ci, (size_t)G->gi.m * sizeof(int32_t), hipMemcpyDeviceToDevice, s), "memcpy");
        hip_check(hipStreamSynchronize(s), "sync");
        G->rp = (i64*)b1.p;
        G->ci = (int32_t*)b2.p;
        b1.p = b2.p = nullptr;
        if (n <= smp_rows_max_n() && (double)G->gi.m >= kBottomUpMinDegree * (double)n) {
          i64* rpt;
          int32_t* cit;
          build_csc(h, R1, ld, G->rp, G->ci, n, G->gi.m, o, s, &rpt, &cit);
          DevBuf b3((size_t)(n + 1) * sizeof(i64)), b4((size_t)std::max<i64>(G->gi.m, 1) * sizeof(int32_t));
          hip_check(hipMemcpyAsync(b3.p, rpt, (size_t)(n + 1) * sizeof(i64), hipMemcpyDeviceToDevice, s), "memcpy");
          hip_check(hipMemcpyAsync(b4.p, cit, (size_t)G->gi.m * sizeof(int32_t), hipMemcpyDeviceToDevice, s),
                    "memcpy");
          hip_check(hipStreamSynchronize(s), "sync");
          G->rpt = (i64*)b3.p;
          G->cit = (int32_t*)b4.p;
          b3.p = b4.p = nullptr;
        }
      }
    } catch (...) {
      if (G->rp) (void)hipFree(G->rp);
      if (G->ci) (void)hipFree(G->ci);
      if (G->rpt) (void)hipFree(G->rpt);
      if (G->cit) (void)hipFree(G->cit);
      delete G;
      throw;
    }
    *g = G;
  });
}

int32_t bmlp_graph_has_closure(bmlp_graph g) { return (g && g->closure) ? 1 : 0; }

bmlp_status bmlp_graph_close(bmlp_graph g) {
  if (!g) return BMLP_OK;
  return guarded([&] {
    DeviceGuard dg(g->c->device);
    (void)hipDeviceSynchronize();
    if (g->rp) (void)hipFree(g->rp);
    if (g->ci) (void)hipFree(g->ci);
    if (g->rpt) (void)hipFree(g->rpt);
    if (g->cit) (void)hipFree(g->cit);
    if (g->closure) (void)hipFree(g->closure);
    delete g;
  });
}

}  // extern "C"

namespace {

// A session query: V (k query rows), or for one-hot queries their source indices src (then V is null and is
// formed only if the query is not answered from the closure; an index outside [0, n) gives an all-zero
// answer row and is latched for bmlp_deferred_error).
void graph_query_core(bmlp_graph g, const uint64_t* V, const int32_t* src, uint64_t* Vstar, int64_t k, int64_t ldv,
                      const bmlp_opts& o, hipStream_t s, StatsRec& sr) {
  bmlp_ctx* h = g->c;
  const i64 n = g->n;
  const int refl = o.smp_reflexive ? 1 : 0;
  int arm = BMLP_ARM_SMP_CLOSURE;
  if (k > 0 && n == 0) hip_check(launch_fill_zero(Vstar, k * ldv, s), "fill_zero");
  if (k > 0 && n > 0) {
    const i64 nw = words_for(n);
    bool use_closure = g->closure != nullptr;
    if (!use_closure) {
      const bool learned = o.dispatch == BMLP_DISPATCH_LEARNED && h->model;
      const bool forced = o.dispatch == BMLP_DISPATCH_FORCED && o.smp_arm != BMLP_ARM_AUTO;
      // the source count is a feature of the model's choice (and of the trace) only
      const double delta0 = src ? (double)k
                                : ((learned && !forced) || h->trace) ? (double)count_bits(h, V, k, n, ldv, s) : 0.0;
      float pred[4] = {0, 0, 0, 0};
      arm = smp_choose_arm(h, o, g->gi, k, 0, refl, delta0, s, learned ? pred : nullptr);
      // how a closure would be built: by squarings (BMLP-RMS), or by the selection from every source
      int build = arm == BMLP_ARM_SMP_CLOSURE_SELECT ? BMLP_ARM_SMP_CLOSURE_SELECT : BMLP_ARM_SMP_CLOSURE;
      if (arm == BMLP_ARM_SMP_CLOSURE || arm == BMLP_ARM_SMP_CLOSURE_SELECT) use_closure = true;
      if (learned && !forced) {
        // the closure's predicted cost: the cheaper of the two builds (the selection from all n sources
        // predicted once per session, by the model's one-launch output at k = n)
        double p_clo = std::exp(pred[2]);
        if (g->gi.n <= smp_rows_max_n()) {
          if (g->p_sel_all_ms < 0.0) {
            float f[kIn], pa[4];
            make_features(f, g->gi, n, 0, 1, 0, (double)n, (double)n, 0.0, 0);
            (void)model_decide(h, f, 0x8u, s, pa);
            g->p_sel_all_ms = std::exp(pa[3]);
          }
          if (g->p_sel_all_ms < p_clo) {
            p_clo = g->p_sel_all_ms;
            build = BMLP_ARM_SMP_CLOSURE_SELECT;
          }
        }
        // ski rental: build the closure once its predicted cost is below the time already spent on
        // this relation plus this query's predicted cost without it
        const double p_iter = std::exp(std::min(pred[0], g->gi.n <= smp_rows_max_n() ? pred[3] : pred[0]));
        if (p_clo <= g->spent_ms + p_iter) use_closure = true;
      }
      if (use_closure) {
        u64* clo = nullptr;
        if (hipMalloc((void**)&clo, (size_t)std::max<i64>(n * nw, 1) * sizeof(u64)) != hipSuccess) {
          (void)hipGetLastError();
          fail(BMLP_ENOMEM, "closure allocation failed");
        }
        try {
          if (build == BMLP_ARM_SMP_CLOSURE_SELECT)
            closure_by_selection(h, g->R1, g->ld, n, clo, nw, g->gi, Csr{g->rp, g->ci, g->rpt, g->cit}, o, s, sr);
          else
            rms_core(h, g->R1, g->ld, clo, nw, n, o, s, sr);
        } catch (...) {
          (void)hipFree(clo);
          throw;
        }
        g->closure = clo;
        g->closure_arm = build;
      } else {
        if (!V) {
          // the query rows of the sources
          u64* qv = ws_bits(h, S_QV, k, ldv, o);
          hip_check(launch_fill_zero(qv, k * ldv, s), "fill_zero");
          hip_check(launch_set_onehot(qv, ldv, src, k, n, h->d_flags + F_DEFER, s), "set_onehot");
          V = qv;
        }
        // the learned schedule's ski rental needs the device time of the query: only then does the
        // query wait for its own end
        const bool rent = learned && !forced;
        if (rent) hip_check(hipEventRecord(h->ev1, s), "hipEventRecord");
        if (h->trace) h->trace->call_arm = arm;
        smp_core(h, g->R1, g->ld, n, V, Vstar, k, ldv, refl, arm, g->gi, 0, Csr{g->rp, g->ci, g->rpt, g->cit}, o, s, sr);
        if (rent) {
          hip_check(hipEventRecord(h->evp1, s), "hipEventRecord");
          hip_check(hipEventSynchronize(h->evp1), "hipEventSynchronize");
          float ms = 0.f;
          hip_check(hipEventElapsedTime(&ms, h->ev1, h->evp1), "hipEventElapsedTime");
          g->spent_ms += ms;
        }
      }
    }
    if (use_closure) {
      // the query that builds the closure reports how it was built; later ones read it off
      arm = g->closure_arm >= 0 ? g->closure_arm : BMLP_ARM_SMP_CLOSURE;
      g->closure_arm = -1;
      if (src)
        hip_check(launch_rows_by_index(g->closure, nw, src, k, n, refl, Vstar, ldv, h->d_flags + F_DEFER, s),
                  "rows_by_index");
      else
        read_off_closure(h, V, ldv, k, g->closure, nw, n, refl, Vstar, o, s, sr);
    }
  }
  g->last_arm = arm;
  if (sr.st) sr.st->arm = arm;
}

}  // namespace

extern "C" {

bmlp_status bmlp_graph_query(bmlp_graph g, const uint64_t* V, uint64_t* Vstar, int64_t k, int64_t ldv,
                             const bmlp_opts* opts, void* stream, bmlp_stats* stats) {
  return guarded([&] {
    need(g != nullptr, BMLP_EINVAL, "null session");
    bmlp_ctx* h = g->c;
    const bmlp_opts o = opts_or_default(opts);
    const i64 n = g->n;
    check_bits_arg(V, "V", k, n, ldv);
    check_bits_arg(Vstar, "Vstar", k, n, ldv);
    need(!overlap(range_of(Vstar, k, ldv), range_of(V, k, ldv)), BMLP_EALIAS, "Vstar overlaps V");
    need(!overlap(range_of(Vstar, k, ldv), range_of(g->R1, n, g->ld)), BMLP_EALIAS, "Vstar overlaps R1");
    DeviceGuard dg(h->device);
    hipStream_t s = (hipStream_t)stream;
    StatsRec sr(stats, h, s, &o);
    graph_query_core(g, V, nullptr, Vstar, k, ldv, o, s, sr);
    sr.finish();
  });
}

bmlp_status bmlp_graph_query_sources(bmlp_graph g, const int32_t* src, uint64_t* Vstar, int64_t k, int64_t ldv,
                                     const bmlp_opts* opts, void* stream, bmlp_stats* stats) {
  return guarded([&] {
    need(g != nullptr, BMLP_EINVAL, "null session");
    bmlp_ctx* h = g->c;
    const bmlp_opts o = opts_or_default(opts);
    const i64 n = g->n;
    need(k >= 0, BMLP_EINVAL, "k < 0");
    if (k > 0) {
      need(src != nullptr, BMLP_EINVAL, "src: null pointer");
      need(((uintptr_t)src & 3u) == 0, BMLP_EALIGN, "src: not 4-byte aligned");
    }
    check_bits_arg(Vstar, "Vstar", k, n, ldv);
    need(!overlap(range_of(Vstar, k, ldv), range_of(g->R1, n, g->ld)), BMLP_EALIAS, "Vstar overlaps R1");
    need(!overlap(range_of(Vstar, k, ldv), Range{(uintptr_t)src, (uintptr_t)(src + k)}), BMLP_EALIAS,
         "Vstar overlaps src");
    DeviceGuard dg(h->device);
    hipStream_t s = (hipStream_t)stream;
    StatsRec sr(stats, h, s, &o);
    graph_query_core(g, nullptr, src, Vstar, k, ldv, o, s, sr);
    sr.finish();
  });
}

int32_t bmlp_graph_last_arm(bmlp_graph g) { return g ? g->last_arm : -1; }

}  // extern "C"
