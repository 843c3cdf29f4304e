// C ABI of libbmlp (declared in include/bmlp.h) and the host fixpoint drivers
// of the BMLP algorithms.  Host code only: every step of the computation runs
// in the kernels of k_bits.hip, k_gemm.hip and k_smp.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/bmlp.h"
#include "bmlp_batch.h"
#include "bmlp_internal.h"

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
  static constexpr int kSlots = 13;
  void* slot[kSlots] = {};
  size_t slot_bytes[kSlots] = {};
  u32* d_flags = nullptr;  // device flags / counters
  u32* h_flags = nullptr;  // pinned host mirror
  hipEvent_t ev0 = nullptr, ev1 = nullptr, evp0 = nullptr, evp1 = nullptr;
  // batched launch: the captured kernel chain, reused while the batch is unchanged
  hipStream_t capture_stream = nullptr;
  hipGraph_t bgraph = nullptr;
  hipGraphExec_t bexec = nullptr;
  uint64_t bkey = 0;
};

namespace {

enum Slot { S_W0 = 0, S_W1, S_W2, S_W3, S_W4, S_DEG, S_RP, S_CI, S_T0, S_T1, S_T2, S_BT, S_BATCH };

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
  void product_begin() {
    if (st) hip_check(hipEventRecord(c->evp0, s), "hipEventRecord");
  }
  void product(i64 m, i64 k, i64 n) {
    if (!st) return;
    hip_check(hipEventRecord(c->evp1, s), "hipEventRecord");
    hip_check(hipEventSynchronize(c->evp1), "hipEventSynchronize");
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, c->evp0, c->evp1), "hipEventElapsedTime");
    const uint64_t ops = (uint64_t)2 * (uint64_t)m * (uint64_t)k * (uint64_t)n;
    st->products += 1;
    st->bool_ops += ops;
    st->product_bool_ops += ops;
    st->product_ms += ms;
    st->bytes_moved += (uint64_t)(m * words_for(k) + k * words_for(n) + 2 * m * words_for(n)) * 8u;
  }
  void finish() {
    if (!st) return;
    hip_check(hipEventRecord(c->ev1, s), "hipEventRecord");
    hip_check(hipEventSynchronize(c->ev1), "hipEventSynchronize");
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, c->ev0, c->ev1), "hipEventElapsedTime");
    st->device_ms = ms;
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
                       i64* ldbt) {
  *ldbt = std::max<i64>(words_for(K), 1);
  u64* bt = ws_bits(c, S_BT, N, *ldbt, o);
  hip_check(launch_transpose(B, K, N, ldb, bt, *ldbt, s), "transpose");
  return bt;
}

// One Boolean product C = Cold | A.B (D, changed optional) with the chosen arm.  The MFMA arm reads B
// transposed: pass BT when the caller has it, else B is transposed into workspace first.
void product(bmlp_ctx* c, const u64* A, i64 lda, const u64* B, i64 ldb, const u64* Cold, i64 ldco, u64* C, i64 ldc,
             u64* D, i64 ldd, i64 M, i64 K, i64 N, u32* changed, int arm, hipStream_t s, StatsRec& sr,
             const u64* BT = nullptr, i64 ldbt = 0) {
  GemmArgs g{A, lda, B, ldb, Cold, ldco, C, ldc, D, ldd, M, K, N, changed};
  if (arm == BMLP_ARM_PRODUCT_MFMA) {
    bmlp_opts dflt;
    bmlp_opts_init(&dflt);
    if (!BT) BT = transpose_b(c, B, ldb, K, N, sr.o ? *sr.o : dflt, s, &ldbt);
    sr.product_begin();
    hip_check(launch_gemm_mfma(g, BT, ldbt, s), "gemm_mfma");
  } else {
    sr.product_begin();
    hip_check(launch_gemm_valu(g, s), "gemm_valu");
  }
  sr.product(M, K, N);
}

int ceil_log2(i64 x) {
  int r = 0;
  while (((i64)1 << r) < x) ++r;
  return r;
}

// Plain choice of the product kernel for an (M x K).(K x N) product: the matrix-core arm once both
// output dimensions fill its 256 x 256 workgroup tiles (measured faster from n = 4,096 up), the
// bit-packed VALU arm (which also splits K) for thin or small products.
int product_arm(const bmlp_opts& o, i64 M, i64 N) {
  if (o.product_arm == BMLP_ARM_PRODUCT_VALU || o.product_arm == BMLP_ARM_PRODUCT_MFMA) return o.product_arm;
  return (M >= 1024 && N >= 1024) ? BMLP_ARM_PRODUCT_MFMA : BMLP_ARM_PRODUCT_VALU;
}

// R1+ into `out` (n x ldo) -- the RMS fixpoint driver shared by rms, the closure arm of smp and the RMS
// route of compose.  `R1` has leading dimension ld1.
void rms_core(bmlp_ctx* c, const u64* R1, i64 ld1, u64* out, i64 ldo, i64 n, const bmlp_opts& o, hipStream_t s,
              StatsRec& sr) {
  const i64 nw = words_for(n);
  const i64 ldi = nw;
  u64* cur = ws_bits(c, S_W0, n, ldi, o);
  u64* nxt = ws_bits(c, S_W1, n, ldi, o);
  const int arm = product_arm(o, n, n);
  hip_check(launch_ewise(4, R1, ld1, nullptr, 0, cur, ldi, n, n, s), "copy");
  if (o.rms_variant == 1) hip_check(launch_set_diag(cur, ldi, n, n, s), "set_diag");
  const int cap = ceil_log2(std::max<i64>(n, 2)) + 2;
  int it = 0;
  for (;;) {
    zero_flag(c, s);
    // variant 0: R <- R | R.R ; variant 1: R' = R.R (I is in R, so R | R.R = R.R)
    product(c, cur, ldi, cur, ldi, cur, ldi, nxt, ldi, nullptr, 0, n, n, n, c->d_flags, arm, s, sr);
    sr.trace(it, arm);
    ++it;
    const u32 changed = read_flag(c, s);
    std::swap(cur, nxt);
    if (!changed) break;
    need(it < cap, BMLP_EITER, "RMS exceeded %d products (n=%lld)", cap, (long long)n);
  }
  if (sr.st) sr.st->iterations = it;
  if (o.rms_variant == 1) {
    // Algorithm 1, last line: R2* = R2* R1
    product(c, cur, ldi, R1, ld1, nullptr, 0, out, ldo, nullptr, 0, n, n, n, nullptr, arm, s, sr);
  } else {
    hip_check(launch_ewise(4, cur, ldi, nullptr, 0, out, ldo, n, n, s), "copy");
  }
  hip_check(launch_zero_pad(out, n, n, ldo, s), "zero_pad");
}

// CSR of the bit matrix R (n x n, ld) in workspace slots S_DEG/S_RP/S_CI.
void build_csr(bmlp_ctx* c, const u64* R, i64 ld, i64 n, const bmlp_opts& o, hipStream_t s, i64** rp_out,
               int32_t** ci_out) {
  int32_t* deg = (int32_t*)ws(c, S_DEG, (size_t)n * sizeof(int32_t), o);
  i64* rp = (i64*)ws(c, S_RP, (size_t)(n + 1) * sizeof(i64), o);
  hip_check(launch_row_popcount(R, n, n, ld, deg, nullptr, s), "row_popcount");
  hip_check(launch_scan_rowptr(deg, n, rp, s), "scan");
  // the scan's last entry is the number of set bits
  hip_check(hipMemcpyAsync(c->h_flags + 4, rp + n, sizeof(i64), hipMemcpyDeviceToHost, s), "memcpy");
  hip_check(hipStreamSynchronize(s), "sync");
  i64 m = 0;
  std::memcpy(&m, c->h_flags + 4, sizeof m);
  int32_t* ci = (int32_t*)ws(c, S_CI, (size_t)std::max<i64>(m, 1) * sizeof(int32_t), o);
  hip_check(launch_bits_to_csr(R, n, n, ld, rp, ci, s), "bits_to_csr");
  *rp_out = rp;
  *ci_out = ci;
}

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

// Plain schedule for the selection, from a timing sweep of the three arms on
// n = 16,384 random digraphs (mean out-degree 1.6 .. 164, k = 1 .. 1024): the
// sparse-frontier arm wins while the mean out-degree is low (its work grows with
// the edges it visits); the dense semi-naive arm wins on dense relations (its
// work is independent of the degree).
int smp_plain_arm(i64 n, i64 k, i64 m) {
  if (n > smp_rows_max_n()) return BMLP_ARM_SMP_DENSE;
  const double deg = n > 0 ? (double)m / (double)n : 0.0;
  if (deg < 12.0) return BMLP_ARM_SMP_SPARSE;
  if (deg < 40.0 && k >= 32) return BMLP_ARM_SMP_SPARSE;
  return BMLP_ARM_SMP_DENSE;
}

// Vstar = V . R1+ (or V . R1* when reflexive).
void smp_core(bmlp_ctx* c, const u64* R1, i64 ld, i64 n, const u64* V, u64* Vstar, i64 k, i64 ldv, int reflexive,
              int arm, const bmlp_opts& o, hipStream_t s, StatsRec& sr) {
  const i64 nw = words_for(n);
  const int parm = product_arm(o, k, n);
  if (sr.st) sr.st->arm = arm;
  if (arm == BMLP_ARM_SMP_SPARSE) {
    need(n <= smp_rows_max_n(), BMLP_EINVAL, "sparse SMP arm supports n <= %lld", (long long)smp_rows_max_n());
    i64* rp;
    int32_t* ci;
    build_csr(c, R1, ld, n, o, s, &rp, &ci);
    hip_check(hipMemsetAsync(c->d_flags + 2, 0, sizeof(u32), s), "hipMemsetAsync");
    hip_check(launch_smp_rows(V, ldv, k, rp, ci, R1, ld, n, reflexive, Vstar, ldv, c->d_flags + 2, s), "smp_rows");
    const u32 rounds = read_flag(c, s, 2);
    need((i64)rounds <= n + 2, BMLP_EITER, "SMP exceeded the round cap");
    if (sr.st) {
      sr.st->iterations = (int32_t)rounds;
      for (u32 r = 0; r < rounds && r < 64; ++r) sr.trace((int)r, arm);
    }
    return;
  }
  if (arm == BMLP_ARM_SMP_CLOSURE) {
    u64* clo = ws_bits(c, S_W2, n, nw, o);
    rms_core(c, R1, ld, clo, nw, n, o, s, sr);
    // V . R1+ (strict) or V | V . R1+ (reflexive)
    product(c, V, ldv, clo, nw, reflexive ? V : nullptr, ldv, Vstar, ldv, nullptr, 0, k, n, n, nullptr, parm, s, sr);
    hip_check(launch_zero_pad(Vstar, k, n, ldv, s), "zero_pad");
    return;
  }
  // dense semi-naive: delta_0 = V.R1 (strict) or V (reflexive); then
  // delta' = (delta . R1) & ~Vis ; Vis |= delta' until delta' is empty.
  u64* da = ws_bits(c, S_W3, k, nw, o);
  u64* db = ws_bits(c, S_W4, k, nw, o);
  const u64* r1t = nullptr;
  i64 ldr1t = 0;
  if (parm == BMLP_ARM_PRODUCT_MFMA) r1t = transpose_b(c, R1, ld, n, n, o, s, &ldr1t);
  int it = 0;
  if (reflexive) {
    hip_check(launch_ewise(4, V, ldv, nullptr, 0, Vstar, ldv, k, n, s), "copy");
    hip_check(launch_ewise(4, V, ldv, nullptr, 0, da, nw, k, n, s), "copy");
  } else {
    product(c, V, ldv, R1, ld, nullptr, 0, Vstar, ldv, da, nw, k, n, n, nullptr, parm, s, sr, r1t, ldr1t);
    sr.trace(it++, arm);
  }
  const i64 cap = n + 2;
  for (;;) {
    zero_flag(c, s);
    product(c, da, nw, R1, ld, Vstar, ldv, Vstar, ldv, db, nw, k, n, n, c->d_flags, parm, s, sr, r1t, ldr1t);
    sr.trace(it++, arm);
    const u32 changed = read_flag(c, s);
    std::swap(da, db);
    if (!changed) break;
    need(it < cap, BMLP_EITER, "SMP exceeded %lld rounds", (long long)cap);
  }
  if (sr.st) sr.st->iterations = it;
  hip_check(launch_zero_pad(Vstar, k, n, ldv, s), "zero_pad");
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
    if (hipMalloc((void**)&c->d_flags, 64 * sizeof(u32)) != hipSuccess ||
        hipHostMalloc((void**)&c->h_flags, 64 * sizeof(u32), hipHostMallocDefault) != hipSuccess ||
        hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
        hipEventCreate(&c->evp0) != hipSuccess || hipEventCreate(&c->evp1) != hipSuccess) {
      (void)hipGetLastError();
      bmlp_destroy(c);
      fail(BMLP_ENOMEM, "handle allocation failed");
    }
    hip_check(hipMemset(c->d_flags, 0, 64 * sizeof(u32)), "hipMemset");
    *h = c;
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
      if (h->bexec) (void)hipGraphExecDestroy(h->bexec);
      if (h->bgraph) (void)hipGraphDestroy(h->bgraph);
      if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
    }
    delete h;
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
        product(h, A, lda, B, ldb, Cold, ldc, C, ldc, nullptr, 0, m, kdim, n, nullptr, product_arm(o, m, n), s, sr);
      }
    }
    if (m > 0) hip_check(launch_zero_pad(C, m, n, ldc, s), "zero_pad");
    if (stats) stats->arm = product_arm(o, m, n);
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
    if (stats) stats->arm = product_arm(o, n, n);
    if (n > 0) rms_core(h, R1, ld, Rstar, ld, n, o, s, sr);
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
    int arm = o.smp_arm;
    if (forced)
      need(arm == BMLP_ARM_SMP_DENSE || arm == BMLP_ARM_SMP_SPARSE || arm == BMLP_ARM_SMP_CLOSURE, BMLP_EINVAL,
           "smp_arm %d is not a selection arm", arm);
    DeviceGuard dg(h->device);
    hipStream_t s = (hipStream_t)stream;
    if (!forced) arm = (n > 0 && k > 0) ? smp_plain_arm(n, k, count_bits(h, R1, n, n, ld, s)) : BMLP_ARM_SMP_SPARSE;
    if (o.check_padding) {
      check_padding(h, R1, n, n, ld, s, "R1");
      check_padding(h, V, k, n, ldv, s, "V");
    }
    StatsRec sr(stats, h, s, &o);
    if (k > 0) {
      if (n == 0) hip_check(launch_fill_zero(Vstar, k * ldv, s), "fill_zero");
      else smp_core(h, R1, ld, n, V, Vstar, k, ldv, o.smp_reflexive ? 1 : 0, arm, o, s, sr);
    }
    if (stats) stats->arm = arm;
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
    int arm = o.compose_arm;
    if (o.dispatch != BMLP_DISPATCH_FORCED || arm == BMLP_ARM_AUTO) arm = BMLP_ARM_COMPOSE_SEMINAIVE;
    need(arm == BMLP_ARM_COMPOSE_RMS || arm == BMLP_ARM_COMPOSE_SEMINAIVE, BMLP_EINVAL,
         "compose_arm %d is not a composition arm", arm);
    DeviceGuard dg(h->device);
    hipStream_t s = (hipStream_t)stream;
    if (o.check_padding) {
      check_padding(h, Rbase, n, n, ld, s, "Rbase");
      check_padding(h, Rstep, n, n, ld, s, "Rstep");
    }
    StatsRec sr(stats, h, s, &o);
    if (n > 0) {
      const i64 nw = words_for(n);
      const int parm = product_arm(o, n, n);
      if (arm == BMLP_ARM_COMPOSE_RMS) {
        // Rs+ by RMS, then P = Rb | Rs+ . Rb
        u64* sp = ws_bits(h, S_W2, n, nw, o);
        bmlp_opts o2 = o;
        o2.rms_variant = 0;
        rms_core(h, Rstep, ld, sp, nw, n, o2, s, sr);
        product(h, sp, nw, Rbase, ld, Rbase, ld, P, ld, nullptr, 0, n, n, n, nullptr, parm, s, sr);
        hip_check(launch_zero_pad(P, n, n, ld, s), "zero_pad");
      } else {
        // P^T = Rb^T . (Rs^T)*: the columns of P are reflexive selections over the transposed step
        // relation, evaluated by the selection driver; then transpose back.
        u64* rbt = ws_bits(h, S_T0, n, nw, o);
        u64* rst = ws_bits(h, S_T1, n, nw, o);
        u64* pt = ws_bits(h, S_T2, n, nw, o);
        hip_check(launch_transpose(Rbase, n, n, ld, rbt, nw, s), "transpose");
        hip_check(launch_transpose(Rstep, n, n, ld, rst, nw, s), "transpose");
        const int sarm = smp_plain_arm(n, n, count_bits(h, rst, n, n, nw, s));
        smp_core(h, rst, nw, n, rbt, pt, n, nw, 1, sarm, o, s, sr);
        hip_check(launch_transpose(pt, n, n, nw, P, ld, s), "transpose");
      }
    }
    if (stats) stats->arm = arm;
    sr.finish();
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
    BatchPlan plan{0, 0, 0, 0};
    size_t buf_words = 0;
    for (int i = 0; i < count; ++i) {
      const bmlp_graph_desc& d = graphs[i];
      plan.rounds = std::max(plan.rounds, ceil_log2(std::max<int64_t>(d.n, 2)) + 2);
      buf_words += (size_t)(2 * d.n * words_for(d.n));
    }
    const size_t table_bytes = ((size_t)count * sizeof(BatchGraph) + 255) & ~(size_t)255;
    const size_t nflags = (size_t)count * plan.rounds + 2 * (size_t)plan.rounds + 1;
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
      plan.total_rows += std::max<int64_t>(d.n, d.k);
      plan.total_tiles += batch_tiles(d.n);
      plan.total_select_tiles += d.k > 0 ? batch_select_tiles(d.k, d.n) : 0;
    }
    // the captured chain is reused while the batch (and its workspace) is unchanged
    uint64_t key = 1469598103934665603ull;
    auto mix = [&](const void* p, size_t nb) {
      const unsigned char* b = (const unsigned char*)p;
      for (size_t i = 0; i < nb; ++i) key = (key ^ b[i]) * 1099511628211ull;
    };
    mix(graphs, sizeof(bmlp_graph_desc) * (size_t)count);
    mix(&base, sizeof base);
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
      const hipError_t le = launch_batch_chain(d_table, count, plan, d_flags, h->capture_stream);
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
      int max_rounds = 0;
      for (int j = 0; j < count; ++j) {
        int r = 0;
        while (r < plan.rounds && fl[(size_t)j * plan.rounds + r]) ++r;
        need(r < plan.rounds, BMLP_EITER, "batched RMS exceeded %d rounds (graph of n=%lld)", plan.rounds,
             (long long)tab[j].n);
        const int prods = r + 1;  // the rounds that changed plus the one that found the fixpoint
        max_rounds = std::max(max_rounds, prods);
        const uint64_t nn = (uint64_t)tab[j].n;
        stats->products += prods + (tab[j].k > 0 ? 1 : 0);
        stats->bool_ops += (uint64_t)prods * 2u * nn * nn * nn + 2u * (uint64_t)tab[j].k * nn * nn;
      }
      stats->iterations = max_rounds;
      stats->arm = BMLP_ARM_SMP_CLOSURE;
      stats->product_bool_ops = stats->bool_ops;
      stats->product_ms = stats->device_ms;
    }
  });
}

}  // extern "C"
