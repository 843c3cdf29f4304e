// Internal declarations shared by the HIP translation units of libbmlp.
// Not part of the public C-ABI (that is include/bmlp.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

typedef uint64_t u64;
typedef uint32_t u32;
typedef int64_t i64;

namespace bmlp {

static inline i64 words_for(i64 n) { return (n + 63) >> 6; }

// ---------------------------------------------------------------- bit kernels
// All bit matrices: row-major, LSB-first uint64 words, leading dimension in
// words.  `nw` = ceil(cols/64) words carry data; words in [nw, ld) are padding.
hipError_t launch_fill_zero(u64* p, i64 nwords, hipStream_t s);
// seeded random bits, each 1 with probability 2^-s_in inside rows < brows and words < bwords, 2^-s_out elsewhere
hipError_t launch_fill_random(u64* a, i64 rows, i64 n, i64 ld, u64 seed, int s_in, int s_out, i64 brows, i64 bwords,
                              hipStream_t s);
hipError_t launch_pack_u8(const uint8_t* d, i64 rows, i64 n, i64 ldd, u64* bits, i64 ld, hipStream_t s);
hipError_t launch_unpack_u8(const u64* bits, i64 rows, i64 n, i64 ld, uint8_t* d, i64 ldd, hipStream_t s);
// bits must be zeroed beforehand; out-of-range pairs set *bad = 1.
hipError_t launch_pack_coo(const int32_t* r, const int32_t* c, i64 m, i64 rows, i64 n, u64* bits, i64 ld,
                           u32* bad, hipStream_t s);
// elementwise: op 0 = or, 1 = and, 2 = andnot (a & ~b), 3 = not a (padding kept 0), 4 = copy a; with
// pred, only when *pred == pred_val
hipError_t launch_ewise(int op, const u64* a, i64 lda, const u64* b, i64 ldb, u64* c, i64 ldc, i64 rows,
                        i64 n, hipStream_t s, const u32* pred = nullptr, u32 pred_val = 0);
// zero the padding words [nw, ld) of every row (nw = ceil(n/64))
hipError_t launch_zero_pad(u64* a, i64 rows, i64 n, i64 ld, hipStream_t s);
// set the diagonal bits (i, i) for i < min(rows, n)
hipError_t launch_set_diag(u64* a, i64 ld, i64 rows, i64 n, hipStream_t s);
// row i of a gets bit idx[i] (0 <= idx[i] < columns; rows zeroed beforehand)
hipError_t launch_set_onehot(u64* a, i64 ld, const int32_t* idx, i64 k, i64 n, u32* bad, hipStream_t s);
hipError_t launch_check_index(const int32_t* idx, i64 k, i64 n, u32* bad, hipStream_t s);
// list of the rows of a (rows x n) with a set bit, in no particular order; *count (zeroed by the caller) += their number
hipError_t launch_nonempty_rows(const u64* a, i64 rows, i64 n, i64 ld, int32_t* list, u32* count, hipStream_t s);
// dst row i = src row list[i] for i < k (n columns; padding words of dst up to ldd zeroed)
hipError_t launch_copy_rows(const u64* src, i64 lds, const int32_t* list, i64 k, i64 n, u64* dst, i64 ldd,
                            hipStream_t s);
// out row i = C row idx[i] (| bit idx[i] when reflexive); padding words up to ldo zeroed; an index outside
// [0, n) gives a zero row and raises *bad
hipError_t launch_rows_by_index(const u64* C, i64 ldc, const int32_t* idx, i64 k, i64 n, int reflexive, u64* out,
                               i64 ldo, u32* bad, hipStream_t s);
// out[rp[r] .. rp[r+1]) = r for r < rows
hipError_t launch_rows_from_rp(const i64* rp, i64 rows, int32_t* out, hipStream_t s);
// out = I | M+ for b <= 64 (M, out: b rows of one significant word)
hipError_t launch_closure64(const u64* M, i64 ldm, i64 b, u64* out, i64 ldo, hipStream_t s);
// A[x][i] = T[x][cols[i]] (| (cols[i] == x) when diag) for rows x < rows of T (n columns); n <= gather_cols_max_n()
hipError_t launch_gather_cols(const u64* T, i64 ldt, i64 rows, i64 n, const int32_t* cols, i64 b, int diag, u64* A,
                              i64 lda, hipStream_t s);
i64 gather_cols_max_n();
// out (cols x rows) = transpose of in (rows x cols); with pred, only when *pred == pred_val (the padding
// words of out beyond ceil(rows/64) are then left as they are: the products never read them)
hipError_t launch_transpose(const u64* in, i64 rows, i64 cols, i64 ldi, u64* out, i64 ldo, hipStream_t s,
                            const u32* pred = nullptr, u32 pred_val = 0);
// nonzero padding bits (columns >= n) in any row -> *bad = 1
hipError_t launch_check_pad(const u64* a, i64 rows, i64 n, i64 ld, u32* bad, hipStream_t s);
// per-row popcount into deg (int32), plus total into *total (u64, must be zeroed)
hipError_t launch_row_popcount(const u64* a, i64 rows, i64 n, i64 ld, int32_t* deg, unsigned long long* total,
                               hipStream_t s);
// number of set bits of the matrix added into *total (must be zeroed)
hipError_t launch_popcount_total(const u64* a, i64 rows, i64 n, i64 ld, unsigned long long* total, hipStream_t s);
// exclusive scan of deg[0..n) into rp[0..n] (int64); single-workgroup; deg and rp 16-byte aligned
hipError_t launch_scan_rowptr(const int32_t* deg, i64 n, i64* rp, hipStream_t s);
// dst[i][j] = src[perm[i]][perm[j]] for a permutation perm of [0, n) (n <= 524,288); dst must not overlap src
hipError_t launch_permute(const u64* src, i64 lds_, const int32_t* perm, i64 n, u64* dst, i64 ldd, hipStream_t s);
// CSC (rpt, cit: in-edges) of an n-node CSR (rp, ci) with m edges; degt and cursor are n int32 of
// workspace (8-byte aligned).  The order inside each CSC segment is unspecified.
hipError_t launch_csc_from_csr(const i64* rp, const int32_t* ci, i64 n, i64 m, int32_t* degt, int32_t* cursor,
                               i64* rpt, int32_t* cit, hipStream_t s);
// CSR column indices of the set bits of each row (rp from launch_scan_rowptr)
hipError_t launch_bits_to_csr(const u64* a, i64 rows, i64 n, i64 ld, const i64* rp, int32_t* ci, hipStream_t s);

// ---------------------------------------------------------------- products
// C = Cold | A.B over the Boolean semiring; D = C & ~Cold (optional);
// *changed |= 1 when any word of C differs from Cold.  The MFMA arm skips output tiles whose Cold bits
// are all set and words of k that are zero in every row of a 128-row block.
//   A: M x K bits (lda), B: K x N bits (ldb), Cold/C/D: M x N bits.
//   Cold may be null (treated as 0).  C may equal Cold (element-wise in place);
//   A and B must not overlap C or D.  Words >= ceil(N/64) are not written.
struct GemmArgs {
  const u64* A; i64 lda;
  const u64* B; i64 ldb;
  const u64* Cold; i64 ldco;
  u64* C; i64 ldc;
  u64* D; i64 ldd;
  i64 M, K, N;
  u32* changed;
  unsigned long long* newbits = nullptr;  // += number of bits of C not in Cold (optional)
  const u32* pred = nullptr;              // when given, the kernel runs only if *pred == pred_val
  u32 pred_val = 0;
  unsigned long long* executed = nullptr;  // += matrix-core ops actually issued (MFMA arm, optional)
  // A likely saturates early (MFMA arm, second tile code): with early set, or early_flag given and nonzero,
  // a whole tile votes on saturation after its first chunk of k, before it loads further chunks
  const u32* early_flag = nullptr;
  bool early = false;
};
enum ProductKernel { PK_VALU = 0, PK_MFMA = 1 };
// variant (autotuner candidates, identical bits): rows per wave of the tile for M > 64: 0 -> 16, 1 -> 8,
// 2 -> 4 (thin products, M <= 64, always take 4)
constexpr int kValuVariants = 3;
hipError_t launch_gemm_valu(const GemmArgs& g, hipStream_t s, int variant = 0);
// MFMA int8 arm: needs B transposed (BT: N x K bits, ldbt) instead of B; K <= 64 * gemm_mfma_max_kwords()
// (the int32 sums stay exact).
// variant: the tile code (autotuner candidates, identical bits):
//   0, 1, 2  256 x 256 tile, operands expanded into e2m1 nibbles while staging (4 words of k per LDS
//            stage); output tiles in row-major, XCD-contiguous or XCD-interleaved order
//   3, 4, 5  raw words in LDS, operands formed in registers (8 words per stage); the same three orders
//   6, 7     the two tile codes with the output tiles in column strips per XCD
// A variant whose alignment needs (16-byte rows for 3, 4, 5 and 7) are not met runs as 0.
constexpr int kMfmaVariants = 8;
hipError_t launch_gemm_mfma(const GemmArgs& g, const u64* BT, i64 ldbt, hipStream_t s, int variant = 0);
bool gemm_mfma_variant_ok(int variant, const GemmArgs& g, const u64* BT, i64 ldbt);
int gemm_mfma_variants();
i64 gemm_mfma_max_kwords();

// ---------------------------------------------------------------- selection
// Per-row fixpoint of the semi-naive selection in one launch (one workgroup
// per query row, bitmaps in LDS): out[r] = V[r] R+ (reflexive: V[r] R*).
// Needs CSR (rp, ci) of R and the bit rows of R (for dense frontier nodes); with the CSC (rpt, cit: the
// in-edges, optional) rounds with a large frontier run bottom-up.  V null stands for the identity (row r
// starts from node r; k <= n), so that out holds the rows of R+ (R* when reflexive).
hipError_t launch_smp_rows(const u64* V, i64 ldv, i64 k, const i64* rp, const int32_t* ci, const i64* rpt,
                           const int32_t* cit, const u64* R, i64 ldr, i64 n, int reflexive, u64* out, i64 ldo,
                           u32* iters_max, hipStream_t s);
i64 smp_rows_max_n();
// One semi-naive round for k rows with the state in global memory: nxt = fr . R1 (CSR),
// fr_out = nxt & ~vis, vis |= fr_out.  Runs only when *pred == pred_val (pred optional).
hipError_t launch_smp_round(const u64* fr, u64* fr_out, i64 ldf, u64* vis, i64 ldvis, i64 k, const i64* rp,
                            const int32_t* ci, const u64* R, i64 ldr, i64 n, u32* changed, unsigned long long* newbits,
                            const u32* pred, u32 pred_val, hipStream_t s);
// Overflow queue of the gathers: room for gather_queue_capacity(k, n) pieces, a 64-bit counter, and the
// bits per piece (at least 64; rows with more set bits than that are split).
struct GatherQueue {
  int2* e;
  unsigned long long* n;
  i64 cap;
  int piece;
  // optional: the set bits of V counted on the device; the kernels then size the pieces from it (twice
  // the mean row, at least 64) instead of from `piece`, for gathers queued before that count reaches the host
  const unsigned long long* bits = nullptr;
};
i64 gather_queue_capacity(i64 k, i64 n);
// out[map(r)] = init | OR of Cl[u, :] over the set bits u of V[r], with init = 0 (0), V[r] (1) or the
// current out[map(r)] (2); map(r) = row_map[r], or r without a map (a map must not repeat a row);
// n <= gather_rows_max_n().  *newbits (optional) += bits of the answers not in init.  out must not
// overlap V or Cl.  With a queue (n <= 16,384), rows with more set bits than q->piece are split over waves.
// With pred, the gather runs only when *pred == pred_val.
hipError_t launch_gather_rows(const u64* V, i64 ldv, i64 k, const u64* Cl, i64 ldc, i64 n, int init, u64* out,
                              i64 ldo, hipStream_t s, const int32_t* row_map = nullptr,
                              unsigned long long* newbits = nullptr, const GatherQueue* q = nullptr,
                              const u32* pred = nullptr, u32 pred_val = 0);
i64 gather_rows_max_n();
// The route of BMLP-RMS squaring t, decided on the device from the bits squaring t - 1 added: recs holds
// kRmsRecWords-word records {new bits u64, running count u64, route u32, early flag u32} per squaring; reads
// record t - 1, writes record t's running count, route (stop / row gathers / dense product / back to the
// host for the semi-naive form or the relabelling) and early flag (rms_early_votes).  One thread.
hipError_t launch_rms_decide(u32* recs, int t, i64 n, int mfma, int may_gather, int may_semi, int dense_ok,
                             i64 gather_max_n, hipStream_t s);
// out[0] += set bits, out[1] = max(out[1], largest row count), out[2] += rows with a set bit
// (out must be zeroed)
hipError_t launch_graph_stats(const u64* a, i64 rows, i64 n, i64 ld, unsigned long long* out, hipStream_t s);
// out[0..2] = (sum, max, nonzero entries) of deg[0..n), one workgroup, plain stores
hipError_t launch_deg_stats(const int32_t* deg, i64 n, unsigned long long* out, hipStream_t s);
// The relabelling of rms_core from row and column counts (n <= 262,144): out (9 u64) = rmax, cmax, heavy
// rows, heavy columns, dead nodes, tiles with a dead row, tiles with a dead column; then perm / inv for
// mode 1 (heavy/light classes) or 2 (dead nodes last), maxes = that out.
hipError_t launch_relabel_classes(const int32_t* rp, const int32_t* cp, i64 n, unsigned long long* out, hipStream_t s);
hipError_t launch_relabel_perm(const int32_t* rp, const int32_t* cp, i64 n, int mode, const unsigned long long* maxes,
                               int32_t* perm, int32_t* inv, hipStream_t s);

}  // namespace bmlp
