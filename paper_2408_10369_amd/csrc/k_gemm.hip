// Boolean-semiring matrix product with OR-accumulate:
//     C = Cold | A.B,   (A.B)_ij = OR_k (A_ik AND B_kj)      (Section 2)
// plus the semi-naive delta D = C & ~Cold and a wave-ballot "changed" flag
// (the fixpoint test of Algorithms 1 and 2: iterates only grow, so "some word
// changed" is the same test as "the matrices differ").
//
// VALU arm (bit-packed).  Row-OR formulation: C[i,:] |= B[k,:] for every set
// bit A[i,k].  A workgroup owns a tile of TR rows x TW words of C.  Each wave
// owns RPW rows; each lane owns WPL words of those rows.  For every chunk of
// 64 k values the workgroup stages B[k0..k0+63, tile words] in LDS; the A word
// of each of the wave's rows is wave-uniform, so the AND mask for (i, k) is a
// scalar value and every lane does one v_and_or per 32 bit-MACs.  Chunks in
// which no row of the tile has a set A bit are skipped entirely (sparse A).
//
// Split-K.  When the output has too few tiles to fill the chip, the k range
// is split over several workgroups and partial results are merged with 64-bit
// atomic ORs.  OR is idempotent and commutative, so the merge is exact.  C is
// first made equal to Cold; a bit is new exactly when the atomic that sets it
// returns an old word without it, which gives D and the changed flag exactly.
#include "bmlp_internal.h"
#include "valu_tile.h"
#include "mfma_tile.h"
#include "mfma_tile2.h"
#include "rms_cost.h"

namespace bmlp {

namespace {

template <int RPW, int WPL>
__global__ void __launch_bounds__(256)
k_gemm_valu(const u64* __restrict__ A, i64 lda, const u64* __restrict__ B, i64 ldb, const u64* __restrict__ Cold,
            i64 ldco, u64* __restrict__ C, i64 ldc, u64* __restrict__ D, i64 ldd, i64 M, i64 K, i64 N,
            u32* __restrict__ changed, int ksplit, int chunks_per_split, unsigned long long* __restrict__ newbits,
            const u32* __restrict__ pred, u32 pred_val) {
  constexpr int TW = 64 * WPL;
  constexpr int TR = 4 * RPW;
  __shared__ u64 Bs[64][TW];
  if (pred && *pred != pred_val) return;  // another arm serves this round
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const i64 nw = (N + 63) >> 6;
  const i64 ctiles = (nw + TW - 1) / TW;
  const i64 rtiles = (M + TR - 1) / TR;
  // block order: row tiles fastest, then column tiles, then k splits, so that
  // concurrently running workgroups share the B chunks they stage
  const i64 tile = blockIdx.x;
  const i64 rt = tile % rtiles;
  const i64 ct = (tile / rtiles) % ctiles;
  const i64 ks = tile / (rtiles * ctiles);
  const i64 row0 = rt * TR + (i64)wave * RPW;
  const i64 w0 = ct * TW;

  u32 acc[RPW][WPL][2];
#pragma unroll
  for (int r = 0; r < RPW; ++r)
#pragma unroll
    for (int wl = 0; wl < WPL; ++wl) acc[r][wl][0] = acc[r][wl][1] = 0u;

  const i64 kwords = (K + 63) >> 6;
  const i64 kw_begin = ks * chunks_per_split;
  const i64 kw_end = (kw_begin + chunks_per_split < kwords) ? kw_begin + chunks_per_split : kwords;
  const bool worked = valu_tile_accumulate<RPW, WPL>(A, lda, B, ldb, M, K, nw, row0, w0, kw_begin, kw_end, Bs, acc);

  int ch = 0;
  u32 pop = 0;
  if (ksplit == 1) {
    // an in-place product (C is Cold, no delta) leaves a tile whose rows of A are all zero as it is
    if (worked || C != Cold || D) ch = valu_tile_store<RPW, WPL>(acc, Cold, ldco, C, ldc, D, ldd, M, nw, row0, w0, &pop);
  } else {
    // C already holds Cold and D is zero (the launcher sees to both)
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      const i64 row = row0 + r;
      if (row >= M) break;
#pragma unroll
      for (int wl = 0; wl < WPL; ++wl) {
        const i64 w = w0 + lane + 64 * wl;
        const u64 v = ((u64)acc[r][wl][1] << 32) | (u64)acc[r][wl][0];
        if (w < nw && v) {
          const u64 old = atomicOr((unsigned long long*)&C[row * ldc + w], (unsigned long long)v);
          const u64 nb = v & ~old;
          if (nb) {
            if (D) atomicOr((unsigned long long*)&D[row * ldd + w], (unsigned long long)nb);
            ch = 1;
            pop += (u32)__popcll(nb);
          }
        }
      }
    }
  }
  __shared__ unsigned long long cslot[4][2];
  block_counts<4>(pop, ch, newbits, changed, cslot);
}

template <int RPW>
hipError_t launch_rpw(const GemmArgs& g, hipStream_t s, i64 target_blocks) {
  constexpr int WPL = 1;
  const i64 nw = words_for(g.N);
  const i64 ctiles = (nw + 64 * WPL - 1) / (64 * WPL);
  const i64 rtiles = (g.M + 4 * RPW - 1) / (4 * RPW);
  const i64 kwords = words_for(g.K);
  const i64 tiles = ctiles * rtiles;
  i64 ksplit = 1;
  if (tiles < target_blocks && kwords > 1) {
    ksplit = (target_blocks + tiles - 1) / tiles;
    if (ksplit > kwords) ksplit = kwords;
  }
  i64 cps = (kwords + ksplit - 1) / ksplit;
  if (cps < 1) cps = 1;
  ksplit = (kwords + cps - 1) / cps;
  if (ksplit < 1) ksplit = 1;
  if (ksplit > 1) {
    // C := Cold (unless C is Cold), D := 0 -- under the product's own condition
    if (g.Cold && g.Cold != g.C) {
      hipError_t e = launch_ewise(4, g.Cold, g.ldco, nullptr, 0, g.C, g.ldc, g.M, g.N, s, g.pred, g.pred_val);
      if (e != hipSuccess) return e;
    } else if (!g.Cold) {
      hipError_t e = launch_ewise(4, g.C, g.ldc, nullptr, 0, g.C, g.ldc, g.M, 0, s, g.pred, g.pred_val);  // zero C rows
      if (e != hipSuccess) return e;
    }
    if (g.D) {
      hipError_t e = launch_ewise(4, g.D, g.ldd, nullptr, 0, g.D, g.ldd, g.M, 0, s, g.pred, g.pred_val);  // zero D rows
      if (e != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL((k_gemm_valu<RPW, WPL>), dim3((unsigned)(tiles * ksplit)), dim3(256), 0, s, g.A, g.lda, g.B,
                     g.ldb, g.Cold, g.ldco, g.C, g.ldc, g.D, g.ldd, g.M, g.K, g.N, g.changed, (int)ksplit, (int)cps,
                     g.newbits, g.pred, g.pred_val);
  return hipGetLastError();
}

// Output tile of workgroup b.  Workgroups are dealt to the 8 XCDs round-robin (b mod 8), and each XCD
// has its own L2.  Orders:
//   0  row-major over the tiles: an XCD gets every row tile and an eighth of the column tiles;
//   1  contiguous: the workgroups of one XCD get a contiguous range of an order that walks groups of
//      ceil(rtiles / 2) row tiles column by column, so each XCD works on half of A's row tiles and a
//      quarter of B's column tiles (a 2 x 4 partition of the output);
//   2  interleaved: XCD x gets the tiles (tr, tc) with tr = x / 4 (mod 2) and tc = x (mod 4), walked in
//      groups of 8 of its row tiles, column by column: the same halving of each XCD's operand footprint,
//      while a block-structured product (its work in one corner) still spreads over all XCDs.  It needs
//      an even number of row tiles and a multiple of 4 column tiles, else order 1 is used;
//   3  column strips: XCD x gets the column tiles [x c/8, (x + 1) c/8) (c = ctiles) and walks them in
//      sub-strips of 8 columns, row by row, so the workgroups an XCD holds at once (one per CU, 32: four
//      rows of 8 columns) share 4 panels of A and 8 of B^T, and the 8 B^T panels of a sub-strip stay in
//      its L2 while the rows go by.  It needs multiples of 8 row tiles and of 64 column tiles, else order 1.
__device__ __forceinline__ void grouped(i64 li, i64 rows, i64 cols, i64 gmax, i64* i, i64* j) {
  const i64 gsz = rows < gmax ? rows : gmax;
  const i64 group = li / (gsz * cols), first = group * gsz;
  const i64 rin = rows - first < gsz ? rows - first : gsz;
  const i64 in = li - group * gsz * cols;
  *i = first + in % rin;
  *j = in / rin;
}
__device__ __forceinline__ void tile_of_block(i64 b, i64 rtiles, i64 ctiles, int order, i64* tr, i64* tc) {
  if (order == 3 && (rtiles & 7) == 0 && (ctiles & 63) == 0) {
    const i64 x = b & 7, li = b >> 3, cw = ctiles >> 3;
    const i64 sub = li / (rtiles * 8), rem = li - sub * rtiles * 8;
    *tr = rem >> 3;
    *tc = x * cw + sub * 8 + (rem & 7);
    return;
  }
  if (order == 2 && (rtiles & 1) == 0 && (ctiles & 3) == 0) {
    const i64 x = b & 7, li = b >> 3;
    i64 i, j;
    grouped(li, rtiles / 2, ctiles / 4, 8, &i, &j);
    *tr = 2 * i + (x >> 2);
    *tc = 4 * j + (x & 3);
    return;
  }
  if (order == 0) {
    *tr = b / ctiles;
    *tc = b % ctiles;
    return;
  }
  const i64 nb = rtiles * ctiles, per = nb / 8;
  const i64 bb = b < 8 * per ? (b % 8) * per + b / 8 : b;
  grouped(bb, rtiles, ctiles, (rtiles + 1) / 2, tr, tc);
}

template <int ORDER>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_gemm_mfma(MfmaTile g, const u32* __restrict__ pred, u32 pred_val) {
  __shared__ MfmaLds L;
  if (pred && *pred != pred_val) return;  // another arm serves this round
  const i64 rtiles = (g.M + kMT - 1) / kMT, ctiles = (g.N + kMT - 1) / kMT;
  i64 tr, tc;
  tile_of_block(blockIdx.x, rtiles, ctiles, ORDER, &tr, &tc);
  mfma_tile(L, g, tr, tc);
}

template <int KC, int SUB, int ORDER>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_gemm_mfma2(MfmaTile g, const u32* __restrict__ pred, u32 pred_val) {
  __shared__ Mfma2Lds<KC> L;
  if (pred && *pred != pred_val) return;  // another arm serves this round
  const i64 rtiles = (g.M + kMT - 1) / kMT, ctiles = (g.N + kMT - 1) / kMT;
  i64 tr, tc;
  tile_of_block(blockIdx.x, rtiles, ctiles, ORDER, &tr, &tc);
  mfma_tile2<KC, SUB>(L, g, tr, tc);
}

// The device-side choice of the next RMS squaring's route (see launch_rms_decide), the same rules the host
// driver applies: stop when the last squaring added nothing or R is all ones (its own square; the running
// count never exceeds R's bits, so it reaches n^2 only then); row gathers while they pay; the semi-naive
// form (driven by the host) when it may pay; else the dense product, unless the relabelling is still due.
__global__ void k_rms_decide(u32* __restrict__ recs, int t, i64 n, int mfma, int may_gather, int may_semi,
                             int dense_ok, i64 gather_max_n) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const unsigned long long* prev = (const unsigned long long*)(recs + (i64)(t - 1) * kRmsRecWords);
  unsigned long long* cur = (unsigned long long*)(recs + (i64)t * kRmsRecWords);
  const unsigned long long added = prev[0];
  const unsigned long long bits = prev[1] + added;
  cur[1] = bits;
  u32 route;
  if (added == 0 || bits >= (unsigned long long)n * (unsigned long long)n) route = RR_STOP;
  else if (may_gather && rms_gather_pays(n, (i64)bits, mfma != 0, gather_max_n)) route = RR_GATHER;
  else if (may_semi && rms_semi_may_pay(n, (i64)added, mfma != 0)) route = RR_HOST;
  else route = dense_ok ? RR_DENSE : RR_HOST;
  recs[(i64)t * kRmsRecWords + 4] = route;
  recs[(i64)t * kRmsRecWords + kRmsRecEarly] = rms_early_votes(n, (i64)bits) ? 1u : 0u;
}

}  // namespace

hipError_t launch_rms_decide(u32* recs, int t, i64 n, int mfma, int may_gather, int may_semi, int dense_ok,
                             i64 gather_max_n, hipStream_t s) {
  hipLaunchKernelGGL(k_rms_decide, dim3(1), dim3(64), 0, s, recs, t, n, mfma, may_gather, may_semi, dense_ok,
                     gather_max_n);
  return hipGetLastError();
}

i64 gemm_mfma_max_kwords() { return kMaxKWords; }

int gemm_mfma_variants() { return kMfmaVariants; }

bool gemm_mfma_variant_ok(int variant, const GemmArgs& g, const u64* BT, i64 ldbt) {
  if (variant < 0 || variant >= kMfmaVariants) return false;
  if (variant <= 2 || variant == 6) return true;
  // the second layout loads rows of A and B^T in 16-byte pieces
  return ((uintptr_t)g.A & 15u) == 0 && ((uintptr_t)BT & 15u) == 0 && (g.lda & 1) == 0 && (ldbt & 1) == 0;
}

hipError_t launch_gemm_mfma(const GemmArgs& g, const u64* BT, i64 ldbt, hipStream_t s, int variant) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  if (words_for(g.K) > kMaxKWords) return hipErrorInvalidValue;
  if (!gemm_mfma_variant_ok(variant, g, BT, ldbt)) variant = 0;
  const i64 tiles = ((g.M + kMT - 1) / kMT) * ((g.N + kMT - 1) / kMT);
  MfmaTile t{g.A, g.lda, BT, ldbt, g.Cold, g.ldco, g.C, g.ldc, g.D, g.ldd, g.M, g.K, g.N,
              g.changed, g.newbits, g.executed, nullptr};
  t.early_flag = g.early_flag;
  t.early = g.early ? 1u : 0u;
  const dim3 grid((unsigned)tiles), block(512);
  switch (variant) {
    case 6: hipLaunchKernelGGL((k_gemm_mfma<3>), grid, block, 0, s, t, g.pred, g.pred_val); break;
    case 7: hipLaunchKernelGGL((k_gemm_mfma2<8, 1, 3>), grid, block, 0, s, t, g.pred, g.pred_val); break;
    case 1: hipLaunchKernelGGL((k_gemm_mfma<1>), grid, block, 0, s, t, g.pred, g.pred_val); break;
    case 2: hipLaunchKernelGGL((k_gemm_mfma<2>), grid, block, 0, s, t, g.pred, g.pred_val); break;
    case 3: hipLaunchKernelGGL((k_gemm_mfma2<8, 1, 0>), grid, block, 0, s, t, g.pred, g.pred_val); break;
    case 4: hipLaunchKernelGGL((k_gemm_mfma2<8, 1, 1>), grid, block, 0, s, t, g.pred, g.pred_val); break;
    case 5: hipLaunchKernelGGL((k_gemm_mfma2<8, 1, 2>), grid, block, 0, s, t, g.pred, g.pred_val); break;
    default: hipLaunchKernelGGL((k_gemm_mfma<0>), grid, block, 0, s, t, g.pred, g.pred_val); break;
  }
  return hipGetLastError();
}


hipError_t launch_gemm_valu(const GemmArgs& g, hipStream_t s, int variant) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  constexpr i64 kTargetBlocks = 1024;  // 4 workgroups per CU on 256 CUs
  if (g.M <= 64) return launch_rpw<4>(g, s, kTargetBlocks);
  if (variant == 1) return launch_rpw<8>(g, s, kTargetBlocks);
  if (variant == 2) return launch_rpw<4>(g, s, kTargetBlocks);
  return launch_rpw<16>(g, s, kTargetBlocks);
}

}  // namespace bmlp
